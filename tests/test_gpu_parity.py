"""GPU parity of the HIP path against the CPU FP64 oracle, through the C ABI.

Tolerances:
  * float64 plans: the only differences from the oracle are rounding order
    and the tap at distance exactly W when u is integral (weight
    exp(-beta W^2) ~ 7e-7, absent for generic inputs), so 1e-9 rel L2.
  * float32 plans: the spec bar, 1e-4 rel L2 against the FP64 oracle;
    the measured error is ~1e-6, so a tighter 2e-5 is asserted where the
    inputs are generic.
  * weights are float64 on both sides; the HIP path forms sin(pi (k_i - k_j))
    from per-sample sin and cos, whose rounding differs from the oracle's direct
    sinc by ~1e-12 relative at worst: 1e-10 relative.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_08575_amd import synth as S

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-9
TOL_F32 = 2e-5
TOL_PATH = 1e-4   # the whole path against the float64 oracle


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def plan(n, dim, dtype, weights="plain", **kw):
    from paper_1706_08575_amd.ftcg import Plan
    return Plan(n, dim=dim, dtype=dtype, weights=weights, **kw)


def run(k, f, n, dtype="f32", weights="plain", alpha=None, tune=None, **kw):
    dim = k.shape[1]
    with plan(n, dim, dtype, weights, **kw) as P:
        if tune:
            P.set_tuning(*tune)
        P.set_points(dev(k))
        if weights == "user":
            P.set_weights(dev(alpha))
        cd = torch.complex64 if dtype == "f32" else torch.complex128
        img = host(P.execute(dev(f, cd)))
        a = host(P.get_weights())
        info = P.info()
    return img, a, info


# ---------------------------------------------------------------------------
# 1D, float64 (the jittered-raster workload)
# ---------------------------------------------------------------------------

def test_1d_f64_weights_and_image():
    k, f, _ = S.make_1d()
    img, a, _ = run(k, f, 256, "f64")
    a_ref = O.frame_weights(k, 8.0)
    assert np.max(np.abs(a - a_ref) / a_ref) < 1e-10
    ref = O.ftcg_image(k, f, a_ref, 256)
    assert O.rel_l2(img, ref) < TOL_F64


def test_1d_f32_image():
    k, f, _ = S.make_1d()
    img, a, _ = run(k, f, 256, "f32")
    ref = O.ftcg_image(k, f, O.frame_weights(k, 8.0), 256)
    assert O.rel_l2(img, ref) < TOL_F32


# ---------------------------------------------------------------------------
# 2D polar-format SAS, 512 x 512 (the plain workload), float32 and float64
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sas512():
    k, f, _ = S.workload_2d_plain()
    a = O.frame_weights(k, 8.0)
    ref = O.ftcg_image(k, f, a, 512)
    return k, f, a, ref


def test_2d_plain_weights(sas512):
    k, f, a_ref, _ = sas512
    _, a, _ = run(k, f, 512, "f32")
    assert np.max(np.abs(a - a_ref) / a_ref) < 1e-10


def test_2d_plain_f32_image(sas512):
    k, f, a_ref, ref = sas512
    img, _, info = run(k, f, 512, "f32")
    err = O.rel_l2(img, ref)
    print(f"2D 512 f32 rel L2 = {err:.3e}, records = {info['n_records']}")
    assert err < TOL_F32


def test_2d_plain_f64_image(sas512):
    k, f, a_ref, ref = sas512
    img, _, _ = run(k, f, 512, "f64")
    assert O.rel_l2(img, ref) < TOL_F64


@pytest.mark.parametrize("tile,accum,copies", [(16, "fixed", 1), (32, "fixed", 1), (64, "fixed", 1),
                                               (128, "fixed", 1), (16, "f64", 1), (32, "f64", 4),
                                               (64, "f64", 1), (64, "f64", 2)])
def test_2d_tilings_agree(sas512, tile, accum, copies):
    k, f, a_ref, ref = sas512
    img, _, info = run(k, f, 512, "f32", tune=(tile, accum, copies))
    assert info["tile"] == tile
    assert O.rel_l2(img, ref) < TOL_F32


def test_tiling_beyond_lds_rejected():
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(512, dim=2) as P:
        for tile, accum, copies in ((128, "f64", 1), (64, "f64", 4), (64, "fixed", 2)):
            with pytest.raises(L.FtcgError) as e:
                P.set_tuning(tile, accum, copies)
            assert e.value.status == L.FTCG_EUNSUPPORTED
        # accumulation code 2 (a matrix-core variant, measured and dropped) is not accepted
        assert L.call("ftcg_plan_set_tuning", P._h, 64, 2, 1) == L.FTCG_EINVAL
    with Plan(64, dim=2, dtype="f64") as P:
        with pytest.raises(L.FtcgError) as e:
            P.set_tuning(64, "fixed", 1)
        assert e.value.status == L.FTCG_EUNSUPPORTED


def test_fixed_accumulation_is_bitwise_reproducible(sas512):
    # integer accumulation does not depend on the order records are binned in
    k, f, _, _ = sas512
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(512, dim=2) as P:
        P.set_tuning(64, "fixed", 1)
        ff = dev(f, torch.complex64)
        P.set_points(dev(k))
        a = host(P.execute(ff))
        P.set_points(dev(k))        # re-binned (atomic slot order may differ)
        b = host(P.execute(ff))
    assert np.array_equal(a, b)


def test_2d_spread_step_vs_oracle():
    k, f, _ = S.make_sas(21, 128, 64, 128)
    n = 128
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(n, dim=2, dtype="f64", weights="none") as P:
        P.set_points(dev(k))
        H = host(P.spread_only(dev(f)))
    Href = O.spread(k, f, n)
    assert O.rel_l2(H, Href) < TOL_F64


@pytest.mark.parametrize("tile", [16, 32, 64, 128])
def test_2d_spread_fixed_dense_tiles_vs_oracle(tile):
    # fixed-point accumulation with a dense cluster (thousands of records in
    # a few tiles: many LDS staging chunks of records per tile, the last one
    # ragged) beside sparse tiles and samples on the periodic seam; tile 128
    # leaves no LDS room for staging and reads the records directly
    from paper_1706_08575_amd.ftcg import Plan
    rng = np.random.default_rng(24)
    n = 128
    kd = rng.uniform(-6.0, 6.0, size=(6001, 2)) + np.array([10.3, -20.7])
    ks = rng.uniform(-0.6 * n, 0.6 * n, size=(1500, 2))
    ks[:20, 1] = -n / 2 + 0.01 * rng.random(20)
    k = np.vstack([kd, ks])
    f = S.random_values(25, k.shape[0])
    with Plan(n, dim=2, dtype="f32", weights="none") as P:
        P.set_tuning(tile, "fixed", 1)
        P.set_points(dev(k))
        ff = dev(f, torch.complex64)
        H = host(P.spread_only(ff))
        P.set_points(dev(k))        # re-binned: the integer sums do not depend on record order
        H2 = host(P.spread_only(ff))
    assert np.array_equal(H, H2)
    Href = O.spread(k, f, n)
    assert O.rel_l2(H, Href) < TOL_PATH


def test_plan_autotuner(tmp_path, monkeypatch):
    # the tuner times every candidate launch on the caller's data, leaves the
    # plan on the fastest, and the result stays within the float32 bar
    monkeypatch.setenv("FTCG_TUNING_CACHE", str(tmp_path / "tune.json"))
    from paper_1706_08575_amd import autotune
    from paper_1706_08575_amd.ftcg import Plan
    k, f, _ = S.make_sas(41, 128, 64, 256)
    with Plan(128, dim=2) as P:
        best, ms = autotune.tune_plan(P, dev(k), dev(f, torch.complex64), reps=1)
        assert "32/fixed" in ms and "64/fixed" in ms
        assert best in {tuple([int(a.split("/")[0]), a.split("/")[1]]) for a in ms}
        img = host(P.execute(dev(f, torch.complex64)))
        again, _ = autotune.tune_plan(P, dev(k), dev(f, torch.complex64))   # from the cache
        assert again == best
    ref = O.ftcg_image(k, f, O.frame_weights(k, 8.0), 128)
    assert O.rel_l2(img, ref) < TOL_F32


def test_2d_fft_step_vs_oracle():
    rng = np.random.default_rng(3)
    n, G = 64, 128
    H = (rng.standard_normal((G, G)) + 1j * rng.standard_normal((G, G)))
    from paper_1706_08575_amd.ftcg import Plan
    for dtype, tol in (("f64", 1e-12), ("f32", 2e-6)):
        with Plan(n, dim=2, dtype=dtype, weights="none") as P:
            cd = torch.complex64 if dtype == "f32" else torch.complex128
            img = host(P.grid_to_image(dev(H, cd)))
        assert O.rel_l2(img, O.grid_to_image(H, n)) < tol, dtype


@pytest.mark.parametrize("n", [8, 16, 32, 256, 1024, 2048])
def test_fft_lengths(n):
    # every supported row length (G = 2n), odd and even log2
    rng = np.random.default_rng(n)
    G = 2 * n
    H = rng.standard_normal((G, G)) + 1j * rng.standard_normal((G, G))
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(n, dim=2, dtype="f32", weights="none") as P:
        img = host(P.grid_to_image(dev(H, torch.complex64)))
    assert O.rel_l2(img, O.grid_to_image(H, n)) < 3e-6


@pytest.mark.parametrize("dim,n,dtype", [(2, 2048, "f64"), (2, 1024, "f64"), (1, 4096, "f32"), (1, 2048, "f64"),
                                         (1, 256, "f32"), (1, 8192, "f32")])
def test_fft_row_shapes(dim, n, dtype):
    # row lengths whose passes run with the first and last stage in registers
    # and two LDS row buffers (2D float64 at G = 4096, 1D rows of 512 .. 8192
    # points in float32 and 4096 in float64), next to ones that do not
    # (2D float64 at G = 2048, 1D 16384 points), against the oracle
    rng = np.random.default_rng(1000 * dim + n)
    G = 2 * n
    shape = (G,) * dim
    H = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    from paper_1706_08575_amd.ftcg import Plan
    cd = torch.complex64 if dtype == "f32" else torch.complex128
    with Plan(n, dim=dim, dtype=dtype, weights="none") as P:
        img = host(P.grid_to_image(dev(H, cd)))
    tol = 3e-6 if dtype == "f32" else 1e-12
    assert O.rel_l2(img, O.grid_to_image(H, n)) < tol


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_single_sample_and_user_weights():
    k = np.array([[0.3, -1.7]])
    f = np.array([2.0 - 1.0j])
    img, a, _ = run(k, f, 32, "f64", weights="user", alpha=np.array([0.25]))
    assert a[0] == 0.25
    assert O.rel_l2(img, O.ftcg_image(k, f, np.array([0.25]), 32)) < TOL_F64


def test_outside_box_wraps_and_tile_borders():
    # samples far outside the k-box, and samples whose grid position sits
    # exactly on tile borders (u = multiple of 64) and on integers
    rng = np.random.default_rng(5)
    n = 64
    k = rng.uniform(-2.2 * n, 2.2 * n, size=(3000, 2))
    k[:50] = (64.0 * rng.integers(0, 2, size=(50, 2)) - n) / 2.0      # u = 0 or 64
    k[50:100] = np.round(k[50:100] * 2.0) / 2.0                         # integral u
    f = S.random_values(6, 3000)
    alpha = rng.uniform(0.5, 1.5, size=3000)
    ref = O.ftcg_image(k, f, alpha, n)
    img, _, _ = run(k, f, n, "f64", weights="user", alpha=alpha)
    # integral u drops one tap of weight e^{-beta W^2} per axis in the HIP path
    assert O.rel_l2(img, ref) < 1e-6
    img32, _, _ = run(k, f, n, "f32", weights="user", alpha=alpha)
    assert O.rel_l2(img32, ref) < TOL_PATH


def test_weights_none_and_lattice():
    # integer lattice: plain weights are exactly 1
    j0, j1 = np.meshgrid(np.arange(32) - 16, np.arange(32) - 16, indexing="ij")
    k = np.stack([j0.ravel(), j1.ravel()], axis=1).astype(np.float64)
    f = S.random_values(7, k.shape[0])
    img, a, _ = run(k, f, 32, "f64")
    assert np.max(np.abs(a - 1.0)) < 1e-14
    img1, a1, _ = run(k, f, 32, "f64", weights="none")
    assert np.all(a1 == 1.0)
    assert O.rel_l2(img, img1) < 1e-13


def test_weights_shared_coordinates_and_duplicates():
    # tensor raster of jittered axes: most pairs share one coordinate exactly
    # (sinc factor exactly 1 on that axis); 20 points repeated bit for bit
    rng = np.random.default_rng(12)
    xa = np.sort(rng.uniform(-20.0, 20.0, 40))
    ya = np.sort(rng.uniform(-20.0, 20.0, 40))
    x0, x1 = np.meshgrid(xa, ya, indexing="ij")
    k = np.stack([x0.ravel(), x1.ravel()], axis=1)
    k = np.concatenate([k, k[rng.choice(k.shape[0], 20, replace=False)]])
    f = S.random_values(13, k.shape[0])
    _, a, _ = run(k, f, 64, "f64")
    a_ref = O.frame_weights(k, 8.0)
    assert np.max(np.abs(a - a_ref) / a_ref) < 1e-10
    # the same in 1D, with repeated values
    k1 = np.concatenate([xa, xa[:7]])[:, None]
    f1 = S.random_values(14, k1.shape[0])
    _, a1, _ = run(k1, f1, 64, "f64")
    a1_ref = O.frame_weights(k1, 8.0)
    assert np.max(np.abs(a1 - a1_ref) / a1_ref) < 1e-10


def test_nonfinite_points_rejected():
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    k = np.zeros((10, 2))
    k[3, 1] = np.nan
    with Plan(32, dim=2) as P:
        with pytest.raises(L.FtcgError) as e:
            P.set_points(dev(k))
        assert e.value.status == L.FTCG_EINVAL
        import ctypes as C
        f = dev(np.zeros(10, np.complex64))
        img = torch.empty((32, 32), dtype=torch.complex64, device="cuda")
        st = L.call("ftcg_execute", P._h, C.c_void_p(f.data_ptr()), C.c_void_p(img.data_ptr()))
        assert st == L.FTCG_ESTATE


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf, 2.0 ** 41, -1e300])
@pytest.mark.parametrize("n,dim,weights", [(32, 2, "plain"), (4096, 2, "plain"), (64, 1, "plain"),
                                           (32, 2, "none")])
def test_rejected_points_then_recovery(bad, n, dim, weights):
    # the binning passes enqueued before the host reads the check run on the
    # rejected points too (fused tile/bin-row binning on the small 2D grid,
    # tile counting on the 65 536-tile grid, the whole tile binning in 1D and
    # without weights); the call reports FTCG_EINVAL, and the plan then takes
    # valid points and matches the oracle
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    rng = np.random.default_rng(5)
    m = 600
    k = rng.uniform(-12.0, 12.0, size=(m, dim))
    kb = k.copy()
    kb[17, dim - 1] = bad
    f = S.random_values(6, m)
    with Plan(n, dim=dim, dtype="f64", weights=weights) as P:
        with pytest.raises(L.FtcgError) as e:
            P.set_points(dev(kb))
        assert e.value.status == L.FTCG_EINVAL
        P.set_points(dev(k))
        a = host(P.get_weights())
        if n <= 64:
            img = host(P.execute(dev(f, torch.complex128)))
    a_ref = O.frame_weights(k, 8.0) if weights == "plain" else np.ones(m)
    assert np.max(np.abs(a - a_ref) / a_ref) < 1e-10
    if n <= 64:
        assert O.rel_l2(img, O.ftcg_image(k, f, a_ref, n)) < TOL_F64


@pytest.mark.parametrize("tile", [32, 128])
def test_deferred_weights_match_finished(sas512, tile):
    # on fused-binning grids the fixed-point spread forms each record's weight
    # from the weight sums; after get_weights the records carry the finished
    # weights and the spread reads those: the same float64 division, so the
    # two images agree bitwise (one set_points, one set of sums)
    k, f, a_ref, ref = sas512
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(512, dim=2, dtype="f32", weights="plain") as P:
        P.set_tuning(tile, "fixed", 1)
        P.set_points(dev(k))
        ff = dev(f, torch.complex64)
        img_deferred = host(P.execute(ff))
        a = host(P.get_weights())
        img_finished = host(P.execute(ff))
    assert np.array_equal(img_deferred, img_finished)
    assert np.max(np.abs(a - a_ref) / a_ref) < 1e-10
    assert O.rel_l2(img_deferred, ref) < TOL_F32


def test_long_bin_row_bitwise_and_oracle():
    # 20 000 samples in a band half a cycle high: one bin row holds nearly all
    # of them, more than the row sort orders in LDS, so its bins are put in
    # caller-index order by the separate pass for long rows. The weights are
    # bitwise equal after re-binning and agree with the oracle.
    rng = np.random.default_rng(77)
    m = 20000
    k = np.stack([rng.uniform(0.0, 0.5, m), rng.uniform(-200.0, 200.0, m)], axis=1)
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(512, dim=2) as P:
        P.set_points(dev(k))
        wa = host(P.get_weights())
        P.set_points(dev(k))
        wb = host(P.get_weights())
    assert np.array_equal(wa, wb)
    a_ref = O.frame_weights(k, 8.0)
    assert np.max(np.abs(wa - a_ref) / a_ref) < 1e-10


@pytest.mark.parametrize("n,pulses,per_pulse,spl,lpg",
                         [(128, 64, 128, 0, 0), (256, 256, 512, 2, 0), (256, 256, 512, 2, 2),
                          (256, 256, 512, 4, 0)])
def test_repeat_is_bitwise_stable(n, pulses, per_pulse, spl, lpg):
    # Run to run, and across re-binning (atomic slot claims reorder samples
    # within their bins and records within their tiles), the weights and the
    # image are bitwise equal: the bin sort puts every bin in caller-index
    # order, a lane's own sums add its pairs in an order fixed by its group,
    # whichever lane takes the group, and round once; the candidate slots and
    # the global sums add terms rounded to a common quantum (exact float64
    # additions, so the atomics' order cannot matter); the spread adds exact
    # integers. spl selects the symmetric (2) and the one-sided (4) weight
    # kernels at 2^17 samples; lpg = 2 takes the symmetric kernel with two
    # lanes per group, whose runs order their groups by work through LDS
    # atomics (the instance of rasters of 2^21 samples and more).
    k, f, _ = S.make_sas(31, n, pulses, per_pulse)
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(n, dim=2) as P:
        if spl:
            P.set_weight_tuning(spl, lpg)
        ff = dev(f, torch.complex64)
        P.set_points(dev(k))
        a = host(P.execute(ff))
        wa = host(P.get_weights())
        b = host(P.execute(ff))
        P.set_points(dev(k))
        wb = host(P.get_weights())
        c = host(P.execute(ff))
    assert np.array_equal(a, b)
    assert np.array_equal(wa, wb)
    assert np.array_equal(a, c)
    a_ref = O.frame_weights(k, 8.0)
    assert np.max(np.abs(wa - a_ref) / a_ref) < 1e-10
