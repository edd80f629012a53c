"""GPU parity of the forward (type-2) transform, ftcg_forward, the adjoint of
the reconstruction (Omega^T after the forward DFT of the deapodized,
zero-padded image; eq:cgmatrix), against the FP64 oracle (oracle.forward,
the same steps in float64; oracle.nudft_forward, the direct sum it
approximates).

Tolerances: float64 plans 1e-9 rel L2 against oracle.forward; float32 plans
2e-5 (spec bar 1e-4); against the direct sum 1e-4 (kernel error of
W = 6, sigma = 2 is about 1e-6). Adjointness with the GPU's own
reconstruction, <A c, I> = <c, A^H I>: in float64 to 1e-12 of the product;
in float32 the two products differ by at most 2e-5 (|A c| |I| + |c| |A^H I|)
when each operator meets the 2e-5 float32 bar (Cauchy-Schwarz on each
side's error). That bound, not a fixed fraction of the product, is the
float32 tolerance: the products cancel heavily (on the test's data
|A c| |I| is about 950 times |<A c, I>|), so rounding that is well inside
the bar can move them by 1e-5 of their size.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_08575_amd import synth as S

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _image(n, d, seed):
    rng = np.random.default_rng(seed)
    shape = (n,) * d
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def run_forward(k, img, n, dtype="f32", tile=0):
    from paper_1706_08575_amd.ftcg import Plan
    cd = torch.complex64 if dtype == "f32" else torch.complex128
    with Plan(n, dim=k.shape[1], dtype=dtype, weights="none") as P:
        if tile:
            P.set_tuning(tile, "fixed" if dtype == "f32" else "f64", 1)
        P.set_points(dev(k))
        return host(P.forward(dev(img, cd)))


def test_forward_1d_f64():
    k, _, _ = S.make_1d()
    k = k.copy()
    k[:5, 0] += 256.0                    # outside the k-box: wraps
    img = _image(256, 1, 1)
    got = run_forward(k, img, 256, "f64")
    assert O.rel_l2(got, O.forward(k, img, 256)) < 1e-9
    assert O.rel_l2(got, O.nudft_forward(k, img)) < 1e-5


@pytest.mark.parametrize("tile", [16, 32, 64, 128])
def test_forward_2d_f32_tilings(tile):
    k, _, _ = S.make_sas(S.seed_for(1) + 60, n=128, pulses=64, per_pulse=128)
    k = k.copy()
    k[:20, 1] = 64.0 - 0.01 * np.arange(20)   # next to the periodic seam
    img = _image(128, 2, 2)
    got = run_forward(k, img, 128, "f32", tile)
    err = O.rel_l2(got, O.forward(k, img, 128))
    assert err < 2e-5, err
    assert O.rel_l2(got, O.nudft_forward(k, img)) < 1e-4


def test_forward_2d_f64():
    k, _, _ = S.make_sas(S.seed_for(1) + 61, n=64, pulses=32, per_pulse=64)
    img = _image(64, 2, 3)
    got = run_forward(k, img, 64, "f64")
    assert O.rel_l2(got, O.forward(k, img, 64)) < 1e-9


@pytest.mark.parametrize("dtype,tol", [("f32", 2e-5), ("f64", 1e-12)])
def test_forward_is_adjoint_of_execute(dtype, tol):
    # <A c, I> = <c, A^H I>, A = the GPU reconstruction with unit weights
    from paper_1706_08575_amd.ftcg import Plan
    k, _, _ = S.make_sas(S.seed_for(1) + 62, n=128, pulses=64, per_pulse=128)
    c = S.random_values(63, len(k))
    img = _image(128, 2, 4)
    cd = torch.complex64 if dtype == "f32" else torch.complex128
    with Plan(128, dim=2, dtype=dtype, weights="none") as P:
        P.set_points(dev(k))
        Ac = host(P.execute(dev(c, cd))).astype(np.complex128)
        AhI = host(P.forward(dev(img, cd))).astype(np.complex128)
    c = c.astype(np.complex64 if dtype == "f32" else np.complex128).astype(np.complex128)
    im = img.astype(np.complex64 if dtype == "f32" else np.complex128).astype(np.complex128)
    lhs = np.vdot(Ac, im)
    rhs = np.vdot(c, AhI)
    if dtype == "f64":
        assert abs(lhs - rhs) < tol * abs(lhs)
    else:
        scale = np.linalg.norm(Ac) * np.linalg.norm(im) + np.linalg.norm(c) * np.linalg.norm(AhI)
        print(f"adjoint f32: |lhs - rhs| = {abs(lhs - rhs):.3e}, |lhs| = {abs(lhs):.3e}, bound {tol * scale:.3e}")
        assert abs(lhs - rhs) < tol * scale


def test_forward_before_points_is_a_state_error():
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(64, dim=2) as P:
        P.m = 4
        with pytest.raises(L.FtcgError) as e:
            P.forward(torch.zeros((64, 64), dtype=torch.complex64, device="cuda"))
        assert e.value.status == L.FTCG_ESTATE


def test_forward_full_size_sampled():
    # the 4096^2 workload's raster (8 388 608 samples): 512 seeded samples
    # against the oracle's forward transform (its full 8192^2 grid in float64)
    from paper_1706_08575_amd.ftcg import Plan
    import os
    k, _, _ = S.workload_2d_precision()
    n = 4096
    rng = np.random.default_rng(40)
    x = (np.arange(n) - n / 2) / n
    env = np.exp(-(x[:, None] ** 2 + x[None, :] ** 2) / 0.05)
    img = (env * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))).astype(np.complex64)
    with Plan(n, dim=2, dtype="f32", weights="none") as P:
        P.set_points(dev(k))
        got = host(P.forward(dev(img)))
    idx = rng.choice(len(k), 512, replace=False)
    H = O.image_to_grid(img.astype(np.complex128), n, workers=os.cpu_count() or 1)
    ref = O.interpolate(k[idx], H)
    err = O.rel_l2(got[idx], ref)
    print(f"full-size forward: 512 sampled values, rel L2 {err:.2e}")
    assert err < 2e-5
