"""The segmented float32 spread (large grids: one workgroup per segment of 2
tile columns by 4 or 8 tile rows, each sample used once per segment it
reaches, boundary rows carried in float between the segment's steps) against
the oracle's spread (the product Omega D fhat of eq:twodcgmatrix) on whole
windows that straddle segment and stripe boundaries, against the per-tile
kernel on the whole grid, and for run-to-run reproducibility.

Workloads: polar SAS rasters at n = 2048 (G = 4096, segments of 4 tile rows):
2^21 samples (about 300 records per tile) and 2^22 samples (about 600 per
tile, so a step's two tiles take several staging chunks).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_08575_amd import synth as S

pytestmark = pytest.mark.gpu

T = 32


def _raster(m, seed):
    q = 2048
    p = int(np.ceil(m / q))
    k, f, _ = S.make_sas(S.seed_for(2) + seed, n=2048, pulses=p, per_pulse=q, m=m)
    return k, f


def _spread(k, f, layout, n=2048):
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(n, dim=2, dtype="f32", weights="plain") as P:
        P.set_spread_layout(layout)
        P.set_points(torch.from_numpy(np.ascontiguousarray(k)).cuda())
        H = P.spread_only(torch.from_numpy(f).to(torch.complex64).cuda())
        a = P.get_weights()
        torch.cuda.synchronize()
        return H, a.cpu().numpy()


@pytest.mark.parametrize("m,seed", [(1 << 21, 1), (1 << 22, 2)])
def test_segments_match_oracle_windows_and_tile_kernel(m, seed):
    k, f = _raster(m, seed)
    n, G = 2048, 4096
    K = 4                       # segment rows at G = 4096 (2048 workgroups)
    Hs, a = _spread(k, f, "auto")
    Ht, a2 = _spread(k, f, "tiles")
    assert np.array_equal(a, a2)
    # whole grid: the two layouts differ by the carried rows' float rounding
    # and by each step's fixed-point quantum
    d = torch.linalg.vector_norm(Hs - Ht).item() / torch.linalg.vector_norm(Ht).item()
    print(f"m = {m}: segmented vs per-tile rel L2 {d:.2e}")
    assert d < 1e-6
    # 48 x 80 windows centred on segment corners (rows k K T, columns 2 j T),
    # on stripe edges inside a segment, and on the busiest tile
    u = np.mod(2.0 * k + G / 2, G)
    busy = np.bincount((u[:, 0] // T).astype(np.int64) * (G // T) + (u[:, 1] // T).astype(np.int64),
                       minlength=(G // T) ** 2)
    rng = np.random.default_rng(seed)
    centres = []
    occupied = np.nonzero(busy)[0]
    for t in rng.choice(occupied, 12, replace=False).tolist() + [int(np.argmax(busy))]:
        tr, tc = t // (G // T), t % (G // T)
        centres.append(((tr // K) * K * T, (tc // 2) * 2 * T))         # segment corner
        centres.append((tr * T + T // 2, (tc // 2) * 2 * T + T))        # stripe's inner edge
    c = a * f
    num = den = 0.0
    worst = 0.0
    h, w = 48, 80
    for (r, cc) in centres:
        r0 = int(np.clip(r - h // 2, 0, G - h))
        c0 = int(np.clip(cc - w // 2, 0, G - w))
        got = Hs[r0:r0 + h, c0:c0 + w].cpu().numpy()
        ref = O.spread_window(k, c, n, r0, c0, h, w)
        e = np.linalg.norm(got - ref)
        nr = np.linalg.norm(ref)
        num += e * e
        den += nr * nr
        if nr > 0:
            worst = max(worst, e / nr)
    tot = float(np.sqrt(num / den))
    print(f"m = {m}: {len(centres)} boundary windows, rel L2 {tot:.2e}, worst {worst:.2e}")
    assert tot < 2e-5
    assert worst < 1e-4


def test_segments_bitwise_reproducible_after_rebinning():
    from paper_1706_08575_amd.ftcg import Plan
    k, f = _raster(1 << 21, 3)
    kd = torch.from_numpy(np.ascontiguousarray(k)).cuda()
    fd = torch.from_numpy(f).to(torch.complex64).cuda()
    with Plan(2048, dim=2, dtype="f32", weights="plain") as P:
        P.set_points(kd)
        h1 = P.spread_only(fd).clone()
        i1 = P.execute(fd).clone()
        P.set_points(kd)
        h2 = P.spread_only(fd)
        i2 = P.execute(fd)
        torch.cuda.synchronize()
        assert torch.equal(h1, h2)
        assert torch.equal(i1, i2)


def test_segments_non_finite_value_stays_local():
    # a NaN sample value poisons the step that holds it (its 64 columns and
    # the rows of that step) and nothing far away, as the per-tile kernel
    # poisons its tile
    k, f = _raster(1 << 20, 4)
    G = 4096
    j = 12345
    f = f.copy()
    f[j] = np.nan
    Hs, _ = _spread(k, f, "auto")
    H = Hs.cpu().numpy()
    u = np.mod(2.0 * k[j] + G / 2, G)
    r, c = int(u[0]), int(u[1])
    assert np.isnan(H[r, c]).any()
    far = np.ones((G, G), dtype=bool)
    far[max(0, r - 80):r + 80, max(0, c - 140):c + 140] = False
    assert np.isfinite(H[far]).all()


@pytest.mark.parametrize("case", ["single", "corners", "wrapped"])
def test_segments_sparse_and_wrapped(case):
    # degenerate inputs on the segmented layout (n = 2048, G = 4096): one
    # sample; samples on segment corners and stripe edges (every other step
    # and segment empty); a raster whose samples lie up to 2.2 n outside the
    # k-box, so that their taps wrap around the grid edges. Every cell against
    # the per-tile kernel, the cells near the samples against the oracle.
    n, G, T, K = 2048, 4096, 32, 4
    rng = np.random.default_rng(17)
    if case == "single":
        u = np.array([[1234.3, 2999.7]])
    elif case == "corners":
        pts = []
        for r in (K * T * 3, K * T * 7 - 1, K * T * 11 + 0.5):
            for c in (2 * T * 5, 2 * T * 9 - 1, 2 * T * 20 + 0.25, 0.0, G - 0.5):
                pts.append([r + rng.uniform(-0.5, 0.5), c])
        u = np.array(pts)
    else:
        u = rng.uniform(0, G, size=(3000, 2))
    k = (u - G / 2) / 2.0
    if case == "wrapped":
        k += rng.integers(-2, 3, size=k.shape) * n * 1.1
    f = (rng.standard_normal(len(k)) + 1j * rng.standard_normal(len(k))).astype(np.complex128)
    Hs, a = _spread(k, f, "auto")
    Ht, _ = _spread(k, f, "tiles")
    d = torch.linalg.vector_norm(Hs - Ht).item() / torch.linalg.vector_norm(Ht).item()
    assert d < 1e-6, d
    c = a * f
    uu = np.mod(2.0 * k + G / 2, G)
    num = den = 0.0
    for (r, cc) in uu[:40]:
        r0 = int(np.clip(int(r) - 16, 0, G - 32))
        c0 = int(np.clip(int(cc) - 16, 0, G - 32))
        got = Hs[r0:r0 + 32, c0:c0 + 32].cpu().numpy()
        ref = O.spread_window(k, c, n, r0, c0, 32, 32)
        num += np.linalg.norm(got - ref) ** 2
        den += np.linalg.norm(ref) ** 2
    err = float(np.sqrt(num / den))
    print(f"{case}: vs per-tile {d:.2e}, windows vs oracle {err:.2e}")
    assert err < 2e-5
