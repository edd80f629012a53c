"""Full-size parity: the 2048 x 4096-sample polar SAS raster (8 388 608
samples, 4096^2 image), in the plan configuration bench.py times, checked
against the oracle on sampled outputs it can compute one by one.

  * weights of 256 seeded samples against the oracle's per-sample
    eq:difopt sum (k-d tree neighbourhoods), 1e-10 relative;
  * image pixels against the exact weighted type-1 sum (the NUDFT of
    Sec. III-A that gridding approximates) at 24 seeded pixels and the 4
    brightest ones, with the GPU weights validated above: the float32
    spec bar, 1e-4 relative L2 over the sampled pixels (the kernel
    error of W = 6, sigma = 2 and float32 rounding are both far below it).
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_08575_amd import synth as S

pytestmark = pytest.mark.gpu


def test_full_size_4096_sampled():
    from paper_1706_08575_amd.ftcg import Plan
    k, f, _ = S.workload_2d_precision()
    n = 4096
    kd = torch.from_numpy(np.ascontiguousarray(k)).cuda()
    fd = torch.from_numpy(f).to(torch.complex64).cuda()
    with Plan(n, dim=2, dtype="f32", weights="plain") as P:
        P.set_points(kd)
        img = P.execute(fd)
        torch.cuda.synchronize()
        img = img.cpu().numpy()
        a = P.get_weights().cpu().numpy()
    rng = np.random.default_rng(4096)
    idx = rng.choice(k.shape[0], 256, replace=False)
    a_ref = O.frame_weights_at(k, idx, 8.0)
    assert np.max(np.abs(a[idx] - a_ref) / a_ref) < 1e-10
    mag = np.abs(img)
    top = np.argsort(mag.ravel())[-4:]
    pix = np.concatenate([rng.integers(0, n * n, 24), top])
    p0, p1 = pix // n, pix % n
    x = np.stack([(p0 - n // 2) / n, (p1 - n // 2) / n], axis=1)
    ref = O.nudft_at(k, a * f, x)
    got = img[p0, p1]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-4


def test_full_size_4096_spread_tiles():
    # every cell of 64 seeded 32 x 32 tiles of the 8192^2 oversampled grid
    # (spread of alpha * fhat, eq:twodcgmatrix), in the launch the step uses,
    # against the oracle's spread restricted to those tiles; tiles drawn among
    # those the sector reaches, plus the 8 with the most samples
    from paper_1706_08575_amd.ftcg import Plan
    k, f, _ = S.workload_2d_precision()
    n, G, T = 4096, 8192, 32
    kd = torch.from_numpy(np.ascontiguousarray(k)).cuda()
    fd = torch.from_numpy(f).to(torch.complex64).cuda()
    u = np.mod(2.0 * k + G / 2, G)
    tid = (u[:, 0] // T).astype(np.int64) * (G // T) + (u[:, 1] // T).astype(np.int64)
    cnt = np.bincount(tid, minlength=(G // T) ** 2)
    rng = np.random.default_rng(8192)
    busy = np.nonzero(cnt)[0]
    tiles = np.concatenate([rng.choice(busy, 56, replace=False), np.argsort(cnt)[-8:]])
    with Plan(n, dim=2, dtype="f32", weights="plain") as P:
        P.set_points(kd)
        H = P.spread_only(fd)
        a = P.get_weights()
        blocks = torch.stack([H[(t // (G // T)) * T:(t // (G // T) + 1) * T, (t % (G // T)) * T:(t % (G // T) + 1) * T]
                              for t in tiles.tolist()])
        torch.cuda.synchronize()
        blocks = blocks.cpu().numpy()
        a = a.cpu().numpy()
    c = a * f
    errs = []
    num = den = 0.0
    for b, t in enumerate(tiles.tolist()):
        r0, c0 = (t // (G // T)) * T, (t % (G // T)) * T
        ref = O.spread_window(k, c, n, r0, c0, T, T)
        e = np.linalg.norm(blocks[b] - ref)
        num += e * e
        den += np.linalg.norm(ref) ** 2
        errs.append(e / np.linalg.norm(ref))
    tot = float(np.sqrt(num / den))
    print(f"64 tiles of the 8192^2 grid: rel L2 {tot:.2e}, worst tile {max(errs):.2e}")
    assert tot < 2e-5
    assert max(errs) < 1e-4


def test_full_size_spread_is_bitwise_reproducible():
    # the 4096^2 workload's spread (fixed-point tiles, more than 256 records
    # in most of them, so staged in two chunks) is bitwise the same after
    # re-binning, which may place the records of a tile in another order
    from paper_1706_08575_amd.ftcg import Plan
    k, f, _ = S.workload_2d_precision()
    kd = torch.from_numpy(np.ascontiguousarray(k)).cuda()
    fd = torch.from_numpy(f).to(torch.complex64).cuda()
    with Plan(4096, dim=2, dtype="f32", weights="plain") as P:
        P.set_points(kd)
        h1 = P.spread_only(fd).clone()
        P.set_points(kd)
        h2 = P.spread_only(fd)
        torch.cuda.synchronize()
        assert torch.equal(h1, h2)


def test_full_size_weights_are_bitwise_reproducible():
    # the 4096^2 workload's frame weights (symmetric kernel, two samples per
    # lane, two lanes per group, groups ordered by work in each run) are
    # bitwise the same after re-binning
    from paper_1706_08575_amd.ftcg import Plan
    k, _, _ = S.workload_2d_precision()
    kd = torch.from_numpy(np.ascontiguousarray(k)).cuda()
    with Plan(4096, dim=2, dtype="f32", weights="plain") as P:
        P.set_points(kd)
        w1 = P.get_weights().clone()
        P.set_points(kd)
        w2 = P.get_weights()
        torch.cuda.synchronize()
        assert torch.equal(w1, w2)
        assert bool(torch.all(w1 > 0)) and bool(torch.all(w1 <= 1 + 1e-12))


@pytest.mark.parametrize("n", [4096, 8192])
def test_fft_full_size_elementwise(n):
    # the inverse-FFT passes, deapodization and crop at G = 8192 and 16384
    # (the two largest row lengths), every output pixel against the oracle on
    # a seeded grid with a smooth envelope (the spread of a sector of samples
    # has most of its energy in a few rows and columns) plus white noise
    from paper_1706_08575_amd.ftcg import Plan
    G = 2 * n
    rng = np.random.default_rng(n)
    x = (np.arange(G) - G / 2) / G
    env = np.exp(-((x[:, None] - 0.1) ** 2 + (x[None, :] + 0.2) ** 2) / 0.02).astype(np.float32)
    H = (env * (rng.standard_normal((G, G), dtype=np.float32)
                + 1j * rng.standard_normal((G, G), dtype=np.float32))).astype(np.complex64)
    H += (1e-3 * (rng.standard_normal((G, G), dtype=np.float32)
                  + 1j * rng.standard_normal((G, G), dtype=np.float32))).astype(np.complex64)
    with Plan(n, dim=2, dtype="f32", weights="none") as P:
        img = P.grid_to_image(torch.from_numpy(H).cuda())
        torch.cuda.synchronize()
        img = img.cpu().numpy()
    ref = O.grid_to_image(H.astype(np.complex128), n, workers=os.cpu_count() or 1)
    del H
    err = O.rel_l2(img, ref)
    rows = np.linalg.norm(img - ref, axis=1) / np.linalg.norm(ref, axis=1)
    cols = np.linalg.norm(img - ref, axis=0) / np.linalg.norm(ref, axis=0)
    print(f"G = {G}: rel L2 {err:.2e}, worst row {rows.max():.2e}, worst column {cols.max():.2e}")
    assert err < 2e-5
    assert rows.max() < 1e-4 and cols.max() < 1e-4
