"""Densest batched shape: 2^22 samples of the polar SAS raster on a 256^2
image (the top of the batched workload's sample-count range at its smallest
image size, about 64 samples per image pixel and 3 200 footprint taps per
grid cell), single plans and a batch item, at tiles 32 and 64.

This is where the fixed-point tile accumulation is stressed most: its
quantum is 2^-31 of the tile's L1 bound, which grows with the records of a
tile (about 42 000 at tile 32 and 125 000 at tile 64 here), and each cell
adds thousands of rounded taps. The whole image is compared with the FP64
oracle (Sec. III-A eq:cgmatrix: Omega D fhat, then the inverse FFT and the
division by w) fed the GPU's own weights, whose float64 values are checked
separately on a seeded subset (eq:difopt, 1e-10 relative).

Bar: the benchmark spec's 1e-4 relative L2; 2e-5 is asserted (the measured error
is printed).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_08575_amd import synth as S

pytestmark = pytest.mark.gpu

N = 256
M = 1 << 22


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def dense():
    from paper_1706_08575_amd.ftcg import Plan
    q = int(np.ceil(np.sqrt(2 * M)))
    p = int(np.ceil(M / q))
    k, f, _ = S.make_sas(S.seed_for(3) + 777, n=N, pulses=p, per_pulse=q, m=M)
    with Plan(N, dim=2) as P:
        P.set_points(dev(k))
        a = host(P.get_weights())
    idx = np.random.default_rng(77).choice(M, 48, replace=False)
    a_ref = O.frame_weights_at(k, idx, 8.0)
    werr = float(np.max(np.abs(a[idx] - a_ref) / a_ref))
    ref = O.ftcg_image(k, f, a, N)
    print(f"densest shape: {M} samples on {N}^2, weights max rel err {werr:.2e} on 48 samples")
    return k, f, a, ref, werr


def test_dense_weights(dense):
    assert dense[4] < 1e-10


@pytest.mark.parametrize("tile", [32, 64])
def test_dense_single_plan(dense, tile):
    from paper_1706_08575_amd.ftcg import Plan
    k, f, a, ref, _ = dense
    with Plan(N, dim=2) as P:
        P.set_tuning(tile, "fixed", 1)
        P.set_points(dev(k))
        img = host(P.execute(dev(f, torch.complex64)))
        nrec = P.info()["n_records"]
    err = O.rel_l2(img, ref)
    print(f"tile {tile}: {nrec} records ({nrec / (N * 2 // tile) ** 2:.0f} per tile), rel L2 {err:.3e}")
    assert err < 2e-5


@pytest.mark.parametrize("tile", [32, 64])
def test_dense_batch_item(dense, tile):
    # the dense item between two small ones, its tiles split over tasks of
    # 16384 records (the autotuner's choice for the batched workload)
    from paper_1706_08575_amd.batch import Batch
    k, f, a, ref, _ = dense
    others = [S.make_sas(S.seed_for(3) + 778 + i, n=n, pulses=64, per_pulse=128) for i, n in enumerate((128, 512))]
    sizes = [128, N, 512]
    ks = [others[0][0], k, others[1][0]]
    fs = [others[0][1], f, others[1][1]]
    with Batch(sizes) as B:
        B.set_tuning(tile=tile, chunk=16384)
        B.set_points([len(x) for x in fs], dev(np.concatenate(ks)))
        out = B.execute(dev(np.concatenate(fs), torch.complex64))
        img = host(B.image(out, 1))
        w = host(B.get_weights())
        info = B.info()
    m0 = len(fs[0])
    assert np.array_equal(w[m0:m0 + M], a)
    err = O.rel_l2(img, ref)
    print(f"batch tile {tile}: {info['split_tiles']} split tiles, rel L2 {err:.3e}")
    assert err < 2e-5
