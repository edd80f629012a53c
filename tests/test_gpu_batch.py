"""GPU tests of batched execution (persistent spreading launch over all
items, batched FFT passes, hipGraph replay) through the C ABI.

Each item of a batch must reproduce the single-plan result exactly: the
fixed-point tile accumulation is exact and uses the same order-independent
tile bound, and the FFT rows run the same code, so a batch item and a
single plan with the same tile size agree bitwise, also when dense tiles are
split over several tasks. Against the FP64 oracle the float32 bar applies.
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


@pytest.fixture(scope="module")
def items():
    # uneven items: sizes 64..256, from sparse to very dense (dense tiles get split)
    spec = [(64, 4000), (256, 65536), (128, 30000), (64, 60000), (256, 9000), (128, 1)]
    out = []
    for i, (n, m) in enumerate(spec):
        q = max(1, int(np.ceil(np.sqrt(2 * m))))
        p = int(np.ceil(m / q))
        k, f, _ = S.make_sas(S.seed_for(3) + 100 + i, n=n, pulses=p, per_pulse=q, m=m)
        out.append((n, k, f))
    return out


def single_image(n, k, f, tile=32):
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(n, dim=2) as P:
        P.set_tuning(tile, "fixed", 1)
        P.set_points(dev(k))
        return host(P.execute(dev(f, torch.complex64))), host(P.get_weights())


def run_batch(items, chunk=4096, graph=True, reps=1):
    from paper_1706_08575_amd.batch import Batch
    sizes = [n for n, _, _ in items]
    K = np.concatenate([k for _, k, _ in items])
    F = np.concatenate([f for _, _, f in items])
    with Batch(sizes) as B:
        B.set_tuning(tile=32, chunk=chunk, graph=graph)
        B.set_points([len(f) for _, _, f in items], dev(K))
        fd = dev(F, torch.complex64)
        for _ in range(reps):
            out = B.execute(fd)
        imgs = [host(B.image(out, i)) for i in range(len(items))]
        w = host(B.get_weights())
        info = B.info()
    return imgs, w, info


def test_batch_items_equal_single_plans(items):
    imgs, w, info = run_batch(items, graph=False)
    off = 0
    for i, (n, k, f) in enumerate(items):
        ref, a = single_image(n, k, f)
        assert np.array_equal(imgs[i], ref), i
        assert np.max(np.abs(w[off:off + len(f)] - a) / a) < 1e-12
        off += len(f)
    assert info["tasks"] >= info["tiles"]


def test_batch_vs_oracle(items):
    imgs, _, _ = run_batch(items)
    for i, (n, k, f) in enumerate(items[:4]):
        ref = O.ftcg_image(k, f, O.frame_weights(k, 8.0), n)
        assert O.rel_l2(imgs[i], ref) < 2e-5, i


def test_split_tiles_are_exact(items):
    a, _, info_a = run_batch(items, chunk=4096)
    b, _, info_b = run_batch(items, chunk=64)
    assert info_b["split_tiles"] > info_a["split_tiles"] >= 0
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_graph_replays_match_eager(items):
    from paper_1706_08575_amd.batch import Batch
    sizes = [n for n, _, _ in items]
    K = np.concatenate([k for _, k, _ in items])
    F = np.concatenate([f for _, _, f in items])
    m = [len(f) for _, _, f in items]
    with Batch(sizes) as E, Batch(sizes) as G:
        E.set_tuning(tile=32, graph=False)
        G.set_tuning(tile=32, graph=True)
        E.set_points(m, dev(K))
        G.set_points(m, dev(K))
        for r in range(4):
            vals = dev(F * (1.0 + 0.5 * r) + (r % 2) * 1j, torch.complex64)
            e = host(E.execute(vals))
            junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
            g = host(G.execute(vals))
            torch.cuda.synchronize()
            assert np.array_equal(e, g), r
            del junk


def test_user_weights_concatenated(items):
    from paper_1706_08575_amd.batch import Batch
    sub = items[:3]
    sizes = [n for n, _, _ in sub]
    K = np.concatenate([k for _, k, _ in sub])
    F = np.concatenate([f for _, _, f in sub])
    A = np.random.default_rng(1).uniform(0.5, 1.5, size=len(F))
    with Batch(sizes, weights="user") as B:
        B.set_points([len(f) for _, _, f in sub], dev(K))
        B.set_weights(dev(A))
        out = B.execute(dev(F, torch.complex64))
        imgs = [host(B.image(out, i)) for i in range(3)]
        assert np.array_equal(host(B.get_weights()), A)
    off = 0
    for i, (n, k, f) in enumerate(sub):
        ref = O.ftcg_image(k, f, A[off:off + len(f)], n)
        assert O.rel_l2(imgs[i], ref) < 2e-5
        off += len(f)
