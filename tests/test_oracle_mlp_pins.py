"""Pins of the learned-weight oracle (16-NN features, MLP, backward, Adam)
against library routines (torch autograd and torch.optim.Adam on the CPU in
float64, a full distance matrix), closed forms and finite differences."""
import numpy as np
import pytest
import torch

import oracle.mlp_ref as M
from paper_1706_08575_amd import synth as S


def rand_params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return {n: scale * rng.standard_normal(s) for n, s in M.PARAM_SHAPES}


def torch_forward(params, X):
    t = {n: torch.tensor(np.asarray(params[n], dtype=np.float64), requires_grad=True) for n, _ in M.PARAM_SHAPES}
    x = torch.tensor(X, dtype=torch.float64)
    h1 = torch.nn.functional.silu(x @ t["W1"] + t["b1"])
    h2 = torch.nn.functional.silu(h1 @ t["W2"] + t["b2"])
    y = (h2 @ t["W3"])[:, 0] + t["b3"][0]
    return y, t


def test_forward_matches_torch():
    p = rand_params(1)
    X = np.random.default_rng(2).standard_normal((50, 32))
    y_ref, _ = torch_forward(p, X)
    assert np.max(np.abs(M.forward(p, X) - y_ref.detach().numpy())) < 1e-12


def test_gradients_match_torch_autograd():
    p = rand_params(3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((40, 32))
    T = rng.standard_normal(40)
    loss, g = M.loss_and_grads(p, X, T)
    y, t = torch_forward(p, X)
    L = torch.mean((y - torch.tensor(T)) ** 2)
    L.backward()
    assert abs(loss - L.item()) < 1e-12
    for n, _ in M.PARAM_SHAPES:
        ref = t[n].grad.numpy()
        assert np.max(np.abs(g[n] - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref))), n


def test_gradients_match_finite_differences():
    p = rand_params(5)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((20, 32))
    T = rng.standard_normal(20)
    _, g = M.loss_and_grads(p, X, T)
    h = 1e-6
    for n, shp in M.PARAM_SHAPES:
        flat = np.asarray(p[n]).ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            pp = {k: np.array(v, dtype=np.float64) for k, v in p.items()}
            pm = {k: np.array(v, dtype=np.float64) for k, v in p.items()}
            pp[n].ravel()[idx] += h
            pm[n].ravel()[idx] -= h
            fd = (M.loss_and_grads(pp, X, T)[0] - M.loss_and_grads(pm, X, T)[0]) / (2 * h)
            an = g[n].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (n, idx, fd, an)


def test_forward_special_case_zero_first_layer():
    p = rand_params(7)
    p["W1"] = np.zeros((32, 64))
    p["b1"] = np.zeros(64)
    X = np.random.default_rng(8).standard_normal((5, 32))
    b2 = p["b2"]
    expect = (b2 / (1.0 + np.exp(-b2))) @ p["W3"][:, 0] + p["b3"][0]
    assert np.max(np.abs(M.forward(p, X) - expect)) < 1e-14


def test_adam_first_step_closed_form_and_torch():
    p = rand_params(9)
    rng = np.random.default_rng(10)
    g = {n: rng.standard_normal(s) for n, s in M.PARAM_SHAPES}
    z = {n: np.zeros(s) for n, s in M.PARAM_SHAPES}
    lr = 1e-3
    P1, M1, V1 = M.adam_step(p, g, z, z, 1, lr)
    for n, _ in M.PARAM_SHAPES:
        # first step: m_hat = g, v_hat = g^2  =>  delta = -lr g / (|g| + eps)
        assert np.max(np.abs(P1[n] - (p[n] - lr * g[n] / (np.abs(g[n]) + 1e-8)))) < 1e-15
    # several steps against torch.optim.Adam
    tp = [torch.tensor(np.asarray(p[n], dtype=np.float64), requires_grad=True) for n, _ in M.PARAM_SHAPES]
    opt = torch.optim.Adam(tp, lr=lr, betas=(0.9, 0.999), eps=1e-8)
    P, Mm, Vv = p, z, z
    for step in range(1, 5):
        gs = {n: rng.standard_normal(s) for n, s in M.PARAM_SHAPES}
        for t_, (n, _) in zip(tp, M.PARAM_SHAPES):
            t_.grad = torch.tensor(gs[n])
        opt.step()
        P, Mm, Vv = M.adam_step(P, gs, Mm, Vv, step, lr)
    for t_, (n, _) in zip(tp, M.PARAM_SHAPES):
        assert np.max(np.abs(P[n] - t_.detach().numpy())) < 1e-14, n


def test_knn_features_vs_full_distance_matrix():
    rng = np.random.default_rng(11)
    k = rng.uniform(-6, 6, size=(300, 2))
    R = 30.0   # the box covers everything: plain k-nearest on the full matrix
    F, base = M.knn_features(k, R)
    D = k[None, :, :] - k[:, None, :]
    D32 = D.astype(np.float32)
    d2 = (D32[..., 0] * D32[..., 0] + D32[..., 1] * D32[..., 1]).astype(np.float64)
    np.fill_diagonal(d2, np.inf)
    for j in (0, 17, 299):
        order = np.lexsort((np.arange(300), d2[j]))[:16]
        assert np.array_equal(F[j].reshape(16, 2), D32[j, order])
        # ranking in float32 agrees with exact distances away from ties
        exact = np.argsort(np.sum(D[j] ** 2, axis=1) + np.where(np.arange(300) == j, np.inf, 0))[:16]
        assert set(exact) == set(order)
        g = np.prod(np.sinc(D[j, order]), axis=1)
        assert abs(base[j] - 1.0 / (1.0 + np.sum(g * g))) < 1e-15
    sub, bsub = M.knn_features(k, R, at=[17, 299])
    assert np.array_equal(sub, F[[17, 299]]) and np.array_equal(bsub, base[[17, 299]])


def test_knn_sparse_neighbourhood_padded():
    k = np.array([[0.0, 0.0], [1.0, 0.5], [20.0, 20.0]])
    F, base = M.knn_features(k, 8.0)
    assert np.array_equal(F[0, :2], [1.0, 0.5])
    assert np.all(F[0, 2:] == 8.0)
    assert np.all(F[2] == 8.0) and base[2] == 1.0


def test_base_estimate_exact_on_lattice():
    # integer lattice: every other lattice point has a zero sinc factor, so the
    # analytic estimate is exactly 1, equal to the plain frame weight
    j0, j1 = np.meshgrid(np.arange(12), np.arange(12), indexing="ij")
    k = np.stack([j0.ravel(), j1.ravel()], axis=1).astype(np.float64)
    _, base = M.knn_features(k, 8.0)
    assert np.max(np.abs(base - 1.0)) < 1e-15


def test_fp16_storage_rounding_is_applied():
    p = S.mlp_init()
    X = np.random.default_rng(12).uniform(-3, 3, size=(64, 32))
    y16 = M.forward(p, X, fp16=True)
    y64 = M.forward(p, X, fp16=False)
    d = np.max(np.abs(y16 - y64))
    assert 0 < d < 1e-2


@pytest.mark.parametrize("plant", ["transposed_W2", "no_bias2", "relu"])
def test_planted_mistakes_fail_torch_pin(plant, monkeypatch):
    good = M.forward

    def wrong(params, X, fp16=False, return_cache=False):
        q = dict(params)
        if plant == "transposed_W2":
            q["W2"] = np.asarray(params["W2"]).T
        if plant == "no_bias2":
            q["b2"] = np.zeros(64)
        if plant == "relu":
            monkeypatch.setattr(M, "silu", lambda z: np.maximum(z, 0.0))
        return good(q, X, fp16, return_cache)
    monkeypatch.setattr(M, "forward", wrong)
    with pytest.raises(AssertionError):
        test_forward_matches_torch()
