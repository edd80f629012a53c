"""FP64 oracle of the learned-weight form: 16-nearest-neighbour geometry
features, the MLP that maps them to a frame-weight correction, its backward
pass and the Adam update.

TEST INFRASTRUCTURE. Imported only by tests, by the package smoke check and by
the benchmark's CPU-baseline leg. Shares no code with the GPU library.

The paper does not contain this part (it is the learned extension of the
frame-optimal weights of Sec. III-C eq:difopt); the definitions below are the
ones the GPU library implements, written out plainly:

  features of sample j: the 16 other samples i with ||k_i - k_j||_inf <= R
    nearest to j in squared Euclidean distance, ranked in float32: with
    d = k_i - k_j formed in float64 and rounded to float32 per axis,
    d2 = dx*dx + dy*dy with each product and the sum rounded to float32 (no
    fused multiply-add); ties broken by the smaller index. The feature is
    (dx_1, dy_1, ..., dx_16, dy_16) as float32, nearest first; missing
    neighbours are (R, R).
  analytic estimate: base_j = 1 / (1 + sum over the 16 of sinc^2(dx) sinc^2(dy)).
  network: y = W3^T s(W2^T s(W1^T x + b1) + b2) + b3 with s(z) = z / (1 + e^-z)
    (SiLU), x the 32 features, widths 32 -> 64 -> 64 -> 1.
  learned weight: alpha_hat_j = base_j * exp(y_j); training target
    y* = log(alpha_j / base_j) with alpha_j the plain frame weight.
  loss: mean over the batch of (y - y*)^2.
  storage precision of the inference kernel ("fp16"): weights, inputs and the
    two hidden activations are rounded to IEEE half before each product;
    accumulation is exact here (float64) and float32 on the GPU.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

K_NN = 16
N_IN = 2 * K_NN
WIDTH = 64
PARAM_SHAPES = (("W1", (N_IN, WIDTH)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
                ("W3", (WIDTH, 1)), ("b3", (1,)))


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _h(a, fp16):
    return a.astype(np.float16).astype(np.float64) if fp16 else np.asarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------

def knn_features(k: np.ndarray, R: float = 8.0, K: int = K_NN, at=None):
    """(features (n, 2K), base (n,)) following the definition in the header,
    for every sample or for the samples listed in ``at``. Neighbour candidates
    come from a k-d tree box query (library primitive); the ordering is a
    plain lexicographic sort on (d2, index)."""
    k = np.asarray(k, dtype=np.float64)
    targets_ = np.arange(k.shape[0]) if at is None else np.asarray(at, dtype=np.int64)
    tree = cKDTree(k)
    feats = np.full((len(targets_), 2 * K), R, dtype=np.float32)
    base = np.empty(len(targets_))
    lists = tree.query_ball_point(k[targets_], r=R, p=np.inf)
    for t, j in enumerate(targets_):
        idx = np.array([i for i in lists[t] if i != j], dtype=np.int64)
        if idx.size == 0:
            base[t] = 1.0
            continue
        d = k[idx] - k[j]
        d32 = d.astype(np.float32)
        d2 = d32[:, 0] * d32[:, 0] + d32[:, 1] * d32[:, 1]     # float32 arithmetic
        order = np.lexsort((idx, d2))[:K]
        sel = d[order]
        feats[t, :2 * len(sel)] = sel.astype(np.float32).ravel()
        g = np.prod(np.sinc(sel), axis=1)
        base[t] = 1.0 / (1.0 + np.sum(g * g))
    return feats, base


# ----------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------

def forward(params: dict, X: np.ndarray, fp16: bool = False, return_cache: bool = False):
    """y (n,) for inputs X (n, 32)."""
    W1, b1, W2, b2, W3, b3 = (np.asarray(params[n], dtype=np.float64) for n, _ in PARAM_SHAPES)
    W1, W2, W3 = _h(W1, fp16), _h(W2, fp16), _h(W3, fp16)
    x = _h(X, fp16)
    z1 = x @ W1 + b1
    h1 = _h(silu(z1), fp16)
    z2 = h1 @ W2 + b2
    h2 = _h(silu(z2), fp16)
    y = (h2 @ W3)[:, 0] + b3[0]
    if return_cache:
        return y, (x, z1, h1, z2, h2, W1, W2, W3)
    return y


def loss_and_grads(params: dict, X: np.ndarray, T: np.ndarray, fp16: bool = False):
    """Mean squared error and its gradient with respect to every parameter
    (backpropagation through the network above; with fp16=True the rounding
    steps are treated as identities in the backward pass)."""
    y, (x, z1, h1, z2, h2, W1, W2, W3) = forward(params, X, fp16, return_cache=True)
    n = X.shape[0]
    r = y - np.asarray(T, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = (2.0 / n) * r                       # (n,)
    g = {}
    g["W3"] = h2.T @ dy[:, None]
    g["b3"] = np.array([dy.sum()])
    dz2 = (dy[:, None] @ W3.T) * silu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * silu_grad(z1)
    g["W1"] = x.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam_step(params: dict, grads: dict, m: dict, v: dict, t: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba): moments, bias correction, step. t >= 1 is
    the index of this step. Returns new (params, m, v)."""
    P, M, V = {}, {}, {}
    for name, _ in PARAM_SHAPES:
        g = np.asarray(grads[name], dtype=np.float64)
        M[name] = beta1 * np.asarray(m[name], dtype=np.float64) + (1.0 - beta1) * g
        V[name] = beta2 * np.asarray(v[name], dtype=np.float64) + (1.0 - beta2) * g * g
        mh = M[name] / (1.0 - beta1 ** t)
        vh = V[name] / (1.0 - beta2 ** t)
        P[name] = np.asarray(params[name], dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return P, M, V


def learned_weights(params: dict, k: np.ndarray, R: float = 8.0, fp16: bool = True):
    """alpha_hat = base * exp(y(features))."""
    X, base = knn_features(k, R)
    return base * np.exp(forward(params, X, fp16=fp16))


def targets(alpha: np.ndarray, base: np.ndarray) -> np.ndarray:
    return np.log(np.asarray(alpha) / np.asarray(base))
