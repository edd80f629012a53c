"""Pins of the iterative density compensation oracle (the cited iterative
quadrature weights of Sec. III-A, w <- w / (Omega^T Omega w)): uniform
lattices give equal weights of h^d (the normalization shared with the frame
weights of eq:difopt), a pure-Python brute force of the iteration on a tiny
raster, and the fixed-point residual falling with the iterations. Planted
mistakes at the end each fail a pin.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.density_ref as OD
from paper_1706_08575_amd import synth as S


def test_uniform_lattices_give_h_to_the_d():
    # equal weights by symmetry (to rounding), equal to h^d up to the kernel's
    # truncation and aliasing (1.4e-5 at W = 6, sigma = 2)
    n = 32
    g = np.arange(n) - n // 2
    cases = [(S.integer_raster_1d(n), 1.0),
             (((np.arange(2 * n) - n) / 2.0).reshape(-1, 1), 0.5),
             (np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2).astype(np.float64), 1.0)]
    for k, h in cases:
        a = O.pipe_menon_weights(k, n, 3)
        d = k.shape[1]
        assert np.max(a) - np.min(a) < 1e-12 * np.max(a)
        assert abs(a[0] / h ** d - 1.0) < 3e-5, (h, d, a[0])


def _brute(k, n, iters, sigma=2.0, W=6):
    # the definition with explicit loops: K[j][i] = sum over grid cells g of
    # phi(g - u_j) phi(g - u_i), taps |g - u| <= W, g taken modulo G
    G = int(sigma * n)
    beta = math.pi * (sigma - 0.5) / (sigma * W)
    u = [sigma * float(x) + G / 2 for x in k[:, 0]]

    def taps(uj):
        out = {}
        for g in range(math.ceil(uj - W), math.floor(uj + W) + 1):
            out[g % G] = out.get(g % G, 0.0) + math.exp(-beta * (g - uj) ** 2)
        return out

    tp = [taps(x) for x in u]
    m = len(u)
    K = [[sum(tp[j][g] * tp[i].get(g, 0.0) for g in tp[j]) for i in range(m)] for j in range(m)]
    w = [1.0] * m
    for _ in range(iters):
        dens = [sum(K[j][i] * w[i] for i in range(m)) for j in range(m)]
        w = [w[j] / dens[j] for j in range(m)]
    return np.array(w) * (math.pi / (sigma * beta))


def test_brute_force_tiny():
    rng = np.random.default_rng(11)
    k = rng.uniform(-9.0, 9.0, size=(14, 1))
    k[0, 0] = 7.9                        # taps wrap across the periodic seam
    ref = _brute(k, 16, 4)
    assert np.max(np.abs(O.pipe_menon_weights(k, 16, 4) - ref) / ref) < 1e-12


def test_fixed_point_residual_falls():
    k, _, _ = S.make_sas(S.seed_for(1) + 70, n=64, pulses=32, per_pulse=64)
    beta = O.kernel_beta(2.0, 6)
    c = (math.pi / (2.0 * beta)) ** 2
    res = []
    for it in (1, 4, 16):
        w = O.pipe_menon_weights(k, 64, it) / c
        dens = O.interpolate(k, O.spread(k, w.astype(np.complex128), 64)).real
        res.append(np.sqrt(np.mean((w * dens - 1.0) ** 2)))
    assert res[0] > res[1] > res[2], res


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

_good_interp = OD.interpolate


def _interp_nearest(k, H, sigma=2.0, W=6, chunk=1 << 14):
    G = H.shape[0]
    u = np.mod(np.rint(sigma * np.asarray(k) + G / 2), G).astype(np.int64)
    return H[tuple(u.T)] if H.ndim > 1 else H[u[:, 0]]


def _pm_times(k, n, iters, sigma=2.0, W=6):
    k = np.asarray(k, dtype=np.float64)
    w = np.ones(k.shape[0])
    for _ in range(iters):
        w = w * _good_interp(k, O.spread(k, w.astype(np.complex128), n, sigma, W), sigma, W).real
    return w * (math.pi / (sigma * O.kernel_beta(sigma, W))) ** k.shape[1]


def _pm_unscaled(k, n, iters, sigma=2.0, W=6):
    k = np.asarray(k, dtype=np.float64)
    w = np.ones(k.shape[0])
    for _ in range(iters):
        w = w / _good_interp(k, O.spread(k, w.astype(np.complex128), n, sigma, W), sigma, W).real
    return w


PLANTS = {
    "interpolation_nearest_cell": ("interpolate", _interp_nearest),
    "multiplies_by_density": ("pipe_menon_weights", _pm_times),
    "missing_normalization": ("pipe_menon_weights", _pm_unscaled),
}
PINS = [test_uniform_lattices_give_h_to_the_d, test_brute_force_tiny, test_fixed_point_residual_falls]


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_density_planted_mistake_is_caught(plant, monkeypatch):
    name, fn = PLANTS[plant]
    monkeypatch.setattr(OD, name, fn)
    if name == "pipe_menon_weights":
        monkeypatch.setattr(O, name, fn)
    failed = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, IndexError, ValueError):
            failed.append(pin.__name__)
    assert failed, plant
