"""Pins of the dense frame approximation oracle (Sec. III-B eq:binv, eq:afr,
eq:afrm; Sec. IV eq:twodframeB): the inner products g(t) against scipy's
adaptive quadrature and a closed form at t = 0 (erfi), exact reproduction of
a finite expansion in the admissible frame zeta_n = e^{2 pi i n x} / w(x)
whose data are formed with the independent quadrature, and the two defining
properties of the minimum-norm solution when samples are fewer than modes.
Planted mistakes at the end each fail a pin.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import erfi

import oracle as O
import oracle.frame_ref as OF


def _g_quad(t, sigma=2.0, W=6):
    beta = math.pi * (sigma - 0.5) / (sigma * W)
    iw = lambda x: math.exp(math.pi ** 2 * (x / sigma) ** 2 / beta) / math.sqrt(math.pi / beta)
    return quad(lambda x: math.cos(2 * math.pi * t * x) * iw(x), -0.5, 0.5, limit=400, epsabs=1e-15,
                epsrel=1e-14)[0]


def test_inner_products_against_adaptive_quadrature():
    ts = np.array([0.0, 0.3, -1.7, 5.7, 12.2, 30.45])
    got = O.g_integral(ts, 16)
    ref = np.array([_g_quad(t) for t in ts])
    assert np.max(np.abs(got - ref)) < 1e-13
    beta = O.kernel_beta(2.0, 6)
    a = math.pi ** 2 / (4 * beta)          # 1 / w(x) = e^{a x^2} / sqrt(pi / beta)
    g0 = math.sqrt(math.pi / a) * erfi(math.sqrt(a) / 2) / math.sqrt(math.pi / beta)
    assert abs(got[0] - g0) < 1e-13


def _expansion_data(k, c, n):
    # fhat_j = <f, phi_j> for f = sum_n c_n zeta_n: sum_n c_n g(k_j - n), per axis
    modes = np.arange(n) - n // 2
    d = k.shape[1]
    G = [np.array([[_g_quad(kj - mm) for mm in modes] for kj in k[:, a]]) for a in range(d)]
    if d == 1:
        return G[0] @ c
    return np.einsum("jp,jq,pq->j", G[0], G[1], c.reshape(n, n))


def test_reproduces_a_finite_expansion():
    rng = np.random.default_rng(12)
    for d, n, m in ((1, 8, 24), (2, 4, 40)):
        k = rng.uniform(-n / 2, n / 2, size=(m, d))
        c = rng.standard_normal(n ** d) + 1j * rng.standard_normal(n ** d)
        fhat = _expansion_data(k, c, n)
        beta = O.frame_coefficients(k, fhat, n)
        assert np.max(np.abs(beta - c)) < 1e-9 * np.max(np.abs(c))
        # and A_fr equals the expansion at the pixels
        x = O.pixel_coords(n)
        modes = np.arange(n) - n // 2
        iw = 1.0 / O.window(x)
        E = np.exp(2j * math.pi * np.outer(x, modes))
        ref = (E @ c) * iw if d == 1 else (E @ c.reshape(n, n) @ E.T) * iw[:, None] * iw[None, :]
        assert np.max(np.abs(O.frame_image(k, fhat, n) - ref)) < 1e-8 * np.max(np.abs(ref))


def test_minimum_norm_when_underdetermined():
    # fewer samples than modes: Psi beta = fhat exactly, and beta lies in the
    # row space of Psi (orthogonal to its null space)
    rng = np.random.default_rng(13)
    n, m = 16, 10
    k = rng.uniform(-8, 8, size=(m, 1))
    fhat = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    Psi = O.frame_matrix(k, n)
    beta = O.frame_coefficients(k, fhat, n)
    assert np.max(np.abs(Psi @ beta - fhat)) < 1e-10 * np.max(np.abs(fhat))
    _, s, Vt = np.linalg.svd(Psi)
    null = Vt[m:]                                  # rows spanning the null space
    assert np.max(np.abs(null @ beta)) < 1e-10 * np.max(np.abs(beta))


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

_good_window = OF.window
_good_g = OF.g_integral


def _window_flat(x, sigma=2.0, W=6):
    return np.ones_like(np.asarray(x, dtype=np.float64))


def _g_shifted_modes(t, n, sigma=2.0, W=6):
    return _good_g(np.asarray(t) + 1.0, n, sigma, W)


def _g_sine(t, n, sigma=2.0, W=6):
    X, Wq = np.polynomial.legendre.leggauss(4 * n + 64)
    x = X / 2.0
    return np.sin(2 * math.pi * np.asarray(t)[..., None] * x + 0.5) @ (Wq / 2.0 / _good_window(x, sigma, W))


PLANTS = {
    "window_missing": ("window", _window_flat),
    "modes_off_by_one": ("g_integral", _g_shifted_modes),
    "wrong_kernel_of_inner_product": ("g_integral", _g_sine),
}
PINS = [test_inner_products_against_adaptive_quadrature, test_reproduces_a_finite_expansion]


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_frame_planted_mistake_is_caught(plant, monkeypatch):
    name, fn = PLANTS[plant]
    monkeypatch.setattr(OF, name, fn)
    monkeypatch.setattr(O, name, fn)
    failed = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, np.linalg.LinAlgError):
            failed.append(pin.__name__)
    assert failed, plant
