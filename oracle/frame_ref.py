"""FP64 oracle of the dense frame approximation A_fr (Sec. III-B eq:binv,
eq:afr, eq:afrm; 2D Sec. IV eq:twodframe, eq:twodframeB), the accuracy
reference that FTCG approximates with a banded C.

TEST INFRASTRUCTURE. Imported only by tests, by the package smoke check and by
the benchmark's CPU-baseline leg. Shares no code with the GPU library.

Readings (also listed in the design notes):
  * Admissible frame: zeta_n(x) = exp(2 pi i n . x) / w(x) (eq:newadm, the
    psi_m = e^{2 pi i m x} / w(x) of eq:afr) with the modes n on the pixel
    grid's frequencies, n_a in -N/2 .. N/2 - 1, and w the window of this
    path, w(x) = Phi(x / sigma) per axis, Phi(t) = sqrt(pi / beta)
    exp(-pi^2 t^2 / beta) (the function the reconstruction divides by).
  * Inner products on the centred FOV [-1/2, 1/2)^d:
    Psi_{j,n} = <phi_j, zeta_n> = prod_a g(k_ja - n_a),
    g(t) = int_{-1/2}^{1/2} cos(2 pi t x) / w(x) dx (w is even and real),
    by Gauss-Legendre quadrature (numpy's nodes) with 4N + 64 points.
  * beta = Psi^dagger fhat (eq:binv): numpy.linalg.lstsq, the least-squares
    solution when there are at least as many samples as modes, the
    minimum-norm one otherwise.
  * A_fr(x_p) = sum_n beta_n exp(2 pi i n . x_p) / w(x_p) (eq:afrm) at the
    pixels x_p = (p - N/2) / N.
"""
from __future__ import annotations

import math

import numpy as np

from .ftcg_ref import kernel_beta, pixel_coords


def window(x: np.ndarray, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """w(x) = Phi(x / sigma), Phi(t) = sqrt(pi / beta) exp(-pi^2 t^2 / beta)."""
    beta = kernel_beta(sigma, W)
    t = np.asarray(x, dtype=np.float64) / sigma
    return math.sqrt(math.pi / beta) * np.exp(-(math.pi ** 2) * t * t / beta)


def g_integral(t: np.ndarray, n: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """g(t) = int_{-1/2}^{1/2} cos(2 pi t x) / w(x) dx, Gauss-Legendre with 4n + 64 nodes."""
    X, Wq = np.polynomial.legendre.leggauss(4 * n + 64)
    x = X / 2.0
    wq = Wq / 2.0 / window(x, sigma, W)
    t = np.asarray(t, dtype=np.float64)
    return np.cos(2 * math.pi * t[..., None] * x) @ wq


def frame_matrix(k: np.ndarray, n: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """Psi (m x N^d): Psi[j, mode] = prod_a g(k_ja - n_a), modes in row-major
    order of (n_0 + N/2, n_1 + N/2)."""
    k = np.asarray(k, dtype=np.float64)
    modes = np.arange(n) - n // 2
    G0 = g_integral(k[:, 0:1] - modes[None, :], n, sigma, W)
    if k.shape[1] == 1:
        return G0
    G1 = g_integral(k[:, 1:2] - modes[None, :], n, sigma, W)
    return (G0[:, :, None] * G1[:, None, :]).reshape(k.shape[0], n * n)


def frame_coefficients(k: np.ndarray, fhat: np.ndarray, n: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """beta = Psi^dagger fhat (numpy lstsq: least squares or minimum norm)."""
    Psi = frame_matrix(k, n, sigma, W)
    beta, *_ = np.linalg.lstsq(Psi, np.asarray(fhat, dtype=np.complex128), rcond=None)
    return beta


def frame_image(k: np.ndarray, fhat: np.ndarray, n: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """A_fr at the pixels: sum_n beta_n exp(2 pi i n . x_p) / w(x_p)."""
    d = np.asarray(k).shape[1]
    beta = frame_coefficients(k, fhat, n, sigma, W)
    x = pixel_coords(n)
    modes = np.arange(n) - n // 2
    E = np.exp(2j * math.pi * np.outer(x, modes))          # E[p, n] = e^{2 pi i n x_p}
    iw = 1.0 / window(x, sigma, W)
    if d == 1:
        return (E @ beta) * iw
    B = beta.reshape(n, n)
    return (E @ B @ E.T) * iw[:, None] * iw[None, :]
