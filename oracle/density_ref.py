"""FP64 oracle of the iterative density compensation the paper cites as the
established way to obtain quadrature weights (Sec. III-A, the iterative
method of its reference on sampling density compensation), used here as a
comparator to the frame-theoretic weights of eq:difopt.

TEST INFRASTRUCTURE. Imported only by tests, by the package smoke check and by
the benchmark's CPU-baseline leg. Shares no code with the GPU library.

Reading (also listed in the design notes). The paper gives no formula for
it; the cited method iterates w <- w / (w * C) evaluated at the samples, C
the convolution kernel of the gridding. Here C is the kernel of this path
applied twice through the oversampled grid, the operator Omega^T Omega of
eq:cgmatrix:

    d_j = sum_g phi(g - u_j) sum_i w_i phi(g - u_i),   w_j <- w_j / d_j,

starting from w = 1, phi the truncated Gaussian taps of spread() and
interpolate() (indices modulo G). The fixed point makes the gridded density
of the weights flat. The result is reported as alpha = w (pi / (sigma beta))^d,
the scale at which a uniform lattice of spacing h (cycles per FOV) gets
alpha = h^d, the value the frame weights take there: per axis the grid sum
of phi(g - a) phi(g - b) over b integrates to pi / beta in grid units, and a
spacing h is sigma h grid cells.
"""
from __future__ import annotations

import math

import numpy as np

from .ftcg_ref import interpolate, kernel_beta, spread


def pipe_menon_weights(k: np.ndarray, n: int, iters: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """alpha after `iters` iterations of w <- w / (Omega^T Omega w), w0 = 1."""
    k = np.asarray(k, dtype=np.float64)
    d = k.shape[1]
    w = np.ones(k.shape[0])
    for _ in range(iters):
        H = spread(k, w.astype(np.complex128), n, sigma, W)
        dens = interpolate(k, H, sigma, W).real
        w = w / dens
    return w * (math.pi / (sigma * kernel_beta(sigma, W))) ** d
