"""FP64 oracle of the banded FTCG coefficient matrix C (Sec. III-C eq:ftcg,
eq:cr; 2D Sec. IV eq:twodftcg) and of its application tau = Omega C fhat.

TEST INFRASTRUCTURE. Imported only by tests, by the package smoke check and by
the benchmark's CPU-baseline leg. Shares no code with the GPU library.

Reading of the paper used here (also listed in the design notes). The paper
writes C = (Psi Omega (Hadamard) B_r)^dagger, calls C a (2r-1)-banded matrix,
and derives it from min ||Psi Omega C - I||_F (eq:difopt with the diagonal
constraint relaxed, eq:dif3). A pseudo-inverse of a band-masked matrix is not
banded in general, so C is read as the band-constrained minimiser of that
norm: the Frobenius norm splits into columns, and column n of C solves

    min over c supported on J(n) of || T c - e_n ||_2,
    J(n) = {n - r + 1, ..., n + r - 1} (clipped to 0 .. M-1),

a least-squares problem with 2r - 1 unknowns, solved here with
numpy.linalg.lstsq (minimum-norm solution). T = Psi Omega is the truncated
Gram matrix of the data frame used for the diagonal weights,
T_in = prod_a sinc(k_ia - k_na) for ||k_i - k_n||_inf <= R, else 0. The band
runs over the samples in the caller's (raster) order: the paper's band of 15
entries of a 900 x 900 T (Sec. V-A) is a band of the flattened 2D raster.
At r = 1 the column problem is the diagonal one of eq:difopt; with the band
covering every sample and no truncation, C = T^dagger (eq:dif3).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def _gram(ki: np.ndarray, kj: np.ndarray, R: float) -> np.ndarray:
    """T[i, j] = prod_a sinc(ki[i, a] - kj[j, a]) where ||ki[i] - kj[j]||_inf <= R, else 0."""
    d = ki[:, None, :] - kj[None, :, :]
    t = np.prod(np.sinc(d), axis=2)
    return np.where(np.max(np.abs(d), axis=2) <= R, t, 0.0)


def band_columns(k: np.ndarray, r: int, R: float = 8.0, cols=None) -> np.ndarray:
    """Columns of the band-constrained C.

    Returns B with B[t, p] = C[n - r + 1 + p, n] for n = cols[t] (all samples
    when cols is None), p = 0 .. 2r-2; entries whose row index falls outside
    0 .. M-1 are 0. Each column is one lstsq over the rows of T that are not
    identically zero on J(n) (the union of the R-boxes of the samples in J(n);
    every other row of T[:, J(n)] is 0 and does not change the problem).
    """
    k = np.asarray(k, dtype=np.float64)
    m, d = k.shape
    if r < 1:
        raise ValueError("r >= 1")
    cols = np.arange(m) if cols is None else np.asarray(cols)
    out = np.zeros((len(cols), 2 * r - 1))
    finite = np.isfinite(R)
    tree = cKDTree(k) if finite else None
    for t, n in enumerate(cols):
        lo, hi = max(0, n - r + 1), min(m - 1, n + r - 1)
        J = np.arange(lo, hi + 1)
        if finite:
            rows = np.unique(np.concatenate([np.asarray(l, dtype=np.int64)
                                             for l in tree.query_ball_point(k[J], r=R, p=np.inf)]))
        else:
            rows = np.arange(m)
        A = _gram(k[rows], k[J], R)
        e = (rows == n).astype(np.float64)
        c, *_ = np.linalg.lstsq(A, e, rcond=None)
        out[t, J - (n - r + 1)] = c
    return out


def band_dense(B: np.ndarray, r: int) -> np.ndarray:
    """The M x M matrix C from its columns B (as band_columns returns them for all samples)."""
    m = B.shape[0]
    C = np.zeros((m, m))
    for n in range(m):
        for p in range(2 * r - 1):
            i = n - r + 1 + p
            if 0 <= i < m:
                C[i, n] = B[n, p]
    return C


def band_apply(B: np.ndarray, fhat: np.ndarray, r: int) -> np.ndarray:
    """c = C fhat (the weighting step of tau = Omega C fhat, eq:ftcg):
    c_i = sum over n with |n - i| <= r - 1 of C[i, n] fhat_n."""
    fhat = np.asarray(fhat, dtype=np.complex128)
    m = B.shape[0]
    c = np.zeros(m, dtype=np.complex128)
    for p in range(2 * r - 1):
        # column n contributes B[n, p] fhat_n to row i = n - r + 1 + p
        n = np.arange(m)
        i = n - r + 1 + p
        ok = (i >= 0) & (i < m)
        np.add.at(c, i[ok], B[n[ok], p] * fhat[n[ok]])
    return c
