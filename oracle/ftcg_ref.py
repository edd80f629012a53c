"""FP64 oracle of the FTCG hot path: weights, spreading, inverse FFT, deapodization.

TEST INFRASTRUCTURE. Imported only by tests, by the package smoke check and by
the benchmark's CPU-baseline leg. Shares no code with the GPU library.

Readings of the paper used here (each also listed in the design notes):
  * Result approximated (Sec. III-A, eq:ffind, eq:cgmatrix): the weighted
    synthesis sum I(x) = sum_j alpha_j fhat_j exp(+2 pi i k_j . x), with
    k in cycles per field of view, x on the centred FOV [-1/2, 1/2)^d, no 1/N.
  * Window (Sec. III-A names a Gaussian without width): in oversampled-grid
    units the spreading kernel is exp(-beta s^2), beta = pi (sigma - 1/2) /
    (sigma W), truncated to |s| <= W (eq:ffind's |m - lambda| <= K, inclusive).
  * The grid is oversampled by sigma: grid index g <-> k = (g - G/2) / sigma,
    G = sigma N, indices taken modulo G.
  * "Divide by w(x)" (psi_m = e^{2 pi i m x} / w(x)): w is the continuous
    Fourier transform of the kernel, Phi(t) = sqrt(pi / beta) exp(-pi^2 t^2 / beta),
    evaluated at t = x / sigma.
  * Diagonal frame weights (eq:difopt): min over diagonal D of ||T D - I||_F
    splits into one least-squares problem per column, alpha_n =
    conj(T_nn) / sum_i |T_in|^2. T = Psi Omega is taken as the Gram matrix of
    the data frame on the FOV, T_in = prod_a sinc(k_ia - k_na), truncated to
    ||k_i - k_n||_inf <= R. T_nn = 1, so alpha_n = 1 / sum_i T_in^2.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
from scipy.spatial import cKDTree


# ----------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------

def kernel_beta(sigma: float, W: int) -> float:
    """Gaussian shape parameter in oversampled-grid units (fast Gaussian
    gridding parameterisation of the Gaussian window named in Sec. III-A)."""
    return math.pi * (sigma - 0.5) / (sigma * W)


def grid_size(n: int, sigma: float) -> int:
    g = sigma * n
    if abs(g - round(g)) > 1e-9 or int(round(g)) % 2:
        raise ValueError("sigma * n must be an even integer")
    return int(round(g))


def pixel_coords(n: int) -> np.ndarray:
    """x_p = (p - n/2) / n, p = 0..n-1: pixel positions on the centred FOV."""
    return (np.arange(n, dtype=np.float64) - n // 2) / n


# ----------------------------------------------------------------------------
# the definition: weighted non-uniform DFT (Sec. III-A, eq:ffind; Sec. IV, eq:twodcg)
# ----------------------------------------------------------------------------

def nudft(k: np.ndarray, c: np.ndarray, n: int, chunk: int = 8192) -> np.ndarray:
    """I[p] = sum_j c_j exp(+2 pi i k_j . x_p) on the n^d pixel grid.

    k: (m, d) float64 with d in {1, 2}; c: (m,) complex (c_j = alpha_j fhat_j).
    Returns complex128 of shape (n,) or (n, n), axis a of the image <-> k[:, a].
    In 2D the exponential factors over the axes, so the sum is a product of
    two per-axis phase matrices (a matmul per chunk of samples).
    """
    k = np.asarray(k, dtype=np.float64)
    c = np.asarray(c, dtype=np.complex128)
    d = k.shape[1]
    x = pixel_coords(n)
    if d == 1:
        out = np.zeros(n, dtype=np.complex128)
        for b in range(0, k.shape[0], chunk):
            e = np.exp(2j * np.pi * np.outer(k[b:b + chunk, 0], x))
            out += c[b:b + chunk] @ e
        return out
    if d == 2:
        out = np.zeros((n, n), dtype=np.complex128)
        for b in range(0, k.shape[0], chunk):
            e0 = np.exp(2j * np.pi * np.outer(k[b:b + chunk, 0], x))
            e1 = np.exp(2j * np.pi * np.outer(k[b:b + chunk, 1], x))
            out += (e0 * c[b:b + chunk, None]).T @ e1
        return out
    raise ValueError("d must be 1 or 2")


def nudft_at(k: np.ndarray, c: np.ndarray, x: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
    """I(x_q) = sum_j c_j exp(+2 pi i k_j . x_q) at arbitrary points x (q, d)."""
    k = np.asarray(k, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1, k.shape[1])
    c = np.asarray(c, dtype=np.complex128)
    out = np.zeros(x.shape[0], dtype=np.complex128)
    for b in range(0, k.shape[0], chunk):
        out += c[b:b + chunk] @ np.exp(2j * np.pi * (k[b:b + chunk] @ x.T))
    return out


# ----------------------------------------------------------------------------
# step 1: frame-optimal diagonal weights (Sec. III-C, eq:dif .. eq:difopt)
# ----------------------------------------------------------------------------

def _gram_entries(ki: np.ndarray, kj: np.ndarray) -> np.ndarray:
    """T_ij = <phi_j, phi_i> on the unit FOV = prod_a sinc(k_ia - k_ja)
    (np.sinc(t) = sin(pi t) / (pi t))."""
    return np.prod(np.sinc(ki - kj), axis=1)


def frame_weights(k: np.ndarray, R: float = 8.0, chunk: int = 1 << 14) -> np.ndarray:
    """alpha_n = 1 / sum_{i : ||k_i - k_n||_inf <= R} T_in^2 (self included).

    This is the column-wise least-squares optimum of min_D ||T D - I||_F over
    diagonal D (eq:difopt), with T the Gram matrix of the data frame. The
    neighbour search is a k-d tree query in the infinity norm (a library
    primitive); R = inf means all samples.
    """
    k = np.asarray(k, dtype=np.float64)
    m = k.shape[0]
    if not np.isfinite(R):
        s = np.zeros(m)
        for b in range(0, m, 256):
            kb = k[b:b + 256]
            g = np.prod(np.sinc(kb[:, None, :] - k[None, :, :]), axis=2)
            s[b:b + 256] = np.sum(g * g, axis=1)
        return 1.0 / s
    tree = cKDTree(k)
    s = np.zeros(m)
    for b in range(0, m, chunk):
        lists = tree.query_ball_point(k[b:b + chunk], r=R, p=np.inf)
        lens = np.fromiter((len(l) for l in lists), dtype=np.int64, count=len(lists))
        nb = np.fromiter((i for l in lists for i in l), dtype=np.int64, count=int(lens.sum()))
        own = np.repeat(np.arange(b, b + len(lists)), lens)
        g = _gram_entries(k[nb], k[own])
        s[b:b + len(lists)] = np.bincount(own - b, weights=g * g, minlength=len(lists))
    return 1.0 / s


def frame_weights_at(k: np.ndarray, idx: np.ndarray, R: float = 8.0) -> np.ndarray:
    """frame_weights(k, R)[idx], computed one sample at a time (for sampled
    checks at sizes where the full vector is too costly)."""
    k = np.asarray(k, dtype=np.float64)
    tree = cKDTree(k)
    out = np.empty(len(idx))
    lists = tree.query_ball_point(k[np.asarray(idx)], r=R, p=np.inf)
    for t, (j, l) in enumerate(zip(idx, lists)):
        g = _gram_entries(k[np.asarray(l)], k[j][None, :])
        out[t] = 1.0 / np.sum(g * g)
    return out


# ----------------------------------------------------------------------------
# step 2: spreading onto the oversampled grid (Omega, eq:cgmatrix / eq:twodcgmatrix)
# ----------------------------------------------------------------------------

def _axis_taps(u: np.ndarray, W: int, beta: float, G: int):
    """Taps of one axis: integer g with |g - u| <= W (2W or 2W+1 of them),
    kernel values exp(-beta (g - u)^2), indices modulo G."""
    lo = np.ceil(u - W)
    g = lo[:, None] + np.arange(2 * W + 1)[None, :]
    dist = g - u[:, None]
    w = np.where(np.abs(dist) <= W, np.exp(-beta * dist * dist), 0.0)
    return np.mod(g, G).astype(np.int64), w


def spread(k: np.ndarray, c: np.ndarray, n: int, sigma: float = 2.0, W: int = 6,
           chunk: int = 1 << 14) -> np.ndarray:
    """H[g] = sum_j c_j prod_a exp(-beta (g_a - u_ja)^2) over |g_a - u_ja| <= W,
    u_j = sigma k_j + G/2, g taken modulo G. Returns complex128 (G,)*d."""
    k = np.asarray(k, dtype=np.float64)
    c = np.asarray(c, dtype=np.complex128)
    d = k.shape[1]
    G = grid_size(n, sigma)
    beta = kernel_beta(sigma, W)
    re = np.zeros(G ** d)
    im = np.zeros(G ** d)
    for b in range(0, k.shape[0], chunk):
        u = sigma * k[b:b + chunk] + G / 2
        cb = c[b:b + chunk]
        i0, w0 = _axis_taps(u[:, 0], W, beta, G)
        if d == 1:
            flat = i0
            wt = w0
        else:
            i1, w1 = _axis_taps(u[:, 1], W, beta, G)
            flat = i0[:, :, None] * G + i1[:, None, :]
            wt = w0[:, :, None] * w1[:, None, :]
        val = wt * cb.reshape((-1,) + (1,) * d)
        re += np.bincount(flat.ravel(), weights=val.real.ravel(), minlength=G ** d)
        im += np.bincount(flat.ravel(), weights=val.imag.ravel(), minlength=G ** d)
    return (re + 1j * im).reshape((G,) * d)


def spread_window(k: np.ndarray, c: np.ndarray, n: int, r0: int, c0: int, h: int, w: int,
                  sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """The same H as spread() (eq:twodcgmatrix, 2D), only on the window of grid
    rows r0 .. r0+h-1 and columns c0 .. c0+w-1 (0 <= r0, r0+h <= G, likewise
    for columns): the samples whose taps can reach the window are selected
    first (by their grid position u taken modulo G), then their taps are
    formed exactly as in spread() and those landing in the window summed.
    For checks of grids too large to hold in float64."""
    k = np.asarray(k, dtype=np.float64)
    c = np.asarray(c, dtype=np.complex128)
    G = grid_size(n, sigma)
    beta = kernel_beta(sigma, W)
    u = np.mod(sigma * k + G / 2, G)

    def near(ua, lo, span):
        # some integer g with |g - u| <= W lies in lo .. lo+span-1 (mod G)
        d = np.mod(ua - (lo - W), G)
        return d <= span - 1 + 2 * W

    sel = np.nonzero(near(u[:, 0], r0, h) & near(u[:, 1], c0, w))[0]
    out = np.zeros((h, w), dtype=np.complex128)
    if sel.size == 0:
        return out
    uu = sigma * k[sel] + G / 2
    i0, w0 = _axis_taps(uu[:, 0], W, beta, G)
    i1, w1 = _axis_taps(uu[:, 1], W, beta, G)
    rr = np.mod(i0 - r0, G)
    cc = np.mod(i1 - c0, G)
    inside = (rr[:, :, None] < h) & (cc[:, None, :] < w)
    val = (w0[:, :, None] * w1[:, None, :]) * c[sel][:, None, None]
    flat = (rr[:, :, None] * w + cc[:, None, :])[inside]
    re = np.bincount(flat, weights=val.real[inside], minlength=h * w)
    im = np.bincount(flat, weights=val.imag[inside], minlength=h * w)
    return (re + 1j * im).reshape(h, w)


# ----------------------------------------------------------------------------
# steps 3-4: inverse FFT, divide by w (deapodize), crop (psi_m = e^{2 pi i m x}/w(x))
# ----------------------------------------------------------------------------

def deapod_factors(n: int, sigma: float = 2.0, W: int = 6) -> np.ndarray:
    """1 / Phi(x_p / sigma) per axis, Phi(t) = sqrt(pi/beta) exp(-pi^2 t^2 / beta)."""
    beta = kernel_beta(sigma, W)
    t = pixel_coords(n) / sigma
    return 1.0 / (math.sqrt(math.pi / beta) * np.exp(-(math.pi ** 2) * t * t / beta))


def grid_to_image(H: np.ndarray, n: int, sigma: float = 2.0, W: int = 6, workers: int = 1) -> np.ndarray:
    """J[q] = sum_g H[g] exp(+2 pi i (g - G/2).(q - G/2) / G) (an unnormalised
    inverse DFT, via scipy.fft in float64), then I[p] = J[p + (G - n)/2] /
    prod_a Phi(x_pa / sigma)."""
    d = H.ndim
    G = H.shape[0]
    axes = tuple(range(d))
    J = scipy.fft.fftshift(scipy.fft.ifftn(scipy.fft.ifftshift(H, axes=axes), axes=axes,
                                           workers=workers), axes=axes) * (G ** d)
    o = (G - n) // 2
    crop = J[(slice(o, o + n),) * d]
    f = deapod_factors(n, sigma, W)
    if d == 1:
        return crop * f
    return crop * f[:, None] * f[None, :]


def ftcg_image(k: np.ndarray, fhat: np.ndarray, alpha: np.ndarray, n: int,
               sigma: float = 2.0, W: int = 6, workers: int = 1) -> np.ndarray:
    """The whole path: c = alpha * fhat (D fhat), H = spread(c) (Omega D fhat),
    image = deapodized, cropped inverse FFT of H."""
    c = np.asarray(alpha, dtype=np.float64) * np.asarray(fhat, dtype=np.complex128)
    return grid_to_image(spread(k, c, n, sigma, W), n, sigma, W, workers=workers)


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_2 / ||ref||_2 over all entries."""
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


# ----------------------------------------------------------------------------
# the forward (type-2) transform: uniform image -> values at the raster, the
# adjoint of the reconstruction above (Omega^T of eq:cgmatrix after the
# forward DFT of the deapodized, zero-padded image)
# ----------------------------------------------------------------------------

def nudft_forward(k: np.ndarray, image: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """fhat_j = sum_p I[p] exp(-2 pi i k_j . x_p): the analysis sum at the raster
    (the data model fhat(lambda) = <f, phi_lambda> of Sec. III-B sampled on
    the pixel grid), direct, in chunks of samples."""
    k = np.asarray(k, dtype=np.float64)
    image = np.asarray(image, dtype=np.complex128)
    d = k.shape[1]
    n = image.shape[0]
    x = pixel_coords(n)
    out = np.zeros(k.shape[0], dtype=np.complex128)
    for b in range(0, k.shape[0], chunk):
        e0 = np.exp(-2j * np.pi * np.outer(k[b:b + chunk, 0], x))
        if d == 1:
            out[b:b + chunk] = e0 @ image
        else:
            e1 = np.exp(-2j * np.pi * np.outer(k[b:b + chunk, 1], x))
            out[b:b + chunk] = np.einsum("jp,pq,jq->j", e0, image, e1)
    return out


def image_to_grid(image: np.ndarray, n: int, sigma: float = 2.0, W: int = 6, workers: int = 1) -> np.ndarray:
    """Adjoint of grid_to_image: multiply by the deapodization factors,
    zero-pad to the centred n^d window of the G^d grid, then
    H[g] = sum_q J[q] exp(-2 pi i (g - G/2).(q - G/2) / G) (an unnormalised
    forward DFT, scipy.fft in float64)."""
    image = np.asarray(image, dtype=np.complex128)
    d = image.ndim
    G = grid_size(n, sigma)
    f = deapod_factors(n, sigma, W)
    o = (G - n) // 2
    J = np.zeros((G,) * d, dtype=np.complex128)
    if d == 1:
        J[o:o + n] = image * f
    else:
        J[o:o + n, o:o + n] = image * f[:, None] * f[None, :]
    axes = tuple(range(d))
    return scipy.fft.fftshift(scipy.fft.fftn(scipy.fft.ifftshift(J, axes=axes), axes=axes, workers=workers),
                              axes=axes)


def interpolate(k: np.ndarray, H: np.ndarray, sigma: float = 2.0, W: int = 6, chunk: int = 1 << 14) -> np.ndarray:
    """fhat_j = sum over the taps g of sample j of H[g mod G] prod_a exp(-beta (g_a - u_ja)^2),
    the same taps as spread() (Omega^T)."""
    k = np.asarray(k, dtype=np.float64)
    d = k.shape[1]
    G = H.shape[0]
    beta = kernel_beta(sigma, W)
    Hf = H.reshape(-1)
    out = np.zeros(k.shape[0], dtype=np.complex128)
    for b in range(0, k.shape[0], chunk):
        u = sigma * k[b:b + chunk] + G / 2
        i0, w0 = _axis_taps(u[:, 0], W, beta, G)
        if d == 1:
            out[b:b + chunk] = np.sum(Hf[i0] * w0, axis=1)
        else:
            i1, w1 = _axis_taps(u[:, 1], W, beta, G)
            flat = i0[:, :, None] * G + i1[:, None, :]
            out[b:b + chunk] = np.sum(Hf[flat] * (w0[:, :, None] * w1[:, None, :]), axis=(1, 2))
    return out


def forward(k: np.ndarray, image: np.ndarray, n: int, sigma: float = 2.0, W: int = 6,
            workers: int = 1) -> np.ndarray:
    """The type-2 gridding transform: interpolate(image_to_grid(image)),
    approximating nudft_forward to the kernel error."""
    return interpolate(k, image_to_grid(image, n, sigma, W, workers=workers), sigma, W)
