"""Pins of the CPU FP64 oracle against facts fixed by the mathematics, not by the
oracle itself: library routines in special cases, closed forms, brute force on
tiny inputs, invariants, and the kernel-width/oversampling error behaviour.
Each pin is chosen so that a plausible mistake in the oracle (a dropped term,
a wrong sign or index, a transposed operand) fails at least one of them; the
planted-mistake tests at the end check that claim for a few such mistakes.
"""
import math

import numpy as np
import pytest
import scipy.fft

import oracle as O
import oracle.ftcg_ref as OR
from paper_1706_08575_amd import synth as S


# ---------------------------------------------------------------------------
# the definition (weighted NUDFT) against library FFTs
# ---------------------------------------------------------------------------

def test_nudft_integer_raster_is_ifft():
    # k_j = j - n/2 on the integer lattice: sum_j c_j e^{2 pi i (j - n/2)(p - n/2)/n}
    # is n * fftshift(ifft(ifftshift(c))) (library routine).
    n = 64
    k = S.integer_raster_1d(n)
    c = S.random_values(3, n)
    ref = n * np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(c)))
    assert np.max(np.abs(O.nudft(k, c, n) - ref)) < 1e-11 * np.max(np.abs(ref))


def test_nudft_2d_integer_raster_is_ifft2():
    n = 16
    j0, j1 = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    k = np.stack([j0.ravel(), j1.ravel()], axis=1).astype(np.float64)
    c = S.random_values(4, n * n)
    ref = n * n * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(c.reshape(n, n))))
    assert np.max(np.abs(O.nudft(k, c, n) - ref)) < 1e-11 * np.max(np.abs(ref))


def test_nudft_at_matches_grid():
    k, f, _ = S.make_sas(11, 32, 8, 16)
    n = 32
    I = O.nudft(k, f, n)
    x = O.pixel_coords(n)
    pts = np.array([[x[3], x[7]], [x[0], x[31]], [x[16], x[16]]])
    v = O.nudft_at(k, f, pts)
    ref = np.array([I[3, 7], I[0, 31], I[16, 16]])
    assert np.max(np.abs(v - ref)) < 1e-10 * np.max(np.abs(I))


# ---------------------------------------------------------------------------
# the gridding pipeline against the definition (brute force on tiny inputs)
# ---------------------------------------------------------------------------

def test_pipeline_1d_vs_nudft():
    k, f, _ = S.make_1d()
    a = O.frame_weights(k, 8.0)
    I = O.ftcg_image(k, f, a, 256)
    ref = O.nudft(k, a * f, 256)
    assert O.rel_l2(I, ref) < 1e-5


def test_pipeline_2d_vs_nudft():
    k, f, _ = S.make_sas(5, 64, 32, 96)
    a = O.frame_weights(k, 8.0)
    I = O.ftcg_image(k, f, a, 64)
    ref = O.nudft(k, a * f, 64)
    assert O.rel_l2(I, ref) < 1e-5


def test_pipeline_2d_odd_spread_outside_box_wraps():
    # samples outside the k-box [-n/2, n/2) wrap on the grid; pixel-centred
    # evaluation of the definition is n-periodic in k, so the result still
    # matches the definition
    rng = np.random.default_rng(7)
    n = 32
    k = rng.uniform(-1.3 * n, 1.3 * n, size=(500, 2))
    c = S.random_values(8, 500)
    I = O.grid_to_image(O.spread(k, c, n), n)
    assert O.rel_l2(I, O.nudft(k, c, n)) < 1e-5


def test_kernel_width_error_slope():
    k, f, _ = S.make_1d()
    a = O.frame_weights(k, 8.0)
    ref = O.nudft(k, a * f, 256)
    errs = [O.rel_l2(O.ftcg_image(k, f, a, 256, W=W), ref) for W in range(2, 9)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    slope = -np.polyfit(np.arange(2, 9), np.log(errs), 1)[0]
    assert 1.8 < slope < 2.7, slope


def test_oversampling_error_monotone():
    k, f, _ = S.make_1d()
    a = O.frame_weights(k, 8.0)
    ref = O.nudft(k, a * f, 256)
    errs = [O.rel_l2(O.ftcg_image(k, f, a, 256, sigma=s), ref) for s in (1.25, 1.5, 2.0)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_trig_polynomial_recovered():
    # samples of a trigonometric polynomial's coefficients on the integer
    # lattice, weights 1: the image is the polynomial at the pixels
    n = 128
    k = S.integer_raster_1d(n)
    a_l = S.random_values(9, n)
    a_l[0] = 0.0  # keep |l| < n/2 strictly
    x = O.pixel_coords(n)
    p = np.exp(2j * np.pi * np.outer(x, k[:, 0])) @ a_l
    alpha = O.frame_weights(k, 8.0)
    assert np.max(np.abs(alpha - 1.0)) < 1e-14
    assert np.max(np.abs(O.nudft(k, alpha * a_l, n) - p)) < 1e-10 * np.max(np.abs(p))
    assert O.rel_l2(O.ftcg_image(k, a_l, alpha, n), p) < 1e-5


def test_unit_sample_at_origin_gives_ones():
    # one sample at k = 0 with value 1: I == 1 everywhere, up to kernel error;
    # this pins the deapodization factors against the kernel
    for d, n in ((1, 256), (2, 64)):
        k = np.zeros((1, d))
        I = O.ftcg_image(k, np.ones(1), np.ones(1), n)
        assert np.max(np.abs(I - 1.0)) < 1e-5, d


def test_fft_step_vs_direct_sum():
    # J[q] = sum_g H[g] e^{+2 pi i (g - G/2)(q - G/2)/G}, checked by a direct sum
    rng = np.random.default_rng(1)
    G, n = 16, 8
    H = rng.standard_normal((G, G)) + 1j * rng.standard_normal((G, G))
    g = np.arange(G) - G // 2
    E = np.exp(2j * np.pi * np.outer(g, g) / G)
    J = E.T @ H @ E  # J[q0, q1] = sum E[g0,q0] H[g0,g1] E[g1,q1]
    o = (G - n) // 2
    f = O.deapod_factors(n)
    ref = J[o:o + n, o:o + n] * f[:, None] * f[None, :]
    assert np.max(np.abs(O.grid_to_image(H, n) - ref)) < 1e-12 * np.max(np.abs(ref))


def test_linearity_and_integer_shift():
    k, f, _ = S.make_sas(12, 32, 12, 24)
    n = 32
    a = np.ones(len(f))
    g = S.random_values(13, len(f))
    I1 = O.ftcg_image(k, f, a, n)
    I2 = O.ftcg_image(k, g, a, n)
    I12 = O.ftcg_image(k, 2.0 * f - 3j * g, a, n)
    assert O.rel_l2(I12, 2.0 * I1 - 3j * I2) < 1e-13
    s = np.array([3.0, -5.0])
    Is = O.ftcg_image(k + s, f, a, n)
    x = O.pixel_coords(n)
    mod = np.exp(2j * np.pi * (s[0] * x[:, None] + s[1] * x[None, :]))
    assert O.rel_l2(Is, I1 * mod) < 1e-12


def test_hermitian_samples_give_real_image():
    rng = np.random.default_rng(2)
    n = 32
    kh = rng.uniform(-12, 12, size=(200, 2))
    ch = S.random_values(14, 200)
    k = np.concatenate([kh, -kh])
    c = np.concatenate([ch, np.conj(ch)])
    I = O.ftcg_image(k, c, np.ones(400), n)
    assert np.max(np.abs(I.imag)) < 1e-12 * np.max(np.abs(I.real))


# ---------------------------------------------------------------------------
# frame weights (eq:difopt)
# ---------------------------------------------------------------------------

def test_weights_integer_lattice_exactly_one():
    for R in (3.0, 8.0, np.inf):
        assert np.max(np.abs(O.frame_weights(S.integer_raster_1d(64), R) - 1.0)) < 1e-15
    j0, j1 = np.meshgrid(np.arange(24) - 12, np.arange(24) - 12, indexing="ij")
    k = np.stack([j0.ravel(), j1.ravel()], axis=1).astype(np.float64)
    assert np.max(np.abs(O.frame_weights(k, 8.0) - 1.0)) < 1e-15


def test_weights_uniform_spacing_tend_to_h():
    # sum_n sinc^2(h n + x) = 1/h for h <= 1 (Poisson summation of the
    # triangle), so interior weights tend to h as R grows
    for h in (0.5, 0.25):
        m = int(256 / h)
        k = (np.arange(m) - m // 2) * h
        a = O.frame_weights(k.reshape(-1, 1), np.inf)
        mid = a[len(a) // 2 - 5: len(a) // 2 + 5]
        assert np.max(np.abs(mid - h)) < 2e-3 * h, (h, mid)


def test_weights_tensor_raster_separable():
    rng = np.random.default_rng(5)
    kx = np.arange(30) - 15 + rng.uniform(-0.25, 0.25, 30)
    ky = 0.7 * (np.arange(26) - 13) + rng.uniform(-0.2, 0.2, 26)
    a1x = O.frame_weights(kx.reshape(-1, 1), 8.0)
    a1y = O.frame_weights(ky.reshape(-1, 1), 8.0)
    X, Y = np.meshgrid(kx, ky, indexing="ij")
    k2 = np.stack([X.ravel(), Y.ravel()], axis=1)
    a2 = O.frame_weights(k2, 8.0)
    # 1/alpha2 = (1/alpha_x)(1/alpha_y) because the infinity-norm box is a product
    assert np.max(np.abs(a2 - np.outer(a1x, a1y).ravel()) / a2) < 1e-13


def test_weights_are_columnwise_least_squares():
    # min over diagonal D of ||T D - I||_F: each column n is a one-unknown
    # least-squares problem min_a ||a T[:, n] - e_n||, solved by numpy lstsq
    rng = np.random.default_rng(6)
    k = np.sort(rng.uniform(-20, 20, 40)).reshape(-1, 1)
    T = np.sinc(k - k.T)
    alpha = O.frame_weights(k, np.inf)
    for nn in range(40):
        e = np.zeros(40)
        e[nn] = 1.0
        sol = np.linalg.lstsq(T[:, nn:nn + 1], e, rcond=None)[0][0]
        assert abs(sol - alpha[nn]) < 1e-13 * abs(sol)
    # and the diagonal optimum beats perturbed diagonals
    base = np.linalg.norm(T @ np.diag(alpha) - np.eye(40))
    for s in (0.99, 1.01):
        assert np.linalg.norm(T @ np.diag(alpha * s) - np.eye(40)) > base


def test_weights_tree_vs_dense_masked():
    rng = np.random.default_rng(8)
    k = rng.uniform(-15, 15, size=(300, 2))
    R = 4.0
    D = np.max(np.abs(k[:, None, :] - k[None, :, :]), axis=2)
    T = np.prod(np.sinc(k[:, None, :] - k[None, :, :]), axis=2) * (D <= R)
    ref = 1.0 / np.sum(T * T, axis=0)
    assert np.max(np.abs(O.frame_weights(k, R) - ref) / ref) < 1e-13
    idx = np.array([0, 17, 299])
    assert np.max(np.abs(O.frame_weights_at(k, idx, R) - ref[idx]) / ref[idx]) < 1e-13


def test_spread_window_is_a_window_of_spread():
    # the windowed spread equals the full (pinned) spread on its window, for
    # interior windows, windows on the periodic seam and samples outside the
    # k-box, and is zero where no sample reaches
    rng = np.random.default_rng(81)
    n = 32
    G = 64
    k = rng.uniform(-0.7 * n, 0.7 * n, size=(900, 2))
    k[:30] = n / 2 - 0.02 * rng.random((30, 2))          # u next to G (taps wrap)
    c = S.random_values(82, k.shape[0])
    H = O.spread(k, c, n)
    for r0, c0, h, w in ((0, 0, 16, 16), (24, 40, 8, 24), (48, 48, 16, 16), (60, 0, 4, 64), (0, 0, G, G)):
        Hw = O.spread_window(k, c, n, r0, c0, h, w)
        assert np.max(np.abs(Hw - H[r0:r0 + h, c0:c0 + w])) < 1e-13 * np.max(np.abs(H))
    kk = np.array([[0.1, 0.2]])
    assert np.all(O.spread_window(kk, np.ones(1), n, 0, 0, 8, 8) == 0)


# ---------------------------------------------------------------------------
# the pins have teeth: each planted mistake in the oracle fails at least one pin
# ---------------------------------------------------------------------------

_good_deapod = OR.deapod_factors
_good_taps = OR._axis_taps


def _taps_shifted(u, W, beta, G):
    g, w = _good_taps(u, W, beta, G)
    return np.mod(g + 1, G), w            # off-by-one grid index


def _taps_no_square(u, W, beta, G):
    lo = np.ceil(u - W)
    g = lo[:, None] + np.arange(2 * W + 1)[None, :]
    dist = g - u[:, None]
    w = np.where(np.abs(dist) <= W, np.exp(-beta * np.abs(dist)), 0.0)  # wrong kernel
    return np.mod(g, G).astype(np.int64), w


def _fft_forward(H, n, sigma=2.0, W=6, workers=1):
    G = H.shape[0]
    ax = tuple(range(H.ndim))
    J = scipy.fft.fftshift(scipy.fft.fftn(scipy.fft.ifftshift(H, axes=ax), axes=ax), axes=ax)
    o = (G - n) // 2
    f = _good_deapod(n, sigma, W)
    return J[o:o + n] * f if H.ndim == 1 else J[o:o + n, o:o + n] * f[:, None] * f[None, :]


PLANTS = {
    "gram_of_sum_not_difference": ("_gram_entries", lambda ki, kj: np.prod(np.sinc(ki + kj), axis=1)),
    "gram_not_squared_in_sum": ("_gram_entries", lambda ki, kj: np.sqrt(np.abs(np.prod(np.sinc(ki - kj), axis=1)))),
    "deapod_of_wrong_kernel": ("deapod_factors", lambda n, sigma=2.0, W=6: _good_deapod(n, sigma, W + 1)),
    "spread_index_off_by_one": ("_axis_taps", _taps_shifted),
    "spread_kernel_not_gaussian": ("_axis_taps", _taps_no_square),
    "fft_forward_not_inverse": ("grid_to_image", _fft_forward),
}

PINS = [test_pipeline_1d_vs_nudft, test_pipeline_2d_vs_nudft, test_unit_sample_at_origin_gives_ones,
        test_trig_polynomial_recovered, test_weights_uniform_spacing_tend_to_h,
        test_weights_are_columnwise_least_squares, test_weights_tree_vs_dense_masked,
        test_weights_tensor_raster_separable]


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_mistake_is_caught(plant, monkeypatch):
    name, fn = PLANTS[plant]
    monkeypatch.setattr(OR, name, fn)
    failed = []
    for pin in PINS:
        try:
            pin()
        except (AssertionError, FloatingPointError, ZeroDivisionError):
            failed.append(pin.__name__)
    assert failed, plant
