"""Pins of the forward (type-2) oracle: the direct analysis sum against library
FFTs on the integer lattice, the gridded transform against the direct sum
(kernel error, including samples outside the k-box), exact adjointness with
the reconstruction (the forward transform is Omega^T F^- P^T applied to the
image: the conjugate transpose of the path of eq:cgmatrix), and the error
falling with the kernel width. Planted mistakes at the end each fail a pin.
"""
import numpy as np
import pytest

import oracle as O
import oracle.ftcg_ref as OR
from paper_1706_08575_amd import synth as S


def _image(n, d, seed):
    rng = np.random.default_rng(seed)
    shape = (n,) * d
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_direct_sum_on_lattice_is_fft():
    n = 32
    I1 = _image(n, 1, 1)
    k1 = S.integer_raster_1d(n)
    ref1 = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(I1)))
    assert np.max(np.abs(O.nudft_forward(k1, I1) - ref1)) < 1e-11 * np.max(np.abs(ref1))
    I2 = _image(n, 2, 2)
    g = np.arange(n) - n // 2
    k2 = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2).astype(np.float64)
    ref2 = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(I2))).reshape(-1)
    assert np.max(np.abs(O.nudft_forward(k2, I2) - ref2)) < 1e-11 * np.max(np.abs(ref2))


def test_forward_vs_direct_sum():
    rng = np.random.default_rng(3)
    n = 64
    k1 = rng.uniform(-0.6 * n, 0.6 * n, size=(700, 1))        # some outside the k-box: wrap
    I1 = _image(n, 1, 4)
    assert O.rel_l2(O.forward(k1, I1, n), O.nudft_forward(k1, I1)) < 1e-5
    n2 = 32
    k2 = rng.uniform(-0.6 * n2, 0.6 * n2, size=(900, 2))
    I2 = _image(n2, 2, 5)
    assert O.rel_l2(O.forward(k2, I2, n2), O.nudft_forward(k2, I2)) < 1e-5


def test_forward_is_adjoint_of_reconstruction():
    # <A c, I> = <c, A^H I> with A the gridding reconstruction (unit weights)
    rng = np.random.default_rng(6)
    for d, n, m in ((1, 64, 300), (2, 16, 400)):
        k = rng.uniform(-0.55 * n, 0.55 * n, size=(m, d))
        c = S.random_values(7, m)
        I = _image(n, d, 8)
        lhs = np.vdot(O.ftcg_image(k, c, np.ones(m), n), I)
        rhs = np.vdot(c, O.forward(k, I, n))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_forward_error_falls_with_width():
    rng = np.random.default_rng(9)
    n = 64
    k = rng.uniform(-0.5 * n, 0.5 * n, size=(400, 1))
    I = _image(n, 1, 10)
    ref = O.nudft_forward(k, I)
    errs = [O.rel_l2(O.forward(k, I, n, W=W), ref) for W in (2, 3, 4, 5, 6)]
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

_good_deapod = OR.deapod_factors
_good_interp = OR.interpolate


def _to_grid_inverse_sign(image, n, sigma=2.0, W=6, workers=1):
    import scipy.fft
    d = image.ndim
    G = OR.grid_size(n, sigma)
    f = _good_deapod(n, sigma, W)
    o = (G - n) // 2
    J = np.zeros((G,) * d, dtype=np.complex128)
    J[(slice(o, o + n),) * d] = image * (f if d == 1 else f[:, None] * f[None, :])
    ax = tuple(range(d))
    return scipy.fft.fftshift(scipy.fft.ifftn(scipy.fft.ifftshift(J, axes=ax), axes=ax), axes=ax) * G ** d


def _to_grid_no_deapod(image, n, sigma=2.0, W=6, workers=1):
    import scipy.fft
    d = image.ndim
    G = OR.grid_size(n, sigma)
    o = (G - n) // 2
    J = np.zeros((G,) * d, dtype=np.complex128)
    J[(slice(o, o + n),) * d] = image
    ax = tuple(range(d))
    return scipy.fft.fftshift(scipy.fft.fftn(scipy.fft.ifftshift(J, axes=ax), axes=ax), axes=ax)


def _interp_shifted(k, H, sigma=2.0, W=6, chunk=1 << 14):
    return _good_interp(np.asarray(k, dtype=np.float64) + 1.0 / sigma, H, sigma, W, chunk)


PLANTS = {
    "fft_inverse_sign": ("image_to_grid", _to_grid_inverse_sign),
    "missing_deapodization": ("image_to_grid", _to_grid_no_deapod),
    "interpolation_off_by_one_cell": ("interpolate", _interp_shifted),
}
PINS = [test_forward_vs_direct_sum, test_forward_is_adjoint_of_reconstruction]


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_forward_planted_mistake_is_caught(plant, monkeypatch):
    name, fn = PLANTS[plant]
    monkeypatch.setattr(OR, name, fn)
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, plant
