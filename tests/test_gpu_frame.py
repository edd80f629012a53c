"""GPU parity of the dense frame approximation (ftcg_frame_approx: Sec. III-B
eq:binv, eq:afr, eq:afrm; Sec. IV eq:twodframeB) against the FP64 oracle
(oracle.frame_image: Gauss-Legendre inner products and numpy lstsq), through
the C ABI, in the least-squares case (samples at least as many as modes) and
the minimum-norm case, on jittered rasters and the noisy grid of Sec. V-A.

Tolerance: both sides are backward-stable float64 least-squares solvers, so
they agree to about the condition number of Psi times the float64 rounding;
1e-8 rel L2 on the images (the condition numbers here are below 1e4).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1706_08575_amd import synth as S

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def run_frame(k, f, n):
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(n, dim=k.shape[1], dtype="f64", weights="none") as P:
        return host(P.frame_approx(dev(k), dev(f, torch.complex128)))


@pytest.mark.parametrize("n,m", [(32, 64), (64, 40)])
def test_frame_1d(n, m):
    rng = np.random.default_rng(n + m)
    k = (np.arange(m) - m / 2 + rng.uniform(-0.25, 0.25, m)).reshape(m, 1) * (n / m if m < n else 1.0)
    f = S.random_values(5, m)
    img = run_frame(k, f, n)
    ref = O.frame_image(k, f, n)
    err = O.rel_l2(img, ref)
    print(f"1D frame n={n} m={m}: rel L2 {err:.2e}")
    assert err < 1e-8


@pytest.mark.parametrize("side,n", [(20, 16), (30, 32)])
def test_frame_2d_noisy_grid(side, n):
    # 20 x 20 raster on 16^2 modes (least squares), 30 x 30 on 32^2 (minimum
    # norm), data of the test function of Sec. V
    k = S.noisy_grid(S.seed_for(5) + side, side)
    f = S.sine_test_fourier(k)
    img = run_frame(k, f, n)
    ref = O.frame_image(k, f, n)
    err = O.rel_l2(img, ref)
    x = (np.arange(n) - n / 2) / n
    truth = S.sine_test_function(np.stack(np.meshgrid(x, x, indexing="ij"), -1))
    psnr = 20 * np.log10(np.max(np.abs(truth)) / np.sqrt(np.mean(np.abs(img - truth) ** 2)))
    print(f"2D frame {side}^2 samples, {n}^2 modes: rel L2 vs oracle {err:.2e}, PSNR vs f {psnr:.2f} dB")
    assert err < 1e-8


def test_frame_rank_deficient_rejected():
    # fewer samples than modes with two samples at one location: Psi^T has
    # two equal columns, R a zero pivot
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    k = np.linspace(-10, 10, 20).reshape(20, 1)
    k[5] = k[4]
    with Plan(32, dim=1, dtype="f64", weights="none") as P:
        with pytest.raises(L.FtcgError) as e:
            P.frame_approx(dev(k), dev(np.ones(20), torch.complex128))
        assert e.value.status == L.FTCG_EINVAL


def test_frame_limits():
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(32, dim=2, dtype="f32", weights="none") as P:     # float64 plans only
        with pytest.raises(L.FtcgError) as e:
            P.frame_approx(dev(np.zeros((4, 2))), dev(np.ones(4), torch.complex128))
        assert e.value.status == L.FTCG_EUNSUPPORTED
    with Plan(128, dim=2, dtype="f64", weights="none") as P:    # 16384 modes
        with pytest.raises(L.FtcgError) as e:
            P.frame_approx(dev(np.zeros((4, 2))), dev(np.ones(4), torch.complex128))
        assert e.value.status == L.FTCG_EUNSUPPORTED
