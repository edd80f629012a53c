"""GPU parity of the iterative density compensation (FTCG_W_DENSITY: the
iterative quadrature weights cited in Sec. III-A, w <- w / (Omega^T Omega w))
against the FP64 oracle (oracle.pipe_menon_weights), through the C ABI.

Tolerances: float64 plans 1e-10 relative per weight. Float32 plans spread and
interpolate in float32 (fixed-point tile sums, float32 taps), about 1e-6
relative per product, and each iteration divides by a fresh product: after
20 iterations 1e-4 relative per weight, 2e-5 rel L2 over the weights. Images
with these weights against the oracle fed the same weights: 2e-5.
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


def run_density(k, f, n, iters, dtype="f32"):
    from paper_1706_08575_amd.ftcg import Plan
    cd = torch.complex64 if dtype == "f32" else torch.complex128
    with Plan(n, dim=k.shape[1], dtype=dtype, weights="density") as P:
        P.set_density_iterations(iters)
        P.set_points(dev(k))
        a = host(P.get_weights())
        img = host(P.execute(dev(f, cd)))
    return a, img


def test_density_1d_f64():
    k, f, _ = S.make_1d()
    a, img = run_density(k, f, 256, 12, "f64")
    ref = O.pipe_menon_weights(k, 256, 12)
    assert np.max(np.abs(a - ref) / ref) < 1e-10
    assert O.rel_l2(img, O.ftcg_image(k, f, ref, 256)) < 1e-9


@pytest.mark.parametrize("n,pulses,per_pulse", [(128, 64, 128), (256, 128, 512)])
def test_density_2d_sas_f32(n, pulses, per_pulse):
    k, f, _ = S.make_sas(S.seed_for(1) + 80, n=n, pulses=pulses, per_pulse=per_pulse)
    a, img = run_density(k, f, n, 20)
    ref = O.pipe_menon_weights(k, n, 20)
    rel = (a - ref) / ref
    print(f"density {n}^2: max rel {np.max(np.abs(rel)):.2e}, rms rel {np.sqrt(np.mean(rel ** 2)):.2e}")
    assert np.max(np.abs(rel)) < 1e-4
    assert np.sqrt(np.mean(rel ** 2)) < 2e-5
    assert O.rel_l2(img, O.ftcg_image(k, f, a, n)) < 2e-5


def test_density_lattice_gpu():
    # a uniform lattice of spacing 1/2 gives equal weights of h^2 = 1/4 up to
    # the kernel's truncation (the same closed form the oracle is pinned to)
    n = 64
    g = (np.arange(2 * n) - n) / 2.0
    k = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    a, _ = run_density(k, np.ones(len(k), dtype=np.complex128), n, 3, "f64")
    assert np.max(np.abs(a / 0.25 - 1.0)) < 3e-5


def test_density_state_errors():
    from paper_1706_08575_amd import _lib as L
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(64, dim=2) as P:
        with pytest.raises(L.FtcgError) as e:
            P.set_density_iterations(5)
        assert e.value.status == L.FTCG_ESTATE
    with Plan(64, dim=2, weights="density") as P:
        for it in (0, 1001):
            with pytest.raises(L.FtcgError) as e:
                P.set_density_iterations(it)
            assert e.value.status == L.FTCG_EINVAL
