"""The allocation-free grid-to-image entry point (ftcg_grid_to_image_noalloc)
against ftcg_grid_to_image of a plan (same kernels, so bit for bit), through
the C ABI: two calls in a row per case, the second on a smaller grid (the
static workspace keeps the first call's contents), 2D and 1D, float32 and
float64, and sizes beyond its workspace rejected before any GPU work."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _grid(G, dim, dtype, seed):
    rng = np.random.default_rng(seed)
    shape = (G,) * dim
    h = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return torch.from_numpy(h.astype(np.complex64 if dtype == "f32" else np.complex128)).cuda()


def _noalloc(dim, n, dtype, H):
    from paper_1706_08575_amd import _lib as L
    cd = H.dtype
    out = torch.empty((n,) * dim, dtype=cd, device="cuda")
    st = L.call("ftcg_grid_to_image_noalloc", dim, n, 6, 2.0, L.FTCG_F32 if dtype == "f32" else L.FTCG_F64,
                C.c_void_p(H.data_ptr()), C.c_void_p(out.data_ptr()),
                C.c_void_p(int(torch.cuda.current_stream().cuda_stream)))
    assert st == L.FTCG_OK, L.status_string(st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _plan(dim, n, dtype, H):
    from paper_1706_08575_amd.ftcg import Plan
    with Plan(n, dim=dim, dtype=dtype, weights="none") as P:
        img = P.grid_to_image(H)
        torch.cuda.synchronize()
        return img.cpu().numpy()


@pytest.mark.parametrize("dim,dtype,sizes", [(2, "f32", (1024, 256)), (2, "f64", (512, 128)),
                                             (1, "f64", (4096, 512)), (1, "f32", (8192, 64))])
def test_noalloc_equals_plan_twice(dim, dtype, sizes):
    for i, n in enumerate(sizes):
        H = _grid(2 * n, dim, dtype, 100 * dim + i)
        got = _noalloc(dim, n, dtype, H)
        ref = _plan(dim, n, dtype, H)
        assert np.array_equal(got, ref), (dim, dtype, n)


def test_noalloc_rejects_beyond_workspace():
    from paper_1706_08575_amd import _lib as L
    H = torch.zeros(8, dtype=torch.complex64, device="cuda")   # never read: rejected before any launch
    for dim, n, dt in ((2, 2048, L.FTCG_F32), (2, 2048, L.FTCG_F64)):
        st = L.call("ftcg_grid_to_image_noalloc", dim, n, 6, 2.0, dt, C.c_void_p(H.data_ptr()),
                    C.c_void_p(H.data_ptr()), None)
        assert st == L.FTCG_EUNSUPPORTED
    st = L.call("ftcg_grid_to_image_noalloc", 2, 100, 6, 2.0, L.FTCG_F32, None, C.c_void_p(H.data_ptr()), None)
    assert st == L.FTCG_EINVAL
