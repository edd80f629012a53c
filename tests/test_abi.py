"""CPU checks of the C ABI: the library loads, exports every entry point that
include/ftcg.h declares, and rejects invalid arguments with the documented
status codes before touching the GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1706_08575_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ftcg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ftcg_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = header_functions()
    for must in ("ftcg_plan_create", "ftcg_set_points", "ftcg_execute", "ftcg_plan_destroy",
                 "ftcg_set_weights", "ftcg_get_weights", "ftcg_status_string"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) <= set(L.EXPORTED)


def test_status_strings():
    for s in range(6):
        assert L.status_string(s).startswith("FTCG_")
    assert "unknown" in L.status_string(99)


def _create(dim=2, n=64, W=6, sigma=2.0, dtype=L.FTCG_F32, wmode=L.FTCG_W_PLAIN, R=8.0):
    h = C.c_void_p()
    nn = (C.c_int64 * 2)(n, n)
    st = L.call("ftcg_plan_create", C.byref(h), dim, nn, W, sigma, dtype, wmode, R, None)
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(dim=3), L.FTCG_EINVAL),
    (dict(n=63), L.FTCG_EINVAL),
    (dict(n=4), L.FTCG_EINVAL),
    (dict(W=1), L.FTCG_EINVAL),
    (dict(W=9), L.FTCG_EINVAL),
    (dict(sigma=1.0), L.FTCG_EINVAL),
    (dict(sigma=2.1), L.FTCG_EINVAL),          # sigma * n not an integer
    (dict(sigma=1.5), L.FTCG_EUNSUPPORTED),    # G = 96 not a power of two
    (dict(R=0.0), L.FTCG_EINVAL),
    (dict(R=float("nan")), L.FTCG_EINVAL),
    (dict(dtype=7), L.FTCG_EINVAL),
    (dict(wmode=9), L.FTCG_EINVAL),
    (dict(n=8192, dtype=L.FTCG_F64), L.FTCG_EUNSUPPORTED),   # G = 16384 float64 row exceeds LDS
])
def test_plan_create_rejects(kw, status):
    st, h = _create(**kw)
    assert st == status
    assert not h.value


def test_null_arguments():
    assert L.call("ftcg_plan_create", None, 2, None, 6, 2.0, 1, 0, 8.0, None) == L.FTCG_EINVAL
    for name, args in (("ftcg_plan_destroy", (None,)), ("ftcg_set_points", (None, 10, None)),
                       ("ftcg_execute", (None, None, None)), ("ftcg_set_weights", (None, None)),
                       ("ftcg_get_weights", (None, None, None)), ("ftcg_plan_set_tuning", (None, 64, 0, 1)),
                       ("ftcg_plan_set_spread_layout", (None, 0)),
                       ("ftcg_plan_info", (None, None, None, None, None)),
                       ("ftcg_spread_only", (None, None, None)), ("ftcg_grid_to_image", (None, None, None)),
                       ("ftcg_plan_enable_timing", (None, 1)), ("ftcg_plan_timing", (None, None, None)),
                       ("ftcg_mlp_create", (None, None)), ("ftcg_mlp_destroy", (None,)),
                       ("ftcg_mlp_set_params", (None, None, 6337)), ("ftcg_mlp_get_params", (None, None, 6337)),
                       ("ftcg_mlp_save", (None, None, None)), ("ftcg_mlp_load", (None, None, 0)),
                       ("ftcg_mlp_features", (None, 1, None, 8.0, None, None, None)),
                       ("ftcg_mlp_forward", (None, 1, None, None)),
                       ("ftcg_mlp_loss_grad", (None, 1, None, None, 0, None, None)),
                       ("ftcg_mlp_train_batch", (None, 1, None, None, 0, 0.0, None)),
                       ("ftcg_mlp_train_raster", (None, 1, None, 8.0, 16, 0.0, 0, None)),
                       ("ftcg_plan_set_mlp", (None, None, 1e-4, 16)),
                       ("ftcg_plan_learned_report", (None, None, None))):
        assert L.call(name, *args) == L.FTCG_EINVAL, name
