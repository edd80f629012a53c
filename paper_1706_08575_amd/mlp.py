"""Learned frame-weight network over the C ABI (ftcg_mlp_*), taking torch
device tensors for data and numpy/dict for parameters. Argument marshalling
only: features, inference, gradients and Adam run in libftcg."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .ftcg import _dptr, _stream_ptr

SHAPES = (("W1", (32, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 1)), ("b3", (1,)))


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[n], dtype=np.float32).ravel() for n, _ in SHAPES])


def unflatten(v: np.ndarray) -> dict:
    out, o = {}, 0
    for n, s in SHAPES:
        c = int(np.prod(s))
        out[n] = np.asarray(v[o:o + c], dtype=np.float32).reshape(s)
        o += c
    return out


class Mlp:
    def __init__(self, params: dict | None = None, stream=None, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._h = C.c_void_p()
        L.check(L.call("ftcg_mlp_create", C.byref(self._h), C.c_void_p(_stream_ptr(stream))), "ftcg_mlp_create")
        if params is not None:
            self.set_params(params)

    def close(self):
        if self._h:
            L.call("ftcg_mlp_destroy", self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_params(self, params: dict) -> None:
        v = np.ascontiguousarray(flatten(params))
        L.check(L.call("ftcg_mlp_set_params", self._h, v.ctypes.data_as(C.c_void_p), v.size), "ftcg_mlp_set_params")

    def get_params(self) -> dict:
        v = np.empty(L.MLP_NPARAM, dtype=np.float32)
        L.check(L.call("ftcg_mlp_get_params", self._h, v.ctypes.data_as(C.c_void_p), v.size), "ftcg_mlp_get_params")
        return unflatten(v)

    def save(self) -> bytes:
        n = C.c_size_t(0)
        L.check(L.call("ftcg_mlp_save", self._h, None, C.byref(n)), "ftcg_mlp_save")
        buf = (C.c_ubyte * n.value)()
        L.check(L.call("ftcg_mlp_save", self._h, C.cast(buf, C.c_void_p), C.byref(n)), "ftcg_mlp_save")
        return bytes(buf)

    def load(self, blob: bytes) -> None:
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        L.check(L.call("ftcg_mlp_load", self._h, C.cast(buf, C.c_void_p), len(blob)), "ftcg_mlp_load")

    def features(self, k: torch.Tensor, R: float = 8.0, with_target: bool = False):
        m = int(k.shape[0])
        feat = torch.empty((m, 32), dtype=torch.float32, device=self.device)
        base = torch.empty(m, dtype=torch.float64, device=self.device)
        tgt = torch.empty(m, dtype=torch.float32, device=self.device) if with_target else None
        L.check(L.call("ftcg_mlp_features", self._h, m, C.c_void_p(_dptr(k, torch.float64, 2 * m, "k")),
                       float(R), C.c_void_p(feat.data_ptr()), C.c_void_p(base.data_ptr()),
                       C.c_void_p(tgt.data_ptr()) if tgt is not None else None), "ftcg_mlp_features")
        return (feat, base, tgt) if with_target else (feat, base)

    def forward(self, feat: torch.Tensor) -> torch.Tensor:
        n = int(feat.shape[0])
        y = torch.empty(n, dtype=torch.float32, device=self.device)
        L.check(L.call("ftcg_mlp_forward", self._h, n, C.c_void_p(_dptr(feat, torch.float32, 32 * n, "feat")),
                       C.c_void_p(y.data_ptr())), "ftcg_mlp_forward")
        return y

    def loss_grad(self, feat: torch.Tensor, target: torch.Tensor, fp16: bool = False):
        n = int(feat.shape[0])
        g = torch.empty(L.MLP_NPARAM, dtype=torch.float32, device=self.device)
        loss = C.c_double(0.0)
        L.check(L.call("ftcg_mlp_loss_grad", self._h, n, C.c_void_p(_dptr(feat, torch.float32, 32 * n, "feat")),
                       C.c_void_p(_dptr(target, torch.float32, n, "target")), 1 if fp16 else 0,
                       C.c_void_p(g.data_ptr()), C.byref(loss)), "ftcg_mlp_loss_grad")
        return loss.value, g

    def train_batch(self, feat: torch.Tensor, target: torch.Tensor, lr: float, fp16: bool = True) -> float:
        n = int(feat.shape[0])
        loss = C.c_double(0.0)
        L.check(L.call("ftcg_mlp_train_batch", self._h, n, C.c_void_p(_dptr(feat, torch.float32, 32 * n, "feat")),
                       C.c_void_p(_dptr(target, torch.float32, n, "target")), 1 if fp16 else 0, float(lr),
                       C.byref(loss)), "ftcg_mlp_train_batch")
        return loss.value

    def train_raster(self, k: torch.Tensor, lr: float, R: float = 8.0, batch: int = 4096, fp16: bool = True) -> float:
        m = int(k.shape[0])
        loss = C.c_double(0.0)
        L.check(L.call("ftcg_mlp_train_raster", self._h, m, C.c_void_p(_dptr(k, torch.float64, 2 * m, "k")),
                       float(R), int(batch), float(lr), 1 if fp16 else 0, C.byref(loss)), "ftcg_mlp_train_raster")
        return loss.value
