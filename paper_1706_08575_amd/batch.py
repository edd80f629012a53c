"""Batched FTCG over the C ABI (ftcg_batch_*): many pings of uneven size in
one persistent spreading launch, replayed from a captured hipGraph. Argument
marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .ftcg import _dptr, _stream_ptr


class Batch:
    def __init__(self, sizes, W: int = 6, sigma: float = 2.0, weights: str = "plain", R: float = 8.0,
                 stream=None, device=None):
        self.sizes = [int(n) for n in sizes]
        self.W, self.sigma, self.R = int(W), float(sigma), float(R)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        wmode = {"plain": L.FTCG_W_PLAIN, "learned": L.FTCG_W_LEARNED, "user": L.FTCG_W_USER,
                 "none": L.FTCG_W_NONE}[weights]
        self._h = C.c_void_p()
        nn = (C.c_int64 * len(self.sizes))(*self.sizes)
        L.check(L.call("ftcg_batch_create", C.byref(self._h), len(self.sizes), nn, int(W), float(sigma), wmode,
                       float(R), C.c_void_p(_stream_ptr(stream))), "ftcg_batch_create")
        self.m = None
        self.img_offsets = np.concatenate([[0], np.cumsum([n * n for n in self.sizes])])

    def close(self):
        if self._h:
            L.call("ftcg_batch_destroy", self._h)
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

    def set_tuning(self, tile: int = 32, chunk: int = 4096, blocks: int | None = None, graph: bool = True):
        if blocks is None:
            blocks = 8 * torch.cuda.get_device_properties(self.device).multi_processor_count
        L.check(L.call("ftcg_batch_set_tuning", self._h, int(tile), int(chunk), int(blocks), 1 if graph else 0),
                "ftcg_batch_set_tuning")

    def set_mlp(self, mlp, audit_threshold: float = 1e-4, audit_samples: int = 4096):
        self._mlp = mlp
        L.check(L.call("ftcg_batch_set_mlp", self._h, mlp._h, float(audit_threshold), int(audit_samples)),
                "ftcg_batch_set_mlp")

    def set_points(self, m, k: torch.Tensor):
        self.m = [int(x) for x in m]
        mm = (C.c_int64 * len(self.m))(*self.m)
        L.check(L.call("ftcg_batch_set_points", self._h, mm, C.c_void_p(_dptr(k, torch.float64, 2 * sum(self.m), "k"))),
                "ftcg_batch_set_points")

    def set_weights(self, alpha: torch.Tensor):
        L.check(L.call("ftcg_batch_set_weights", self._h, C.c_void_p(_dptr(alpha, torch.float64, sum(self.m), "alpha"))),
                "ftcg_batch_set_weights")

    def get_weights(self) -> torch.Tensor:
        out = torch.empty(sum(self.m), dtype=torch.float64, device=self.device)
        L.check(L.call("ftcg_batch_get_weights", self._h, C.c_void_p(out.data_ptr())), "ftcg_batch_get_weights")
        return out

    def execute(self, fhat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        total = int(self.img_offsets[-1])
        if out is None:
            out = torch.empty(total, dtype=torch.complex64, device=self.device)
        L.check(L.call("ftcg_batch_execute", self._h, C.c_void_p(_dptr(fhat, torch.complex64, sum(self.m), "fhat")),
                       C.c_void_p(_dptr(out, torch.complex64, total, "images"))), "ftcg_batch_execute")
        return out

    def image(self, images: torch.Tensor, i: int) -> torch.Tensor:
        a, b = int(self.img_offsets[i]), int(self.img_offsets[i + 1])
        return images[a:b].view(self.sizes[i], self.sizes[i])

    def info(self) -> dict:
        v = [C.c_int64() for _ in range(4)]
        L.check(L.call("ftcg_batch_info", self._h, *[C.byref(x) for x in v]), "ftcg_batch_info")
        return dict(zip(("tasks", "split_tiles", "records", "tiles"), (x.value for x in v)))
