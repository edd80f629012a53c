"""Plan object over the C ABI, taking torch device tensors.

PyTorch only provides device memory and the HIP stream here; every step of
weighting, binning, spreading, FFT and deapodization runs in libftcg.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dptr(t: torch.Tensor, dtype: torch.dtype, numel: int, name: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


class Plan:
    """One FTCG reconstruction geometry: image size n (per axis), dimension,
    kernel half-width W, oversampling sigma, precision, weight mode and the
    weight neighbourhood R. See include/ftcg.h for the conventions."""

    def __init__(self, n: int, dim: int = 2, W: int = 6, sigma: float = 2.0, dtype: str = "f32",
                 weights: str = "plain", R: float = 8.0, stream=None, device=None):
        self.n, self.dim, self.W, self.sigma, self.R = int(n), int(dim), int(W), float(sigma), float(R)
        self.dtype = {"f32": L.FTCG_F32, "f64": L.FTCG_F64}[dtype]
        self.wmode = {"plain": L.FTCG_W_PLAIN, "learned": L.FTCG_W_LEARNED, "user": L.FTCG_W_USER,
                      "none": L.FTCG_W_NONE, "band": L.FTCG_W_BAND, "density": L.FTCG_W_DENSITY}[weights]
        self.cdtype = torch.complex64 if self.dtype == L.FTCG_F32 else torch.complex128
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream
        self._h = C.c_void_p()
        nn = (C.c_int64 * dim)(*([self.n] * dim))
        L.check(L.call("ftcg_plan_create", C.byref(self._h), self.dim, nn, self.W, self.sigma, self.dtype,
                       self.wmode, self.R, C.c_void_p(_stream_ptr(stream))), "ftcg_plan_create")
        self.m = 0
        self._k = None

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if self._h:
            L.call("ftcg_plan_destroy", self._h)
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

    # -- calls -----------------------------------------------------------------
    def set_points(self, k: torch.Tensor) -> None:
        """k: (m, dim) float64 device tensor, cycles per FOV."""
        m = int(k.shape[0])
        L.check(L.call("ftcg_set_points", self._h, m, C.c_void_p(_dptr(k, torch.float64, m * self.dim, "k"))),
                "ftcg_set_points")
        self.m = m

    def set_weights(self, alpha: torch.Tensor) -> None:
        L.check(L.call("ftcg_set_weights", self._h, C.c_void_p(_dptr(alpha, torch.float64, self.m, "alpha"))),
                "ftcg_set_weights")

    def get_weights(self, out: torch.Tensor | None = None):
        if out is None:
            out = torch.empty(self.m, dtype=torch.float64, device=self.device)
        fb = C.c_int(0)
        L.check(L.call("ftcg_get_weights", self._h, C.c_void_p(_dptr(out, torch.float64, self.m, "alpha")),
                       C.byref(fb)), "ftcg_get_weights")
        self.used_fallback = bool(fb.value)
        return out

    def forward(self, image: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Type-2 transform of an n^dim image at the plan's raster (m values)."""
        if out is None:
            out = torch.empty(self.m, dtype=self.cdtype, device=self.device)
        L.check(L.call("ftcg_forward", self._h, C.c_void_p(_dptr(image, self.cdtype, self.n ** self.dim, "image")),
                       C.c_void_p(_dptr(out, self.cdtype, self.m, "fhat"))), "ftcg_forward")
        return out

    def frame_approx(self, k: torch.Tensor, fhat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Dense frame approximation of raster k (m x dim float64) with values
        fhat (complex128) on this float64 plan's n^dim pixels."""
        m = int(k.shape[0])
        if out is None:
            out = torch.empty((self.n,) * self.dim, dtype=torch.complex128, device=self.device)
        L.check(L.call("ftcg_frame_approx", self._h, m, C.c_void_p(_dptr(k, torch.float64, m * self.dim, "k")),
                       C.c_void_p(_dptr(fhat, torch.complex128, m, "fhat")),
                       C.c_void_p(_dptr(out, torch.complex128, self.n ** self.dim, "image"))), "ftcg_frame_approx")
        return out

    def set_density_iterations(self, iters: int) -> None:
        """Iterations of a weights="density" plan (applies from the next set_points)."""
        L.check(L.call("ftcg_plan_set_density_iterations", self._h, int(iters)), "ftcg_plan_set_density_iterations")

    def set_band(self, r: int) -> None:
        """Band half-width r of a weights="band" plan (applies from the next set_points)."""
        L.check(L.call("ftcg_plan_set_band", self._h, int(r)), "ftcg_plan_set_band")
        self.band_r = int(r)

    def get_band(self) -> torch.Tensor:
        """Banded C by columns: (m, 2r - 1) float64, [n, p] = C[n - r + 1 + p, n]."""
        r = C.c_int(0)
        nb = 2 * getattr(self, "band_r", 1) - 1
        out = torch.empty((self.m, nb), dtype=torch.float64, device=self.device)
        L.check(L.call("ftcg_get_band", self._h, C.c_void_p(_dptr(out, torch.float64, self.m * nb, "band")),
                       C.byref(r)), "ftcg_get_band")
        return out

    def execute(self, fhat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.n,) * self.dim, dtype=self.cdtype, device=self.device)
        L.check(L.call("ftcg_execute", self._h, C.c_void_p(_dptr(fhat, self.cdtype, self.m, "fhat")),
                       C.c_void_p(_dptr(out, self.cdtype, self.n ** self.dim, "image"))), "ftcg_execute")
        return out

    def spread_only(self, fhat: torch.Tensor, grid: torch.Tensor | None = None) -> torch.Tensor:
        G = self.info()["grid_size"]
        if grid is None:
            grid = torch.empty((G,) * self.dim, dtype=self.cdtype, device=self.device)
        L.check(L.call("ftcg_spread_only", self._h, C.c_void_p(_dptr(fhat, self.cdtype, self.m, "fhat")),
                       C.c_void_p(_dptr(grid, self.cdtype, G ** self.dim, "grid"))), "ftcg_spread_only")
        return grid

    def grid_to_image(self, grid: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        G = self.info()["grid_size"]
        if out is None:
            out = torch.empty((self.n,) * self.dim, dtype=self.cdtype, device=self.device)
        L.check(L.call("ftcg_grid_to_image", self._h, C.c_void_p(_dptr(grid, self.cdtype, G ** self.dim, "grid")),
                       C.c_void_p(_dptr(out, self.cdtype, self.n ** self.dim, "image"))), "ftcg_grid_to_image")
        return out

    def info(self) -> dict:
        g, r, t = C.c_int64(), C.c_int64(), C.c_int64()
        tile = C.c_int()
        L.check(L.call("ftcg_plan_info", self._h, C.byref(g), C.byref(r), C.byref(t), C.byref(tile)),
                "ftcg_plan_info")
        return {"grid_size": g.value, "n_records": r.value, "n_tiles": t.value, "tile": tile.value}

    def set_tuning(self, tile: int = 0, accum: str | None = None, lds_copies: int = 1) -> None:
        """tile: 0 (automatic) or 16/32/64/128; accum: "fixed" (float32 plans'
        default) or "f64"; lds_copies: partial tiles for "f64"."""
        if accum is None:
            accum = "fixed" if self.dtype == L.FTCG_F32 else "f64"
        a = {"fixed": L.FTCG_ACCUM_FIXED, "f64": L.FTCG_ACCUM_F64}[accum]
        L.check(L.call("ftcg_plan_set_tuning", self._h, int(tile), a, int(lds_copies)), "ftcg_plan_set_tuning")

    def set_spread_layout(self, layout: str = "auto") -> None:
        """"auto" (segments of tile rows on large float32 grids) or "tiles"
        (one workgroup per tile); applies from the next execute."""
        v = {"auto": 0, "tiles": 1}[layout]
        L.check(L.call("ftcg_plan_set_spread_layout", self._h, v), "ftcg_plan_set_spread_layout")

    def set_weight_tuning(self, samples_per_lane: int = 0, lanes_per_group: int = 0) -> None:
        """Launch shape of the frame-weight kernel (0 = automatic); applies
        from the next weight computation."""
        L.check(L.call("ftcg_plan_set_weight_tuning", self._h, int(samples_per_lane), int(lanes_per_group)),
                "ftcg_plan_set_weight_tuning")

    def set_mlp(self, mlp, audit_threshold: float = 1e-4, audit_samples: int = 4096) -> None:
        """Attach a learned-weight network (FTCG_W_LEARNED plans); the plan
        keeps a reference so the network outlives it."""
        self._mlp = mlp
        L.check(L.call("ftcg_plan_set_mlp", self._h, mlp._h, float(audit_threshold), int(audit_samples)),
                "ftcg_plan_set_mlp")

    def learned_report(self) -> dict:
        est = C.c_double(0.0)
        fb = C.c_int(0)
        L.check(L.call("ftcg_plan_learned_report", self._h, C.byref(est), C.byref(fb)), "ftcg_plan_learned_report")
        return {"audit_estimate": est.value, "used_fallback": bool(fb.value)}

    def enable_timing(self, on: bool = True) -> None:
        L.check(L.call("ftcg_plan_enable_timing", self._h, 1 if on else 0), "ftcg_plan_enable_timing")

    def timing(self) -> dict:
        ms = (C.c_double * L.TIMING_STEPS)()
        cnt = (C.c_int64 * L.TIMING_STEPS)()
        L.check(L.call("ftcg_plan_timing", self._h, ms, cnt), "ftcg_plan_timing")
        return {L.STEP_NAMES[i]: (ms[i], cnt[i]) for i in range(L.TIMING_STEPS) if cnt[i]}
