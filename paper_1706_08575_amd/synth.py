"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module only draws sample locations and sample values. It holds none of
the reconstruction arithmetic (no weights, no gridding, no transforms): the
values it returns are the exact Fourier data of a known scene, so both sides
of every parity check start from the same arrays.

Conventions (both dimensions):
  * the field of view is the centred unit box [-1/2, 1/2)^d;
  * a sample location k is in cycles per field of view;
  * the Fourier datum is fhat(k) = integral over the FOV of f(x) exp(-2 pi i k.x) dx.

Draw order is fixed and listed in each generator, so a seed names one input.
The paper's experiments are synthetic (Sec. V); the geometries below stand in
for its jittered rasters (Sec. V-A) and its side-scan/polar-format SAS-like
raster (Sec. V-C), at the sizes of the benchmark workloads.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 1706_08575


def seed_for(config_index: int) -> int:
    """Seed of workload ``config_index`` (0 = 1D, 1 = 2D plain, 2 = precision,
    3 = batched, 4 = learned)."""
    return SEED_BASE + int(config_index)


# ----------------------------------------------------------------------------
# 1D: jittered raster, piecewise-smooth function with closed-form coefficients
# ----------------------------------------------------------------------------

@dataclass
class Scene1D:
    jumps: np.ndarray      # (3,) sorted jump positions in (-0.45, 0.45)
    levels: np.ndarray     # (4,) piece levels
    cos_amp: np.ndarray    # (3,) amplitudes b_l of cos(2 pi l x + phi_l), l = 1..3
    cos_phase: np.ndarray  # (3,) phases phi_l

    def evaluate(self, x: np.ndarray) -> np.ndarray:
        """f(x) on [-1/2, 1/2)."""
        x = np.asarray(x, dtype=np.float64)
        edges = np.concatenate(([-0.5], self.jumps, [0.5]))
        f = np.zeros_like(x)
        for i, v in enumerate(self.levels):
            f += np.where((x >= edges[i]) & (x < edges[i + 1]), v, 0.0)
        for l, (b, ph) in enumerate(zip(self.cos_amp, self.cos_phase), start=1):
            f += b * np.cos(2 * np.pi * l * x + ph)
        return f

    def fourier(self, k: np.ndarray) -> np.ndarray:
        """Exact fhat(k) = int_{-1/2}^{1/2} f(x) exp(-2 pi i k x) dx (complex128)."""
        k = np.asarray(k, dtype=np.float64)
        edges = np.concatenate(([-0.5], self.jumps, [0.5]))
        out = np.zeros(k.shape, dtype=np.complex128)
        for i, v in enumerate(self.levels):
            a, b = edges[i], edges[i + 1]
            # int_a^b e^{-2 pi i k x} dx = (b - a) e^{-i pi k (a + b)} sinc(k (b - a))
            out += v * (b - a) * np.exp(-1j * np.pi * k * (a + b)) * np.sinc(k * (b - a))
        for l, (b, ph) in enumerate(zip(self.cos_amp, self.cos_phase), start=1):
            # cos(2 pi l x + ph) = (e^{i(2 pi l x + ph)} + e^{-i(...)}) / 2
            out += 0.5 * b * (np.exp(1j * ph) * np.sinc(k - l) + np.exp(-1j * ph) * np.sinc(k + l))
        return out


def make_1d(seed: int = seed_for(0), n: int = 256, m: int = 512):
    """1D workload: k_j = j - m/2 + U(-1/4, 1/4) (the admissible jittered
    raster of Sec. V), values = exact coefficients of a piecewise-smooth scene.

    Draw order: jitter (m), jump positions (3), levels (4), cosine amplitudes
    (3), cosine phases (3).
    Returns (k (m,1) float64, fhat (m,) complex128, scene).
    """
    rng = np.random.default_rng(seed)
    jitter = rng.uniform(-0.25, 0.25, size=m)
    jumps = np.sort(rng.uniform(-0.45, 0.45, size=3))
    levels = rng.uniform(-1.0, 1.0, size=4)
    cos_amp = rng.uniform(-0.5, 0.5, size=3)
    cos_phase = rng.uniform(0.0, 2 * np.pi, size=3)
    k = (np.arange(m, dtype=np.float64) - m // 2 + jitter).reshape(m, 1)
    scene = Scene1D(jumps, levels, cos_amp, cos_phase)
    return k, scene.fourier(k[:, 0]), scene


# ----------------------------------------------------------------------------
# 2D: polar-format (annular sector) SAS raster, point scatterers + speckle
# ----------------------------------------------------------------------------

@dataclass
class Scene2D:
    pos: np.ndarray   # (S, 2) scatterer positions in [-0.4, 0.4]^2
    amp: np.ndarray   # (S,) complex amplitudes

    def fourier(self, k: np.ndarray, chunk: int = 1 << 18) -> np.ndarray:
        """Exact fhat(k) = sum_s a_s exp(-2 pi i k . x_s) for point scatterers
        (float64; evaluated with multithreaded torch CPU ops, chunked)."""
        import torch
        k = np.asarray(k, dtype=np.float64)
        out = np.empty(k.shape[0], dtype=np.complex128)
        pos_t = torch.from_numpy(np.ascontiguousarray(self.pos.T))
        amp = torch.from_numpy(np.ascontiguousarray(self.amp))
        for b in range(0, k.shape[0], chunk):
            ph = (-2.0 * math.pi) * (torch.from_numpy(k[b:b + chunk]) @ pos_t)     # (c, S)
            e = torch.polar(torch.ones_like(ph), ph)
            out[b:b + chunk] = (e @ amp).numpy()
        return out


def sas_geometry(n: int):
    """Annular-sector constants for an n x n image: k0 = 2.25 n and the
    baseband shift kc that centres the sector in range."""
    k0 = 2.25 * n
    kc = k0 * (0.8 * math.cos(math.radians(10.0)) + 1.2) / 2.0
    return k0, kc


def sas_raster(rng: np.random.Generator, n: int, pulses: int, per_pulse: int,
               m: int | None = None, jitter_scale: float = 1.0) -> np.ndarray:
    """Polar-format raster: pulse angles theta_p over +/-10 deg with N(0, 0.02 deg)
    angle jitter, range wavenumbers r_q over [0.8, 1.2] k0, per-sample position
    jitter N(0, 0.01^2) cycles/FOV. Optionally truncated to the first m samples.

    Draw order: angle jitter (pulses), position jitter (pulses*per_pulse*2).
    """
    k0, kc = sas_geometry(n)
    theta = (np.radians(-10.0 + 20.0 * (np.arange(pulses) + 0.5) / pulses)
             + np.radians(0.02 * jitter_scale) * rng.standard_normal(pulses))
    r = k0 * (0.8 + 0.4 * (np.arange(per_pulse) + 0.5) / per_pulse)
    kx = (r[None, :] * np.cos(theta)[:, None] - kc).reshape(-1)
    ky = (r[None, :] * np.sin(theta)[:, None]).reshape(-1)
    k = np.stack([kx, ky], axis=1)
    k += (0.01 * jitter_scale) * rng.standard_normal(k.shape)
    if m is not None:
        k = k[:m]
    return np.ascontiguousarray(k)


def sas_scene(rng: np.random.Generator, n_scatter: int = 40) -> Scene2D:
    """Draw order: positions (S*2), amplitudes (S), phases (S)."""
    pos = rng.uniform(-0.4, 0.4, size=(n_scatter, 2))
    mag = rng.uniform(5.0, 20.0, size=n_scatter)
    phase = rng.uniform(0.0, 2 * np.pi, size=n_scatter)
    return Scene2D(pos, mag * np.exp(1j * phase))


def speckle(rng: np.random.Generator, m: int, sigma: float = 1.0) -> np.ndarray:
    """Circular complex Gaussian CN(0, sigma^2): re, im ~ N(0, sigma^2/2).
    Draw order: re (m), im (m)."""
    s = sigma / math.sqrt(2.0)
    re = rng.standard_normal(m)
    im = rng.standard_normal(m)
    return s * (re + 1j * im)


def make_sas(seed: int, n: int, pulses: int, per_pulse: int, m: int | None = None,
             n_scatter: int = 40, speckle_sigma: float = 1.0, jitter_scale: float = 1.0):
    """2D SAS workload. Draw order: raster (see sas_raster), scene (see
    sas_scene), speckle (see speckle).
    Returns (k (m,2) float64, fhat (m,) complex128, scene)."""
    rng = np.random.default_rng(seed)
    k = sas_raster(rng, n, pulses, per_pulse, m=m, jitter_scale=jitter_scale)
    scene = sas_scene(rng, n_scatter)
    fhat = scene.fourier(k) + speckle(rng, k.shape[0], speckle_sigma)
    return k, fhat, scene


# named workloads ------------------------------------------------------------

def workload_2d_plain(seed: int = seed_for(1)):
    """256 pulses x 512 samples, 512 x 512 image."""
    return make_sas(seed, n=512, pulses=256, per_pulse=512)


def workload_2d_precision(seed: int = seed_for(2)):
    """2048 pulses x 4096 samples (8 388 608 points), 4096 x 4096 image."""
    return make_sas(seed, n=4096, pulses=2048, per_pulse=4096)


@dataclass
class BatchItem:
    n: int
    m: int
    pulses: int
    per_pulse: int
    seed: int


def batch_items(seed: int = seed_for(3), n_items: int = 64,
                log2_lo: float = 16.0, log2_hi: float = 22.0,
                sizes=(256, 512, 1024, 2048)) -> list[BatchItem]:
    """Batched workload descriptors: M_i = round(2^U(lo, hi)), N_i uniform over
    ``sizes``, Q_i = ceil(sqrt(2 M_i)), P_i = ceil(M_i / Q_i) (last pulse
    truncated). Draw order: log2 M (n), size index (n), per-item seeds (n)."""
    rng = np.random.default_rng(seed)
    lm = rng.uniform(log2_lo, log2_hi, size=n_items)
    si = rng.integers(0, len(sizes), size=n_items)
    seeds = rng.integers(0, 2**31 - 1, size=n_items)
    items = []
    for i in range(n_items):
        m = int(round(2.0 ** lm[i]))
        q = int(math.ceil(math.sqrt(2 * m)))
        p = int(math.ceil(m / q))
        items.append(BatchItem(int(sizes[si[i]]), m, p, q, int(seeds[i])))
    return items


def make_batch_item(item: BatchItem):
    return make_sas(item.seed, n=item.n, pulses=item.pulses, per_pulse=item.per_pulse, m=item.m)


def train_pattern(pattern_index: int, seed: int = seed_for(4), n: int = 256,
                  pulses: int = 128, per_pulse: int = 512, vary_jitter: bool = True) -> np.ndarray:
    """Training raster number ``pattern_index`` (geometry only, no values):
    128 x 512 = 2^16 samples at n = 256. Jitter scale is drawn log-uniformly
    from [1/2, 2] when ``vary_jitter``. Draw order: jitter scale (1), raster."""
    rng = np.random.default_rng([seed, int(pattern_index)])
    js = float(2.0 ** rng.uniform(-1.0, 1.0)) if vary_jitter else 1.0
    return sas_raster(rng, n, pulses, per_pulse, jitter_scale=js)


def workload_learned_eval(seed: int = seed_for(4) + 1000):
    """Evaluation input of the learned-weight form: 512 x 2048 = 2^20 samples,
    1024 x 1024 image."""
    return make_sas(seed, n=1024, pulses=512, per_pulse=2048)


def integer_raster_1d(n: int) -> np.ndarray:
    """k_j = j - n/2, j = 0..n-1 (the uniform lattice)."""
    return (np.arange(n, dtype=np.float64) - n // 2).reshape(n, 1)


def random_values(seed: int, m: int) -> np.ndarray:
    """Unit-variance circular complex Gaussian values (for linearity and
    property tests). Draw order: re (m), im (m)."""
    rng = np.random.default_rng(seed)
    return speckle(rng, m, 1.0)


# ----------------------------------------------------------------------------
# initial parameters of the learned-weight MLP (32 -> 64 -> 64 -> 1)
# ----------------------------------------------------------------------------

MLP_SHAPES = (("W1", (32, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 1)), ("b3", (1,)))


def mlp_init(seed: int = SEED_BASE + 40) -> dict:
    """Float32 initial parameters, each entry U(-1/sqrt(fan_in), 1/sqrt(fan_in))
    (the last layer scaled by 0.1 so the initial correction is small).
    Draw order: the shapes above, in order."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, shp in MLP_SHAPES:
        fan_in = shp[0] if len(shp) == 2 else (64 if name != "b1" else 32)
        lim = 1.0 / math.sqrt(fan_in)
        v = rng.uniform(-lim, lim, size=shp)
        if name in ("W3", "b3"):
            v = 0.1 * v
        out[name] = v.astype(np.float32)
    return out


# ----------------------------------------------------------------------------
# the 2D experiments of Sec. V: noisy grid raster, test function
# ----------------------------------------------------------------------------

def noisy_grid(seed: int, side: int) -> np.ndarray:
    """Noisy grid raster of Sec. V-A: lambda = (n1, n2) + U(-1/4, 1/4)^2 for
    n_a = -side/2 .. side/2 - 1, raster order n1-major. Draw order: jitter
    (side^2 x 2)."""
    rng = np.random.default_rng(seed)
    g = np.arange(side) - side // 2
    base = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2).astype(np.float64)
    return base + rng.uniform(-0.25, 0.25, size=base.shape)


def sine_test_function(x: np.ndarray) -> np.ndarray:
    """f(x) = sin(4 pi x1) sin(2 pi x2) (the test function of Sec. V), x (..., 2)."""
    x = np.asarray(x, dtype=np.float64)
    return np.sin(4 * np.pi * x[..., 0]) * np.sin(2 * np.pi * x[..., 1])


def sine_test_fourier(k: np.ndarray) -> np.ndarray:
    """Exact fhat(k) = int over [-1/2, 1/2)^2 of f(x) e^{-2 pi i k.x} dx for the
    test function: per axis int sin(2 pi c x) e^{-2 pi i k x} dx =
    (sinc(k - c) - sinc(k + c)) / (2i), c = 2 and 1."""
    k = np.asarray(k, dtype=np.float64)
    f0 = (np.sinc(k[:, 0] - 2.0) - np.sinc(k[:, 0] + 2.0)) / 2j
    f1 = (np.sinc(k[:, 1] - 1.0) - np.sinc(k[:, 1] + 1.0)) / 2j
    return f0 * f1
