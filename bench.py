"""Benchmark of the FTCG hot path on one MI355X.

A step is one pass of the whole path over one synthetic input already
resident in HBM: input check + tile binning, neighbour binning + float64
frame weights, weighting + spreading, both inverse-FFT passes, deapodization
and crop (ftcg_set_points followed by ftcg_execute).

Prints ONE JSON line. `value` is Msamples/s gridded end to end (samples per
step / step time); images/s, the spreading-only rate, the per-step times
(HIP events recorded by the library on its stream over the timed region),
the roofline of the dominant kernel, the error against the FP64 oracle and
the oracle's own CPU rate are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Msamples/s gridded + images/s at rel L2 <=1e-4 vs FP64 oracle (plain vs batched/learned)"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
SPREAD_HBM_TARGET = 0.5
# Work unit of the frame-weight sum (eq:difopt with the Gram entries as sinc
# products): one ordered in-box pair (i, n), i != n, of the 2D sum costs
# about 20 float64 operations (per axis the difference, sin(pi d) from the
# per-sample sine and cosine, pi d; then the products, the division, the
# square and the accumulation). The formula itself counts 15 per ordered
# pair; 20 is the figure the work is planned against. In 1D: 8.
FLOPS_PER_PAIR = {1: 8, 2: 20}

WORKLOADS = {
    # name: (description, builder)
    "sas512_plain": "2D polar-format SAS, plain weights, 256 pulses x 512 samples, 512x512 image, FP32 spread/FFT",
    "sas4096_precision": "2D polar-format SAS, 2048 pulses x 4096 samples (8 388 608), 4096x4096 image, "
                         "FP32 spread/FFT, FP64 weights and deapodization",
    "jitter1d_f64": "1D jittered raster, 512 samples, 256 pixels, FP64",
    "batch64_sas": "64 SAS pings, 2^16..2^22 samples each, images 256..2048 squared, plain weights, "
                   "one persistent spreading launch per step, hipGraph replay",
    "learned1024_sas": "2D SAS 512 x 2048 samples (2^20), 1024x1024 image, learned weights (trained MLP) "
                       "with audit against plain weights",
}


def make_inputs(name):
    from paper_1706_08575_amd import synth as S
    if name == "sas512_plain":
        k, f, _ = S.workload_2d_plain()
        return k, f, 512, "f32"
    if name == "sas4096_precision":
        k, f, _ = S.workload_2d_precision()
        return k, f, 4096, "f32"
    if name == "jitter1d_f64":
        k, f, _ = S.make_1d()
        return k, f, 256, "f64"
    raise SystemExit(f"unknown workload {name}")


def step_bytes(step, m, nrec, n, G, dim, dtype):
    """Algorithmic HBM bytes of one launch of each step."""
    cs = 8 if dtype == "f32" else 16
    rs = 4 if dtype == "f32" else 8
    if step == "spread":
        # read per sample: dim offsets + one complex value; write every grid cell once
        return m * (dim * rs + cs) + G ** dim * cs
    if step == "fft1":
        return G * G * cs + n * G * cs
    if step == "fft2_deapod":
        return (n * G * cs + n * n * cs) if dim == 2 else (G * cs + n * cs)
    if step == "bin":
        if dim == 2:
            # 2D weights bin tiles and bin rows together: read k, write one
            # record (2 offsets, cell, index) per record and one row-grouped
            # sample (k, index, bin column: 24 B) per sample
            return m * 8 * dim + nrec * 16 + m * 24
        # read k, write one record (offset, cell, index) + weight per record
        return m * 8 * dim + nrec * (16 + rs)
    if step == "weight_bin":
        if dim == 2:
            # the row sort: read the row-grouped samples, write the bin-ordered
            # sample (k, sin, cos: 48 B), its caller index, the caller-to-bin
            # map and the self term of its sum
            return m * (24 + 48 + 4 + 4 + 8)
        # read k twice (count, scatter), bin id written and read, write the
        # bin-ordered sample (k, sin, cos), its index and the inverse map
        return m * (2 * 8 * dim + 4 + 4 + 24 * dim + 4 + 4)
    return None


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    table (profiles/pmc_traffic.md), or None when there is no row for it or the
    kernel's sources changed since the counters were taken. A name ending in
    '<' matches the one instantiation of that template the workload ran."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "pmc_traffic.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    for line in lines:
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) != 8 or cells[2] != workload:
            continue
        if not (cells[0] == kernel or (kernel.endswith("<") and cells[0].startswith(kernel))):
            continue
        h = hashlib.sha256()
        try:
            for f in cells[7].split():
                with open(os.path.join(here, f), "rb") as fh:
                    h.update(fh.read())
        except OSError:
            return None
        if h.hexdigest()[:16] != cells[6]:
            return None
        return {"bytes": float(cells[5]), "fetch_kib": float(cells[3]), "write_kib": float(cells[4]),
                "kernel": cells[0], "source": "profiles/pmc_traffic.md"}
    return None


def count_box_pairs(k, R, sample=None):
    """Number of ordered pairs (i, n), i != n, with ||k_i - k_n||_inf <= R,
    exact or estimated from a seeded random subset of n."""
    from scipy.spatial import cKDTree
    tree = cKDTree(k)
    if sample is None or sample >= len(k):
        return int(np.sum(tree.query_ball_point(k, r=R, p=np.inf, return_length=True))) - len(k)
    rng = np.random.default_rng(0)
    idx = rng.choice(len(k), size=sample, replace=False)
    c = tree.query_ball_point(k[idx], r=R, p=np.inf, return_length=True)
    return int(round((np.mean(c) - 1.0) * len(k)))


def cpu_baseline(name, k, f, n, R=8.0):
    """The oracle as it stands on a bounded sample: its weights (k-d tree +
    numpy) and spreading (numpy bincount) run on one thread, its FFT
    (scipy.fft) on all host cores."""
    import oracle as O
    m = len(f)
    workers = os.cpu_count() or 1
    t0 = time.perf_counter()
    if m <= 200_000:
        a = O.frame_weights(k, R)
        img = O.ftcg_image(k, f, a, n, workers=workers)
        dt = time.perf_counter() - t0
        return {"value": m / dt / 1e6, "unit": "Msamples/s", "cores": workers, "kind": "oracle",
                "sample": f"whole workload: {m} samples, {n}^{k.shape[1]} image (weights + spread on one "
                          f"thread, FFT + deapod on {workers})",
                "seconds": dt}, img, a
    # large workloads: weights of a contiguous 1/64 of the samples (their
    # neighbour sums use the whole raster), spreading of the same subset onto
    # the full grid, and the full-grid FFT; the rate is scaled to all samples
    # for the per-sample stages and counted once for the FFT
    sub = slice(0, m // 64)
    t0 = time.perf_counter()
    idx = np.arange(m)[sub]
    a_sub = O.frame_weights_at(k, idx, R)
    t_w = time.perf_counter() - t0
    t0 = time.perf_counter()
    H = O.spread(k[sub], a_sub * f[sub], n)
    t_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.grid_to_image(H, n, workers=workers)
    t_f = time.perf_counter() - t0
    per_sample = (t_w + t_s) / len(idx)
    total = per_sample * m + t_f
    return {"value": m / total / 1e6, "unit": "Msamples/s", "cores": workers, "kind": "oracle",
            "sample": f"weights + spreading (one thread) of {len(idx)} of {m} samples (scaled "
                      f"x{m / len(idx):.0f}) + one full {2 * n}^2 FFT/deapod on {workers} threads; "
                      f"measured {t_w + t_s + t_f:.1f} s",
            "seconds_projected": total, "stage_seconds": {"weights_sample": t_w, "spread_sample": t_s,
                                                          "fft_full": t_f}}, None, None


def sampled_parity(k, f, alpha_gpu, img, n, pixels=24, weights=256, seed=4096, R=8.0):
    """Errors of a full-size run the oracle cannot redo whole: weights of
    seeded samples against the oracle's per-sample sum, and seeded pixels
    plus the brightest ones against the oracle's exact weighted sum (fed the
    GPU's weights, which the first check validates)."""
    import oracle as O
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(f), weights, replace=False)
    a_ref = O.frame_weights_at(k, idx, R)
    werr = float(np.max(np.abs(alpha_gpu[idx] - a_ref) / a_ref))
    top = np.argsort(np.abs(img).ravel())[-4:]
    pix = np.concatenate([rng.integers(0, n * n, pixels), top])
    p0, p1 = pix // n, pix % n
    x = np.stack([(p0 - n // 2) / n, (p1 - n // 2) / n], axis=1)
    ref = O.nudft_at(k, alpha_gpu * f, x)
    got = img[p0, p1]
    return {"weights_max_rel_err": werr, "weights_checked": weights,
            "image_rel_l2_sampled": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "pixels_checked": int(len(pix)), "reference": "oracle.nudft_at with the GPU weights (exact sum)"}


MODEL_PATH = os.path.join(ROOT, "paper_1706_08575_amd", "models", "mlp_sas.bin")


def bench_batched(steps: int, warmup: int, tune: bool = True) -> dict:
    """Batched form: 64 SAS pings of uneven size (2^16..2^22 samples, images
    256..2048 squared), plain weights, one persistent spreading launch per
    step under a replayed hipGraph. A step = set_points of all items (weights,
    binning, task tables) + one batched execute."""
    import torch

    from paper_1706_08575_amd import synth as S
    from paper_1706_08575_amd.batch import Batch
    from paper_1706_08575_amd import autotune

    items = S.batch_items()
    t0 = time.perf_counter()
    data = [S.make_batch_item(it) for it in items]
    t_gen = time.perf_counter() - t0
    sizes = [it.n for it in items]
    m = [it.m for it in items]
    K = torch.from_numpy(np.concatenate([d[0] for d in data])).cuda()
    F = torch.from_numpy(np.concatenate([d[1] for d in data])).to(torch.complex64).cuda()
    B = Batch(sizes)
    tuned = None
    if tune:
        tuned, _ = autotune.tune_batch(B, m, K, F, reps=1)
    else:
        B.set_tuning(tile=32, chunk=4096)
        B.set_points(m, K)
    out = B.execute(F)
    for _ in range(warmup):
        B.set_points(m, K)
        out = B.execute(F, out)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(steps):
        B.set_points(m, K)
        out = B.execute(F, out)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - ta) / steps
    # execute alone (geometry fixed): the graph replay
    tb = time.perf_counter()
    for _ in range(steps):
        out = B.execute(F, out)
    torch.cuda.synchronize()
    sec_exec = (time.perf_counter() - tb) / steps
    info = B.info()
    # parity against the oracle: the two densest items (samples per pixel,
    # where the fixed-point tiles hold the most records), fed the GPU's
    # weights, and the smallest item, with the oracle's own weights
    import oracle as O
    w_all = B.get_weights().cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(m)])
    dens = np.array(m, dtype=np.float64) / np.array(sizes, dtype=np.float64) ** 2
    errs = {}
    for i in list(np.argsort(dens)[-2:]) + [int(np.argmin(m))]:
        k, f = data[i][0], data[i][1]
        a = w_all[offs[i]:offs[i + 1]] if dens[i] > 1.0 else O.frame_weights(k, 8.0)
        ref = O.ftcg_image(k, f, a, sizes[i], workers=os.cpu_count() or 1)
        errs[int(i)] = {"n": sizes[i], "m": m[i], "samples_per_pixel": float(dens[i]),
                        "rel_l2": O.rel_l2(B.image(out, int(i)).cpu().numpy(), ref),
                        "oracle_weights": "GPU's (checked separately)" if dens[i] > 1.0 else "oracle's"}
    B.close()
    mt = int(sum(m))
    return {"workload": "batch64_sas", "items": len(items), "samples": mt, "ms_per_step": sec * 1e3,
            "images_per_s": len(items) / sec, "msamples_per_s": mt / sec / 1e6,
            "execute_only_ms": sec_exec * 1e3, "execute_only_images_per_s": len(items) / sec_exec,
            "tuned_tile_chunk": tuned, "tasks": info["tasks"], "split_tiles": info["split_tiles"],
            "records": info["records"], "rel_l2_vs_oracle_items": errs,
            "input_generation_s": t_gen}


def bench_learned(steps: int, warmup: int) -> dict:
    """Learned form: 512 pulses x 2048 samples (2^20), 1024x1024 image. The
    network (trained by paper_1706_08575_amd.train on 10k rasters) predicts the
    weights; the audit recomputes plain weights of 4096 samples and falls
    back when the relative RMS weight error exceeds 1e-4. Reported: the audited
    form (same accuracy as plain), the form without fallback (its weight and
    image error against the plain form), and the plain form on the same input."""
    import torch

    from paper_1706_08575_amd import synth as S
    from paper_1706_08575_amd.ftcg import Plan
    from paper_1706_08575_amd.mlp import Mlp

    k, f, _ = S.workload_learned_eval()
    m = len(f)
    K = torch.from_numpy(k).cuda()
    F = torch.from_numpy(f).to(torch.complex64).cuda()
    net = Mlp()
    trained = os.path.exists(MODEL_PATH)
    if trained:
        with open(MODEL_PATH, "rb") as fh:
            net.load(fh.read())
    else:
        net.set_params(S.mlp_init())
        for i in range(500):
            net.train_raster(torch.from_numpy(S.train_pattern(i)).cuda(), lr=3e-3 * (1 - i / 500) + 1e-5)

    def timed(P):
        out = torch.empty((1024, 1024), dtype=torch.complex64, device="cuda")
        for _ in range(warmup):
            P.set_points(K)
            P.execute(F, out)
        torch.cuda.synchronize()
        P.enable_timing(True)
        P.timing()
        t0 = time.perf_counter()
        for _ in range(steps):
            P.set_points(K)
            P.execute(F, out)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        st = {s_: ms / steps for s_, (ms, c) in P.timing().items()}   # ms per step in each stage
        P.enable_timing(False)
        return sec, out, st

    res = {"workload": "learned1024_sas", "samples": m, "model": "trained 10k rasters" if trained else
           "fallback: 500 rasters trained in-run"}
    with Plan(1024, dim=2, weights="plain") as P:
        sec_p, img_p, st_p = timed(P)
        a_p = P.get_weights()
    res["plain"] = {"ms_per_step": sec_p * 1e3, "images_per_s": 1 / sec_p, "stage_ms": st_p}
    for name, thr in (("audited_1e-4", 1e-4), ("no_fallback", float("inf"))):
        with Plan(1024, dim=2, weights="learned") as P:
            P.set_mlp(net, audit_threshold=thr, audit_samples=4096)
            sec, img, st = timed(P)
            rep = P.learned_report()
            a = P.get_weights()
        werr = torch.sqrt(torch.mean(((a - a_p) / a_p) ** 2)).item()
        ierr = (torch.linalg.vector_norm(img - img_p) / torch.linalg.vector_norm(img_p)).item()
        res[name] = {"ms_per_step": sec * 1e3, "images_per_s": 1 / sec, "stage_ms": st,
                     "audit_estimate": rep["audit_estimate"], "used_fallback": rep["used_fallback"],
                     "weights_rel_rms_vs_plain": werr, "image_rel_l2_vs_plain_gpu": ierr}
    net.close()
    return res


def _timed_steps(P, step, steps, warmup):
    """Mean seconds of `step` over `steps` calls after `warmup`, then the same
    steps with the library's HIP events (ms per step in each stage)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    P.enable_timing(True)
    P.timing()
    for _ in range(steps):
        step()
    st = {s_: ms / steps for s_, (ms, c) in P.timing().items()}
    P.enable_timing(False)
    return sec, st


def bench_band(steps: int, warmup: int, r: int = 8) -> dict:
    """Banded FTCG (Sec. III-C eq:ftcg, eq:cr) on the 512^2 SAS workload with the
    paper's band of 15 (r = 8): a step = set_points (neighbour bins, band of
    T^2, per-column normal equations) + execute (c = C fhat, spread, FFT).
    Parity: 32 seeded columns of C against the oracle's lstsq, and the image
    against the oracle fed the GPU's C."""
    import torch
    import oracle as O
    from paper_1706_08575_amd import synth as S
    from paper_1706_08575_amd.ftcg import Plan
    k, f, _ = S.workload_2d_plain()
    n, m = 512, len(f)
    kd = torch.from_numpy(k).cuda()
    fd = torch.from_numpy(f).to(torch.complex64).cuda()
    with Plan(n, dim=2, weights="band") as P:
        P.set_band(r)
        out = torch.empty((n, n), dtype=torch.complex64, device="cuda")

        def step():
            P.set_points(kd)
            P.execute(fd, out)

        sec, st = _timed_steps(P, step, steps, warmup)
        B = P.get_band().cpu().numpy()
        img = out.cpu().numpy()
    cols = np.random.default_rng(8).choice(m, 32, replace=False)
    Bref = O.band_columns(k, r, 8.0, cols=cols)
    cerr = float(np.max(np.abs(B[cols] - Bref)) / np.max(np.abs(Bref)))
    ref = O.ftcg_image(k, O.band_apply(B, f, r), np.ones(m), n, workers=os.cpu_count() or 1)
    pairs = count_box_pairs(k, 8.0)
    gram_ms = st.get("band_gram", float("nan"))
    ach = pairs * (2 * r - 1) * FLOPS_PER_PAIR[2] / (gram_ms * 1e-3) / 1e12
    return {"workload": "sas512_band_r8", "samples": m, "r": r, "ms_per_step": sec * 1e3, "images_per_s": 1 / sec,
            "msamples_per_s": m / sec / 1e6, "stage_ms": st, "rel_l2_vs_oracle_same_C": O.rel_l2(img, ref),
            "C_max_rel_err_32_columns": cerr,
            "band_gram_roofline": {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": ach / FP64_PEAK_TFLOPS,
                                   "work": f"{pairs} ordered in-box pairs x {2 * r - 1} products x "
                                           f"{FLOPS_PER_PAIR[2]} FP64 flops"}}


def bench_forward(steps: int, warmup: int) -> dict:
    """Forward (type-2) transform on the 4096^2 workload's raster (8.4M samples):
    a step = deapodize + pad + two forward FFT passes + interpolation. Parity:
    512 seeded values against the oracle's forward transform."""
    import torch
    import oracle as O
    from paper_1706_08575_amd import synth as S
    from paper_1706_08575_amd.ftcg import Plan
    k, _, _ = S.workload_2d_precision()
    n, m, G = 4096, len(k), 8192
    rng = np.random.default_rng(40)
    x = (np.arange(n) - n / 2) / n
    env = np.exp(-(x[:, None] ** 2 + x[None, :] ** 2) / 0.05)
    img = (env * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))).astype(np.complex64)
    with Plan(n, dim=2, weights="none") as P:
        P.set_points(torch.from_numpy(k).cuda())
        imd = torch.from_numpy(img).cuda()
        out = torch.empty(m, dtype=torch.complex64, device="cuda")
        sec, st = _timed_steps(P, lambda: P.forward(imd, out), steps, warmup)
        got = out.cpu().numpy()
        nrec = P.info()["n_records"]
    idx = rng.choice(m, 512, replace=False)
    ref = O.interpolate(k[idx], O.image_to_grid(img.astype(np.complex128), n, workers=os.cpu_count() or 1))
    fft_bytes = (n * n * 8 + G * n * 8) + (G * n * 8 + G * G * 8)
    interp_bytes = G * G * 8 + m * 8 + nrec * 16
    fms, ims = st.get("forward_fft", float("nan")), st.get("forward_interp", float("nan"))
    return {"workload": "sas4096_forward", "samples": m, "ms_per_step": sec * 1e3,
            "msamples_per_s": m / sec / 1e6, "stage_ms": st,
            "rel_l2_vs_oracle_512_sampled": O.rel_l2(got[idx], ref),
            "hbm": {"fft_passes": {"bytes": fft_bytes, "GB/s": fft_bytes / (fms * 1e-3) / 1e9,
                                   "frac_hbm": fft_bytes / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS},
                    "interp": {"bytes": interp_bytes, "GB/s": interp_bytes / (ims * 1e-3) / 1e9,
                               "frac_hbm": interp_bytes / (ims * 1e-3) / 1e9 / HBM_PEAK_GBS}}}


def bench_density(steps: int, warmup: int, iters: int = 20) -> dict:
    """Iterative density compensation (the cited iterative quadrature weights)
    on the 512^2 SAS workload, 20 iterations: a step = set_points (binning +
    20 x (spread + interpolation)) + execute. Parity against the oracle's
    iteration on a 128^2 raster (the oracle's cost grows with samples x
    iterations); the weights are compared with the frame weights."""
    import torch
    import oracle as O
    from paper_1706_08575_amd import synth as S
    from paper_1706_08575_amd.ftcg import Plan
    k, f, _ = S.workload_2d_plain()
    n, m = 512, len(f)
    kd = torch.from_numpy(k).cuda()
    fd = torch.from_numpy(f).to(torch.complex64).cuda()
    with Plan(n, dim=2, weights="density") as P:
        P.set_density_iterations(iters)
        out = torch.empty((n, n), dtype=torch.complex64, device="cuda")

        def step():
            P.set_points(kd)
            P.execute(fd, out)

        sec, st = _timed_steps(P, step, steps, warmup)
        a_pm = P.get_weights().cpu().numpy()
    with Plan(n, dim=2, weights="plain") as Q:
        Q.set_points(kd)
        a_fr = Q.get_weights().cpu().numpy()
    ks, fs, _ = S.make_sas(S.seed_for(1) + 80, n=128, pulses=64, per_pulse=128)
    with Plan(128, dim=2, weights="density") as P:
        P.set_density_iterations(iters)
        P.set_points(torch.from_numpy(ks).cuda())
        a_s = P.get_weights().cpu().numpy()
    ref = O.pipe_menon_weights(ks, 128, iters)
    rel = (a_s - ref) / ref
    return {"workload": "sas512_density20", "samples": m, "iterations": iters, "ms_per_step": sec * 1e3,
            "images_per_s": 1 / sec, "stage_ms": st,
            "parity_128": {"samples": len(ks), "max_rel": float(np.max(np.abs(rel))),
                           "rms_rel": float(np.sqrt(np.mean(rel ** 2)))},
            "vs_frame_weights": {"mean_density": float(a_pm.mean()), "mean_frame": float(a_fr.mean()),
                                 "rel_rms_difference": float(np.sqrt(np.mean(((a_pm - a_fr) / a_fr) ** 2)))}}


def bench_frame() -> dict:
    """Dense frame approximation (Sec. III-B eq:binv, eq:afr) on the noisy-grid
    raster of Sec. V-A with the test function of Sec. V, timed once per case,
    against the oracle; beside it the PSNR (peak |f| over the RMS error at the
    pixels) of the frame approximation, of banded FTCG (r = 8, the paper's band
    of 15) and of diagonal FTCG on the same data (the paper's comparison; its
    raster sizes are not given, so its figures are not reproduced)."""
    import torch
    import oracle as O
    from paper_1706_08575_amd import synth as S
    from paper_1706_08575_amd.ftcg import Plan
    res = {}
    for side, n in ((16, 16), (30, 32)):
        k = S.noisy_grid(S.seed_for(5) + side, side)
        f = S.sine_test_fourier(k)
        x = (np.arange(n) - n / 2) / n
        truth = S.sine_test_function(np.stack(np.meshgrid(x, x, indexing="ij"), -1))

        def psnr(img):
            return float(20 * np.log10(np.max(np.abs(truth)) / np.sqrt(np.mean(np.abs(img - truth) ** 2))))

        kd = torch.from_numpy(k).cuda()
        fd = torch.from_numpy(f).cuda()
        with Plan(n, dim=2, dtype="f64", weights="none") as P:
            P.frame_approx(kd, fd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            img = P.frame_approx(kd, fd)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            img = img.cpu().numpy()
        ref = O.frame_image(k, f, n)
        out = {"samples": len(k), "modes": n * n, "ms": ms, "rel_l2_vs_oracle": O.rel_l2(img, ref),
               "psnr_db": {"frame": psnr(img)}}
        for name, w, r in (("ftcg_band_r8", "band", 8), ("ftcg_diagonal", "plain", 1)):
            with Plan(n, dim=2, dtype="f64", weights=w) as P:
                if w == "band":
                    P.set_band(r)
                P.set_points(kd)
                out["psnr_db"][name] = psnr(P.execute(fd).cpu().numpy())
        res[f"noisy_grid_{side}x{side}_modes_{n}x{n}"] = out
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sas4096_precision", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--accum", default=None, choices=["fixed", "f64"])
    ap.add_argument("--copies", type=int, default=1)
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and learned forms")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--only-forms", default=None,
                    help="comma-separated forms to run alone (band, forward, density, frame_approx), "
                         "printing one JSON object of their results (for profiling them)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1706_08575_amd.ftcg import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only_forms:
        run = {"band": lambda: bench_band(steps=5, warmup=2), "forward": lambda: bench_forward(steps=10, warmup=5),
               "density": lambda: bench_density(steps=5, warmup=2), "frame_approx": bench_frame}
        print(json.dumps({name: run[name]() for name in args.only_forms.split(",")}))
        return
    if args.workload in ("batch64_sas", "learned1024_sas"):
        if args.workload == "batch64_sas":
            r = bench_batched(steps=args.steps, warmup=args.warmup, tune=args.tile == 0)
            value, ms, dt = r["msamples_per_s"], r["ms_per_step"], "f32 spread/FFT, f64 weights/deapod"
        else:
            r = bench_learned(steps=args.steps, warmup=args.warmup)
            ms = r["no_fallback"]["ms_per_step"]
            value, dt = r["samples"] / ms / 1e3, "f32 spread/FFT, fp16/fp32 MLP, f64 audit/deapod"
        print(json.dumps({"metric": METRIC, "value": value, "unit": "Msamples/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dt,
                          "data": "synthetic", "config": {"workload": args.workload,
                                                           "description": WORKLOADS[args.workload]},
                          "result": r, "roofline": None, "cpu_baseline": None}))
        return
    k, f, n, dtype = make_inputs(args.workload)
    m, dim = len(f), k.shape[1]
    cdt = torch.complex64 if dtype == "f32" else torch.complex128
    kd = torch.from_numpy(k).to(dev)
    fd = torch.from_numpy(f).to(cdt).to(dev)
    out = torch.empty((n,) * dim, dtype=cdt, device=dev)

    P = Plan(n, dim=dim, dtype=dtype, weights="plain", R=8.0)
    if args.tile or args.copies != 1 or args.accum:
        P.set_tuning(args.tile, args.accum, args.copies)

    def step():
        P.set_points(kd)
        P.execute(fd, out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region 1: the steps alone (value, ms_per_step)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # timed region 2: the same steps with the library's HIP events around
    # every kernel step on the plan's stream (per-kernel durations, roofline)
    P.enable_timing(True)
    P.timing()  # reset
    torch.cuda.synchronize()
    te0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    te1 = time.perf_counter()
    stages = P.timing()
    P.enable_timing(False)
    info = P.info()
    img = out.cpu().numpy()
    alpha = P.get_weights().cpu().numpy()
    sec = (t1 - t0) / args.steps
    G = info["grid_size"]

    if args.copy_calibration:
        x = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    # ms per step in each stage (a stage may be timed in several intervals
    # per step: the binning before and after the weights)
    stage_ms = {s_: ms / args.steps for s_, (ms, c) in stages.items()}
    stage_count = {s_: c for s_, (ms, c) in stages.items()}
    # roofline of the dominant kernel among the stages that are one kernel
    # each (the weight sum, the spread, the FFT passes; the binning stages
    # run several short kernels)
    single = [s_ for s_ in ("weights", "spread", "fft1", "fft2_deapod") if s_ in stage_ms]
    dom = max(single, key=stage_ms.get)
    if dom == "weights":
        pairs = count_box_pairs(k, 8.0, sample=None if m <= 200_000 else 20000)
        flops = pairs * FLOPS_PER_PAIR[dim]
        launch_ms = stage_ms[dom] * args.steps / stage_count[dom]     # mean event time of one launch
        ach = flops / (launch_ms * 1e-3) / 1e12
        kname = "k_frame_weights_sym<" if dim == 2 else "k_frame_weights_1d<"
        tr = measured_traffic(kname, args.workload)
        kname = tr["kernel"] if tr else kname + "...>"
        roof = {"kernel": kname, "bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS, "traffic": tr["bytes"] if tr else None,
                "launch_ms": launch_ms,
                "work_per_launch": f"{pairs} ordered in-box pairs (i != n) x {FLOPS_PER_PAIR[dim]} FP64 flops"
                                   + (" (the symmetric kernel forms each unordered pair once)" if dim == 2 else ""),
                "algorithmic_bytes_per_launch": m * (48 + 8)}
    else:
        b = step_bytes(dom, m, info["n_records"], n, G, dim, dtype)
        launch_ms = stage_ms[dom] * args.steps / stage_count[dom]
        ach = b / (launch_ms * 1e-3) / 1e9
        kname = {"spread": "k_spread2d_fx" if dim == 2 else "k_spread1d", "fft1": "k_fft_rows (pass 1)",
                 "fft2_deapod": "k_fft_rows (pass 2)"}.get(dom, dom)
        tr = measured_traffic(kname + "<", args.workload) if dom == "spread" else None
        roof = {"kernel": kname, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": tr["bytes"] if tr else None, "launch_ms": launch_ms,
                "bytes_per_launch": b}
    # every HBM-bound step, for reference
    steps_hbm = {}
    for s_ in ("spread", "fft1", "fft2_deapod", "bin", "weight_bin"):
        if s_ in stage_ms:
            b = step_bytes(s_, m, info["n_records"], n, G, dim, dtype)
            steps_hbm[s_] = {"ms": stage_ms[s_], "GB/s": b / (stage_ms[s_] * 1e-3) / 1e9,
                             "frac_hbm": b / (stage_ms[s_] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    spread_target = None
    if "spread" in steps_hbm:
        fr = steps_hbm["spread"]["frac_hbm"]
        spread_target = {"frac_hbm": fr, "target": SPREAD_HBM_TARGET, "met": fr >= SPREAD_HBM_TARGET,
                         "ms": stage_ms["spread"], "ms_at_target": step_bytes("spread", m, info["n_records"], n, G,
                                                                               dim, dtype) / (SPREAD_HBM_TARGET *
                                                                                              HBM_PEAK_GBS * 1e6)}

    cpu = None
    rel = None
    parity = None
    if not args.no_cpu:
        cpu, img_ref, a_ref = cpu_baseline(args.workload, k, f, n)
        if img_ref is not None:
            import oracle as O
            rel = O.rel_l2(img, img_ref)
            rel_w = float(np.max(np.abs(alpha - a_ref) / a_ref))
            cpu["weights_max_rel_err"] = rel_w
            parity = {"image_rel_l2": rel, "weights_max_rel_err": rel_w, "reference": "whole oracle image"}
        elif dim == 2:
            parity = sampled_parity(k, f, alpha, img, n)
            rel = parity["image_rel_l2_sampled"]

    forms = None
    if not args.no_forms:
        forms = {"batched": bench_batched(steps=3, warmup=1),
                 "learned": bench_learned(steps=max(3, min(args.steps, 10)), warmup=1),
                 "band": bench_band(steps=5, warmup=2),
                 "forward": bench_forward(steps=10, warmup=5),
                 "density": bench_density(steps=5, warmup=2),
                 "frame_approx": bench_frame()}

    res = {
        "metric": METRIC,
        "value": m / sec / 1e6,
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 spread/FFT, f64 weights/deapod" if dtype == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "n": n, "m": m,
                   "dim": dim, "W": 6, "sigma": 2.0, "R": 8.0, "weights": "plain", "grid": G,
                   "tile": info["tile"], "records": info["n_records"], "lds_copies": args.copies,
                   "accum": args.accum or ("fixed" if dtype == "f32" else "f64")},
        "ms_per_step_with_stage_events": (te1 - te0) / args.steps * 1e3,
        "images_per_s": 1.0 / sec,
        "spread_msamples_per_s": m / (stage_ms["spread"] * 1e-3) / 1e6 if "spread" in stage_ms else None,
        "rel_l2_vs_oracle": rel,
        "parity": parity,
        "stage_ms": stage_ms,
        "hbm_steps": steps_hbm,
        "spread_vs_hbm_target": spread_target,
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": forms,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
