"""Train the learned frame-weight network on jittered annular training rasters.

Every raster (128 pulses x 512 samples = 2^16 samples at n = 256, jitter
scale drawn per raster) is labelled on the GPU by the plain float64 frame
weights; features, labels, forward, backward and Adam all run in libftcg
(ftcg_mlp_train_raster). Rasters are generated on the host one ahead of the
GPU. The learning rate follows a linear warm-up and a cosine decay.

    python -m paper_1706_08575_amd.train --rasters 10000 --out model.bin

Prints one progress line per `--log-every` rasters and a final evaluation on
held-out rasters: the relative RMS error of the predicted weights against the
plain ones, next to that of the analytic 16-neighbour estimate alone.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

EVAL_BASE = 1_000_000   # held-out raster indices start here


def lr_at(i: int, n: int, lr: float, warm: int = 50, floor: float = 0.01) -> float:
    if i < warm:
        return lr * (i + 1) / warm
    t = (i - warm) / max(1, n - warm)
    return lr * (floor + (1.0 - floor) * 0.5 * (1.0 + math.cos(math.pi * t)))


def evaluate(net, n_eval: int = 8, R: float = 8.0) -> dict:
    import torch

    from . import synth as S
    from .ftcg import Plan
    e_net, e_base = [], []
    for q in range(n_eval):
        k = torch.from_numpy(S.train_pattern(EVAL_BASE + q)).cuda()
        with Plan(256, dim=2, weights="learned", R=R) as P:
            P.set_mlp(net, audit_threshold=float("inf"))
            P.set_points(k)
            a = P.get_weights()
        with Plan(256, dim=2, weights="plain", R=R) as Q:
            Q.set_points(k)
            plain = Q.get_weights()
        _, base = net.features(k, R)
        e_net.append(torch.mean(((a - plain) / plain) ** 2).item())
        e_base.append(torch.mean(((base - plain) / plain) ** 2).item())
    return {"rel_rms_network": math.sqrt(np.mean(e_net)), "rel_rms_analytic_estimate": math.sqrt(np.mean(e_base)),
            "held_out_rasters": n_eval}


def train(rasters: int, out: str | None, lr: float = 3e-3, batch: int = 4096, log_every: int = 250,
          seed_params: int | None = None, R: float = 8.0) -> dict:
    import torch

    from . import synth as S
    from .mlp import Mlp

    torch.cuda.set_device(0)
    net = Mlp(S.mlp_init() if seed_params is None else S.mlp_init(seed_params))
    pool = cf.ThreadPoolExecutor(max_workers=2)
    nxt = pool.submit(S.train_pattern, 0)
    t0 = time.perf_counter()
    hist = []
    run = 0.0
    for i in range(rasters):
        k = nxt.result()
        if i + 1 < rasters:
            nxt = pool.submit(S.train_pattern, i + 1)
        loss = net.train_raster(torch.from_numpy(k).cuda(), lr=lr_at(i, rasters, lr), R=R, batch=batch)
        run = loss if i == 0 else 0.98 * run + 0.02 * loss
        if (i + 1) % log_every == 0 or i + 1 == rasters:
            dt = time.perf_counter() - t0
            hist.append({"raster": i + 1, "loss_ema": run, "seconds": dt})
            print(f"train: raster {i + 1}/{rasters} loss(ema) {run:.3e} lr {lr_at(i, rasters, lr):.2e} "
                  f"{dt:.1f} s", flush=True)
    pool.shutdown()
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    ev = evaluate(net, R=R)
    res = {"rasters": rasters, "samples": rasters * 65536, "batch": batch, "lr": lr, "seconds": seconds,
           "history": hist, "eval": ev}
    print("train: " + json.dumps(ev), flush=True)
    if out:
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        with open(out, "wb") as fh:
            fh.write(net.save())
        with open(os.path.splitext(out)[0] + ".json", "w") as fh:
            json.dump(res, fh, indent=1)
    net.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rasters", type=int, default=10000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--log-every", type=int, default=250)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    train(args.rasters, args.out, args.lr, args.batch, args.log_every)


if __name__ == "__main__":
    main()
