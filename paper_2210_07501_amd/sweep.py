"""Batched sweep: many independent channels of uneven size in one context,
each solved to residual 1e-8 and retired on convergence.

    python -m paper_2210_07501_amd.sweep [--n 256] [--seed 2210] [--cap 3000000] [--precision fp32]

Channels follow the batched-sweep distribution (inputs.batched_sweep): nx in
{128, 256, 512}, ny = nx / 2, s1, s2, layer fraction and property ratios
drawn from the seed.  The tile shape is chosen by lbm_autotune on the full
batch; the step loop runs as hipGraph replays of 100 steps with device-side
retirement (lbm_solve).  Float32 channels whose residual levels off just above
the tolerance are finished in float64 (warmstart.run_to_tolerance; --no-finish
turns this off).  Prints one JSON line: wall time, converged count, steps per
channel (median, max, by size) and the effective update rate.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbm, warmstart as ws


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=2210)
    ap.add_argument("--cap", type=int, default=3_000_000)
    ap.add_argument("--chunk", type=int, default=100_000)
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--no-finish", action="store_true",
                    help="do not finish stalled float32 channels in float64")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    cfgs = inputs.batched_sweep(a.n, seed=a.seed)
    prec = lbm.LBM_FP32_DEV if a.precision == "fp32" else lbm.LBM_FP64
    ctx = lbm.lbm_create(cfgs, precision=prec)
    lbm.lbm_init(ctx)
    nodes, dev_bytes = lbm.lbm_info(ctx)
    (tx, ty), ms = lbm.lbm_autotune(ctx, 10)
    log("sweep: %d channels, %d nodes, %.2f GB; autotuned tile %dx%d (%.3f ms per launch)"
        % (len(cfgs), nodes, dev_bytes / 1e9, tx, ty, ms))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ws.run_to_tolerance(ctx, cfgs, prec, 1e-8, a.cap, a.chunk, True, not a.no_finish, t0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = np.array([r["steps"] for r in res])
    conv = np.array([r["r"] <= 1e-8 for r in res])
    sizes = np.array([c["nx"] * c["ny"] for c in cfgs])
    updates = float(np.sum(steps * sizes))
    by_size = {}
    for nx in sorted(set(c["nx"] for c in cfgs)):
        m = np.array([c["nx"] == nx for c in cfgs])
        by_size[str(nx)] = dict(channels=int(m.sum()), converged=int(conv[m].sum()),
                                median_steps=int(np.median(steps[m])), max_steps=int(steps[m].max()))
    out = dict(channels=len(cfgs), nodes=int(nodes), precision=a.precision, tile=[tx, ty],
               finished_fp64=int(sum(bool(r.get("finished_fp64")) for r in res)),
               tile_ms_full_batch=round(ms, 4), cap=a.cap, wall_s=round(wall, 1), converged=int(conv.sum()),
               median_steps=int(np.median(steps)), max_steps=int(steps.max()), by_nx=by_size,
               node_updates=updates, effective_glups=round(updates / wall / 1e9, 2),
               unconverged=[dict(index=int(k), r=float(res[k]["r"]), nx=int(cfgs[k]["nx"]),
                                 u_int_peak=float(res[k]["u_int_peak"])) for k in np.where(~conv)[0]])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
