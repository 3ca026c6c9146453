"""Train and evaluate the warm-start network.

    python -m paper_2210_07501_amd.train_warmstart train --n-train 1024 --out weights.npz
    python -m paper_2210_07501_amd.train_warmstart evaluate --weights weights.npz --n-eval 256

train: generates steady states of n-train channels (256 x 128, the batched
sweep distribution with nx = 256, seeds 10000 + i) with the batched
float32-deviation solver (each channel to residual 1e-8, or the step cap),
builds the network inputs and targets on the GPU, trains the network with
the library's kernels, and saves the float32 master weights.

evaluate: on held-out seeds 900000 + i, compares
  warm:        network inference + one batched float32 solve from the prediction;
  cold batch:  one batched float32 solve from rest;
  cold single: plain float64 solves from rest, one channel at a time (the
               first n-single channels; the warm solve is repeated on the
               same subset so both sides cover the same channels);
and the network's raw relative error per output against the converged
fields.  Prints one JSON line.
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


def generate(cfgs, cap, chunk=25_000):
    """Steady states of cfgs: (device fields [n][4][ny][nx] float64, steps, residuals)."""
    ctx, wall, res = ws.solve_batch(cfgs, lbm.LBM_FP32_DEV, tol=1e-8, cap=cap, chunk=chunk)
    F = ws.fields_tensor(ctx, len(cfgs))
    lbm.lbm_destroy(ctx)
    return F, wall, res


def cmd_train(a):
    import torch
    from . import nn
    torch.cuda.set_device(0)
    cfgs = inputs.warmstart_set(a.n_train, 10_000)
    log("train: generating %d steady states (cap %d steps)" % (len(cfgs), a.cap))
    F, wall, res = generate(cfgs, a.cap)
    steps = np.array([r["steps"] for r in res])
    conv = np.array([r["r"] <= 1e-8 for r in res])
    log("train: data in %.1f s; converged %d / %d; median steps %d" % (wall, conv.sum(), len(cfgs), np.median(steps)))
    net = ws.WarmStartNet(seed=a.seed)
    X = net.features(cfgs)
    ny, nx = int(cfgs[0]["ny"]), int(cfgs[0]["nx"])
    Y = torch.empty((len(cfgs), ny, nx, 4), dtype=torch.float32, device="cuda")
    nn.nn_targets(cfgs, F, Y)
    del F
    # train on steady states only: a channel stopped by the cap is not one
    # (--keep-unconverged: every channel, for short timing runs)
    keep = torch.tensor(np.nonzero(conv | a.keep_unconverged)[0], dtype=torch.long, device="cuda")
    X, Y = X[keep].contiguous(), Y[keep].contiguous()
    log("train: %d channels as training data" % X.shape[0])
    log("train: target rms per output", [float(v) for v in torch.sqrt(torch.mean(Y ** 2, dim=(0, 1, 2))).cpu()])
    t0 = time.perf_counter()
    hist = ws.train(net, X, Y, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, time_limit=a.time_limit)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    net.save(a.out)
    out = dict(n_train=len(cfgs), n_used=int(X.shape[0]), data_wall_s=round(wall, 1), data_converged=int(conv.sum()),
               data_median_steps=int(np.median(steps)), data_max_steps=int(steps.max()), cap=a.cap,
               epochs=len(hist), train_s=round(t_train, 1), loss_first=hist[0], loss_last=hist[-1],
               params=ws.n_params(), weights=a.out)
    print(json.dumps(out), flush=True)


def cmd_evaluate(a):
    import torch
    torch.cuda.set_device(0)
    cfgs = inputs.warmstart_set(a.n_eval, 900_000)
    net = ws.WarmStartNet()
    net.load_state(a.weights)
    # warm, whole held-out set
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = net.predict_fields(cfgs, phi_from_net=a.phi == "net")
    torch.cuda.synchronize()
    t_nn = time.perf_counter() - t0
    ctx_w, wall_w, res_w = ws.solve_batch(cfgs, lbm.LBM_FP32_DEV, cap=a.cap, init_fields=pred)
    lbm.lbm_destroy(ctx_w)
    log("evaluate: warm batch %.1f s (+ %.2f s inference)" % (wall_w, t_nn))
    # cold batch
    ctx_c, wall_c, res_c = ws.solve_batch(cfgs, lbm.LBM_FP32_DEV, cap=a.cap)
    ref = ws.fields_tensor(ctx_c, len(cfgs))
    lbm.lbm_destroy(ctx_c)
    log("evaluate: cold batch %.1f s" % wall_c)
    err = ws.relative_errors(pred, ref, phi0=ws.cold_phi(cfgs))
    # cold single float64 on a subset, and warm on the same subset
    sub = cfgs[:a.n_single]
    t_single, steps_single = 0.0, []
    for k, c in enumerate(sub):
        ctx, wall, res = ws.solve_batch([c], lbm.LBM_FP64, cap=a.cap, verbose=False)
        lbm.lbm_destroy(ctx)
        t_single += wall
        steps_single.append(res[0]["steps"])
        log("evaluate: single float64 %d/%d: %d steps, %.2f s" % (k + 1, len(sub), res[0]["steps"], wall))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred_s = net.predict_fields(sub, phi_from_net=a.phi == "net")
    torch.cuda.synchronize()
    t_nn_s = time.perf_counter() - t0
    ctx, wall_ws, res_ws = ws.solve_batch(sub, lbm.LBM_FP32_DEV, cap=a.cap, init_fields=pred_s, verbose=False)
    lbm.lbm_destroy(ctx)
    ctx, wall_cs, res_cs = ws.solve_batch(sub, lbm.LBM_FP32_DEV, cap=a.cap, verbose=False)
    lbm.lbm_destroy(ctx)

    def stats(res):
        s = np.array([r["steps"] for r in res])
        ok = np.array([r["r"] <= 1e-8 for r in res])
        return dict(median_steps=int(np.median(s)), mean_steps=float(s.mean()), max_steps=int(s.max()),
                    converged=int(ok.sum()), n=len(res))

    sw, sc = np.array([r["steps"] for r in res_w]), np.array([r["steps"] for r in res_c])
    out = dict(
        n_eval=len(cfgs), cap=a.cap, phi=a.phi,
        warm_batch=dict(wall_s=round(wall_w + t_nn, 2), inference_s=round(t_nn, 3), **stats(res_w)),
        cold_batch=dict(wall_s=round(wall_c, 2), **stats(res_c)),
        step_ratio_cold_over_warm_median=float(np.median(sc / np.maximum(sw, 1))),
        nn_relative_error_median={k: float(np.median(v)) for k, v in err.items()},
        subset=dict(n=len(sub), cold_single_fp64_s=round(t_single, 2),
                    cold_single_fp64_median_steps=int(np.median(steps_single)),
                    warm_batch_s=round(wall_ws + t_nn_s, 2), cold_batch_s=round(wall_cs, 2),
                    speedup_cold_fp64_over_warm=round(t_single / (wall_ws + t_nn_s), 2),
                    speedup_cold_batch_over_warm=round(wall_cs / (wall_ws + t_nn_s), 2),
                    warm=stats(res_ws), cold=stats(res_cs)),
    )
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-train", type=int, default=1024)
    t.add_argument("--cap", type=int, default=200_000)
    t.add_argument("--epochs", type=int, default=60)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--time-limit", type=float, default=None)
    t.add_argument("--out", required=True)
    t.add_argument("--keep-unconverged", action="store_true",
                   help="train on every generated channel, also those stopped by the cap (timing runs)")
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", required=True)
    e.add_argument("--n-eval", type=int, default=256)
    e.add_argument("--n-single", type=int, default=16)
    e.add_argument("--cap", type=int, default=400_000)
    e.add_argument("--phi", choices=("net", "cold"), default="net",
                   help="hand-off phi: cold-start profile plus the predicted deviation, or the profile alone")
    a = ap.parse_args()
    lbm.load()
    {"train": cmd_train, "evaluate": cmd_evaluate}[a.cmd](a)


if __name__ == "__main__":
    main()
