"""Learned warm start: a small convolutional network that predicts the
near-steady fields (u, v, T, phi) of a channel from its wall-heating law and
properties, trained on steady states that the batched LBM solver itself
produces.  The LBM then starts from the prediction (lbm_init_device) and must
still reach the same residual; the cold start from rest remains the
fallback and the reference for the network's error.

Every tensor operation runs in the library's HIP kernels (include/lbm_nn.h):
3x3 convolutions forward and backward on BF16 matrix cores with FP32
accumulation, pooling, upsampling, ReLU backward, skip additions, MSE and
Adam.  This module only allocates buffers (PyTorch), orders the calls and
loops over mini-batches.

Network (NHWC, channels padded to multiples of 32; every conv 3x3 + bias,
ReLU except the last; x periodic, zero padding in y):
  level 0 (ny x nx):  c0 10(->32) -> 32, c1 32 -> 32           s0 = c1
  level 1 (1/2):      c2 32 -> 64, c3 64 -> 64                  s1 = c3
  level 2 (1/4):      c4 64 -> 96, c5 96 -> 96
  level 1:            c6 96 -> 64 on up(c5); a1 = c6 + s1; c7 64 -> 64
  level 0:            c8 64 -> 32 on up(c7); a0 = c8 + s0; c9 32 -> 4(->32), linear
About 317k real parameters.  Inputs: 10 planes (nn_features); outputs
u / U_s, v / U_s, (T - T_ref) / dT, phi.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, lbm, nn

CPAD = 32            # padded input / output channel count
NFEAT = 10           # real input planes
NOUT = 4             # real outputs
# name: (ci_pad, ci_real, co_pad, co_real, level)
LAYERS = {
    "c0": (32, NFEAT, 32, 32, 0), "c1": (32, 32, 32, 32, 0),
    "c2": (32, 32, 64, 64, 1), "c3": (64, 64, 64, 64, 1),
    "c4": (64, 64, 96, 96, 2), "c5": (96, 96, 96, 96, 2),
    "c6": (96, 96, 64, 64, 1), "c7": (64, 64, 64, 64, 1),
    "c8": (64, 64, 32, 32, 0), "c9": (32, 32, 32, NOUT, 0),
}


def n_params():
    return sum(co_r * 9 * ci_r + co_r for ci, ci_r, co, co_r, _ in LAYERS.values())


class WarmStartNet:
    def __init__(self, seed: int = 0, device=None):
        import torch
        self.torch = torch
        self.dev = device or torch.device("cuda", torch.cuda.current_device())
        rng = np.random.default_rng(seed)
        self.p = {}
        for name, (ci, ci_r, co, co_r, _) in LAYERS.items():
            w = np.zeros((co, 9, ci), dtype=np.float32)
            std = math.sqrt(2.0 / (9 * ci_r)) if name != "c9" else math.sqrt(1.0 / (9 * ci_r))
            w[:co_r, :, :ci_r] = rng.normal(0.0, std, size=(co_r, 9, ci_r))
            self.p[name] = {"w": torch.from_numpy(w).to(self.dev), "b": torch.zeros(co, device=self.dev)}
        self._derived()
        self.step_count = 0
        self.bufs = {}

    # ---- parameters -------------------------------------------------------
    def _derived(self):
        t = self.torch
        for name, (ci, _, co, _, _) in LAYERS.items():
            q = self.p[name]
            q["w16"] = t.empty((co, 9, ci), dtype=t.bfloat16, device=self.dev)
            q["wf"] = t.empty((ci, 9, co), dtype=t.bfloat16, device=self.dev)
            nn.nn_cast_weights(q["w"], q["w16"], q["wf"], co, ci)
            for k in ("gw", "mw", "vw"):
                q[k] = t.zeros_like(q["w"])
            for k in ("gb", "mb", "vb"):
                q[k] = t.zeros_like(q["b"])

    def state_dict(self):
        out = {}
        for name in LAYERS:
            out[name + ".w"] = self.p[name]["w"].detach().cpu().numpy()
            out[name + ".b"] = self.p[name]["b"].detach().cpu().numpy()
        return out

    def save(self, path: str):
        np.savez(path, **self.state_dict())

    def load_state(self, path_or_dict):
        d = np.load(path_or_dict, allow_pickle=False) if isinstance(path_or_dict, str) else path_or_dict
        for name in LAYERS:
            self.p[name]["w"].copy_(self.torch.from_numpy(np.asarray(d[name + ".w"], dtype=np.float32)))
            self.p[name]["b"].copy_(self.torch.from_numpy(np.asarray(d[name + ".b"], dtype=np.float32)))
        self._derived()

    # ---- buffers ----------------------------------------------------------
    def _buffers(self, n, h, w):
        key = (n, h, w)
        if key in self.bufs:
            return self.bufs[key]
        self.bufs.clear()
        t = self.torch
        bf = t.bfloat16
        hw = [(h, w), (h // 2, w // 2), (h // 4, w // 4)]

        def T(level, c, dtype=bf):
            hh, ww = hw[level]
            return t.empty((n, hh, ww, c), dtype=dtype, device=self.dev)

        B = {"x": T(0, CPAD)}
        for name in ("c0", "c1", "c8", "a0"):
            B[name] = T(0, 32)
        B["u0"] = T(0, 64)
        for name in ("c2", "c3", "c6", "a1", "c7"):
            B[name] = T(1, 64)
        B["p0"] = T(1, 32)
        B["u1"] = T(1, 96)
        B["p1"] = T(2, 64)
        for name in ("c4", "c5"):
            B[name] = T(2, 96)
        B["y32"] = T(0, NOUT, t.float32)
        # gradients
        B["gy"] = T(0, 32)
        B["g_a0"] = T(0, 32)
        B["G8"] = T(0, 32)
        B["g_u0"] = T(0, 64)
        B["tmp0"] = T(0, 32)
        B["g_c0"] = T(0, 32)
        B["g_c7"] = T(1, 64)
        B["g_a1"] = T(1, 64)
        B["G6"] = T(1, 64)
        B["g_u1"] = T(1, 96)
        B["tmp1"] = T(1, 64)
        B["g_c2"] = T(1, 64)
        B["g_p0"] = T(1, 32)
        B["g_c5"] = T(2, 96)
        B["g_c4"] = T(2, 96)
        B["g_p1"] = T(2, 64)
        ws = 0
        for name, (ci, _, co, _, lev) in LAYERS.items():
            hh, ww = hw[lev]
            ws = max(ws, nn.nn_conv3x3_wgrad_workspace(n, hh, ww, ci, co))
        B["work"] = t.empty(ws, dtype=t.uint8, device=self.dev)
        B["lwork"] = t.empty(8 * ((n * h * w + 255) // 256), dtype=t.uint8, device=self.dev)
        B["loss"] = t.zeros(1, dtype=t.float64, device=self.dev)
        B["hw"] = hw
        self.bufs[key] = B
        return B

    # ---- forward / backward -------------------------------------------------
    def _conv(self, name, x, y16, n, hw, relu=True, y32=None):
        ci, _, co, _, lev = LAYERS[name]
        h, w = hw[lev]
        q = self.p[name]
        nn.nn_conv3x3_fwd(x, q["w16"], q["b"], y16, y32, NOUT if y32 is not None else 0, n, h, w, ci, co,
                          1 if relu else 0)

    def forward(self, x, n, h, w):
        """x: [n][h][w][32] bf16 features; returns the [n][h][w][4] float32
        output buffer (valid until the next call)."""
        B = self._buffers(n, h, w)
        hw = B["hw"]
        if x is not B["x"]:
            B["x"].copy_(x)
        c = self._conv
        c("c0", B["x"], B["c0"], n, hw)
        c("c1", B["c0"], B["c1"], n, hw)
        nn.nn_pool2(0, B["c1"], B["p0"], n, hw[0][0], hw[0][1], 32)
        c("c2", B["p0"], B["c2"], n, hw)
        c("c3", B["c2"], B["c3"], n, hw)
        nn.nn_pool2(0, B["c3"], B["p1"], n, hw[1][0], hw[1][1], 64)
        c("c4", B["p1"], B["c4"], n, hw)
        c("c5", B["c4"], B["c5"], n, hw)
        nn.nn_up2(0, B["c5"], B["u1"], n, hw[2][0], hw[2][1], 96)
        c("c6", B["u1"], B["c6"], n, hw)
        nn.nn_add(B["c6"], B["c3"], B["a1"])
        c("c7", B["a1"], B["c7"], n, hw)
        nn.nn_up2(0, B["c7"], B["u0"], n, hw[1][0], hw[1][1], 64)
        c("c8", B["u0"], B["c8"], n, hw)
        nn.nn_add(B["c8"], B["c1"], B["a0"])
        c("c9", B["a0"], None, n, hw, relu=False, y32=B["y32"])
        return B["y32"]

    def _wgrad(self, name, x, dy, n, hw):
        ci, _, co, _, lev = LAYERS[name]
        h, w = hw[lev]
        q = self.p[name]
        B = self.bufs[(n, hw[0][0], hw[0][1])]
        nn.nn_conv3x3_bwd_weight(x, dy, q["gw"], q["gb"], B["work"], 0, n, h, w, ci, co)

    def _dgrad(self, name, dy, dx, n, hw):
        ci, _, co, _, lev = LAYERS[name]
        h, w = hw[lev]
        nn.nn_conv3x3_bwd_data(dy, self.p[name]["wf"], dx, n, h, w, ci, co)

    def backward(self, n, h, w, probe=None):
        """Parameter gradients (into gw, gb) from the output gradient in gy.
        probe(name, x, dy, dx), if given, is called right after each
        convolution's weight and data gradients, with the layer's input, the
        output gradient it was given and the input gradient it produced (None
        for c0), before later calls overwrite them in place."""
        B = self.bufs[(n, h, w)]
        hw = B["hw"]
        (h0, w0), (h1, w1), (h2, w2) = hw

        def layer(name, x, dy, dx):
            self._wgrad(name, x, dy, n, hw)
            if dx is not None:
                self._dgrad(name, dy, dx, n, hw)
            if probe is not None:
                probe(name, x, dy, dx)

        layer("c9", B["a0"], B["gy"], B["g_a0"])
        nn.nn_relu_bwd(B["g_a0"], B["c8"], B["G8"])
        layer("c8", B["u0"], B["G8"], B["g_u0"])
        nn.nn_up2(1, B["g_u0"], B["g_c7"], n, h1, w1, 64)
        nn.nn_relu_bwd(B["g_c7"], B["c7"], B["g_c7"])
        layer("c7", B["a1"], B["g_c7"], B["g_a1"])
        nn.nn_relu_bwd(B["g_a1"], B["c6"], B["G6"])
        layer("c6", B["u1"], B["G6"], B["g_u1"])
        nn.nn_up2(1, B["g_u1"], B["g_c5"], n, h2, w2, 96)
        nn.nn_relu_bwd(B["g_c5"], B["c5"], B["g_c5"])
        layer("c5", B["c4"], B["g_c5"], B["g_c4"])
        nn.nn_relu_bwd(B["g_c4"], B["c4"], B["g_c4"])
        layer("c4", B["p1"], B["g_c4"], B["g_p1"])
        nn.nn_pool2(1, B["g_p1"], B["tmp1"], n, h1, w1, 64)
        nn.nn_add(B["g_a1"], B["tmp1"], B["g_a1"])                   # grad of s1 = c3
        nn.nn_relu_bwd(B["g_a1"], B["c3"], B["g_a1"])
        layer("c3", B["c2"], B["g_a1"], B["g_c2"])
        nn.nn_relu_bwd(B["g_c2"], B["c2"], B["g_c2"])
        layer("c2", B["p0"], B["g_c2"], B["g_p0"])
        nn.nn_pool2(1, B["g_p0"], B["tmp0"], n, h0, w0, 32)
        nn.nn_add(B["g_a0"], B["tmp0"], B["g_a0"])                   # grad of s0 = c1
        nn.nn_relu_bwd(B["g_a0"], B["c1"], B["g_a0"])
        layer("c1", B["c0"], B["g_a0"], B["g_c0"])
        nn.nn_relu_bwd(B["g_c0"], B["c0"], B["g_c0"])
        layer("c0", B["x"], B["g_c0"], None)

    def loss_grad(self, target, n, h, w):
        """MSE of the last forward output against target [n][h][w][4];
        leaves the output gradient in gy; returns the loss (device scalar)."""
        B = self.bufs[(n, h, w)]
        nn.nn_mse(B["y32"], target, B["gy"], 32, n * h * w, NOUT, B["loss"], B["lwork"])
        return B["loss"]

    def adam(self, lr, weight_decay=0.0):
        self.step_count += 1
        for name, (ci, _, co, _, _) in LAYERS.items():
            q = self.p[name]
            nn.nn_adam(q["w"], q["w16"], q["wf"], q["gw"], q["mw"], q["vw"], co, ci, self.step_count, lr,
                       weight_decay=weight_decay)
            nn.nn_adam(q["b"], None, None, q["gb"], q["mb"], q["vb"], 0, 0, self.step_count, lr)

    # ---- channels <-> tensors ------------------------------------------------
    def features(self, cfgs):
        t = self.torch
        ny, nx = int(cfgs[0]["ny"]), int(cfgs[0]["nx"])
        x = t.empty((len(cfgs), ny, nx, CPAD), dtype=t.bfloat16, device=self.dev)
        nn.nn_features(cfgs, x, CPAD)
        return x

    def predict_fields(self, cfgs, batch: int = 32, phi_from_net: bool = True):
        """Device float64 fields [n][phi|ux|uy|T][ny][nx] for lbm_init_device.
        phi: the cold-start profile plus the network's deviation on the
        interface band, shifted to keep sum phi (phi_from_net), or the
        cold-start profile alone."""
        t = self.torch
        ny, nx = int(cfgs[0]["ny"]), int(cfgs[0]["nx"])
        out = t.empty((len(cfgs), 4, ny, nx), dtype=t.float64, device=self.dev)
        for s in range(0, len(cfgs), batch):
            part = cfgs[s:s + batch]
            x = self.features(part)
            y = self.forward(x, len(part), ny, nx)
            nn.nn_to_fields(part, y, out[s:s + len(part)], phi_from_net)
        return out


# ---------------------------------------------------------------------------
# Data generation, training and evaluation.

def log(*a):
    import sys
    print(*a, file=sys.stderr, flush=True)


def run_to_tolerance(ctx, cfgs, precision, tol=1e-8, cap=400_000, chunk=50_000, verbose=True, finish_fp64=True,
                     t0=None):
    """Step an initialised context until every channel has r <= tol or the
    cap; returns the per-channel residual records.

    Float32 contexts: on weakly driven channels the float32 residual can
    level off just above the tolerance (rounding of the capillary and
    Marangoni forces).  With finish_fp64, a channel whose residual is below
    1e-7 but has fallen less than fourfold over the last 100 000 steps
    counts as stalled (a float32 floor, or a decay too slow to be worth
    waiting for in float32);
    stalled channels move at once into a float64 context (lbm_get_state /
    lbm_set_state, exact), which finishes them within the remaining cap, and
    are retired from the float32 context with the finished state written
    back.  Their records then hold the float64 residual, the total steps and
    "finished_fp64": True.

    Fallback: a channel whose state turns non-finite (a diverged warm start,
    a prediction with non-finite values) is retired by the residual check
    with LBM_EDIVERGED; it is started again from rest in the same context
    (lbm_restart), once, and its record carries "restarted_cold": True and
    the steps it has taken in all (those spent before the divergence
    included).  A channel that diverges again from rest stays retired and
    is reported with "diverged": True."""
    t0 = time.perf_counter() if t0 is None else t0
    n = len(cfgs)
    watch = finish_fp64 and precision == lbm.LBM_FP32_DEV
    back = max(1, -(-100_000 // chunk))         # chunks in 100 000 steps
    hist = []
    finished = {}
    done = 0

    def finish(todo, fp32_steps):
        if verbose:
            log("  solve: finishing %d channel(s) in float64 after %d steps" % (len(todo), done))
        c64 = lbm.lbm_create([cfgs[k] for k in todo], precision=lbm.LBM_FP64)
        for q, k in enumerate(todo):
            lbm.lbm_set_state(c64, q, lbm.lbm_get_state(ctx, k))
        rc64, _ = lbm.lbm_solve(c64, tol, cap - done)
        if rc64 not in (lbm.LBM_OK, lbm.LBM_EDIVERGED):
            raise lbm.LBMError(rc64, "lbm_solve (float64 finish)")
        for q, k in enumerate(todo):
            r64 = lbm.lbm_residual(c64, q)
            lbm.lbm_set_state(ctx, k, lbm.lbm_get_state(c64, q))
            lbm.lbm_retire(ctx, k)
            r64["steps"] = fp32_steps[k] + r64["steps"]
            r64["finished_fp64"] = True
            finished[k] = r64
        lbm.lbm_destroy(c64)

    restarted = set()
    first = True
    while done < cap:
        # a short first solve catches a start that diverges at once (a bad
        # prediction) before a whole chunk goes by
        step = min(1000 if first else chunk, cap - done)
        rc, active = lbm.lbm_solve(ctx, tol, step)
        done += step
        if rc == lbm.LBM_EDIVERGED:
            bad = [k for k in range(n) if k not in restarted and k not in finished
                   and lbm.lbm_residual(ctx, k)["diverged"]]
            for k in bad:
                lbm.lbm_restart(ctx, k)          # the cold start from rest
                restarted.add(k)
            active += len(bad)
            if verbose and bad:
                log("  solve: %d channel(s) diverged, restarted from rest: %s" % (len(bad), bad))
        elif rc != lbm.LBM_OK:
            raise lbm.LBMError(rc, "lbm_solve")
        if verbose:
            log("  solve: %d steps, %d of %d active, %.1f s" % (done, active, n, time.perf_counter() - t0))
        if active == 0:
            break
        if first:
            first = False
            continue
        if watch:
            res = [lbm.lbm_residual(ctx, k) for k in range(n)]
            hist.append([r["r"] for r in res])
            live = [k for k in range(n) if res[k]["r"] > tol and k not in finished]
            if len(hist) > back and done < cap:
                stalled = [k for k in live if hist[-1][k] < 1e-7 and hist[-1][k] > 0.25 * hist[-1 - back][k]]
                if stalled:
                    finish(stalled, {k: res[k]["steps"] for k in stalled})
    res = [lbm.lbm_residual(ctx, k) for k in range(n)]
    for k, r in finished.items():
        res[k] = r
    for k in range(n):
        res[k]["restarted_cold"] = k in restarted
    return res


def solve_batch(cfgs, precision, tol=1e-8, cap=400_000, chunk=50_000, init_fields=None, tile=None, verbose=True,
                finish_fp64=True):
    """Batched solve to r <= tol (each channel retires on convergence), with
    the float64 finish of run_to_tolerance.  Returns (ctx, wall seconds,
    per-channel residual records)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = lbm.lbm_create(cfgs, precision=precision)
    if tile:
        lbm.lbm_set_tile(ctx, *tile)
    if init_fields is None:
        lbm.lbm_init(ctx)
    else:
        lbm.lbm_init_device(ctx, init_fields)
    res = run_to_tolerance(ctx, cfgs, precision, tol, cap, chunk, verbose, finish_fp64, t0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ctx, wall, res


def fields_tensor(ctx, n):
    """Converged fields of every channel as one device float64 tensor [n][4][ny][nx]."""
    import torch
    F = []
    for k in range(n):
        f = lbm.lbm_fields(ctx, k)
        F.append(np.stack([f["phi"], f["ux"], f["uy"], f["T"]]))
    return torch.from_numpy(np.stack(F)).cuda()


def train(net, X, Y, epochs, batch=16, lr=2e-3, lr_min=2e-5, warmup=100, seed=0, time_limit=None):
    """Mini-batch Adam on (X [N][h][w][32] bf16, Y [N][h][w][4] float32)."""
    import torch
    N, h, w = X.shape[0], X.shape[1], X.shape[2]
    steps_per_epoch = N // batch
    if steps_per_epoch == 0:
        raise ValueError("training needs at least one batch: %d samples, batch %d" % (N, batch))
    total = epochs * steps_per_epoch
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.perf_counter()
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(X.device)
        acc = torch.zeros((), dtype=torch.float64, device=X.device)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb = X.index_select(0, idx)
            yb = Y.index_select(0, idx)
            net.forward(xb, batch, h, w)
            loss = net.loss_grad(yb, batch, h, w)
            acc += loss[0]
            net.backward(batch, h, w)
            f = min(1.0, (k + 1) / warmup)
            lr_k = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * k / max(1, total))) if k >= warmup else lr * f
            net.adam(lr_k)
            k += 1
        ep_loss = float(acc) / steps_per_epoch
        hist.append(ep_loss)
        log("  epoch %d loss %.4e (%.1f s)" % (ep, ep_loss, time.perf_counter() - t0))
        if time_limit and time.perf_counter() - t0 > time_limit:
            break
    return hist


def cold_phi(cfgs):
    """Cold-start phi profile of each channel, [n][ny][nx] float64 on the GPU."""
    import torch
    out = []
    for c in cfgs:
        j = torch.arange(int(c["ny"]), dtype=torch.float64, device="cuda")
        ph = 0.5 * (1 + torch.tanh(2 * ((c["b"] - 0.5) - j) / c["W"]))
        out.append(ph[:, None].expand(int(c["ny"]), int(c["nx"])))
    return torch.stack(out)


def relative_errors(pred, ref, T_ref=1.0, phi0=None):
    """Per-output relative L2 errors of [n][4][ny][nx] fields (phi, ux, uy, T):
    T - T_ref relative to its own norm; u, v relative to |u|; phi relative to
    the norm of its deviation from phi0 (the cold-start profile) when given,
    else to its own norm."""
    import torch
    out = {}
    names = ("phi", "ux", "uy", "T")
    unorm = torch.sqrt(torch.sum(ref[:, 1] ** 2 + ref[:, 2] ** 2, dim=(1, 2)))
    for c, name in enumerate(names):
        d = torch.sqrt(torch.sum((pred[:, c] - ref[:, c]) ** 2, dim=(1, 2)))
        if name in ("ux", "uy"):
            den = unorm
        elif name == "T":
            den = torch.sqrt(torch.sum((ref[:, 3] - T_ref) ** 2, dim=(1, 2)))
        elif phi0 is not None:
            den = torch.sqrt(torch.sum((ref[:, 0] - phi0) ** 2, dim=(1, 2)))
        else:
            den = torch.sqrt(torch.sum(ref[:, 0] ** 2, dim=(1, 2)))
        out[name] = (d / den).cpu().numpy()
    return out
