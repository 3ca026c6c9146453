"""Float64 numpy reference of the warm-start network -- TEST INFRASTRUCTURE
ONLY (tests, the smoke check and the benchmark baseline may import it; the
product path never does, and it shares no code with the HIP kernels or their
Python orchestration).

Every operation is written from its plain definition, in NHWC layout:

  conv3x3:  y[n, i, j, o] = b[o] + sum_{t, c} x[n, i + dy_t, (j + dx_t) mod W, c] w[o, t, c]
            with tap t = 3 (dy + 1) + (dx + 1), dy, dx in {-1, 0, 1}; rows
            outside [0, H) contribute zero (the channel's walls), columns wrap
            (the channel is periodic).
  relu, 2x2 average pooling, nearest-neighbour x2 upsampling, skip addition,
  mean squared error over the real output channels.

The backward pass applies the chain rule to those definitions (adjoint of
each linear map); the test suite pins it against central finite
differences of the forward pass.

Architecture (a small U-Net; c = (in, out) channels, every conv 3x3 with
bias, ReLU except the last):
  level 0:  c0 (Cin -> 32), c1 (32 -> 32)           s0 = c1 output
  pool      c2 (32 -> 64),  c3 (64 -> 64)           s1 = c3 output
  pool      c4 (64 -> 96),  c5 (96 -> 96)
  up        c6 (96 -> 64);  a1 = c6 + s1;  c7 (64 -> 64)
  up        c8 (64 -> 32);  a0 = c8 + s0;  c9 (32 -> Cout), linear
The channel widths are parameters (`widths`) so that tests can shrink them.
"""
from __future__ import annotations

import numpy as np


def conv3x3(x, w, b):
    """x [N, H, W, C], w [O, 9, C], b [O] -> [N, H, W, O]."""
    N, H, W, C = x.shape
    O = w.shape[0]
    y = np.zeros((N, H, W, O)) + b
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        sh = np.zeros_like(x)
        lo, hi = max(0, -dy), min(H, H - dy)       # output rows whose source row exists
        sh[:, lo:hi] = np.roll(x, -dx, axis=2)[:, lo + dy:hi + dy]
        y += sh @ w[:, t, :].T
    return y


def conv3x3_backward(x, w, dy_out):
    """Gradients of conv3x3 with respect to x, w and b."""
    N, H, W, C = x.shape
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    db = dy_out.sum(axis=(0, 1, 2))
    for t in range(9):
        dy, dxs = t // 3 - 1, t % 3 - 1
        lo, hi = max(0, -dy), min(H, H - dy)
        sh = np.zeros_like(x)
        sh[:, lo:hi] = np.roll(x, -dxs, axis=2)[:, lo + dy:hi + dy]
        dw[:, t, :] = np.einsum("nijo,nijc->oc", dy_out, sh)
        # adjoint of the shift: g[:, lo:hi] lands on source rows lo+dy:hi+dy, columns rolled back
        g = np.zeros_like(x)
        g[:, lo:hi] = dy_out[:, lo:hi] @ w[:, t, :]
        back = np.zeros_like(x)
        back[:, lo + dy:hi + dy] = g[:, lo:hi]
        dx += np.roll(back, dxs, axis=2)
    return dx, dw, db


def relu(x):
    return np.maximum(x, 0.0)


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) * 0.25


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(g):
    N, H, W, C = g.shape
    return g.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def mse(pred, target):
    """Mean over all entries; returns (loss, d loss / d pred)."""
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


LAYERS = ("c0", "c1", "c2", "c3", "c4", "c5", "c6", "c7", "c8", "c9")


def layer_shapes(cin, cout, widths=(32, 64, 96)):
    w0, w1, w2 = widths
    return {"c0": (cin, w0), "c1": (w0, w0), "c2": (w0, w1), "c3": (w1, w1), "c4": (w1, w2),
            "c5": (w2, w2), "c6": (w2, w1), "c7": (w1, w1), "c8": (w1, w0), "c9": (w0, cout)}


def init_params(cin, cout, widths=(32, 64, 96), seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for name, (ci, co) in layer_shapes(cin, cout, widths).items():
        p[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(co, 9, ci))
        p[name + ".b"] = rng.normal(0.0, 0.05, size=co)
    return p


def forward(p, x):
    """Returns the output [N, H, W, Cout] and the activations the backward
    pass needs."""
    a = {}

    def conv(name, inp, act=True):
        y = conv3x3(inp, p[name + ".w"], p[name + ".b"])
        return relu(y) if act else y

    a["x"] = x
    a["c0"] = conv("c0", x)
    a["c1"] = conv("c1", a["c0"])
    a["p0"] = pool2(a["c1"])
    a["c2"] = conv("c2", a["p0"])
    a["c3"] = conv("c3", a["c2"])
    a["p1"] = pool2(a["c3"])
    a["c4"] = conv("c4", a["p1"])
    a["c5"] = conv("c5", a["c4"])
    a["u1"] = up2(a["c5"])
    a["c6"] = conv("c6", a["u1"])
    a["a1"] = a["c6"] + a["c3"]
    a["c7"] = conv("c7", a["a1"])
    a["u0"] = up2(a["c7"])
    a["c8"] = conv("c8", a["u0"])
    a["a0"] = a["c8"] + a["c1"]
    a["y"] = conv("c9", a["a0"], act=False)
    return a["y"], a


def backward(p, a, gy):
    """Gradients of sum(gy * y) with respect to every parameter."""
    g = {}

    def conv_b(name, inp, gout):
        dx, dw, db = conv3x3_backward(inp, p[name + ".w"], gout)
        g[name + ".w"] = dw
        g[name + ".b"] = db
        return dx

    def relu_b(gout, out):
        return gout * (out > 0)

    g_a0 = conv_b("c9", a["a0"], gy)
    g_u0 = conv_b("c8", a["u0"], relu_b(g_a0, a["c8"]))
    g_c7 = up2_backward(g_u0)
    g_a1 = conv_b("c7", a["a1"], relu_b(g_c7, a["c7"]))
    g_u1 = conv_b("c6", a["u1"], relu_b(g_a1, a["c6"]))
    g_c5 = up2_backward(g_u1)
    g_c4 = conv_b("c5", a["c4"], relu_b(g_c5, a["c5"]))
    g_p1 = conv_b("c4", a["p1"], relu_b(g_c4, a["c4"]))
    g_c3 = g_a1 + pool2_backward(g_p1)
    g_c2 = conv_b("c3", a["c2"], relu_b(g_c3, a["c3"]))
    g_p0 = conv_b("c2", a["p0"], relu_b(g_c2, a["c2"]))
    g_c1 = g_a0 + pool2_backward(g_p0)
    g_c0 = conv_b("c1", a["c0"], relu_b(g_c1, a["c1"]))
    conv_b("c0", a["x"], relu_b(g_c0, a["c0"]))
    return g


def loss_and_grads(p, x, target, nout):
    """MSE over the first nout output channels and its parameter gradients."""
    y, a = forward(p, x)
    loss, d = mse(y[..., :nout], target)
    gy = np.zeros_like(y)
    gy[..., :nout] = d
    return loss, backward(p, a, gy), y
