"""Pins of the float64 network oracle (CPU): each operation against its
definition written out as loops, backward passes against central finite
differences of the forward pass, pooling/upsampling against their adjoints."""
import numpy as np
import pytest

from oracle import nn_oracle as nn


def conv_loops(x, w, b):
    N, H, W, C = x.shape
    O = w.shape[0]
    y = np.zeros((N, H, W, O))
    for n in range(N):
        for i in range(H):
            for j in range(W):
                for o in range(O):
                    s = b[o]
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            ii = i + dy
                            if ii < 0 or ii >= H:
                                continue          # wall: zero padding
                            jj = (j + dx) % W      # periodic
                            t = 3 * (dy + 1) + (dx + 1)
                            s += np.dot(x[n, ii, jj], w[o, t])
                    y[n, i, j, o] = s
    return y


def test_conv_matches_loops():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 5, 2))
    w = rng.normal(size=(3, 9, 2))
    b = rng.normal(size=3)
    assert np.allclose(nn.conv3x3(x, w, b), conv_loops(x, w, b), rtol=0, atol=1e-13)


def test_conv_single_tap_is_a_shift():
    # only tap (dy, dx) = (1, -1) set: y[i, j] = x[i + 1, j - 1], zero in the last row
    x = np.arange(1 * 4 * 6 * 1, dtype=float).reshape(1, 4, 6, 1)
    w = np.zeros((1, 9, 1))
    w[0, 3 * 2 + 0, 0] = 1.0
    y = nn.conv3x3(x, w, np.zeros(1))
    for i in range(4):
        for j in range(6):
            ref = x[0, i + 1, (j - 1) % 6, 0] if i + 1 < 4 else 0.0
            assert y[0, i, j, 0] == ref


def fd(f, v, idx, eps=1e-6):
    old = v[idx]
    v[idx] = old + eps
    fp = f()
    v[idx] = old - eps
    fm = f()
    v[idx] = old
    return (fp - fm) / (2 * eps)


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 5, 3))
    w = rng.normal(size=(2, 9, 3))
    b = rng.normal(size=2)
    g = rng.normal(size=(2, 4, 5, 2))
    dx, dw, db = nn.conv3x3_backward(x, w, g)
    L = lambda: float(np.sum(g * nn.conv3x3(x, w, b)))
    for idx in [(0, 0, 0, 0), (1, 3, 4, 2), (0, 2, 1, 1), (1, 0, 4, 0)]:
        assert dx[idx] == pytest.approx(fd(L, x, idx), rel=1e-7, abs=1e-9)
    for idx in [(0, 0, 0), (1, 8, 2), (0, 4, 1), (1, 5, 0)]:
        assert dw[idx] == pytest.approx(fd(L, w, idx), rel=1e-7, abs=1e-9)
    for o in range(2):
        assert db[o] == pytest.approx(fd(L, b, (o,)), rel=1e-7, abs=1e-9)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(2, 6, 8, 3))
    yc = rng.normal(size=(2, 3, 4, 3))
    assert np.sum(nn.pool2(x) * yc) == pytest.approx(np.sum(x * nn.pool2_backward(yc)), rel=1e-13)
    assert np.sum(nn.up2(yc) * x) == pytest.approx(np.sum(yc * nn.up2_backward(x)), rel=1e-13)
    # definitions: pooling averages a 2x2 block, upsampling copies
    assert nn.pool2(x)[1, 2, 3, 1] == pytest.approx(x[1, 4:6, 6:8, 1].mean(), rel=1e-14)
    assert np.array_equal(nn.up2(yc)[0, 5, 7], yc[0, 2, 3])
    assert np.allclose(nn.pool2(nn.up2(yc)), yc, rtol=0, atol=1e-15)


def test_mse_gradient():
    rng = np.random.default_rng(4)
    p = rng.normal(size=(3, 5, 4))
    t = rng.normal(size=(3, 5, 4))
    loss, d = nn.mse(p, t)
    assert loss == pytest.approx(np.sum((p - t) ** 2) / p.size, rel=1e-14)
    L = lambda: nn.mse(p, t)[0]
    for idx in [(0, 0, 0), (2, 4, 3), (1, 2, 1)]:
        assert d[idx] == pytest.approx(fd(L, p, idx), rel=1e-7)


def test_network_gradients_match_finite_differences():
    """Whole U-Net (shrunk widths) on an 8 x 8 image: loss gradients of
    sampled weights and biases of every layer against central differences."""
    rng = np.random.default_rng(5)
    cin, cout, nout = 3, 5, 4
    p = nn.init_params(cin, cout, widths=(4, 5, 6), seed=6)
    x = rng.normal(size=(2, 8, 8, cin))
    t = rng.normal(size=(2, 8, 8, nout))
    loss, g, _ = nn.loss_and_grads(p, x, t, nout)
    L = lambda: nn.loss_and_grads(p, x, t, nout)[0]
    for name in nn.LAYERS:
        w = p[name + ".w"]
        for idx in [(0, 4, 0), (w.shape[0] - 1, 7, w.shape[2] - 1), (w.shape[0] // 2, 1, w.shape[2] // 2)]:
            assert g[name + ".w"][idx] == pytest.approx(fd(L, w, idx), rel=1e-5, abs=1e-10), (name, idx)
        bvec = p[name + ".b"]
        assert g[name + ".b"][0] == pytest.approx(fd(L, bvec, (0,)), rel=1e-5, abs=1e-10), name
