"""Warm-start network kernels against the float64 numpy oracle
(oracle/nn_oracle.py), on bfloat16-rounded inputs.

Bounds: float32 outputs of a convolution agree to 2e-5 of the output scale
(float32 accumulation of bf16 products); bf16 outputs to one bf16 rounding
(2^-8 relative) plus that; weight gradients (float32) to 2e-5 of their
scale.  The whole-network gradient check compares every layer's weight
gradient in relative 2-norm; activations and their gradients are stored in
bf16 between layers, so the bound there is 3e-2."""
import numpy as np
import pytest

from oracle import nn_oracle as O
from paper_2210_07501_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm, nn
    lbm.load()
    nn.load()
    return torch, nn


def bf(torch, a):
    """numpy float64 -> (bf16 cuda tensor, the float64 values it holds)."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda().to(torch.bfloat16)
    return t, t.float().cpu().numpy().astype(np.float64)


def f32(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("ci,co,relu", [(32, 32, 1), (64, 96, 0), (96, 64, 1), (32, 64, 0), (96, 96, 1)])
def test_conv_forward(env, ci, co, relu):
    torch, nn = env
    rng = np.random.default_rng(ci + co)
    n, h, w = 2, 5, 128
    x, xr = bf(torch, rng.normal(size=(n, h, w, ci)))
    wt, wr = bf(torch, rng.normal(size=(co, 9, ci)) / np.sqrt(9 * ci))
    b = rng.normal(size=co).astype(np.float32)
    y16 = torch.empty((n, h, w, co), dtype=torch.bfloat16, device="cuda")
    y32 = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    nn.nn_conv3x3_fwd(x, wt, f32(torch, b), y16, y32, co, n, h, w, ci, co, relu)
    ref = O.conv3x3(xr, wr, b.astype(np.float64))
    if relu:
        ref = O.relu(ref)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(host(y32) - ref)) <= 2e-5 * scale
    assert np.all(np.abs(host(y16) - ref) <= 2.0 ** -8 * np.abs(ref) + 2e-5 * scale)


@pytest.mark.parametrize("n,h,w,ci,co", [
    (1, 3, 256, 64, 32),    # one row per work-group (LDS-staged path)
    (3, 2, 128, 32, 96),    # two rows per work-group, each group straddles two images
    (1, 5, 64, 96, 64),     # four rows per work-group, ragged: the last group has one row
    (2, 3, 192, 32, 32),    # a width outside 64 / 128 / 256: the unstaged path
])
def test_conv_forward_row_widths(env, n, h, w, ci, co):
    """Every launch shape of the forward convolution, periodic in x and
    zero-padded in y, against the oracle."""
    torch, nn = env
    rng = np.random.default_rng(n * h * w + ci + co)
    x, xr = bf(torch, rng.normal(size=(n, h, w, ci)))
    wt, wr = bf(torch, rng.normal(size=(co, 9, ci)) / np.sqrt(9 * ci))
    b = rng.normal(size=co).astype(np.float32)
    y32 = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    nn.nn_conv3x3_fwd(x, wt, f32(torch, b), None, y32, co, n, h, w, ci, co, 0)
    ref = O.conv3x3(xr, wr, b.astype(np.float64))
    assert np.max(np.abs(host(y32) - ref)) <= 2e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("ci,co", [(32, 32), (64, 96), (96, 64)])
def test_conv_backward(env, ci, co):
    torch, nn = env
    rng = np.random.default_rng(7 * ci + co)
    n, h, w = 2, 6, 64
    x, xr = bf(torch, rng.normal(size=(n, h, w, ci)))
    wt32 = f32(torch, rng.normal(size=(co, 9, ci)) / np.sqrt(9 * ci))
    w16 = torch.empty((co, 9, ci), dtype=torch.bfloat16, device="cuda")
    wf = torch.empty((ci, 9, co), dtype=torch.bfloat16, device="cuda")
    nn.nn_cast_weights(wt32, w16, wf, co, ci)
    wr = host(w16)
    assert np.array_equal(host(wf), np.transpose(wr[:, ::-1, :], (2, 1, 0)))   # flipped copy
    dy, dyr = bf(torch, rng.normal(size=(n, h, w, co)))
    dx = torch.empty((n, h, w, ci), dtype=torch.bfloat16, device="cuda")
    nn.nn_conv3x3_bwd_data(dy, wf, dx, n, h, w, ci, co)
    dw = torch.empty((co, 9, ci), dtype=torch.float32, device="cuda")
    db = torch.empty(co, dtype=torch.float32, device="cuda")
    work = torch.empty(nn.nn_conv3x3_wgrad_workspace(n, h, w, ci, co), dtype=torch.uint8, device="cuda")
    nn.nn_conv3x3_bwd_weight(x, dy, dw, db, work, 0, n, h, w, ci, co)
    rdx, rdw, rdb = O.conv3x3_backward(xr, wr, dyr)
    s = np.max(np.abs(rdx))
    assert np.all(np.abs(host(dx) - rdx) <= 2.0 ** -8 * np.abs(rdx) + 2e-5 * s)
    assert np.max(np.abs(host(dw) - rdw)) <= 2e-5 * np.max(np.abs(rdw))
    assert np.max(np.abs(host(db) - rdb)) <= 2e-5 * np.max(np.abs(rdb))
    # accumulate mode adds
    nn.nn_conv3x3_bwd_weight(x, dy, dw, db, work, 1, n, h, w, ci, co)
    assert np.max(np.abs(host(dw) - 2 * rdw)) <= 4e-5 * np.max(np.abs(rdw))


@pytest.mark.parametrize("n,h,w,c", [(3, 4, 256, 96), (1, 2, 128, 64)])
def test_pool_and_up_wide_rows(env, n, h, w, c):
    """Pooling and upsampling on rows wider than one block of 8-channel
    groups (w c / 8 > 256), against the oracle."""
    torch, nn = env
    rng = np.random.default_rng(n * h * w * c)
    x, xr = bf(torch, rng.normal(size=(n, h, w, c)))
    p = torch.empty((n, h // 2, w // 2, c), dtype=torch.bfloat16, device="cuda")
    nn.nn_pool2(0, x, p, n, h, w, c)
    assert np.allclose(host(p), O.pool2(xr), rtol=2.0 ** -8, atol=1e-6)
    gf = torch.empty((n, h, w, c), dtype=torch.bfloat16, device="cuda")
    nn.nn_pool2(1, p, gf, n, h, w, c)
    assert np.allclose(host(gf), O.pool2_backward(host(p)), rtol=2.0 ** -8, atol=1e-6)
    u = torch.empty((n, 2 * h, 2 * w, c), dtype=torch.bfloat16, device="cuda")
    nn.nn_up2(0, x, u, n, h, w, c)
    assert np.array_equal(host(u), O.up2(xr))
    gx = torch.empty((n, h, w, c), dtype=torch.bfloat16, device="cuda")
    nn.nn_up2(1, u, gx, n, h, w, c)
    assert np.allclose(host(gx), O.up2_backward(host(u)), rtol=2.0 ** -8, atol=1e-6)


def test_small_kernels(env):
    torch, nn = env
    rng = np.random.default_rng(11)
    n, h, w, c = 2, 6, 8, 32
    x, xr = bf(torch, rng.normal(size=(n, h, w, c)))
    p = torch.empty((n, h // 2, w // 2, c), dtype=torch.bfloat16, device="cuda")
    nn.nn_pool2(0, x, p, n, h, w, c)
    assert np.allclose(host(p), O.pool2(xr), rtol=2.0 ** -8, atol=1e-6)
    gc, gcr = bf(torch, rng.normal(size=(n, h // 2, w // 2, c)))
    gf = torch.empty((n, h, w, c), dtype=torch.bfloat16, device="cuda")
    nn.nn_pool2(1, gc, gf, n, h, w, c)
    assert np.allclose(host(gf), O.pool2_backward(gcr), rtol=2.0 ** -8, atol=1e-6)
    u = torch.empty((n, 2 * h, 2 * w, c), dtype=torch.bfloat16, device="cuda")
    nn.nn_up2(0, x, u, n, h, w, c)
    assert np.array_equal(host(u), O.up2(xr))
    gu, gur = bf(torch, rng.normal(size=(n, 2 * h, 2 * w, c)))
    gx = torch.empty_like(x)
    nn.nn_up2(1, gu, gx, n, h, w, c)
    assert np.allclose(host(gx), O.up2_backward(gur), rtol=2.0 ** -8, atol=1e-6)
    y, yr = bf(torch, rng.normal(size=(n, h, w, c)))
    s = torch.empty_like(x)
    nn.nn_add(x, y, s)
    assert np.allclose(host(s), xr + yr, rtol=2.0 ** -8, atol=1e-6)
    r = torch.empty_like(x)
    nn.nn_relu_bwd(x, y, r)
    assert np.array_equal(host(r), xr * (yr > 0))
    # unaligned views with an odd count take the one-element-per-thread kernels
    xs, ys = x.view(-1)[1:38], y.view(-1)[3:40]
    s2 = torch.zeros(64, dtype=torch.bfloat16, device="cuda")[1:38]
    nn.nn_add(xs, ys, s2)
    assert np.allclose(host(s2), xr.reshape(-1)[1:38] + yr.reshape(-1)[3:40], rtol=2.0 ** -8, atol=1e-6)
    r2 = torch.zeros(64, dtype=torch.bfloat16, device="cuda")[1:38]
    nn.nn_relu_bwd(xs, ys, r2)
    assert np.array_equal(host(r2), xr.reshape(-1)[1:38] * (yr.reshape(-1)[3:40] > 0))


def test_mse_and_adam(env):
    torch, nn = env
    rng = np.random.default_rng(12)
    npix, nch, cpad = 1000, 4, 32
    pr = rng.normal(size=(npix, nch)).astype(np.float32)
    tg = rng.normal(size=(npix, nch)).astype(np.float32)
    g = torch.empty((npix, cpad), dtype=torch.bfloat16, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    work = torch.empty(8 * ((npix + 255) // 256), dtype=torch.uint8, device="cuda")
    nn.nn_mse(f32(torch, pr), f32(torch, tg), g, cpad, npix, nch, loss, work)
    ref_loss, ref_g = O.mse(pr.astype(np.float64), tg.astype(np.float64))
    assert float(loss.cpu()[0]) == pytest.approx(ref_loss, rel=1e-6)
    gh = host(g)
    assert np.allclose(gh[:, :nch], ref_g, rtol=2.0 ** -8, atol=0)
    assert np.all(gh[:, nch:] == 0)
    # Adam, two steps, against the formula in float64
    co, ci = 32, 32
    w0 = rng.normal(size=(co, 9, ci)).astype(np.float32)
    grads = [rng.normal(size=(co, 9, ci)).astype(np.float32) for _ in range(2)]
    wt = f32(torch, w0)
    m = torch.zeros_like(wt)
    v = torch.zeros_like(wt)
    w16 = torch.empty((co, 9, ci), dtype=torch.bfloat16, device="cuda")
    wf = torch.empty((ci, 9, co), dtype=torch.bfloat16, device="cuda")
    lr, b1, b2, eps, wd = 1e-3, 0.9, 0.999, 1e-8, 1e-4
    W, M, V = w0.astype(np.float64), 0.0, 0.0
    for k, gr in enumerate(grads, start=1):
        nn.nn_adam(wt, w16, wf, f32(torch, gr), m, v, co, ci, k, lr, b1, b2, eps, wd)
        M = b1 * M + (1 - b1) * gr
        V = b2 * V + (1 - b2) * gr.astype(np.float64) ** 2
        W = W - lr * ((M / (1 - b1 ** k)) / (np.sqrt(V / (1 - b2 ** k)) + eps) + wd * W)
    assert np.max(np.abs(wt.cpu().numpy() - W)) <= 1e-6
    assert np.array_equal(host(w16), host(wt.to(torch.bfloat16)))
    assert np.array_equal(host(wf), np.transpose(host(w16)[:, ::-1, :], (2, 1, 0)))


def test_features_targets_and_handoff(env):
    """Input planes against their definitions; targets against their
    definitions (phi: the scaled deviation from the cold-start profile on the
    interface band); the hand-off inverts them, keeps sum phi and the bulk
    phi exact; lbm_init_device equals lbm_init from host fields."""
    torch, nn = env
    from paper_2210_07501_amd import lbm
    cfgs = inputs.warmstart_set(3, 900_000)
    ny, nx = cfgs[0]["ny"], cfgs[0]["nx"]
    x = torch.empty((3, ny, nx, 32), dtype=torch.bfloat16, device="cuda")
    nn.nn_features(cfgs, x, 32)
    X = host(x)
    for k, c in enumerate(cfgs):
        i = np.arange(nx)
        j = np.arange(ny)
        ph = 0.5 * (1 + np.tanh(2 * ((c["b"] - 0.5) - j) / c["W"]))
        planes = [np.broadcast_to(c["dT"] * np.cos(2 * np.pi * i / (nx / c["n_waves"])) + c["T_h"] - c["T_ref"], (ny, nx)),
                  np.broadcast_to(ph[:, None], (ny, nx)),
                  np.broadcast_to(((c["mu_a"] + ph * (c["mu_b"] - c["mu_a"])) / c["mu_b"])[:, None], (ny, nx)),
                  np.broadcast_to(((c["k_a"] + ph * (c["k_b"] - c["k_a"])) / c["k_b"])[:, None], (ny, nx)),
                  np.full((ny, nx), c["sigma_T"] / 2e-4), np.full((ny, nx), c["sigma_TT"] / 3e-4),
                  np.broadcast_to(((j + 0.5) / ny)[:, None], (ny, nx)), np.full((ny, nx), c["b"] / ny),
                  np.full((ny, nx), np.log(c["mu_a"] / c["mu_b"]) / np.log(5.0)),
                  np.full((ny, nx), np.log(c["k_a"] / c["k_b"]) / np.log(5.0))]
        for q, pl in enumerate(planes):
            assert np.allclose(X[k, :, :, q], pl, rtol=2.0 ** -8, atol=1e-7), (k, q)
        assert np.all(X[k, :, :, 10:] == 0)
    rng = np.random.default_rng(13)
    F = np.stack([np.stack([np.clip(rng.uniform(-0.1, 1.1, (ny, nx)), 0, 1), rng.normal(0, 1e-5, (ny, nx)),
                            rng.normal(0, 1e-5, (ny, nx)), 1 + rng.normal(0, 0.3, (ny, nx))]) for _ in range(3)])
    Fd = torch.from_numpy(F).cuda()
    tgt = torch.empty((3, ny, nx, 4), dtype=torch.float32, device="cuda")
    nn.nn_targets(cfgs, Fd, tgt)
    T = tgt.cpu().numpy()
    back = torch.empty_like(Fd)
    nn.nn_to_fields(cfgs, tgt, back, phi_from_net=True)
    Bk = back.cpu().numpy()
    # default hand-off: the cold-start phi profile, the network's u, v, T
    cold = torch.empty_like(Fd)
    nn.nn_to_fields(cfgs, tgt, cold)
    Ch = cold.cpu().numpy()
    # u, v, T: the targets are float32, each field comes back to float32 rounding of its scale
    for c in (1, 2, 3):
        ref = F[:, c] - (1.0 if c == 3 else 0.0)
        assert np.max(np.abs(Bk[:, c] - F[:, c])) <= 2e-7 * np.max(np.abs(ref)), c
    for k, c in enumerate(cfgs):
        us = nn.nn_velocity_scale(c)
        assert us == pytest.approx(0.01 * (abs(c["sigma_T"]) + c["sigma_TT"]) / c["mu_b"], rel=1e-12)
        assert np.allclose(T[k, :, :, 0], F[k, 1] / us, rtol=1e-6, atol=1e-6)
        # phi: 50 (phi - phi_cold) on the band |y - (b - 1/2)| <= 3 W, zero outside
        j = np.arange(ny)
        zeta = (c["b"] - 0.5) - j
        ph = 0.5 * (1 + np.tanh(2 * zeta / c["W"]))
        band = np.abs(zeta) <= 3 * c["W"]
        dev = (F[k, 0] - ph[:, None]) * band[:, None]
        assert np.allclose(T[k, :, :, 3], 50 * dev, rtol=0, atol=5e-6)
        # hand-off: phi_cold + deviation + the rigid shift that restores sum phi
        g = np.where(band, 1 / np.cosh(2 * zeta / c["W"]) ** 2, 0.0)
        S = np.sum(T[k, :, :, 3].astype(np.float64)) / 50
        expect = ph[:, None] + T[k, :, :, 3].astype(np.float64) / 50 - S / (nx * g.sum()) * g[:, None]
        assert np.max(np.abs(Bk[k, 0] - expect)) < 1e-12
        assert np.array_equal(Bk[k, 0][~band], Ch[k, 0][~band])    # bulk phi untouched
        assert Bk[k, 0].sum() == pytest.approx(Ch[k, 0].sum(), rel=1e-12)
    for k, c in enumerate(cfgs):
        ph = 0.5 * (1 + np.tanh(2 * ((c["b"] - 0.5) - np.arange(ny)) / c["W"]))
        assert np.allclose(Ch[k, 0], np.broadcast_to(ph[:, None], (ny, nx)), rtol=0, atol=1e-15)
        assert np.array_equal(Ch[k, 1:], Bk[k, 1:])
    for prec in (0, 1):
        a = lbm.lbm_create(cfgs, precision=prec)
        b = lbm.lbm_create(cfgs, precision=prec)
        lbm.lbm_init_device(a, back)
        Fh = back.cpu().numpy()
        lbm.lbm_init(b, [tuple(Fh[k]) for k in range(3)])
        for k in range(3):
            assert np.array_equal(lbm.lbm_get_state(a, k), lbm.lbm_get_state(b, k))


def test_network_gradients_against_oracle(env):
    """Whole U-Net, batch of 2 channels of 8 x 256: loss and every layer's
    weight and bias gradient against the float64 oracle evaluated with the
    network's bf16 weights and inputs."""
    torch, nn = env
    from paper_2210_07501_amd import warmstart as ws
    net = ws.WarmStartNet(seed=3)
    rng = np.random.default_rng(14)
    n, h, w = 2, 8, 256
    # non-zero biases so that they matter
    for name in ws.LAYERS:
        net.p[name]["b"].copy_(torch.from_numpy(rng.normal(0, 0.1, net.p[name]["b"].shape[0]).astype(np.float32)))
    x = torch.zeros((n, h, w, 32), dtype=torch.bfloat16, device="cuda")
    x[..., :10] = torch.from_numpy(rng.normal(size=(n, h, w, 10)).astype(np.float32)).cuda().to(torch.bfloat16)
    tgt = rng.normal(size=(n, h, w, 4)).astype(np.float32)
    net.forward(x, n, h, w)
    loss = float(net.loss_grad(f32(torch, tgt), n, h, w).cpu()[0])
    net.backward(n, h, w)
    p = {}
    for name in ws.LAYERS:
        p[name + ".w"] = host(net.p[name]["w16"])
        p[name + ".b"] = net.p[name]["b"].cpu().numpy().astype(np.float64)
    ref_loss, g, _ = O.loss_and_grads(p, host(x), tgt.astype(np.float64), 4)
    print("loss gpu %.6e oracle %.6e" % (loss, ref_loss), flush=True)
    assert loss == pytest.approx(ref_loss, rel=1e-2)
    for name in ws.LAYERS:
        gw = net.p[name]["gw"].cpu().numpy()
        gb = net.p[name]["gb"].cpu().numpy()
        ew = np.linalg.norm(gw - g[name + ".w"]) / np.linalg.norm(g[name + ".w"])
        eb = np.linalg.norm(gb - g[name + ".b"]) / max(np.linalg.norm(g[name + ".b"]), 1e-30)
        print("layer %s: weight-gradient error %.2e, bias %.2e" % (name, ew, eb), flush=True)
        assert ew <= 3e-2 and eb <= 3e-2, name


def test_training_reduces_loss(env):
    """A few hundred Adam steps on a fixed synthetic regression (smooth
    targets built from the inputs) cut the loss by more than 10x."""
    torch, nn = env
    from paper_2210_07501_amd import warmstart as ws
    net = ws.WarmStartNet(seed=4)
    rng = np.random.default_rng(15)
    N, h, w = 16, 8, 256
    xf = rng.normal(size=(N, h, w, 8)).astype(np.float32)
    X = torch.zeros((N, h, w, 32), dtype=torch.bfloat16, device="cuda")
    X[..., :8] = torch.from_numpy(xf).cuda().to(torch.bfloat16)
    Y = np.stack([xf[..., 0] * 0.5 + xf[..., 1], np.tanh(xf[..., 2]), xf[..., 3] * xf[..., 4] * 0.2,
                  0.3 * np.ones_like(xf[..., 0])], axis=-1).astype(np.float32)
    hist = ws.train(net, X, f32(torch, Y), epochs=150, batch=8, lr=2e-3, warmup=20)
    print("loss history", hist[0], hist[-1], flush=True)
    assert hist[-1] < hist[0] / 10
