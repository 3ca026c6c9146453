"""Warm-start network kernels against the float64 numpy oracle
(oracle/nn_oracle.py), on bfloat16-rounded inputs.

Bounds: float32 outputs of a convolution agree to 2e-5 of the output scale
(float32 accumulation of bf16 products); bf16 outputs to one bf16 rounding
(2^-8 relative) plus that; weight gradients (float32) to 2e-5 of their
scale.  The whole network is checked layer by layer, each layer on the bf16
values the GPU stored for it, with the same per-element bounds."""
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


@pytest.mark.parametrize("ci,co,w", [(32, 32, 256), (64, 32, 256), (32, 64, 256), (32, 64, 128), (64, 32, 128),
                                     (64, 64, 128), (96, 64, 128), (64, 96, 128), (64, 96, 64), (96, 96, 64),
                                     (96, 64, 64)])
@pytest.mark.parametrize("rs", [1, 2, 8])
def test_conv_forward_row_walk(env, ci, co, w, rs):
    """The row-walking kernel (rows of 256, 128 and 64 pixels, every channel
    pair it is compiled for, the 96-channel pairs with their output channels
    split over two work-groups) with 1, 2 and 8 steps per work-group: 3
    images of 8 steps, so the walks start at image boundaries and the
    input-row ring turns over; bias and ReLU, bf16 and float32 outputs."""
    torch, nn = env
    R = 256 // w
    n, h = 3, 8 * R
    rng = np.random.default_rng(1000 * rs + ci + co + w)
    x, xr = bf(torch, rng.normal(size=(n, h, w, ci)))
    wt, wr = bf(torch, rng.normal(size=(co, 9, ci)) / np.sqrt(9 * ci))
    b = rng.normal(size=co).astype(np.float32)
    y16 = torch.empty((n, h, w, co), dtype=torch.bfloat16, device="cuda")
    y32 = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    print("case: walk ci %d co %d w %d steps %d" % (ci, co, w, rs), flush=True)
    nn.nn_set_conv_walk(rs)
    try:
        nn.nn_conv3x3_fwd(x, wt, f32(torch, b), y16, y32, co, n, h, w, ci, co, 1)
        torch.cuda.synchronize()
    finally:
        nn.nn_set_conv_walk(0)
    ref = O.relu(O.conv3x3(xr, wr, b.astype(np.float64)))
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(host(y32) - ref)) <= 2e-5 * scale
    assert np.all(np.abs(host(y16) - ref) <= 2.0 ** -8 * np.abs(ref) + 2e-5 * scale)


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


@pytest.mark.parametrize("n,h,w,ci,co", [
    (2, 160, 256, 32, 32),   # 256-pixel steps, two per chunk
    (1, 96, 256, 64, 32),    # 128-pixel steps in 256-pixel rows
    (2, 130, 128, 64, 64),   # 128-pixel steps, two per chunk
    (1, 40, 64, 96, 96),     # 64-pixel steps, four per chunk
    (2, 3, 192, 32, 32),     # a width outside 64 / 128 / 256: 64-pixel steps, short last chunk
    (1, 256, 256, 64, 32),   # 256 default chunks, cut to one round of resident blocks
])
def test_conv_weight_gradient_step_sizes(env, n, h, w, ci, co):
    """The weight gradient at every step size its kernel uses, with chunks
    of several steps and a short last chunk, and with the chunk count cut to
    what one round of resident blocks covers: dw and db against the oracle,
    and accumulate mode."""
    torch, nn = env
    rng = np.random.default_rng(n * h * w + 3 * ci + co)
    x, xr = bf(torch, rng.normal(size=(n, h, w, ci)))
    dy, dyr = bf(torch, rng.normal(size=(n, h, w, co)))
    wr = np.zeros((co, 9, ci))
    rdx, rdw, rdb = O.conv3x3_backward(xr, wr, dyr)
    dw = torch.empty((co, 9, ci), dtype=torch.float32, device="cuda")
    db = torch.empty(co, dtype=torch.float32, device="cuda")
    work = torch.empty(nn.nn_conv3x3_wgrad_workspace(n, h, w, ci, co), dtype=torch.uint8, device="cuda")
    print("case: wgrad n %d h %d w %d ci %d co %d" % (n, h, w, ci, co), flush=True)
    nn.nn_conv3x3_bwd_weight(x, dy, dw, db, work, 0, n, h, w, ci, co)
    assert np.max(np.abs(host(dw) - rdw)) <= 2e-5 * np.max(np.abs(rdw))
    assert np.max(np.abs(host(db) - rdb)) <= 2e-5 * np.max(np.abs(rdb))
    nn.nn_conv3x3_bwd_weight(x, dy, dw, db, work, 1, n, h, w, ci, co)
    assert np.max(np.abs(host(dw) - 2 * rdw)) <= 4e-5 * np.max(np.abs(rdw))
    assert np.max(np.abs(host(db) - 2 * rdb)) <= 4e-5 * np.max(np.abs(rdb))


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


# inputs of each convolution and the layer whose output feeds it (forward)
FWD_IN = {"c0": "x", "c1": "c0", "c2": "p0", "c3": "c2", "c4": "p1", "c5": "c4", "c6": "u1", "c7": "a1",
          "c8": "u0", "c9": "a0"}


def bf16_close(got, ref, scale):
    """Within one bfloat16 rounding of ref, plus float32 accumulation slack."""
    return np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 2e-5 * scale)


def test_network_gradients_against_oracle(env):
    """Whole U-Net, batch of 2 channels of 8 x 256, checked layer by layer
    and element by element against the float64 oracle, each layer on the
    very bf16 values the GPU gave it:
      forward: every convolution's output against the oracle convolution of
        its stored input with the bf16 weights (one bf16 rounding), and every
        pooling, upsampling and skip addition between them;
      backward: every layer's weight and bias gradients (float32, 2e-5 of
        their scale) and input gradient (one bf16 rounding) against the
        oracle's conv3x3_backward of its stored input and output gradient,
        and every output gradient a layer was given against the oracle chain
        rule (ReLU mask, upsampling and pooling adjoints, skip sums) applied
        to the GPU's own upstream gradients;
    and the loss against the oracle's."""
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
    B = net.bufs[(n, h, w)]
    A = {k: host(B[k]) for k in ("x", "c0", "c1", "p0", "c2", "c3", "p1", "c4", "c5", "u1", "c6", "a1", "c7", "u0",
                                 "c8", "a0")}
    y32 = B["y32"].cpu().numpy().astype(np.float64)
    Wt = {name: host(net.p[name]["w16"]) for name in ws.LAYERS}
    bias = {name: net.p[name]["b"].cpu().numpy().astype(np.float64) for name in ws.LAYERS}
    # forward, layer by layer
    for name in ws.LAYERS:
        ref = O.conv3x3(A[FWD_IN[name]], Wt[name], bias[name])
        if name == "c9":
            ref = ref[..., :ws.NOUT]
            assert np.max(np.abs(y32 - ref)) <= 2e-5 * np.max(np.abs(ref)), name
        else:
            ref = O.relu(ref)
            assert bf16_close(A[name], ref, np.max(np.abs(ref))), name
    for out, ref in (("p0", O.pool2(A["c1"])), ("p1", O.pool2(A["c3"])), ("u1", O.up2(A["c5"])),
                     ("u0", O.up2(A["c7"])), ("a1", A["c6"] + A["c3"]), ("a0", A["c8"] + A["c1"])):
        assert bf16_close(A[out], ref, np.max(np.abs(ref))), out
    loss = float(net.loss_grad(f32(torch, tgt), n, h, w).cpu()[0])
    gy = host(B["gy"])
    seen = {}
    net.backward(n, h, w, probe=lambda name, X, DY, DX: seen.__setitem__(
        name, (host(X), host(DY), None if DX is None else host(DX))))
    # the loss and its gradient
    p = {}
    for name in ws.LAYERS:
        p[name + ".w"], p[name + ".b"] = Wt[name], bias[name]
    ref_loss, _, _ = O.loss_and_grads(p, A["x"], tgt.astype(np.float64), 4)
    print("loss gpu %.6e oracle %.6e" % (loss, ref_loss), flush=True)
    assert loss == pytest.approx(ref_loss, rel=1e-2)
    l_y, d_y = O.mse(y32, tgt.astype(np.float64))
    assert loss == pytest.approx(l_y, rel=1e-6)
    ref_gy = np.zeros_like(gy)
    ref_gy[..., :4] = d_y
    assert bf16_close(gy, ref_gy, np.max(np.abs(ref_gy)))
    assert np.all(gy[..., 4:] == 0)
    # each layer's own gradients, on the inputs it was given
    for name in ws.LAYERS:
        X, DY, DX = seen[name]
        assert np.array_equal(X, A[FWD_IN[name]]), name
        rdx, rdw, rdb = O.conv3x3_backward(X, Wt[name], DY)
        gw = net.p[name]["gw"].cpu().numpy().astype(np.float64)
        gb = net.p[name]["gb"].cpu().numpy().astype(np.float64)
        ew = np.max(np.abs(gw - rdw)) / np.max(np.abs(rdw))
        eb = np.max(np.abs(gb - rdb)) / max(np.max(np.abs(rdb)), 1e-30)
        print("layer %s: weight-gradient max error / scale %.2e, bias %.2e" % (name, ew, eb), flush=True)
        assert ew <= 2e-5 and eb <= 2e-5, name
        if DX is not None:
            assert bf16_close(DX, rdx, np.max(np.abs(rdx))), name
    # the output gradient each layer was given: the chain rule on the GPU's own upstream gradients
    dx = {name: seen[name][2] for name in ws.LAYERS}
    relu_b = lambda g, out: g * (out > 0)
    chain = {
        "c9": ref_gy,
        "c8": relu_b(dx["c9"], A["c8"]),
        "c7": relu_b(O.up2_backward(dx["c8"]), A["c7"]),
        "c6": relu_b(dx["c7"], A["c6"]),
        "c5": relu_b(O.up2_backward(dx["c6"]), A["c5"]),
        "c4": relu_b(dx["c5"], A["c4"]),
        "c3": relu_b(dx["c7"] + O.pool2_backward(dx["c4"]), A["c3"]),
        "c2": relu_b(dx["c3"], A["c2"]),
        "c1": relu_b(dx["c9"] + O.pool2_backward(dx["c2"]), A["c1"]),
        "c0": relu_b(dx["c1"], A["c0"]),
    }
    for name in ws.LAYERS:
        ref = chain[name]
        assert bf16_close(seen[name][1], ref, np.max(np.abs(ref))), name


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
