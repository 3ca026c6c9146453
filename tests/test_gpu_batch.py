"""Batched channels, the hipGraph step loop and the tile autotuner.

A channel's arithmetic does not depend on the other channels of its context,
on the graph that replays its steps, or on the order in which tiles are
scheduled: batched, graph-replayed runs must reproduce single-channel eager
runs bit for bit (float64 and float32).  The autotuner must leave the state
untouched."""
import numpy as np
import pytest

from paper_2210_07501_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = {(64, 8), (32, 8), (64, 4), (16, 16), (64, 16), (128, 8)}


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm as L
    L.load()
    return L


def channels():
    return [inputs.cfg(nx=16, ny=10, b=5.0, sigma_TT=2e-4, mu_a=0.3, mu_b=0.3, k_a=0.3, k_b=0.3),
            inputs.perturbed_params(inputs.cfg(nx=96, ny=40, n_waves=2, b=12.0, sigma_T=-2e-4), 4),
            inputs.cfg(nx=128, ny=64, b=32.0, sigma_TT=2e-4),
            inputs.cfg(nx=200, ny=30, n_waves=5, b=9.0, sigma_T=1e-4, sigma_TT=3e-4, mu_a=0.02, k_a=0.5)]


@pytest.mark.parametrize("prec", [0, 1])
def test_batched_solve_matches_single_channel_runs(lbm, prec):
    cfgs = channels()
    print("case: batched solve vs single channels, precision", prec, flush=True)
    tol, cap = 1e-6, 3000
    ctx = lbm.lbm_create(cfgs, precision=prec)
    lbm.lbm_init(ctx)
    rc, active = lbm.lbm_solve(ctx, tol, cap)
    assert rc == 0
    steps = [lbm.lbm_residual(ctx, k)["steps"] for k in range(len(cfgs))]
    assert min(steps) < cap, steps          # at least one channel retired early
    assert active == sum(s == cap for s in steps)
    for k, c in enumerate(cfgs):
        one = lbm.lbm_create(c, precision=prec)
        lbm.lbm_init(one)
        lbm.lbm_solve(one, tol, cap)
        r1 = lbm.lbm_residual(one)
        assert r1["steps"] == steps[k]
        assert r1["r"] == lbm.lbm_residual(ctx, k)["r"]
        assert np.array_equal(lbm.lbm_get_state(one), lbm.lbm_get_state(ctx, k))
        lbm.lbm_destroy(one)


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_match_eager_steps(lbm, prec):
    """1000 steps as ten graph replays (tolerance 1e-300: nothing retires) equal
    1000 eager lbm_step calls; the check records agree too."""
    cfgs = channels()[1:3]
    a = lbm.lbm_create(cfgs, precision=prec)
    b = lbm.lbm_create(cfgs, precision=prec)
    for c in (a, b):
        lbm.lbm_init(c)
    rc, active = lbm.lbm_solve(a, 1e-300, 1000)
    assert rc == 0 and active == 2
    lbm.lbm_step(b, 1000)
    for k in range(2):
        ra, rb = lbm.lbm_residual(a, k), lbm.lbm_residual(b, k)
        assert ra["steps"] == rb["steps"] == 1000
        assert ra["r"] == rb["r"] and ra["sum_phi"] == rb["sum_phi"]
        assert np.array_equal(lbm.lbm_get_state(a, k), lbm.lbm_get_state(b, k))


@pytest.mark.parametrize("prec", [0, 1])
def test_autotune_leaves_state_and_picks_a_supported_shape(lbm, prec):
    cfgs = channels()
    ctx = lbm.lbm_create(cfgs, precision=prec)
    ref = lbm.lbm_create(cfgs, precision=prec)
    for c in (ctx, ref):
        lbm.lbm_init(c)
        lbm.lbm_step(c, 150)
    before = [lbm.lbm_get_state(ctx, k) for k in range(len(cfgs))]
    shape, ms = lbm.lbm_autotune(ctx, 3)
    print("autotune", shape, ms, flush=True)
    assert tuple(shape) in SHAPES and ms > 0
    for k in range(len(cfgs)):
        assert np.array_equal(lbm.lbm_get_state(ctx, k), before[k])
        assert lbm.lbm_residual(ctx, k)["steps"] == 150
    # stepping on with the chosen shape matches the default shape to rounding
    lbm.lbm_step(ctx, 100)
    lbm.lbm_step(ref, 100)
    for k in range(len(cfgs)):
        x, y = lbm.lbm_get_state(ctx, k), lbm.lbm_get_state(ref, k)
        for d in range(3):
            # float32: the halo and own-node sums round differently per shape
            assert np.max(np.abs(x[d] - y[d])) <= (1e-12 if prec == 0 else 1e-6) * np.max(np.abs(y[d]))


@pytest.mark.parametrize("prec", [0, 1])
def test_retire_on_request(lbm, prec):
    """lbm_retire stops one channel at the current step: its state and step
    count stay as they were while the rest of the batch goes on, and the
    rest match their single-channel runs bitwise."""
    cfgs = channels()[:2]
    print("case: retire on request, precision", prec, flush=True)
    ctx = lbm.lbm_create(cfgs, precision=prec)
    lbm.lbm_init(ctx)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_retire(ctx, 0)                 # before the first step
    assert e.value.status == lbm.LBM_ESTATE
    lbm.lbm_step(ctx, 250)
    held = lbm.lbm_get_state(ctx, 0)
    lbm.lbm_retire(ctx, 0)
    lbm.lbm_retire(ctx, 0)                     # a second call changes nothing
    rc, active = lbm.lbm_solve(ctx, 1e-300, 300)
    assert active == 1
    lbm.lbm_step(ctx, 50)
    assert np.array_equal(lbm.lbm_get_state(ctx, 0), held)
    assert lbm.lbm_residual(ctx, 0)["steps"] == 250
    n1 = lbm.lbm_residual(ctx, 1)["steps"]       # lbm_solve stops at a check boundary
    assert n1 >= 500
    one = lbm.lbm_create([cfgs[1]], precision=prec)
    lbm.lbm_init(one)
    lbm.lbm_step(one, n1)
    assert np.array_equal(lbm.lbm_get_state(ctx, 1), lbm.lbm_get_state(one, 0))


@pytest.mark.parametrize("prec", [0, 1])
def test_info_counts_the_device_bytes_held(lbm, prec):
    """lbm_info: every live allocation of the context, which at least holds
    the two population buffers and the float64 residual snapshot; the
    temporaries of lbm_fields, lbm_get_state and lbm_set_state are released."""
    cs = channels()
    nodes = sum(c["nx"] * c["ny"] for c in cs)
    elem = 8 if prec == 0 else 4
    ctx = lbm.lbm_create(cs, precision=prec)
    lbm.lbm_init(ctx)
    n, b0 = lbm.lbm_info(ctx)
    print("nodes", n, "device bytes", b0, "per node %.1f" % (b0 / n), flush=True)
    assert n == nodes
    floor = (2 * 27 * elem + 4 * 8) * nodes
    per_node_tables = 0 if prec == 0 else 16          # float32: T references and phi offsets, twice
    assert floor <= b0 <= floor + per_node_tables * nodes + (1 << 20)
    lbm.lbm_step(ctx, 10)
    lbm.lbm_fields(ctx, 2)
    pop = lbm.lbm_get_state(ctx, 1)
    lbm.lbm_set_state(ctx, 1, pop)
    assert lbm.lbm_info(ctx) == (n, b0)


@pytest.mark.parametrize("prec", [0, 1])
def test_profiled_steps_advance_the_state_like_plain_steps(lbm, prec):
    """lbm_profile_steps launches plain steps only (no checks).  In float64 a
    check step writes the same populations as a plain one, so 150 profiled
    steps equal 150 stepped ones bit for bit; in float32 the skipped checks
    keep the old storage references, which changes the rounding only.  The
    checks that follow report their own step index."""
    cs = channels()
    a = lbm.lbm_create(cs, precision=prec)
    lbm.lbm_init(a)
    ms = lbm.lbm_profile_steps(a, 150)
    assert ms > 0
    b = lbm.lbm_create(cs, precision=prec)
    lbm.lbm_init(b)
    lbm.lbm_step(b, 150)
    for k in range(len(cs)):
        pa, pb = lbm.lbm_get_state(a, k), lbm.lbm_get_state(b, k)
        if prec == 0:
            assert np.array_equal(pa, pb), k
        else:
            for d in range(3):
                scale = np.max(np.abs(pb[d]))
                assert np.max(np.abs(pa[d] - pb[d])) <= 1e-6 * scale, (k, d)
    lbm.lbm_step(a, 151)
    r = lbm.lbm_residual(a, 0)
    assert r["steps"] == 301 and not r["diverged"] and np.isfinite(r["r"])
