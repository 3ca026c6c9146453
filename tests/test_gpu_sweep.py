"""The batched sweep at its full size, in the launch configuration the
benchmark times: 256 channels of the sweep distribution (seed 2210: nx in
{128, 256, 512}, ny = nx / 2, one heating wavelength, parameters drawn from
the seed; 14.6 M nodes) in one context with 64 x 8 tiles, every channel in
every launch.  200 steps (two of them check steps) in float64 and in
float32-deviation storage; then one sampled channel of each size against the
float64 oracle node by node, and against the same channel run alone (the
batch must not change a channel's arithmetic: bit for bit).

Bars: float64 populations 1e-11 relative max-norm; float32 populations
f <= 1e-6, g <= 1e-8, h <= 1e-7 (the bars of the float32 parity tests)."""
import numpy as np
import pytest

from paper_2210_07501_amd import inputs
from tests._parity import compare_state, rel_maxnorm, run_oracle

pytestmark = pytest.mark.gpu

STEPS = 200
TOL_POP32 = {"f": 1e-6, "g": 1e-8, "h": 1e-7}


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm as L
    L.load()
    return L


@pytest.fixture(scope="module")
def sweep():
    cfgs = inputs.batched_sweep(256, seed=2210)
    picks = [next(k for k, c in enumerate(cfgs) if c["nx"] == nx) for nx in (128, 256, 512)]
    return cfgs, picks


@pytest.fixture(scope="module")
def oracle_states(sweep):
    cfgs, picks = sweep
    print("case: oracle, sweep channels %s, %d steps" % (picks, STEPS), flush=True)
    return {k: run_oracle(cfgs[k], STEPS).pop for k in picks}


@pytest.mark.parametrize("prec", [0, 1])
def test_full_sweep_batch_sampled_channels(lbm, sweep, oracle_states, prec):
    cfgs, picks = sweep
    print("case: 256-channel sweep batch, precision %d, %d steps" % (prec, STEPS), flush=True)
    ctx = lbm.lbm_create(cfgs, precision=prec)
    nodes, _ = lbm.lbm_info(ctx)
    assert nodes == sum(c["nx"] * c["ny"] for c in cfgs) > 14_000_000
    lbm.lbm_init(ctx)
    lbm.lbm_step(ctx, STEPS)
    states = {k: lbm.lbm_get_state(ctx, k) for k in picks}
    lbm.lbm_destroy(ctx)
    for k in picks:
        c = cfgs[k]
        if prec == 0:
            errs = compare_state(states[k], oracle_states[k])
        else:
            errs = {n: rel_maxnorm(states[k][d], oracle_states[k][d]) for d, n in enumerate("fgh")}
            assert all(errs[n] <= TOL_POP32[n] for n in errs), (k, errs)
        print("  channel %d (%dx%d): %s" % (k, c["nx"], c["ny"], errs), flush=True)
        one = lbm.lbm_create(c, precision=prec)
        lbm.lbm_init(one)
        lbm.lbm_step(one, STEPS)
        assert np.array_equal(lbm.lbm_get_state(one), states[k])
        lbm.lbm_destroy(one)
