"""Float32-deviation path (populations stored in float32 as deviations from
reference equilibria; the phase-field and hydrodynamic collisions, the
residual and the sums in float64) against the float64 oracle on the same
seeded inputs.

Tolerances are the float32 error budget of this storage scheme, measured and
stated per quantity (relative max-norm of each distribution; u on the scale
of the peak interface velocity):
  populations f <= 1e-6, g <= 1e-8, h <= 1e-7 after 2000 steps;
  u <= 1e-5 of the peak interface velocity after 2000 steps of the small
  channel, at equal densities and at density ratio 2 (measured 1.4e-7 and
  1.7e-7; the step is deterministic, so the figures reproduce exactly for a
  given build);
  sum phi drifts by < 1e-8 relative over 2000 steps;
  the same population bars at the full 4096 x 2048 size after 3 steps."""
import numpy as np
import pytest

from oracle import analytic as an
from paper_2210_07501_amd import inputs
from tests._parity import rel_maxnorm, run_oracle

pytestmark = pytest.mark.gpu

TOL_POP = {"f": 1e-6, "g": 1e-8, "h": 1e-7}


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm as L
    L.load()
    return L


def run32(L, cfg, steps, fields=None, tile=None):
    ctx = L.lbm_create(cfg, precision=L.LBM_FP32_DEV)
    if tile:
        L.lbm_set_tile(ctx, *tile)
    L.lbm_init(ctx, None if fields is None else [fields])
    L.lbm_step(ctx, steps)
    return ctx


def check_pops(pop, ref, scale=1.0):
    errs = {n: rel_maxnorm(pop[d], ref[d]) for d, n in enumerate("fgh")}
    bad = {n: e for n, e in errs.items() if not e <= TOL_POP[n] * scale}
    assert not bad, "float32 population error %s (all %s)" % (bad, errs)
    return errs


def test_small_channel_2000_steps_fp32(lbm):
    cfg = inputs.small_channel()
    print("case: small channel float32, 2000 steps", flush=True)
    ctx = run32(lbm, cfg, 2000)
    o = run_oracle(cfg, 2000)
    errs = check_pops(lbm.lbm_get_state(ctx), o.pop)
    F, R = lbm.lbm_fields(ctx), o.fields()
    upk = np.nanmax(np.abs(an.interface_profile(R["ux"], R["phi"])))
    du = max(np.max(np.abs(F["ux"] - R["ux"])), np.max(np.abs(F["uy"] - R["uy"])))
    print("float32 errors: populations", errs, "u / peak interface u", du / upk, flush=True)
    assert du <= 1e-5 * upk
    assert rel_maxnorm(F["phi"], R["phi"]) <= 1e-6
    assert rel_maxnorm(F["T"], R["T"]) <= 1e-7


@pytest.mark.parametrize("seed", [0, 3])
def test_seeded_variants_fp32(lbm, seed):
    cfg = inputs.perturbed_params(inputs.small_channel(), seed)
    fields = inputs.perturbed_fields(cfg, seed)
    ctx = run32(lbm, cfg, 600, fields=fields)
    check_pops(lbm.lbm_get_state(ctx), run_oracle(cfg, 600, fields=fields).pop)


@pytest.mark.parametrize("shape", [dict(nx=100, ny=36, n_waves=2, b=17.0), dict(nx=4, ny=12, n_waves=1, b=6.0)])
def test_ragged_fp32(lbm, shape):
    cfg = inputs.cfg(sigma_T=-1e-4, sigma_TT=2e-4, mu_a=0.05, k_a=0.3, **shape)
    fields = inputs.perturbed_fields(cfg, 7, amp=0.8)
    ctx = run32(lbm, cfg, 300, fields=fields)
    check_pops(lbm.lbm_get_state(ctx), run_oracle(cfg, 300, fields=fields).pop)


@pytest.mark.parametrize("tile", [(32, 8), (64, 4), (16, 16), (64, 16), (128, 8)])
def test_tile_shapes_fp32(lbm, tile):
    cfg = inputs.perturbed_params(inputs.small_channel(), 5)
    fields = inputs.perturbed_fields(cfg, 5)
    ctx = run32(lbm, cfg, 200, fields=fields, tile=tile)
    check_pops(lbm.lbm_get_state(ctx), run_oracle(cfg, 200, fields=fields).pop)


def test_batched_fp32(lbm):
    cfgs = [inputs.cfg(nx=128, ny=64, b=32.0, sigma_TT=1e-4),
            inputs.cfg(nx=96, ny=40, n_waves=2, b=12.0, sigma_T=-2e-4, mu_a=0.3, k_a=0.05)]
    fields = [inputs.perturbed_fields(c, 21 + k) for k, c in enumerate(cfgs)]
    ctx = lbm.lbm_create(cfgs, precision=lbm.LBM_FP32_DEV)
    lbm.lbm_init(ctx, fields)
    lbm.lbm_step(ctx, 250)
    for k, c in enumerate(cfgs):
        check_pops(lbm.lbm_get_state(ctx, k), run_oracle(c, 250, fields=fields[k]).pop)


def test_state_roundtrip_fp32(lbm):
    cfg = inputs.cfg(nx=64, ny=32, b=16.0, sigma_TT=1e-4)
    o = run_oracle(cfg, 150)
    ctx = lbm.lbm_create(cfg, precision=lbm.LBM_FP32_DEV)
    lbm.lbm_init(ctx)
    lbm.lbm_set_state(ctx, 0, o.pop)
    back = lbm.lbm_get_state(ctx)
    # float32 storage of small deviations: far below the population scale
    for d in range(3):
        assert rel_maxnorm(back[d], o.pop[d]) < 1e-8
    lbm.lbm_step(ctx, 100)
    o.step(100)
    check_pops(lbm.lbm_get_state(ctx), o.pop)


def test_phi_conservation_fp32(lbm):
    cfg = inputs.perturbed_params(inputs.small_channel(), 6)
    fields = inputs.perturbed_fields(cfg, 6)
    ctx = run32(lbm, cfg, 101, fields=fields)
    r0 = lbm.lbm_residual(ctx)
    lbm.lbm_step(ctx, 2000)
    r1 = lbm.lbm_residual(ctx)
    assert abs(r1["sum_phi"] - r0["sum_phi"]) / r0["sum_phi"] < 1e-8


def test_full_size_throughput_channel_fp32(lbm):
    """4096 x 2048, 8 wavelengths, in the launch configuration of the
    benchmark (64 x 8 tiles; a check step then two every-step launches):
    float32 storage against the float64 oracle on every node."""
    cfg = inputs.throughput_channel()
    print("case: 4096x2048 float32, 3 steps", flush=True)
    ctx = run32(lbm, cfg, 3)
    pop = lbm.lbm_get_state(ctx)
    del ctx
    errs = check_pops(pop, run_oracle(cfg, 3).pop)
    print("float32 full-size population errors", errs, flush=True)


def test_density_ratio_fp32(lbm):
    """Unequal densities (rho_b = 2 below) in float32 storage, the 128 x 64
    channel heated from rest, 2000 steps: the same bars as at equal
    densities -- u within 1e-5 of the peak interface velocity (measured
    1.7e-7; rho and u enter the g collision in float64, so 1/rho is not
    rounded into the momentum at every step) and the population bars."""
    cfg = dict(inputs.small_channel(), rho_b=2.0)
    print("case: density ratio 2, float32, small channel 2000 steps", flush=True)
    ctx = run32(lbm, cfg, 2000)
    o = run_oracle(cfg, 2000)
    errs = check_pops(lbm.lbm_get_state(ctx), o.pop)
    F, R = lbm.lbm_fields(ctx), o.fields()
    upk = np.nanmax(np.abs(an.interface_profile(R["ux"], R["phi"])))
    du = max(np.max(np.abs(F["ux"] - R["ux"])), np.max(np.abs(F["uy"] - R["uy"])))
    print("float32 density-ratio errors", errs, "u / peak interface u", du / upk, flush=True)
    assert du <= 1e-5 * upk

