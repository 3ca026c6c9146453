"""The 256 x 128 sub-run of the throughput channel (the 4096 x 2048 workload
scaled by 1/16: 8 heating wavelengths of 32 cells, lower layer 38 cells,
viscosity ratio 0.5, conductivity ratio 2, sigma_T = -5e-5, sigma_TT = 2e-4),
20000 steps from rest, float64 and float32-deviation paths against the
float64 oracle.

Heating barely reaches the interface here (peak interface velocity ~4.3e-8),
so this is the case where deviation storage matters most.  Errors printed as
a table; bounds:
  float64: populations <= 1e-11 relative max-norm, u <= 1e-11 of the
           velocity scale max|g| / (rho c_s^2);
  float32: phi, T <= 1e-7 relative max-norm; u <= 1e-5 of the peak interface
           velocity (measured 8.8e-7, 3.8e-14 absolute).

On this weakly driven channel the float32 path used to miss its velocity bar
by 20x (2.0e-4).  Builds that promoted one group of the step's float32
arithmetic to float64 at a time located the cause: the float32 interface
normal, whose deviation n_y - n0_y was formed as the difference of two terms
first order in the phi deviation while the result is second order, and the
float32 arithmetic of the phase-field collision.  Fixing either alone left
1.6e-4 (normal) or 2.6e-4 (collision); both together reach the level of a
step done entirely in float64 with float32 storage (9.5e-7).  The step now forms n_y - n0_y
without cancellation and runs the phase-field collision in float64.
"""
import numpy as np
import pytest

from oracle import analytic as an
from paper_2210_07501_amd import inputs
from tests._parity import TOL64, rel_maxnorm, run_oracle

pytestmark = pytest.mark.gpu
STEPS = 20000


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm as L
    L.load()
    return L


@pytest.fixture(scope="module")
def ref():
    cfg = inputs.throughput_channel(scale=16)
    print("case: throughput sub-run 256x128, oracle %d steps" % STEPS, flush=True)
    o = run_oracle(cfg, STEPS)
    return cfg, o, o.fields()


def run(L, cfg, prec):
    ctx = L.lbm_create(cfg, precision=prec)
    L.lbm_init(ctx)
    L.lbm_step(ctx, STEPS)
    out = L.lbm_fields(ctx), L.lbm_get_state(ctx)
    L.lbm_destroy(ctx)
    return out


def table(F, R, upk):
    du = max(np.max(np.abs(F["ux"] - R["ux"])), np.max(np.abs(F["uy"] - R["uy"])))
    return {"phi": rel_maxnorm(F["phi"], R["phi"]), "T": rel_maxnorm(F["T"], R["T"]),
            "p": rel_maxnorm(F["p"], R["p"]), "u_abs": du, "u/peak": du / upk}


def test_subrun_float64(lbm, ref):
    cfg, o, R = ref
    F, pop = run(lbm, cfg, lbm.LBM_FP64)
    upk = np.nanmax(np.abs(an.interface_profile(R["ux"], R["phi"])))
    print("float64 sub-run errors", table(F, R, upk), flush=True)
    for d in range(3):
        assert rel_maxnorm(pop[d], o.pop[d]) <= TOL64
    uscale = np.max(np.abs(o.pop[1])) * 3.0
    assert max(np.max(np.abs(F["ux"] - R["ux"])), np.max(np.abs(F["uy"] - R["uy"]))) <= TOL64 * uscale


def test_subrun_float32(lbm, ref):
    cfg, o, R = ref
    F, _ = run(lbm, cfg, lbm.LBM_FP32_DEV)
    upk = np.nanmax(np.abs(an.interface_profile(R["ux"], R["phi"])))
    t = table(F, R, upk)
    print("float32 sub-run errors", t, flush=True)
    assert t["phi"] <= 1e-7 and t["T"] <= 1e-7
    assert t["u/peak"] <= 1e-5
