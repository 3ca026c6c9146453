"""Degenerate cases of the method on the HIP path, both precisions.

With no temperature variation along the interface, the Marangoni term has
nothing to act on and a flat interface carries no net force, so the fluid
stays at rest (Sec. 2 with Delta T = 0; Sec. 6 setting):

  flat, isothermal walls      no flow;
  vertical gradient only      T varies in y alone (T_h != T_c, Delta T = 0):
                              no flow, and every field stays x-invariant.

What is left of u is not rounding alone: the regularised normal leaves a
static normal force in the far tails of the profile, balanced by pressure,
with u_y ~ 1e-14 and u_x = 0 exactly on the oracle.  These tests bound a
spurious current far below what population parity at 1e-11 would admit:

  float64: |u_x| and |u - u_oracle| <= 2e-15 on every node (the rounding
           level of u; measured 5.4e-16 for u_x), and the oracle's own
           |u_y| <= 3e-14;
  float32: |u| <= 1e-10, 1e-6 of the 1e-4 interface velocities of the
           studied channels (an order below the float32 velocity bar);
  x-variation of phi, T, p relative to their scale: 1e-12 in float64 (a
           node's own phi sum and its halo copy in the neighbouring tile
           are added in different orders, and the difference accumulates
           over the steps: measured 8.9e-14 after 2000 steps), 2^-22 in
           float32 (four float32 ulps at phi = 1; measured one).
  Measured u: float64 |u_x| 5.4e-16, |u_y - u_y oracle| 1.1e-15;
           float32 |u_x| 7e-13, |u_y| 7e-12."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2210_07501_amd import inputs

pytestmark = pytest.mark.gpu

CASES = {
    "flat": (inputs.cfg(nx=128, ny=64, b=32.0, dT=0.0, sigma_T=-1e-4, sigma_TT=1e-4), 2000),
    "vertical": (inputs.cfg(nx=128, ny=64, b=32.0, dT=0.0, T_h=1.5, T_c=0.5,
                            sigma_T=-1e-4, sigma_TT=2e-4), 1000),
}
U64_BAR, U64_ORACLE, U32_BAR = 2e-15, 3e-14, 1e-10
XINV_BAR = {0: 1e-12, 1: 2.0 ** -22}
_oracle_fields = {}


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm as L
    L.load()
    return L


def oracle_fields(name):
    if name not in _oracle_fields:
        cfg, steps = CASES[name]
        o = orc.Oracle(cfg)
        o.init_cold()
        o.step(steps)
        _oracle_fields[name] = o.fields()
    return _oracle_fields[name]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_no_flow_without_temperature_variation_along_the_interface(lbm, name, prec):
    cfg, steps = CASES[name]
    print("case:", name, "128x64,", steps, "steps, precision", prec, flush=True)
    ctx = lbm.lbm_create(cfg, precision=prec)
    lbm.lbm_init(ctx)
    lbm.lbm_step(ctx, steps)
    F = lbm.lbm_fields(ctx)
    assert not lbm.lbm_residual(ctx)["diverged"]
    O = oracle_fields(name)
    ux, uy = float(np.max(np.abs(F["ux"]))), float(np.max(np.abs(F["uy"])))
    dux = float(np.max(np.abs(F["ux"] - O["ux"])))
    duy = float(np.max(np.abs(F["uy"] - O["uy"])))
    xvar = {k: float(np.max(np.abs(F[k] - F[k][:, :1])) / np.max(np.abs(F[k]))) for k in ("phi", "T", "p")}
    print("max |u_x| %.3e |u_y| %.3e; vs oracle %.3e %.3e; oracle |u_y| %.3e; x-variation %s"
          % (ux, uy, dux, duy, np.max(np.abs(O["uy"])), xvar), flush=True)
    if prec == 0:
        assert np.max(np.abs(O["ux"])) == 0.0 and np.max(np.abs(O["uy"])) <= U64_ORACLE
        assert ux <= U64_BAR and dux <= U64_BAR and duy <= U64_BAR
    else:
        assert ux <= U32_BAR and uy <= U32_BAR
    for k, v in xvar.items():
        assert v <= XINV_BAR[prec], (k, v)
    if name == "vertical":
        # heat is conducted from the hot bottom wall to the cold top wall
        assert np.all(np.diff(F["T"][:, 0]) < 0)
