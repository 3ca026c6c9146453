"""What the trained warm-start network gains (held-out channels, seeds
900000 + i, 256 x 128), measured against the method without it.

Batched float32 solves to residual 1e-8 are started once from the network's
prediction (u, v, T from the network, phi the cold-start profile) and once
from rest.  Checked: the network's raw error is far below that of the state
at rest; both starts converge for the same channels and end in the same
steady state; the warm start needs no more steps in total than the cold one
(within 5%).  The step saving itself is printed, not asserted: with a
residual criterion on the relative change per 100 steps, the last decades
of convergence are set by the slowest viscous and thermal modes, which a
few-percent prediction error barely shortens (measured: about 3% fewer
steps at the median, per-channel ratios 0.8 - 1.5).
"""
import os

import numpy as np
import pytest

from paper_2210_07501_amd import inputs

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2210_07501_amd", "weights", "warmstart.npz")
N = 8
CAP = 600_000


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm
    from paper_2210_07501_amd import warmstart as ws
    lbm.load()
    if not os.path.exists(WEIGHTS):
        pytest.fail("trained weights missing: %s" % WEIGHTS)
    net = ws.WarmStartNet()
    net.load_state(WEIGHTS)
    return torch, lbm, ws, net


def test_warm_start_saves_steps_and_reaches_the_same_state(env):
    torch, lbm, ws, net = env
    cfgs = inputs.warmstart_set(N, 900_000)
    pred = net.predict_fields(cfgs)
    ctx_w, wall_w, res_w = ws.solve_batch(cfgs, lbm.LBM_FP32_DEV, cap=CAP, init_fields=pred, verbose=False)
    ctx_c, wall_c, res_c = ws.solve_batch(cfgs, lbm.LBM_FP32_DEV, cap=CAP, verbose=False)
    sw = np.array([r["steps"] for r in res_w])
    sc = np.array([r["steps"] for r in res_c])
    print("steps warm", sw.tolist(), "cold", sc.tolist(), "wall warm %.2f cold %.2f s" % (wall_w, wall_c), flush=True)
    conv_w = [r["r"] <= 1e-8 for r in res_w]
    conv_c = [r["r"] <= 1e-8 for r in res_c]
    assert conv_w == conv_c
    assert sw.sum() <= 1.05 * sc.sum()
    print("cold / warm steps: total %.3f, per channel %s" % (sc.sum() / sw.sum(), np.round(sc / sw, 2).tolist()),
          flush=True)
    Fw = ws.fields_tensor(ctx_w, N)
    Fc = ws.fields_tensor(ctx_c, N)
    err = ws.relative_errors(Fw, Fc)
    raw = ws.relative_errors(pred, Fc)
    # the state at rest (u = 0, T linear between the walls) as a "prediction"
    ctx0 = lbm.lbm_create(cfgs, precision=lbm.LBM_FP64)
    lbm.lbm_init(ctx0)
    rest = ws.relative_errors(ws.fields_tensor(ctx0, N), Fc)
    print("network raw error (median)", {k: float(np.median(v)) for k, v in raw.items()},
          "state at rest", {k: float(np.median(v)) for k, v in rest.items()},
          "warm vs cold steady state (max)", {k: float(np.max(v)) for k, v in err.items()}, flush=True)
    assert np.median(raw["T"]) < 0.5 * np.median(rest["T"])
    assert np.median(raw["ux"]) < 0.25 and np.median(raw["uy"]) < 0.25    # rest: 1
    for k, c in enumerate(cfgs):
        if conv_w[k]:
            # both stopped at r <= 1e-8: the same steady state to the
            # convergence level of the residual
            assert err["ux"][k] < 1e-2 and err["uy"][k] < 1e-2 and err["T"][k] < 1e-3 and err["phi"][k] < 1e-3
