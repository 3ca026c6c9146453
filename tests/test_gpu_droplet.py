"""Thermocapillary migration of a droplet (Sec. 5.1): the one workload here
where curvature and a genuinely two-dimensional interface matter.

Domain 8R x 16R with R = 20, uniform temperature gradient 0.1 between the
walls, mu = k = 0.2, sigma_T = -1e-4.  The paper compares its 2D droplet with
the 3D Young-Goldstein-Block velocity U_YGB = 1.333e-4 and finds about 80% of
it (as do the other 2D schemes it cites).  Checked: the droplet moves toward
the hot wall at a terminal velocity within [0.75, 0.85] U_YGB (measured 0.791),
keeps sum phi (float64: 1e-12; float32: 1e-7 over 1e5 steps), and float32
agrees with float64; a smaller droplet matches the float64 oracle step by
step (curvature and its stencils)."""
import json
import os

import numpy as np
import pytest

from oracle import analytic as an
from paper_2210_07501_amd import inputs
from tests._parity import compare_state, run_oracle

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_numbers.json")))["ygb_droplet"]
CHUNK, N_CHUNKS = 5000, 20


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm as L
    L.load()
    return L


def migrate(L, prec):
    cfg, fields = inputs.droplet()
    ctx = L.lbm_create(cfg, precision=prec)
    L.lbm_init(ctx, [fields])
    y = np.arange(cfg["ny"], dtype=np.float64)[:, None]
    cen, mass = [], []
    for _ in range(N_CHUNKS):
        L.lbm_step(ctx, CHUNK)
        phi = L.lbm_fields(ctx)["phi"]
        cen.append(float((phi * y).sum() / phi.sum()))
        mass.append(float(phi.sum()))
    L.lbm_destroy(ctx)
    v = np.diff(cen) / CHUNK
    return cfg, np.array(cen), v, np.array(mass)


@pytest.fixture(scope="module")
def run64(lbm):
    print("case: droplet 160x320 float64, %d steps" % (CHUNK * N_CHUNKS), flush=True)
    return migrate(lbm, lbm.LBM_FP64)


def test_droplet_migrates_toward_hot_at_the_2d_fraction_of_ygb(run64):
    cfg, cen, v, mass = run64
    U = an.ygb_velocity(cfg["sigma_T"], 0.1, 20.0, cfg["mu_b"], cfg["k_a"] / cfg["k_b"], cfg["mu_a"] / cfg["mu_b"])
    assert U == pytest.approx(GOLD["printed_U_YGB"], rel=1e-3)
    terminal = v[-5:].mean()
    ratio = terminal / U
    print("droplet terminal velocity %.4e, U_YGB %.4e, ratio %.3f (paper: about %.2f)"
          % (terminal, U, ratio, GOLD["printed_ratio_2d"]), flush=True)
    assert np.all(v > 0)                           # toward the hot (top) wall
    assert abs(ratio - GOLD["printed_ratio_2d"]) <= 0.05
    assert np.std(v[-5:]) < 0.01 * terminal        # terminal
    assert np.max(np.abs(mass - mass[0])) <= 1e-12 * mass[0]


def test_droplet_float32_matches_float64(lbm, run64):
    _, _, v64, _ = run64
    _, _, v32, mass32 = migrate(lbm, lbm.LBM_FP32_DEV)
    print("float32 / float64 terminal velocity %.5f" % (v32[-5:].mean() / v64[-5:].mean()), flush=True)
    assert abs(v32[-5:].mean() / v64[-5:].mean() - 1) < 1e-2
    # float32 storage keeps sum phi to the rounding of the small stored rest
    # populations: measured 4e-8 relative over these 1e5 steps
    assert np.max(np.abs(mass32 - mass32[0])) <= 1e-7 * mass32[0]


def test_small_droplet_matches_oracle(lbm):
    """R = 8 (64 x 128): 300 steps, every population against the oracle."""
    cfg, fields = inputs.droplet(R=8.0)
    ctx = lbm.lbm_create(cfg)
    lbm.lbm_init(ctx, [fields])
    lbm.lbm_step(ctx, 300)
    compare_state(lbm.lbm_get_state(ctx), run_oracle(cfg, 300, fields=fields).pop)
