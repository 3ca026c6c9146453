"""Helpers for the GPU-vs-oracle parity tests (test infrastructure)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc

# Float64 bar (relative max-norm), for populations and phi, T, p; the
# velocity is compared on the scale of the momentum populations, max|g| /
# (rho c_s^2), because u itself is ~1e-6 of the population scale.
TOL64 = 1e-11


def rel_maxnorm(a, ref):
    s = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(np.asarray(a) - np.asarray(ref)))) / (s if s > 0 else 1.0)


def compare_state(gpu_pop, orc_pop, tol=TOL64):
    errs = {}
    for d, name in enumerate("fgh"):
        errs[name] = rel_maxnorm(gpu_pop[d], orc_pop[d])
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, "population mismatch %s (all: %s)" % (bad, errs)
    return errs


def compare_fields(gf, of, g_scale, tol=TOL64):
    errs = {k: rel_maxnorm(gf[k], of[k]) for k in ("phi", "T", "p")}
    uscale = 3.0 * g_scale
    errs["u"] = max(float(np.max(np.abs(gf["ux"] - of["ux"]))), float(np.max(np.abs(gf["uy"] - of["uy"])))) / uscale
    umax = max(float(np.max(np.abs(of["ux"]))), float(np.max(np.abs(of["uy"]))))
    errs["u_rel_own_peak"] = (errs["u"] * uscale / umax) if umax > 0 else 0.0
    bad = {k: v for k, v in errs.items() if k != "u_rel_own_peak" and not v <= tol}
    assert not bad, "field mismatch %s (all: %s)" % (bad, errs)
    return errs


def run_oracle(cfg, steps, fields=None):
    o = orc.Oracle(cfg)
    if fields is None:
        o.init_cold()
    else:
        o.init_fields(*fields)
    o.step(steps)
    return o


def oracle_sensitivity(cfg, steps, fields=None, seed=1):
    """Conditioning of a case: relative max-norm change of the oracle's
    populations (f, g, h) and phi after `steps` when its initial populations
    are perturbed by one ulp (relative 2^-52, seeded signs).  Two float64
    implementations that round differently cannot agree more closely than
    this, whatever the bar."""
    a = run_oracle(cfg, 0, fields)
    b = run_oracle(cfg, 0, fields)
    rng = np.random.default_rng(seed)
    b.set_state(b.pop * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=b.pop.shape)))
    a.step(steps)
    b.step(steps)
    out = {name: rel_maxnorm(b.pop[d], a.pop[d]) for d, name in enumerate("fgh")}
    out["phi"] = rel_maxnorm(b.fields()["phi"], a.fields()["phi"])
    return out
