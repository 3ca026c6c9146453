"""The seeded synthetic workloads match the recipes stated for them
(sizes, ranges, determinism); the module holds no lattice Boltzmann
arithmetic, only parameter draws and initial fields."""
import numpy as np

from paper_2210_07501_amd import inputs


def test_batched_sweep_recipe():
    cs = inputs.batched_sweep()
    assert len(cs) == 256
    assert cs == inputs.batched_sweep()                       # seeded: same draw every time
    assert cs != inputs.batched_sweep(seed=2211)
    nodes = 0
    for c in cs:
        assert c["nx"] in (128, 256, 512) and c["ny"] == c["nx"] // 2 and c["n_waves"] == 1
        assert -2e-4 <= c["sigma_T"] <= 2e-4 and 0.0 <= c["sigma_TT"] <= 3e-4
        assert 0.25 * c["ny"] - 0.5 <= c["b"] <= 0.75 * c["ny"] + 0.5 and c["b"] == round(c["b"])
        assert 0.2 <= c["mu_a"] / c["mu_b"] <= 5.0 and 0.2 <= c["k_a"] / c["k_b"] <= 5.0
        assert c["mu_b"] == 0.1 and c["k_b"] == 0.1 and c["rho_a"] == c["rho_b"] == 1.0
        nodes += c["nx"] * c["ny"]
    assert abs(nodes / 1e6 - 14.6) < 0.1                      # the sweep's 14.6 M nodes
    # every size is drawn, and the ratios span their range
    assert {c["nx"] for c in cs} == {128, 256, 512}
    mr = np.log([c["mu_a"] / c["mu_b"] for c in cs]) / np.log(5.0)
    assert mr.min() < -0.9 and mr.max() > 0.9


def test_warmstart_sets():
    train = inputs.warmstart_set(8, 10_000)
    held = inputs.warmstart_set(8, 900_000)
    assert all(c["nx"] == 256 and c["ny"] == 128 for c in train + held)
    assert train == inputs.warmstart_set(8, 10_000)
    assert not any(a == b for a in train for b in held)       # disjoint seeds, different channels
    assert held[3] == inputs.batched_sweep(1, seed=900_003, nx_choices=(256,))[0]


def test_fixed_workloads():
    t = inputs.throughput_channel()
    assert (t["nx"], t["ny"], t["n_waves"], t["b"]) == (4096, 2048, 8, 614.0)
    assert (t["mu_a"], t["k_a"], t["sigma_T"], t["sigma_TT"]) == (0.05, 0.2, -5e-5, 2e-4)
    s = inputs.throughput_channel(16)
    assert (s["nx"], s["ny"], s["n_waves"], s["b"]) == (256, 128, 8, 38.0)
    c0 = inputs.small_channel()
    assert (c0["nx"], c0["ny"], c0["b"], c0["sigma_T"], c0["sigma_TT"]) == (128, 64, 32.0, 0.0, 1e-4)
    for kind, (s1, s2) in (("srf", (0.0, 2e-4)), ("nf", (-2e-4, 0.0))):
        a = inputs.analytic_channel(kind)
        assert (a["nx"], a["ny"], a["b"], a["sigma_T"], a["sigma_TT"]) == (512, 256, 128.0, s1, s2)


def test_perturbed_fields_recipe():
    c = inputs.small_channel()
    phi, ux, uy, T = inputs.perturbed_fields(c, 3)
    assert phi.shape == T.shape == (64, 128)
    assert np.all((phi > 0) & (phi < 1)) and not ux.any() and not uy.any()
    # interface height from the phi column sums: b plus a displacement of at
    # most 4 * 1.5 cells
    h = phi.sum(axis=0)
    assert np.all(np.abs(h - c["b"]) <= 6.0 + 1e-6)
    # temperature: the linear conduction profile plus noise of at most 1e-2
    y = np.arange(64)[:, None] + 0.5
    x = np.arange(128)[None, :]
    Tb = c["T_h"] + c["dT"] * np.cos(2 * np.pi * x / 128)
    lin = Tb + (c["T_c"] - Tb) * y / 64
    assert 0 < np.max(np.abs(T - lin)) <= 1e-2
    assert np.array_equal(inputs.perturbed_fields(c, 3)[3], T)
