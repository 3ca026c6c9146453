"""Pins of the oracle's moment maps (App. B) against the mathematics that
defines them, independent of the oracle's own formulas."""
import itertools

import numpy as np
import pytest

from oracle import oracle as orc

# Moment order of the paper, Sec. 4.1: (00, 10, 01, 20, 02, 11, 21, 12, 22).
ORDER = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]


def velocity_set():
    # The standard D2Q9 lattice: rest, 4 axis links, 4 diagonals (Sec. 4.1).
    return (np.array([0, 1, 0, -1, 0, 1, -1, -1, 1]),
            np.array([0, 0, 1, 0, -1, 1, 1, -1, -1]))


def test_velocity_set_is_d2q9():
    _, _, _, ex, ey = orc.tables()
    pairs = {(int(a), int(b)) for a, b in zip(ex, ey)}
    assert pairs == set(itertools.product((-1, 0, 1), repeat=2))
    ex0, ey0 = velocity_set()
    assert np.array_equal(ex, ex0) and np.array_equal(ey, ey0)


def test_P_rows_are_raw_moment_monomials():
    # App. B, Eq. (tensorP): row (m, n) of P is e_x^m e_y^n.
    P, _, _, ex, ey = orc.tables()
    for r, (m, n) in enumerate(ORDER):
        assert np.array_equal(P[r], (ex.astype(float) ** m) * (ey.astype(float) ** n))


def test_Pinv_is_inverse_of_P():
    P, Pi, _, _, _ = orc.tables()
    assert np.max(np.abs(Pi @ P - np.eye(9))) == 0.0
    assert np.max(np.abs(P @ Pi - np.eye(9))) == 0.0


def test_weights_from_rest_moments():
    # The textbook D2Q9 weights are P^-1 applied to the raw moments of the
    # rest Maxwellian, (1, 0, 0, 1/3, 1/3, 0, 0, 0, 1/9).
    _, Pi, w, _, _ = orc.tables()
    rest = np.array([1, 0, 0, 1 / 3, 1 / 3, 0, 0, 0, 1 / 9])
    assert np.allclose(Pi @ rest, w, rtol=0, atol=1e-15)
    assert np.allclose(w, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, rtol=0, atol=1e-17)


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.3, -0.2), (-0.11, 0.07), (1e-3, 2e-3)])
def test_F_gives_central_moments_by_brute_force(u):
    # Sec. 4.1: kappa_mn = sum_a f_a (e_ax - u_x)^m (e_ay - u_y)^n, computed
    # here directly from the definition and compared with F(u) P f.
    ux, uy = u
    P, _, _, ex, ey = orc.tables()
    rng = np.random.default_rng(1)
    f = rng.uniform(0.0, 1.0, 9)
    direct = np.array([np.sum(f * (ex - ux) ** m * (ey - uy) ** n) for (m, n) in ORDER])
    via = orc.build_F(ux, uy) @ (P @ f)
    assert np.max(np.abs(direct - via)) < 1e-15


@pytest.mark.parametrize("u", [(0.3, -0.2), (-0.05, 0.4)])
def test_F_inverse_is_F_of_minus_u(u):
    # App. B: F^-1 = F(-u).
    ux, uy = u
    assert np.max(np.abs(orc.build_F(-ux, -uy) @ orc.build_F(ux, uy) - np.eye(9))) < 1e-15


def test_printed_F_row_22_differs_from_binomial():
    # The printed row (22) of F (App. B) has -u_x u_y^2 and -u_x^2 u_y in the
    # columns of kappa'_10, kappa'_01; the binomial expansion (which Sec. 4.1
    # prescribes) gives twice that.  The oracle follows the expansion.
    ux, uy = 0.3, -0.2
    F = orc.build_F(ux, uy)
    assert F[8, 1] == pytest.approx(-2 * ux * uy * uy)
    assert F[8, 2] == pytest.approx(-2 * ux * ux * uy)
    printed = F.copy()
    printed[8, 1] = -ux * uy * uy
    printed[8, 2] = -ux * ux * uy
    assert np.max(np.abs(orc.build_F(-ux, -uy) @ printed - np.eye(9))) > 1e-3


def test_round_trip_without_relaxation():
    # P^-1 F(-u) F(u) P f = f on one node.
    P, Pi, _, _, _ = orc.tables()
    rng = np.random.default_rng(2)
    f = rng.uniform(0.0, 0.2, 9)
    ux, uy = 0.07, -0.03
    back = Pi @ (orc.build_F(-ux, -uy) @ (orc.build_F(ux, uy) @ (P @ f)))
    assert np.max(np.abs(back - f)) < 1e-16 * 10


def test_ace_collision_conserves_phi_and_fixes_rest_equilibrium():
    _, _, w, _, _ = orc.tables()
    rng = np.random.default_rng(3)
    f = rng.uniform(0.0, 0.2, 9)
    phi = f.sum()
    out = orc.collide_f_node(f, phi, 0.01, -0.02, 0.6, 0.8, 0.1, 0.02, 1.5)
    assert out.sum() == pytest.approx(phi, rel=1e-15)
    # rest equilibrium with no sharpening flux is a fixed point
    eq = w * 0.7
    out = orc.collide_f_node(eq, 0.7, 0.0, 0.0, 0.0, 0.0, 0.0, 0.02, 1.5)
    assert np.max(np.abs(out - eq)) < 1e-16


def test_ace_collision_first_moment():
    # Sec. 4.1: the post-collision first central moments relax at omega_phi
    # to M theta n; with u = 0 the raw first moment is that central moment.
    _, _, w, ex, ey = orc.tables()
    rng = np.random.default_rng(4)
    f = w * 0.5 + rng.uniform(-1e-3, 1e-3, 9)
    phi = f.sum()
    jx, jy = np.sum(f * ex), np.sum(f * ey)
    M, theta, om, nx, ny = 0.02, 0.25, 1.2, 0.6, -0.8
    out = orc.collide_f_node(f, phi, 0.0, 0.0, nx, ny, theta, M, om)
    assert np.sum(out * ex) == pytest.approx(jx + om * (M * theta * nx - jx), rel=1e-13)
    assert np.sum(out * ey) == pytest.approx(jy + om * (M * theta * ny - jy), rel=1e-13)


def test_energy_collision_conserves_T():
    rng = np.random.default_rng(5)
    h = rng.uniform(0.0, 0.3, 9)
    T = h.sum()
    out = orc.collide_h_node(h, T, 0.02, 0.01, 1.3)
    assert out.sum() == pytest.approx(T, rel=1e-15)


def test_hydro_collision_momentum_and_pressure_sources():
    # Sec. 4.2: with u from rho c_s^2 u = sum g e + c_s^2 F_t / 2 and
    # p = sum g + F_p.u / 2, one collision adds c_s^2 F_t to the momentum
    # moment and Gamma = F_p.u to the zeroth moment.
    _, _, w, ex, ey = orc.tables()
    rng = np.random.default_rng(6)
    g = w / 3 + rng.uniform(-1e-3, 1e-3, 9)
    rho = 1.3
    Ftx, Fty, Fpx, Fpy = 2e-4, -1e-4, 3e-4, 5e-5
    cs2 = 1 / 3
    ux = (np.sum(g * ex) + 0.5 * cs2 * Ftx) / (rho * cs2)
    uy = (np.sum(g * ey) + 0.5 * cs2 * Fty) / (rho * cs2)
    Gam = Fpx * ux + Fpy * uy
    p = g.sum() + 0.5 * Gam
    out = orc.collide_g_node(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, 1.4)
    assert np.sum(out * ex) - np.sum(g * ex) == pytest.approx(cs2 * Ftx, rel=1e-9)
    assert np.sum(out * ey) - np.sum(g * ey) == pytest.approx(cs2 * Fty, rel=1e-9)
    assert out.sum() - g.sum() == pytest.approx(Gam, rel=1e-9)


def test_hydro_collision_shear_relaxation():
    # Sec. 4.2: without forces, the deviatoric and off-diagonal second central
    # moments relax at omega_nu; the trace goes to its equilibrium 2 p c_s^2.
    _, _, w, ex, ey = orc.tables()
    rng = np.random.default_rng(7)
    g = w / 3 + rng.uniform(-1e-3, 1e-3, 9)
    rho, om = 1.0, 1.37
    cs2 = 1 / 3
    ux, uy = np.sum(g * ex) / (rho * cs2), np.sum(g * ey) / (rho * cs2)
    p = g.sum()
    vphi = p - rho * cs2

    def central(v, m, n):
        return np.sum(v * (ex - ux) ** m * (ey - uy) ** n)

    out = orc.collide_g_node(g, p, rho, ux, uy, 0.0, 0.0, 0.0, 0.0, om)
    d_in = central(g, 2, 0) - central(g, 0, 2)
    d_eq = vphi * (ux * ux - uy * uy)
    assert central(out, 2, 0) - central(out, 0, 2) == pytest.approx(d_in + om * (d_eq - d_in), rel=1e-9)
    o_in = central(g, 1, 1)
    assert central(out, 1, 1) == pytest.approx(o_in + om * (vphi * ux * uy - o_in), rel=1e-9)
    assert central(out, 2, 0) + central(out, 0, 2) == pytest.approx(
        2 * p * cs2 + vphi * (ux * ux + uy * uy), rel=1e-12)
