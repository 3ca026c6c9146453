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


def _central(v, ex, ey, ux, uy, m, n):
    # central moment by its definition, sum_a v_a (e_ax - u_x)^m (e_ay - u_y)^n
    return float(np.sum(v * (ex - ux) ** m * (ey - uy) ** n))


@pytest.mark.parametrize("rho,om", [(1.0, 1.37), (1.8, 0.62)])
def test_hydro_collision_all_central_moments_with_forces(rho, om):
    # Sec. 4.2, Eq. (centralmomentrelaxationtwofluidmotion) with the source
    # moments sigma_mn printed there, at a node carrying a surface-tension force
    # F_t and a pressure force F_p: every post-collision central moment of the
    # oracle's output (computed here by brute force from its definition) equals
    #   eta_mn + omega_mn (eta_mn^eq - eta_mn) + (1 - omega_mn / 2) sigma_mn,
    # with omega_2d = omega_11 = omega_nu and every other rate 1, the diagonal
    # pair evolved as trace 2s and deviator 2d.  This separates the (1 - omega/2)
    # factor of the shear modes (dropping it moves eta_2d by omega sigma_2d / 2).
    _, _, w, ex, ey = orc.tables()
    rng = np.random.default_rng(17)
    g = w / 3 + rng.uniform(-2e-3, 2e-3, 9)
    cs2 = 1 / 3
    Ftx, Fty, Fpx, Fpy = 3e-3, -2e-3, 4e-3, 2.5e-3
    ux = (np.sum(g * ex) + 0.5 * cs2 * Ftx) / (rho * cs2)
    uy = (np.sum(g * ey) + 0.5 * cs2 * Fty) / (rho * cs2)
    Gam = Fpx * ux + Fpy * uy
    p = g.sum() + 0.5 * Gam
    vphi = p - rho * cs2
    out = orc.collide_g_node(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, om)
    c_in = {(m, n): _central(g, ex, ey, ux, uy, m, n) for m in range(3) for n in range(3)}
    c_out = {(m, n): _central(out, ex, ey, ux, uy, m, n) for m in range(3) for n in range(3)}
    eq = {(0, 0): p, (1, 0): -vphi * ux, (0, 1): -vphi * uy,
          (2, 0): p * cs2 + vphi * ux * ux, (0, 2): p * cs2 + vphi * uy * uy, (1, 1): vphi * ux * uy,
          (2, 1): -vphi * (ux * ux + cs2) * uy, (1, 2): -vphi * (uy * uy + cs2) * ux,
          (2, 2): cs2 ** 3 * rho + vphi * (ux * ux + cs2) * (uy * uy + cs2)}
    src = {(0, 0): Gam, (1, 0): cs2 * Ftx - ux * Gam, (0, 1): cs2 * Fty - uy * Gam,
           (2, 0): 2 * cs2 * Fpx * ux + (ux * ux + cs2) * Gam, (0, 2): 2 * cs2 * Fpy * uy + (uy * uy + cs2) * Gam,
           (1, 1): cs2 * (Fpx * uy + Fpy * ux) + ux * uy * Gam, (2, 1): 0.0, (1, 2): 0.0, (2, 2): 0.0}

    def relax(x, x_eq, s, rate):
        return x + rate * (x_eq - x) + (1 - rate / 2) * s

    want = {k: relax(c_in[k], eq[k], src[k], 1.0) for k in [(0, 0), (1, 0), (0, 1), (2, 1), (1, 2), (2, 2)]}
    want[(1, 1)] = relax(c_in[(1, 1)], eq[(1, 1)], src[(1, 1)], om)
    two_s = relax(c_in[(2, 0)] + c_in[(0, 2)], eq[(2, 0)] + eq[(0, 2)], src[(2, 0)] + src[(0, 2)], 1.0)
    two_d = relax(c_in[(2, 0)] - c_in[(0, 2)], eq[(2, 0)] - eq[(0, 2)], src[(2, 0)] - src[(0, 2)], om)
    want[(2, 0)] = 0.5 * (two_s + two_d)
    want[(0, 2)] = 0.5 * (two_s - two_d)
    scale = max(abs(v) for v in c_out.values())
    for k in want:
        assert abs(c_out[k] - want[k]) <= 1e-13 * scale, (k, c_out[k], want[k])
    # the shear-mode sources are large enough here to show the factor: dropping
    # it would move eta_2d and eta_11 by far more than the tolerance
    assert abs(om / 2 * (src[(2, 0)] - src[(0, 2)])) > 1e4 * 1e-13 * scale
    assert abs(om / 2 * src[(1, 1)]) > 1e4 * 1e-13 * scale


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.04, -0.03)])
def test_ace_collision_all_central_moments(u):
    # Sec. 4.1: post-collision central moments of the conservative Allen-Cahn
    # collision -- the first relax at omega_phi to M theta n, every other one
    # equals its equilibrium (phi, -, -, phi c_s^2, phi c_s^2, 0, 0, 0, phi c_s^4)
    # -- checked by brute force on the oracle's output at a moving node.
    _, _, w, ex, ey = orc.tables()
    ux, uy = u
    rng = np.random.default_rng(18)
    f = w * 0.6 + rng.uniform(-1e-3, 1e-3, 9)
    phi = f.sum()
    cs2 = 1 / 3
    M, theta, om, nx, ny = 0.02, 0.25, 1.2, 0.6, -0.8
    out = orc.collide_f_node(f, phi, ux, uy, nx, ny, theta, M, om)
    k10, k01 = _central(f, ex, ey, ux, uy, 1, 0), _central(f, ex, ey, ux, uy, 0, 1)
    want = {(0, 0): phi, (1, 0): k10 + om * (M * theta * nx - k10), (0, 1): k01 + om * (M * theta * ny - k01),
            (2, 0): phi * cs2, (0, 2): phi * cs2, (1, 1): 0.0, (2, 1): 0.0, (1, 2): 0.0, (2, 2): phi * cs2 * cs2}
    for k, v in want.items():
        assert abs(_central(out, ex, ey, ux, uy, *k) - v) < 1e-15, k


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.05, 0.02)])
def test_energy_collision_all_central_moments(u):
    # Sec. 4.3: the first central moments of h relax at omega_T to zero, the
    # others take the equilibrium (T, 0, 0, T c_s^2, T c_s^2, 0, 0, 0, T c_s^4).
    _, _, w, ex, ey = orc.tables()
    ux, uy = u
    rng = np.random.default_rng(19)
    h = w * 1.1 + rng.uniform(-2e-3, 2e-3, 9)
    T = h.sum()
    cs2 = 1 / 3
    om = 1.3
    out = orc.collide_h_node(h, T, ux, uy, om)
    c10, c01 = _central(h, ex, ey, ux, uy, 1, 0), _central(h, ex, ey, ux, uy, 0, 1)
    want = {(0, 0): T, (1, 0): (1 - om) * c10, (0, 1): (1 - om) * c01, (2, 0): T * cs2, (0, 2): T * cs2,
            (1, 1): 0.0, (2, 1): 0.0, (1, 2): 0.0, (2, 2): T * cs2 * cs2}
    for k, v in want.items():
        assert abs(_central(out, ex, ey, ux, uy, *k) - v) < 1e-15, k
