"""Closed-form Stokes-flow solution of the paper (Sec. 2, App. A, App. C) in
float64 -- TEST INFRASTRUCTURE ONLY (tests, smoke check and benchmark
baseline may import it; the product path never does).

Coordinates are the paper's: origin on the interface, fluid a on top
(0 <= y <= a), fluid b below (-b <= y <= 0), heating wavelength l,
omega = 2 pi / l, hot spot at x = 0.

Velocity convention: the paper's stream-function definition (Sec. 2) is
garbled; the printed velocity components u^gamma, v^gamma are used as they
stand.  They equal u = d psi / dy, v = -d psi / dx of
psi = U_t [C2 y cosh wy + (C3 + C4 y) sinh wy] sin wx
    + U_tt/2 [D2 y cosh 2wy + (D3 + D4 y) sinh 2wy] sin 2wx,
which is divergence-free; the tests check that and the boundary conditions.

Two results here are not printed in the paper but follow from its solution:
the Stokes pressure of each layer, and the interface shape to first order in
the capillary number (the paper keeps the interface flat).  Both are pinned
by the tests against the momentum and normal-stress balances they solve.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np


@dataclass
class Channel:
    """Geometry, properties and surface-tension law of the two-layer channel."""
    a: float                 # top (fluid a) thickness
    b: float                 # bottom (fluid b) thickness
    l: float                 # heating wavelength
    mu_b: float              # dynamic viscosity of the bottom fluid
    mu_ratio: float = 1.0    # mu_a / mu_b  (Eq. three)
    k_ratio: float = 1.0     # k_a / k_b
    sigma_T: float = 0.0     # Eq. (ST_SRF) linear coefficient
    sigma_TT: float = 0.0    # Eq. (ST_SRF) quadratic coefficient
    T_ref: float = 1.0
    T_h: float = 1.0
    T_c: float = 1.0
    dT: float = 1.0

    @property
    def omega(self) -> float:
        return 2.0 * np.pi / self.l

    @property
    def at(self) -> float:   # a tilde
        return self.a * self.omega

    @property
    def bt(self) -> float:   # b tilde
        return self.b * self.omega


def f_fun(at, bt, kt):
    """App. A, Eq. (f)."""
    return 1.0 / (kt * np.sinh(bt) * np.cosh(at) + np.sinh(at) * np.cosh(bt))


def g_fun(at, bt, kt):
    """Sec. 2: g = sinh(a~) f(a~, b~, k~)."""
    return np.sinh(at) * f_fun(at, bt, kt)


def h_fun(at, bt, mt):
    """Sec. 2: h(a~, b~, mu~) in the expression for U_t."""
    Da = np.sinh(at) ** 2 - at ** 2
    Db = np.sinh(bt) ** 2 - bt ** 2
    return Da * Db / (mt * Db * (np.sinh(2 * at) - 2 * at) + Da * (np.sinh(2 * bt) - 2 * bt))


def h1_fun(at, bt, mt):
    """Sec. 2: h~_1(a~, b~, mu~) = h(2a~, 2b~, mu~), written out as printed."""
    Da = np.sinh(2 * at) ** 2 - 4 * at ** 2
    Db = np.sinh(2 * bt) ** 2 - 4 * bt ** 2
    return Da * Db / (mt * Db * (np.sinh(4 * at) - 4 * at) + Da * (np.sinh(4 * bt) - 4 * bt))


def interface_mean_T(c: Channel) -> float:
    """Linear part of the temperature on the interface (Eq. Ta at y = 0)."""
    return (c.T_c * c.k_ratio * c.b + c.T_h * c.a) / (c.a + c.b * c.k_ratio)


def U_t(c: Channel) -> float:
    """Sec. 2, Eq. (Umaxexpression)."""
    g = g_fun(c.at, c.bt, c.k_ratio)
    h = h_fun(c.at, c.bt, c.mu_ratio)
    return -(c.dT / c.mu_b) * g * h * (c.sigma_T + 2 * c.sigma_TT * (interface_mean_T(c) - c.T_ref))


def U_tt(c: Channel) -> float:
    """Sec. 2: U_tt = -(sigma_TT dT^2 / mu_b) g^2 h~_1."""
    g = g_fun(c.at, c.bt, c.k_ratio)
    return -(c.sigma_TT * c.dT ** 2 / c.mu_b) * g ** 2 * h1_fun(c.at, c.bt, c.mu_ratio)


def constants(c: Channel):
    """Sec. 2: C_j^gamma and D_j^gamma (j = 1..4) as printed."""
    a, b, at, bt = c.a, c.b, c.at, c.bt
    Db1 = np.sinh(bt) ** 2 - bt ** 2
    Da1 = np.sinh(at) ** 2 - at ** 2
    Db2 = np.sinh(2 * bt) ** 2 - 4 * bt ** 2
    Da2 = np.sinh(2 * at) ** 2 - 4 * at ** 2
    C = {
        "b": (0.0, np.sinh(bt) ** 2 / Db1, -b * bt / Db1, (np.sinh(2 * bt) - 2 * bt) / (2 * Db1)),
        "a": (0.0, np.sinh(at) ** 2 / Da1, -a * at / Da1, -(np.sinh(2 * at) - 2 * at) / (2 * Da1)),
    }
    D = {
        "b": (0.0, np.sinh(2 * bt) ** 2 / Db2, -2 * b * bt / Db2, (np.sinh(4 * bt) - 4 * bt) / (2 * Db2)),
        "a": (0.0, np.sinh(2 * at) ** 2 / Da2, -2 * a * at / Da2, -(np.sinh(4 * at) - 4 * at) / (2 * Da2)),
    }
    return C, D


def temperature(c: Channel, x, y):
    """Eqs. (Ta), (Tb): two-layer conduction field (k jump at y = 0)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w, kt, f = c.omega, c.k_ratio, f_fun(c.at, c.bt, c.k_ratio)
    den = c.a + c.b * kt
    Ta = ((c.T_c - c.T_h) * y + c.T_c * kt * c.b + c.T_h * c.a) / den \
        + c.dT * f * np.sinh(c.at - w * y) * np.cos(w * x)
    Tb = (kt * (c.T_c - c.T_h) * y + c.T_c * kt * c.b + c.T_h * c.a) / den \
        + c.dT * f * (np.sinh(c.at) * np.cosh(w * y) - kt * np.sinh(w * y) * np.cosh(c.at)) * np.cos(w * x)
    return np.where(y >= 0, Ta, Tb)


def velocity(c: Channel, x, y):
    """Sec. 2: u^gamma(x, y), v^gamma(x, y) for gamma = a (y >= 0), b (y < 0)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = c.omega
    Ut, Utt = U_t(c), U_tt(c)
    C, D = constants(c)
    out_u, out_v = [], []
    for key in ("a", "b"):
        _, C2, C3, C4 = C[key]
        _, D2, D3, D4 = D[key]
        u = Ut * ((C2 + w * (C3 + C4 * y)) * np.cosh(w * y) + (C4 + w * C2 * y) * np.sinh(w * y)) * np.sin(w * x) \
            + 0.5 * Utt * ((D2 + 2 * w * (D3 + D4 * y)) * np.cosh(2 * w * y)
                           + (D4 + 2 * w * D2 * y) * np.sinh(2 * w * y)) * np.sin(2 * w * x)
        v = -w * Ut * (C2 * y * np.cosh(w * y) + (C3 + C4 * y) * np.sinh(w * y)) * np.cos(w * x) \
            - w * Utt * (D2 * y * np.cosh(2 * w * y) + (D3 + D4 * y) * np.sinh(2 * w * y)) * np.cos(2 * w * x)
        out_u.append(u)
        out_v.append(v)
    upper = y >= 0
    return np.where(upper, out_u[0], out_u[1]), np.where(upper, out_v[0], out_v[1])


def interface_velocity(c: Channel, x):
    """Sec. 2 boundary condition iii: u(x, 0) = U_t sin wx + U_tt/2 sin 2wx."""
    x = np.asarray(x, dtype=np.float64)
    return U_t(c) * np.sin(c.omega * x) + 0.5 * U_tt(c) * np.sin(2 * c.omega * x)


def pressure(c: Channel, x, y):
    """Stokes pressure of the Sec. 2 flow, grad p = mu_gamma lap u in each
    layer.  For a stream-function term A F(y) sin kx with
    F = C2 y cosh ky + (C3 + C4 y) sinh ky, lap psi = 2 k A (C2 sinh ky +
    C4 cosh ky) sin kx, so p = -2 mu k A (C2 cosh ky + C4 sinh ky) cos kx
    (first harmonic: k = w, A = U_t; second: k = 2w, A = U_tt / 2).  Each
    layer's pressure is defined up to its own constant, taken as 0 here."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = c.omega
    Ut, Utt = U_t(c), U_tt(c)
    C, D = constants(c)
    out = []
    for key, mu in (("a", c.mu_b * c.mu_ratio), ("b", c.mu_b)):
        _, C2, _, C4 = C[key]
        _, D2, _, D4 = D[key]
        out.append(-2 * mu * w * Ut * (C2 * np.cosh(w * y) + C4 * np.sinh(w * y)) * np.cos(w * x)
                   - 2 * mu * w * Utt * (D2 * np.cosh(2 * w * y) + D4 * np.sinh(2 * w * y)) * np.cos(2 * w * x))
    return np.where(y >= 0, out[0], out[1])


def surface_tension(c: Channel, sigma0: float, T):
    """Eq. (ST_SRF): sigma(T) = sigma0 + sigma_T (T - T_ref) + sigma_TT (T - T_ref)^2."""
    d = np.asarray(T, dtype=np.float64) - c.T_ref
    return sigma0 + c.sigma_T * d + c.sigma_TT * d * d


def small_deformation(c: Channel, sigma0: float, n: int = 4096):
    """Interface height h(x) to first order in the capillary number (not in
    the paper, which treats the interface as flat; it follows from the flat
    solution's normal stresses).  With fluid b below and n = +y, the normal
    stress balance on y = h(x) reads, to first order,
        sigma(T(x, 0)) (-h'') = (p_b - p_a)(x, 0) - 2 (mu_b - mu_a) dv/dy(x, 0) + c0,
    where dv/dy(x, 0) = -du/dx of the interface velocity (the same on both
    sides), c0 is the undetermined difference of the layers' pressure levels,
    fixed by h' being periodic (h'' of zero mean), and h has zero mean (each
    layer keeps its volume).  Returns (x, h) on n points of one wavelength."""
    x = np.arange(n) * (c.l / n)
    w = c.omega
    zero = np.zeros_like(x)
    jump = pressure(c, x, zero - 1e-300) - pressure(c, x, zero)
    dvdy = -(w * U_t(c) * np.cos(w * x) + w * U_tt(c) * np.cos(2 * w * x))
    J = jump - 2 * c.mu_b * (1 - c.mu_ratio) * dvdy
    sig = surface_tension(c, sigma0, temperature(c, x, zero))
    c0 = -np.mean(J / sig) / np.mean(1 / sig)
    hpp = -(J + c0) / sig
    k = 2 * np.pi * np.fft.rfftfreq(n, d=c.l / n)
    H = np.fft.rfft(hpp)
    H[1:] = -H[1:] / k[1:] ** 2
    H[0] = 0.0
    return x, np.fft.irfft(H, n)


def U_s(c: Channel) -> float:
    """App. C, Eq. (U_s): characteristic thermocapillary velocity."""
    C1 = (c.T_h * (c.a / c.b) + c.T_c * c.k_ratio) / ((c.a / c.b) + c.k_ratio)
    C2 = c.dT * np.sinh(c.at) / (c.k_ratio * np.cosh(c.at) * np.sinh(c.bt) + np.cosh(c.bt) * np.sinh(c.at))
    return (c.dT / c.mu_b) * (c.b / c.l) * (c.sigma_T + 2 * c.sigma_TT * (C1 + C2 - c.T_ref))


def capillary_number(c: Channel, sigma0: float) -> float:
    """Eq. (ReMaCa): Ca = U mu_b / sigma_0 with U = |U_s|."""
    return abs(U_s(c)) * c.mu_b / sigma0


def ygb_velocity(sigma_T: float, gradT: float, R: float, mu_b: float,
                 k_ratio: float, mu_ratio: float) -> float:
    """Sec. 5.1: U* = -sigma_T |grad T| R / mu_b, U_YGB = 2 U* / ((2 + k~)(2 + 3 mu~))."""
    Ustar = -sigma_T * abs(gradT) * R / mu_b
    return 2 * Ustar / ((2 + k_ratio) * (2 + 3 * mu_ratio))


def channel_from_config(cfg: dict) -> Channel:
    """Map a lattice configuration (walls half-way outside rows 0 and ny-1,
    interface plane at y = b - 1/2) to the analytic channel."""
    nx, ny, b = int(cfg["nx"]), int(cfg["ny"]), float(cfg["b"])
    rho_b = float(cfg.get("rho_b", 1.0))
    return Channel(a=ny - b, b=b, l=nx / int(cfg["n_waves"]), mu_b=float(cfg["mu_b"]),
                   mu_ratio=float(cfg["mu_a"]) / float(cfg["mu_b"]),
                   k_ratio=float(cfg["k_a"]) / float(cfg["k_b"]),
                   sigma_T=float(cfg["sigma_T"]), sigma_TT=float(cfg["sigma_TT"]),
                   T_ref=float(cfg["T_ref"]), T_h=float(cfg["T_h"]), T_c=float(cfg["T_c"]),
                   dT=float(cfg["dT"]))


def lattice_coords(cfg: dict):
    """Paper coordinates (x, y) of lattice node centres, arrays [ny][nx]."""
    nx, ny, b = int(cfg["nx"]), int(cfg["ny"]), float(cfg["b"])
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    X, Y = np.meshgrid(i, j - (b - 0.5))
    return X, Y


def count_rolls(uy: np.ndarray, cfg: dict) -> int:
    """Number of convection rolls: sign changes (periodic in x) of the
    vertical velocity along the mid-line of each layer, summed over the two
    layers.  Values below 1e-3 of the row's peak are ignored."""
    ny = uy.shape[0]
    b = float(cfg["b"])
    rows = [int(round(b / 2.0 - 0.5)), int(round(b + (ny - b) / 2.0 - 0.5))]
    total = 0
    for r in rows:
        v = uy[r]
        thr = 1e-3 * np.max(np.abs(v))
        s = np.sign(np.where(np.abs(v) > thr, v, 0.0))
        s = s[s != 0]
        if s.size == 0:
            continue
        total += int(np.sum(s != np.roll(s, 1)))
    return total


def interface_profile(ux: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """u_x(x) on the phi = 1/2 level, linearly interpolated between the two
    rows whose phi brackets 1/2 (one crossing per column is assumed)."""
    ny, nx = phi.shape
    out = np.zeros(nx)
    for i in range(nx):
        col = phi[:, i] - 0.5
        k = np.nonzero((col[:-1] >= 0) & (col[1:] < 0))[0]
        if k.size == 0:
            out[i] = np.nan
            continue
        j = int(k[0])
        t = col[j] / (col[j] - col[j + 1])
        out[i] = (1 - t) * ux[j, i] + t * ux[j + 1, i]
    return out


def interface_height(phi: np.ndarray) -> np.ndarray:
    """Row coordinate of the phi = 1/2 level in each column, linearly
    interpolated between the two rows that bracket it (first crossing from
    the bottom; NaN where there is none)."""
    ny, nx = phi.shape
    out = np.full(nx, np.nan)
    for i in range(nx):
        col = phi[:, i] - 0.5
        k = np.nonzero((col[:-1] >= 0) & (col[1:] < 0))[0]
        if k.size:
            j = int(k[0])
            out[i] = j + col[j] / (col[j] - col[j + 1])
    return out


def diffuse_interface_velocity(cfg: dict, x=None):
    """Interface velocity u_x(x, y = 0) of the Sec. 2 solution with the
    Marangoni stress spread over the diffuse interface as the lattice spreads
    it: node row y_s of the cold-start tanh profile carries the fraction
    delta_s = 1.5 W |grad phi|^2 (isotropic y-derivative of the sampled tanh)
    of the stress, and its response at y = 0 is the sharp solution for an
    interface at y_s (layers b + y_s and a - y_s).  Exact superposition for
    equal viscosities and conductivities (the temperature field is then the
    same harmonic field for every y_s); an estimate otherwise."""
    ch = channel_from_config(cfg)
    W = float(cfg["W"])
    ny, b = int(cfg["ny"]), float(cfg["b"])
    j = np.arange(-2, ny + 2)
    y = j - (b - 0.5)
    phi = 0.5 * (1 + np.tanh(2 * (-y) / W))
    g = np.zeros_like(phi)
    g[1:-1] = (phi[2:] - phi[:-2]) / 2
    ds = 1.5 * W * g ** 2
    if x is None:
        x = np.arange(int(cfg["nx"]), dtype=float)
    x = np.asarray(x, dtype=float)
    tot = np.zeros_like(x)
    for k in range(2, len(j) - 2):
        if ds[k] < 1e-14:
            continue
        cs = dataclasses.replace(ch, a=ch.a - y[k], b=ch.b + y[k])
        u, _ = velocity(cs, x, np.full_like(x, -y[k]))
        tot += ds[k] * u
    return tot
