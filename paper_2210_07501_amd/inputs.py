"""Seeded synthetic workloads shared by the tests, the benchmark and the
oracle checks.  This module only builds parameter dictionaries and initial
fields from seeds; it contains none of the lattice Boltzmann arithmetic.

Parameter dictionary keys (lattice units, rho c_p = 1):
  nx, ny        lattice size; x periodic, walls half-way outside rows 0, ny-1
  n_waves       heating wavelengths along x (l = nx / n_waves)
  b             thickness of the bottom fluid b (phi = 1); interface plane y = b - 1/2
  W, M_phi      interface width and Allen-Cahn mobility
  rho_a, rho_b, mu_a, mu_b, k_a, k_b   top (a) and bottom (b) properties
  sigma0, sigma_T, sigma_TT, T_ref     surface-tension law sigma(T)
  T_h, dT, T_c  bottom wall T_h + dT cos(2 pi x / l), top wall T_c
  Fx_ext, Fy_ext external body force (zero in every channel workload)

The paper's channel studies (Secs. 5.2, 6) use no dataset; every workload
here is synthetic and deterministic.
"""
from __future__ import annotations

import numpy as np

# Defaults for every channel: bottom fluid is the reference (nu_b = alpha_b = 0.1).
BASE = dict(
    n_waves=1, W=4.0, M_phi=0.02,
    rho_a=1.0, rho_b=1.0, mu_a=0.1, mu_b=0.1, k_a=0.1, k_b=0.1,
    sigma0=5e-3, sigma_T=0.0, sigma_TT=0.0, T_ref=1.0,
    T_h=1.0, dT=1.0, T_c=1.0, Fx_ext=0.0, Fy_ext=0.0,
)


def cfg(**kw) -> dict:
    d = dict(BASE)
    d.update(kw)
    return d


def small_channel() -> dict:
    """128 x 64 channel, one heating wavelength, two 32-cell layers,
    self-rewetting law s1 = 0, s2 = 1e-4 (2000-step parity workload)."""
    return cfg(nx=128, ny=64, b=32.0, sigma_TT=1e-4)


def analytic_channel(kind: str = "srf") -> dict:
    """512 x 256 channel, one wavelength, 128-cell layers; SRF: s1 = 0,
    s2 = 2e-4, NF: s1 = -2e-4, s2 = 0."""
    if kind == "srf":
        return cfg(nx=512, ny=256, b=128.0, sigma_T=0.0, sigma_TT=2e-4)
    if kind == "nf":
        return cfg(nx=512, ny=256, b=128.0, sigma_T=-2e-4, sigma_TT=0.0)
    raise ValueError(kind)


def throughput_channel(scale: int = 1) -> dict:
    """4096 x 2048 channel, 8 heating wavelengths, bottom layer 0.3 of the
    height, viscosity ratio 0.5, conductivity ratio 2, s1 = -5e-5, s2 = 2e-4.
    scale = 16 gives the 256 x 128 sub-run with the same geometry ratios."""
    nx, ny = 4096 // scale, 2048 // scale
    return cfg(nx=nx, ny=ny, n_waves=8, b=float(round(0.3 * ny)),
               mu_a=0.05, k_a=0.2, sigma_T=-5e-5, sigma_TT=2e-4)


def batched_sweep(n: int = 256, seed: int = 2210, nx_choices=(128, 256, 512)) -> list:
    """Independent channels with seed-drawn sizes and parameters:
    nx ~ U{128, 256, 512}, ny = nx / 2, one wavelength; s1 ~ U[-2e-4, 2e-4],
    s2 ~ U[0, 3e-4], lower-layer fraction ~ U[0.25, 0.75], viscosity and
    conductivity ratios log-uniform in [0.2, 5] (top fluid relative to the
    bottom reference fluid)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx = int(rng.choice(np.asarray(nx_choices)))
        s1 = float(rng.uniform(-2e-4, 2e-4))
        s2 = float(rng.uniform(0.0, 3e-4))
        frac = float(rng.uniform(0.25, 0.75))
        mr = float(np.exp(rng.uniform(np.log(0.2), np.log(5.0))))
        kr = float(np.exp(rng.uniform(np.log(0.2), np.log(5.0))))
        ny = nx // 2
        out.append(cfg(nx=nx, ny=ny, b=float(round(frac * ny)), sigma_T=s1, sigma_TT=s2,
                       mu_a=0.1 * mr, k_a=0.1 * kr))
    return out


def warmstart_set(n: int, seed0: int) -> list:
    """Warm-start workloads: the batched-sweep distribution with nx = 256,
    one channel per seed seed0 + i."""
    out = []
    for i in range(n):
        out.append(batched_sweep(1, seed=seed0 + i, nx_choices=(256,))[0])
    return out


def perturbed_fields(c: dict, seed: int, amp: float = 1.5, noise: float = 1e-2):
    """Seeded initial fields (phi, ux, uy, T), each [ny][nx] float64, that
    break the symmetries of the flat channel: the interface plane is displaced
    by sum_{m=1..4} A_m cos(2 pi m x / l + ph_m), A_m ~ U[0, amp], and the
    interior temperature carries noise * U[-1, 1] on top of the linear
    conduction profile.  The interface shape is a tanh of width W."""
    rng = np.random.default_rng(seed)
    nx, ny = int(c["nx"]), int(c["ny"])
    l = nx / int(c["n_waves"])
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    disp = np.zeros(nx)
    for m in range(1, 5):
        A = rng.uniform(0.0, amp)
        ph = rng.uniform(0.0, 2 * np.pi)
        disp += A * np.cos(2 * np.pi * m * x / l + ph)
    yint = float(c["b"]) - 0.5 + disp
    phi = 0.5 * (1.0 + np.tanh(2.0 * (yint[None, :] - y[:, None]) / float(c["W"])))
    Tb = float(c["T_h"]) + float(c["dT"]) * np.cos(2 * np.pi * x / l)
    T = Tb[None, :] + (float(c["T_c"]) - Tb[None, :]) * (y[:, None] + 0.5) / ny
    T = T + noise * rng.uniform(-1.0, 1.0, size=(ny, nx))
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    return phi, ux, uy, T


def perturbed_params(c: dict, seed: int) -> dict:
    """Viscosity and conductivity ratios drawn log-uniform in [0.2, 5]."""
    rng = np.random.default_rng(10_000 + seed)
    d = dict(c)
    d["mu_a"] = float(c["mu_b"]) * float(np.exp(rng.uniform(np.log(0.2), np.log(5.0))))
    d["k_a"] = float(c["k_b"]) * float(np.exp(rng.uniform(np.log(0.2), np.log(5.0))))
    return d


def droplet(R: float = 20.0, W: float = 4.0, M_phi: float = 0.02, scale: float = 1.0):
    """Thermocapillary migration of a droplet (Sec. 5.1): domain 8R x 16R,
    periodic in x, walls at the bottom (T = 0) and top (T = 32 R / 20, a
    uniform gradient of 0.1), droplet of radius R (fluid b, phi = 1) at the
    centre, mu = k = 0.2 in both fluids, sigma0 = 2.5e-3, sigma_T = -1e-4,
    T_ref at mid-height.  Returns (config, fields) with fields = (phi, ux,
    uy, T) for lbm_init: fluid at rest, tanh droplet of width W, linear T."""
    R = R * scale
    nx, ny = int(round(8 * R)), int(round(16 * R))
    G = 0.1
    T_bot, T_top = 0.0, G * ny
    c = cfg(nx=nx, ny=ny, b=ny / 2.0, W=W, M_phi=M_phi, mu_a=0.2, mu_b=0.2, k_a=0.2, k_b=0.2,
            sigma0=2.5e-3, sigma_T=-1e-4, sigma_TT=0.0, T_ref=0.5 * (T_bot + T_top),
            T_h=T_bot, dT=0.0, T_c=T_top)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    xc, yc = nx / 2.0 - 0.5, ny / 2.0 - 0.5
    r = np.sqrt((x[None, :] - xc) ** 2 + (y[:, None] - yc) ** 2)
    phi = 0.5 * (1.0 + np.tanh(2.0 * (R - r) / W))
    T = np.broadcast_to(T_bot + G * (y[:, None] + 0.5), (ny, nx)).copy()
    z = np.zeros((ny, nx))
    return c, (phi, z, z.copy(), T)

