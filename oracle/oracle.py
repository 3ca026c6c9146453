"""Python side of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It builds ``liblbm_oracle.so`` from
``lbm_oracle.c`` with gcc (no HIP, no code shared with the product library)
and wraps it with ctypes.  Population arrays use the layout
``[dist (f, g, h)][alpha (0..8)][y][x]`` in float64.

The steady-state residual follows the reading stated for the solver: every K
steps, r = max(||u^n - u^{n-K}||_2 / ||u^n||_2,
               ||T^n - T^{n-K}||_2 / ||T^n - T_ref||_2) / K.
The paper itself defines no residual.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_lock = threading.Lock()
_lib = None


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("n_waves", ctypes.c_int),
        ("b", ctypes.c_double), ("W", ctypes.c_double), ("M_phi", ctypes.c_double),
        ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double),
        ("mu_a", ctypes.c_double), ("mu_b", ctypes.c_double),
        ("k_a", ctypes.c_double), ("k_b", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("sigma_T", ctypes.c_double),
        ("sigma_TT", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("T_h", ctypes.c_double), ("dT", ctypes.c_double), ("T_c", ctypes.c_double),
        ("Fx_ext", ctypes.c_double), ("Fy_ext", ctypes.c_double),
        ("p0", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (FP64, no fast-math, no FMA
    contraction, OpenMP over lattice rows)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                   "-shared", "-std=c99", "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OrcParams)
        L.orc_step.argtypes = [pp, dp, dp]
        L.orc_run.argtypes = [pp, dp, ctypes.c_long]
        L.orc_macros.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.orc_init_fields.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_init_cold.argtypes = [pp, dp]
        L.orc_cold_fields.argtypes = [pp, dp, dp, dp, dp]
        L.orc_build_F.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        L.orc_tables.argtypes = [dp, dp, dp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.orc_collide_f_node.argtypes = [dp] + [ctypes.c_double] * 8 + [dp]
        L.orc_collide_g_node.argtypes = [dp] + [ctypes.c_double] * 9 + [dp]
        L.orc_collide_h_node.argtypes = [dp] + [ctypes.c_double] * 4 + [dp]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(cfg: dict) -> OrcParams:
    """Fill the oracle's own parameter struct from a plain config dict."""
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        if name == "p0":
            p.p0 = float(cfg.get("p0", 1.0 / 3.0))
        else:
            setattr(p, name, type(getattr(p, name))(cfg[name]))
    return p


def tables():
    P = np.zeros(81); Pi = np.zeros(81); w = np.zeros(9)
    ex = (ctypes.c_int * 9)(); ey = (ctypes.c_int * 9)()
    lib().orc_tables(_dp(P), _dp(Pi), _dp(w), ex, ey)
    return P.reshape(9, 9), Pi.reshape(9, 9), w, np.array(ex[:]), np.array(ey[:])


def build_F(ux: float, uy: float) -> np.ndarray:
    F = np.zeros(81)
    lib().orc_build_F(ux, uy, _dp(F))
    return F.reshape(9, 9)


def collide_f_node(f, phi, ux, uy, nx, ny, theta, M, w_phi):
    f = np.ascontiguousarray(f, dtype=np.float64); out = np.zeros(9)
    lib().orc_collide_f_node(_dp(f), phi, ux, uy, nx, ny, theta, M, w_phi, _dp(out))
    return out


def collide_g_node(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, w_nu):
    g = np.ascontiguousarray(g, dtype=np.float64); out = np.zeros(9)
    lib().orc_collide_g_node(_dp(g), p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, w_nu, _dp(out))
    return out


def collide_h_node(h, T, ux, uy, w_T):
    h = np.ascontiguousarray(h, dtype=np.float64); out = np.zeros(9)
    lib().orc_collide_h_node(_dp(h), T, ux, uy, w_T, _dp(out))
    return out


class Oracle:
    """One channel on the CPU: populations in float64, stepped by the C code."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.p = make_params(cfg)
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self.pop = np.zeros((3, 9, self.ny, self.nx))
        self.steps = 0

    def init_cold(self):
        lib().orc_init_cold(ctypes.byref(self.p), _dp(self.pop))
        self.steps = 0

    def init_fields(self, phi, ux, uy, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx)
                for a in (phi, ux, uy, T)]
        lib().orc_init_fields(ctypes.byref(self.p), *[_dp(a) for a in arrs], _dp(self.pop))
        self.steps = 0

    def cold_fields(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(4)]
        lib().orc_cold_fields(ctypes.byref(self.p), *[_dp(a) for a in out])
        return out

    def set_state(self, pop):
        self.pop[...] = np.asarray(pop, dtype=np.float64).reshape(self.pop.shape)

    def step(self, n: int = 1):
        if n > 0:
            rc = lib().orc_run(ctypes.byref(self.p), _dp(self.pop), int(n))
            if rc != 0:
                raise MemoryError("oracle step failed")
            self.steps += n

    def fields(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(5)]
        lib().orc_macros(ctypes.byref(self.p), _dp(self.pop), *[_dp(a) for a in out])
        return dict(zip(("phi", "ux", "uy", "T", "p"), out))

    def run_to_steady(self, tol: float = 1e-8, K: int = 100, max_steps: int = 10**7):
        """Step until the residual (see module docstring) is <= tol."""
        prev = self.fields()
        r = np.inf
        while self.steps < max_steps:
            self.step(K)
            cur = self.fields()
            r = residual(prev, cur, K, self.cfg["T_ref"])
            prev = cur
            if r <= tol:
                break
        return r


def residual(prev: dict, cur: dict, K: int, T_ref: float) -> float:
    du = np.sqrt(np.sum((cur["ux"] - prev["ux"]) ** 2 + (cur["uy"] - prev["uy"]) ** 2))
    nu = np.sqrt(np.sum(cur["ux"] ** 2 + cur["uy"] ** 2))
    dT = np.sqrt(np.sum((cur["T"] - prev["T"]) ** 2))
    nT = np.sqrt(np.sum((cur["T"] - T_ref) ** 2))
    ru = du / nu if nu > 0 else (0.0 if du == 0 else np.inf)
    rT = dT / nT if nT > 0 else (0.0 if dT == 0 else np.inf)
    return max(ru, rT) / K


def max_threads() -> int:
    return int(lib().orc_max_threads())


def set_threads(n: int) -> None:
    """Threads for later steps (timing only; results do not depend on it)."""
    lib().orc_set_threads(int(n))
