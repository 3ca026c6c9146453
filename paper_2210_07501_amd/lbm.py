"""Thin ctypes binding of liblbm.so (include/lbm.h), same names as the C ABI.

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (through the allocator hooks) and the HIP
stream.  If the shared library has not been built, importing this module
raises -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY may name another build of the same library (tuning variants)
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_FP64, LBM_FP32_DEV = 0, 1

# Every function declared in include/lbm.h.
EXPORTS = ("lbm_create", "lbm_init", "lbm_init_device", "lbm_step", "lbm_solve", "lbm_fields", "lbm_residual",
           "lbm_get_state", "lbm_set_state", "lbm_retire", "lbm_restart", "lbm_profile_steps", "lbm_set_tile", "lbm_autotune",
           "lbm_info",
           "lbm_destroy", "lbm_strerror")


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("n_waves", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("b", ctypes.c_double), ("W", ctypes.c_double), ("M_phi", ctypes.c_double),
        ("rho_a", ctypes.c_double), ("rho_b", ctypes.c_double),
        ("mu_a", ctypes.c_double), ("mu_b", ctypes.c_double),
        ("k_a", ctypes.c_double), ("k_b", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("sigma_T", ctypes.c_double),
        ("sigma_TT", ctypes.c_double), ("T_ref", ctypes.c_double),
        ("T_h", ctypes.c_double), ("dT", ctypes.c_double), ("T_c", ctypes.c_double),
        ("Fx_ext", ctypes.c_double), ("Fy_ext", ctypes.c_double),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load():
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbm.so not built: run `python -m paper_2210_07501_amd.build` "
                           "(there is no CPU fallback)")
    # PyTorch ships its own HIP runtime.  Load it first so that the library
    # binds to that same runtime (same soname): loaded the other way round,
    # the process maps two runtimes and torch's device memory and streams are
    # foreign to the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    L.lbm_create.argtypes = [ctypes.POINTER(lbm_params), ctypes.c_int32, ctypes.c_int32, vp,
                             ALLOC_FN, FREE_FN, vp, ctypes.POINTER(vp)]
    L.lbm_init.argtypes = [vp, dp]
    L.lbm_init_device.argtypes = [vp, vp]
    L.lbm_step.argtypes = [vp, ctypes.c_int64]
    L.lbm_solve.argtypes = [vp, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]
    L.lbm_fields.argtypes = [vp, ctypes.c_int32, dp, dp, dp, dp, dp]
    L.lbm_residual.argtypes = [vp, ctypes.c_int32, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
    L.lbm_get_state.argtypes = [vp, ctypes.c_int32, dp]
    L.lbm_set_state.argtypes = [vp, ctypes.c_int32, dp]
    L.lbm_profile_steps.argtypes = [vp, ctypes.c_int64, dp]
    L.lbm_set_tile.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.lbm_retire.argtypes = [vp, ctypes.c_int32]
    L.lbm_restart.argtypes = [vp, ctypes.c_int32, dp]
    L.lbm_autotune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               dp]
    L.lbm_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_destroy.restype = None
    L.lbm_strerror.argtypes = [ctypes.c_int]
    L.lbm_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lbm_destroy", "lbm_strerror"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class LBMError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().lbm_strerror(status).decode()
        super().__init__("%s failed: %s (status %d)" % (where, msg, status))
        self.status = status


def _check(rc: int, where: str):
    if rc != LBM_OK:
        raise LBMError(rc, where)
    return rc


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(cfg: dict) -> lbm_params:
    p = lbm_params()
    for name, typ in lbm_params._fields_:
        if name == "reserved":
            p.reserved = 0
        else:
            setattr(p, name, int(cfg[name]) if typ is ctypes.c_int32 else float(cfg[name]))
    return p


class _TorchAllocator:
    """Device memory from PyTorch's caching allocator, handed to the library
    through the lbm_alloc_fn / lbm_free_fn hooks."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.last_error = None
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception as e:          # reported by lbm_create (an exception must not cross the C frame)
            self.last_error = "%s allocating %d bytes: %s" % (type(e).__name__, int(nbytes), e)
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


def lbm_create(cfgs, precision: int = LBM_FP64, stream=None, torch_alloc: bool = True, device=None):
    """Create a context for the channel configs (a dict or a list of dicts).
    Returns an opaque handle object (pass it to the other calls)."""
    L = load()
    if isinstance(cfgs, dict):
        cfgs = [cfgs]
    arr = (lbm_params * len(cfgs))(*[make_params(c) for c in cfgs])
    alloc = None
    st = None
    if stream is not None:
        st = ctypes.c_void_p(int(stream))
    if torch_alloc:
        import torch
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        alloc = _TorchAllocator(dev)
        if stream is None:
            # torch's current stream (handle 0 is the null stream, which the
            # library also takes for NULL)
            st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream or None)
    h = ctypes.c_void_p()
    a_cb = alloc.alloc_cb if alloc else ALLOC_FN()
    f_cb = alloc.free_cb if alloc else FREE_FN()
    rc = L.lbm_create(arr, len(cfgs), int(precision), st, a_cb, f_cb, None, ctypes.byref(h))
    if rc != LBM_OK and alloc is not None and alloc.last_error:
        raise LBMError(rc, "lbm_create (%s)" % alloc.last_error)
    _check(rc, "lbm_create")
    return _Ctx(h, cfgs, alloc, precision)


class _Ctx:
    def __init__(self, h, cfgs, alloc, precision):
        self.h = h
        self.cfgs = list(cfgs)
        self.alloc = alloc   # keeps the callbacks and tensors alive
        self.precision = precision

    def shape(self, inst: int):
        c = self.cfgs[inst]
        return int(c["ny"]), int(c["nx"])

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value:
            try:
                lbm_destroy(self)
            except Exception:
                pass


def lbm_init(ctx: _Ctx, fields=None):
    """fields: None (cold start) or a list (one per channel) of (phi, ux, uy, T) arrays."""
    if fields is None:
        _check(load().lbm_init(ctx.h, None), "lbm_init")
        return
    parts = []
    for k, f in enumerate(fields):
        ny, nx = ctx.shape(k)
        for a in f:
            parts.append(np.ascontiguousarray(a, dtype=np.float64).reshape(ny * nx))
    buf = np.ascontiguousarray(np.concatenate(parts))
    _check(load().lbm_init(ctx.h, _dp(buf)), "lbm_init")


def lbm_init_device(ctx: _Ctx, fields):
    """fields: a float64 CUDA tensor (or device address) holding, for each
    channel in order, phi, ux, uy, T ([ny][nx] each)."""
    ptr = fields if isinstance(fields, int) else fields.data_ptr()
    if not isinstance(fields, int):
        need = sum(4 * nx * ny for ny, nx in (ctx.shape(k) for k in range(len(ctx.cfgs))))
        if not (fields.is_cuda and fields.dtype.itemsize == 8 and fields.is_floating_point()
                and fields.is_contiguous() and fields.numel() == need):
            raise ValueError("lbm_init_device: need a contiguous float64 device tensor of %d values" % need)
    _check(load().lbm_init_device(ctx.h, ctypes.c_void_p(ptr)), "lbm_init_device")


def lbm_step(ctx: _Ctx, n: int):
    _check(load().lbm_step(ctx.h, int(n)), "lbm_step")


def lbm_solve(ctx: _Ctx, r_tol: float, max_steps: int):
    """Returns (status, n_active); status is LBM_OK or LBM_EDIVERGED."""
    na = ctypes.c_int32(0)
    rc = load().lbm_solve(ctx.h, float(r_tol), int(max_steps), ctypes.byref(na))
    if rc not in (LBM_OK, LBM_EDIVERGED):
        _check(rc, "lbm_solve")
    return rc, int(na.value)


def lbm_fields(ctx: _Ctx, inst: int = 0):
    ny, nx = ctx.shape(inst)
    out = [np.zeros((ny, nx)) for _ in range(5)]
    _check(load().lbm_fields(ctx.h, int(inst), *[_dp(a) for a in out]), "lbm_fields")
    return dict(zip(("phi", "ux", "uy", "T", "p"), out))


def lbm_residual(ctx: _Ctx, inst: int = 0):
    v = [ctypes.c_double() for _ in range(4)]
    s = ctypes.c_int64()
    rc = load().lbm_residual(ctx.h, int(inst), *[ctypes.byref(x) for x in v], ctypes.byref(s))
    if rc not in (LBM_OK, LBM_EDIVERGED):
        _check(rc, "lbm_residual")
    return dict(r=v[0].value, sum_phi=v[1].value, sum_mass=v[2].value, u_int_peak=v[3].value,
                steps=int(s.value), diverged=(rc == LBM_EDIVERGED))


def lbm_get_state(ctx: _Ctx, inst: int = 0):
    ny, nx = ctx.shape(inst)
    pop = np.zeros((3, 9, ny, nx))
    _check(load().lbm_get_state(ctx.h, int(inst), _dp(pop)), "lbm_get_state")
    return pop


def lbm_set_state(ctx: _Ctx, inst: int, pop):
    ny, nx = ctx.shape(inst)
    a = np.ascontiguousarray(pop, dtype=np.float64).reshape(3, 9, ny, nx)
    _check(load().lbm_set_state(ctx.h, int(inst), _dp(a)), "lbm_set_state")


def lbm_profile_steps(ctx: _Ctx, n: int) -> float:
    ms = ctypes.c_double()
    _check(load().lbm_profile_steps(ctx.h, int(n), ctypes.byref(ms)), "lbm_profile_steps")
    return ms.value


def lbm_retire(ctx: _Ctx, inst: int):
    _check(load().lbm_retire(ctx.h, int(inst)), "lbm_retire")


def lbm_restart(ctx: _Ctx, inst: int, fields=None):
    """Start channel inst again: from rest (fields None) or from (phi, ux, uy, T)."""
    buf = None
    if fields is not None:
        ny, nx = ctx.shape(inst)
        buf = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).reshape(ny * nx)
                                                   for a in fields]))
    _check(load().lbm_restart(ctx.h, int(inst), _dp(buf)), "lbm_restart")


def lbm_set_tile(ctx: _Ctx, tx: int, ty: int):
    _check(load().lbm_set_tile(ctx.h, int(tx), int(ty)), "lbm_set_tile")


def lbm_autotune(ctx: _Ctx, reps: int = 20):
    """Pick the fastest compiled tile shape for this context; returns
    ((tx, ty), ms per step launch)."""
    tx, ty, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(load().lbm_autotune(ctx.h, int(reps), ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(ms)), "lbm_autotune")
    return (tx.value, ty.value), ms.value


def lbm_info(ctx: _Ctx):
    n = ctypes.c_int64()
    b = ctypes.c_int64()
    _check(load().lbm_info(ctx.h, ctypes.byref(n), ctypes.byref(b)), "lbm_info")
    return int(n.value), int(b.value)


def lbm_destroy(ctx: _Ctx):
    if ctx.h is not None and ctx.h.value:
        load().lbm_destroy(ctx.h)
        ctx.h = ctypes.c_void_p()


def lbm_strerror(status: int) -> str:
    return load().lbm_strerror(int(status)).decode()
