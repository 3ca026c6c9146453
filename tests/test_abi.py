"""The C-ABI library: it loads, exports every function include/lbm.h
declares, and rejects invalid parameters before touching a device.  No
compute calls here (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2210_07501_amd import inputs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
NN_HEADER = os.path.join(ROOT, "include", "lbm_nn.h")


def declared_functions(header=HEADER, prefix="lbm_"):
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(%s[a-z0-9_]+)\s*\(" % prefix, txt))
    # typedef'd function-pointer types are not exports
    names -= {"lbm_alloc_fn", "lbm_free_fn"}
    return names


def test_library_exports_every_declared_function():
    L = lbm.load()
    names = declared_functions()
    assert names, "no declarations parsed"
    assert names == set(lbm.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_library_exports_every_network_function():
    from paper_2210_07501_amd import nn
    L = nn.load()
    names = declared_functions(NN_HEADER, "nn_")
    assert names, "no declarations parsed"
    assert names == set(nn.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_params_struct_layout():
    # 4 int32 followed by 18 doubles, no padding
    assert ctypes.sizeof(lbm.lbm_params) == 4 * 4 + 18 * 8
    txt = open(HEADER).read()
    body = txt[txt.index("typedef struct {"):txt.index("} lbm_params;")]
    doubles = sum(len(re.findall(r"\b[A-Za-z_0-9]+\b", decl)) for decl in re.findall(r"double\s+([^;]+);", body))
    assert doubles == 18


def _create(cfg, n_inst=1, prec=0):
    L = lbm.load()
    arr = (lbm.lbm_params * n_inst)(*[lbm.make_params(cfg)] * n_inst)
    h = ctypes.c_void_p()
    rc = L.lbm_create(arr, n_inst, prec, None, lbm.ALLOC_FN(), lbm.FREE_FN(), None, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("bad", [
    dict(nx=2), dict(ny=3), dict(n_waves=3), dict(n_waves=0), dict(W=0.0), dict(b=3.0),
    dict(b=62.0), dict(M_phi=0.0), dict(mu_a=-0.1), dict(k_b=0.0), dict(rho_a=0.0),
    dict(sigma_T=float("nan")), dict(T_h=float("inf")),
    # channel size: 27 x 8 x nx x ny must stay below 2^32 (4096 x 4864 is just over)
    dict(nx=4096, ny=4864, b=2432.0),
])
def test_create_rejects_invalid_parameters(bad):
    cfg = inputs.small_channel()
    cfg.update(bad)
    rc, h = _create(cfg)
    assert rc == lbm.LBM_EINVAL
    assert not h.value


def test_create_rejects_bad_arguments():
    rc, _ = _create(inputs.small_channel(), n_inst=0)
    assert rc == lbm.LBM_EINVAL
    rc, _ = _create(inputs.small_channel(), prec=7)
    assert rc == lbm.LBM_EINVAL
    L = lbm.load()
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_init(None, None) == lbm.LBM_EINVAL
    assert L.lbm_set_tile(None, 32, 8) == lbm.LBM_EINVAL
    assert L.lbm_retire(None, 0) == lbm.LBM_EINVAL


def test_strerror():
    for s in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(lbm.lbm_strerror(s), str)


def test_network_calls_reject_bad_shapes():
    """Shape and pointer checks of the network entry points return before
    any launch (dummy non-null addresses are never dereferenced)."""
    from paper_2210_07501_amd import nn
    L = nn.load()
    p = ctypes.c_void_p(256)
    E = lbm.LBM_EINVAL
    # pooling / upsampling: c a multiple of 8, even sizes for pooling, non-null buffers
    assert L.nn_pool2(0, p, p, 1, 4, 64, 12, None) == E
    assert L.nn_pool2(0, p, p, 1, 5, 64, 32, None) == E
    assert L.nn_pool2(0, None, p, 1, 4, 64, 32, None) == E
    assert L.nn_up2(0, p, p, 1, 4, 64, 4, None) == E
    assert L.nn_up2(1, p, None, 1, 4, 64, 32, None) == E
    # convolution: widths multiple of 64, channels multiple of 32 up to 96
    assert L.nn_conv3x3_fwd(p, p, None, p, None, 0, 1, 4, 96, 32, 32, 0, None) == E
    assert L.nn_conv3x3_fwd(p, p, None, p, None, 0, 1, 4, 64, 48, 32, 0, None) == E
    assert L.nn_conv3x3_fwd(p, p, None, p, None, 0, 1, 4, 64, 32, 128, 0, None) == E
    assert L.nn_conv3x3_bwd_data(p, p, p, 1, 4, 64, 32, 16, None) == E
    # weight gradient: a workspace smaller than the one asked for
    need = nn.nn_conv3x3_wgrad_workspace(1, 4, 64, 32, 32)
    assert L.nn_conv3x3_bwd_weight(p, p, p, None, p, need - 4, 0, 1, 4, 64, 32, 32, None) == E
    # elementwise: negative counts
    assert L.nn_add(p, p, p, -1, None) == E
    assert L.nn_relu_bwd(p, p, p, -1, None) == E
    # the row-walking tuning knob: 0 (automatic) to 64 steps per work-group
    assert L.nn_set_conv_walk(-1) == E
    assert L.nn_set_conv_walk(65) == E
    assert L.nn_set_conv_walk(8) == lbm.LBM_OK
    assert L.nn_set_conv_walk(0) == lbm.LBM_OK
