"""The allocation-free loss entry point (nn_mse_noalloc, include/lbm_nn.h)
against the workspace one (nn_mse): same kernels, so the loss and the
gradient must agree bit for bit -- on two calls in a row, the second on a
smaller input (the static scratch keeps the first call's partial sums,
which the second must not see).  Also: sizes beyond the static scratch are
refused before any launch.  Through the C ABI; no allocation in the call
(the tensors are made beforehand)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_loss_matches_the_workspace_loss():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm, nn
    L = nn.load()
    g = torch.Generator(device="cuda").manual_seed(11)
    for npix, nch, cpad in ((1_000_003, 4, 32), (70_001, 3, 8)):
        print("case: nn_mse_noalloc npix=%d nch=%d cpad=%d" % (npix, nch, cpad), flush=True)
        pred = torch.randn((npix, nch), generator=g, device="cuda", dtype=torch.float32)
        tgt = torch.randn((npix, nch), generator=g, device="cuda", dtype=torch.float32)
        work = torch.empty(((npix + 255) // 256,), device="cuda", dtype=torch.float64)
        d_ref = torch.full((npix, cpad), 7.0, device="cuda", dtype=torch.bfloat16)
        d_new = torch.full((npix, cpad), 5.0, device="cuda", dtype=torch.bfloat16)
        l_ref = torch.zeros(1, device="cuda", dtype=torch.float64)
        l_new = torch.zeros(1, device="cuda", dtype=torch.float64)
        nn.nn_mse(pred, tgt, d_ref, cpad, npix, nch, l_ref, work)
        nn.nn_mse_noalloc(pred, tgt, d_new, cpad, npix, nch, l_new)
        torch.cuda.synchronize()
        assert l_new.item() == l_ref.item()
        assert torch.equal(d_new.view(torch.int16), d_ref.view(torch.int16))
        # the float64 reference of the definition, mean squared difference
        want = float(np.mean((pred.double() - tgt.double()).cpu().numpy() ** 2))
        assert abs(l_new.item() - want) <= 1e-6 * want
        # loss only (no gradient buffer)
        l2 = torch.zeros(1, device="cuda", dtype=torch.float64)
        nn.nn_mse_noalloc(pred, tgt, None, cpad, npix, nch, l2)
        torch.cuda.synchronize()
        assert l2.item() == l_ref.item()


def test_noalloc_loss_refuses_sizes_beyond_its_scratch():
    import torch
    from paper_2210_07501_amd import lbm, nn
    L = nn.load()
    loss = torch.zeros(1, device="cuda", dtype=torch.float64)
    dummy = torch.zeros(4, device="cuda", dtype=torch.float32)
    # 2^25 pixels fit, one more block does not; refused on the host, nothing launched
    rc = L.nn_mse_noalloc(ctypes.c_void_p(dummy.data_ptr()), ctypes.c_void_p(dummy.data_ptr()), None, 4,
                          (1 << 25) + 256, 4, ctypes.c_void_p(loss.data_ptr()), None)
    assert rc == lbm.LBM_EINVAL
