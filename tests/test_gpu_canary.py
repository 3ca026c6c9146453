"""Halo canary: a channel whose every population is NaN sits between two
ragged channels in one batch (sizes that leave partial tiles in x and y).
The fused kernel's halo pulls, ghost rows and partial tiles must never read
another channel's populations: after 150 steps (one check step included)
the two neighbours are finite and bit for bit what they are when run alone,
in both precisions.  The NaN channel is set up through lbm_init_device,
whose device fields are not checked on the host (lbm_set_state and lbm_init
refuse non-finite values); its populations stay NaN in both buffers after
it is retired at its first check.  No kernel faults here: the NaN values are
data."""
import numpy as np
import pytest

from paper_2210_07501_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available()
    from paper_2210_07501_amd import lbm as L
    L.load()
    return L


@pytest.mark.parametrize("prec", [0, 1])
def test_nan_channel_does_not_leak_into_its_neighbours(lbm, prec):
    a = inputs.cfg(nx=100, ny=37, n_waves=2, b=17.0, sigma_T=-1e-4, sigma_TT=2e-4)
    b = inputs.cfg(nx=70, ny=21, b=10.0, sigma_TT=1e-4)
    c = inputs.cfg(nx=130, ny=45, b=25.0, sigma_T=5e-5, mu_a=0.05, k_a=0.3)
    print("case: NaN channel between two ragged channels, precision", prec, flush=True)
    import torch
    fa, fc = inputs.perturbed_fields(a, 3, amp=0.8), inputs.perturbed_fields(c, 4, amp=0.8)
    dev = torch.from_numpy(np.concatenate([np.stack(fa).ravel(), np.full(4 * b["nx"] * b["ny"], np.nan),
                                           np.stack(fc).ravel()])).cuda()
    ctx = lbm.lbm_create([a, b, c], precision=prec)
    lbm.lbm_init_device(ctx, dev)
    lbm.lbm_step(ctx, 150)
    assert lbm.lbm_residual(ctx, 1)["diverged"]
    for k, (cfg, f) in ((0, (a, fa)), (2, (c, fc))):
        alone = lbm.lbm_create(cfg, precision=prec)
        lbm.lbm_init_device(alone, torch.from_numpy(np.stack(f).ravel()).cuda())
        lbm.lbm_step(alone, 150)
        got, want = lbm.lbm_get_state(ctx, k), lbm.lbm_get_state(alone, 0)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, want)
        assert not lbm.lbm_residual(ctx, k)["diverged"]
