"""The binding refuses arguments whose sizes, types or layouts do not match
what the handle and the run settings imply, before anything is enqueued (the
kernels read every buffer at the implied size)."""
import numpy as np
import pytest
import torch

from paper_2602_19775_amd import workloads as W

from test_gpu_parity import _x0

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


def test_mass_action_arguments(ssa):
    net = W.dimerization_2a()
    B = 128
    cfg = W.RunConfig(seed=1, n_steps=100, obs_kind=W.OBS_BINS, n_bins=5, t_obs=20.0)
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    with pytest.raises(ValueError):
        ssa.forward(h, cfg, th.double(), x0)                       # wrong dtype
    with pytest.raises(ValueError):
        ssa.forward(h, cfg, th, x0[:-1])                           # one count short
    with pytest.raises(ValueError):
        ssa.forward(h, cfg, th, x0.cpu())                          # host memory
    f = ssa.forward(h, cfg, th, x0)
    d_obs = torch.zeros(h.obs_total(cfg.obs_kind, cfg.n_bins), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ssa.backward(h, cfg, th, x0, f, d_obs[:-1])                # dL/dobs too short
    with pytest.raises(ValueError):
        ssa.backward(h, cfg, th, x0, f, d_obs.float())
    with pytest.raises(ValueError):
        ssa.backward(h, cfg, th, x0, f, d_obs, d_params=torch.empty(1, device="cuda"))
    big = ssa.Net([net], [2 * B], t_obs=[cfg.t_obs])
    with pytest.raises(ValueError):
        ssa.forward(big, cfg, th, _x0([net], [2 * B]), buffers=f)   # buffers of a smaller handle
    with pytest.raises(ValueError):
        ssa.step_batch(h, cfg, th, x0, torch.zeros(B - 1, dtype=torch.float64, device="cuda"), 0)
    # a non-contiguous dL/dobs is taken as its contiguous copy
    wide = torch.zeros((d_obs.numel(), 2), dtype=torch.float64, device="cuda")
    dp = ssa.backward(h, cfg, th, x0, f, wide[:, 0])
    dp0 = ssa.backward(h, cfg, th, x0, f, d_obs)
    torch.cuda.synchronize()
    assert torch.equal(dp, dp0)


def test_gene_network_arguments(ssa):
    from test_gpu_grn import workload
    w = workload(2, 2, 20, n_in=64, n_out=4, seed=0)
    g = ssa.Grn(w.net, w.n_images, w.n_rep)
    th = torch.tensor(w.theta, device="cuda")
    x = torch.tensor(w.images, device="cuda")
    with pytest.raises(ValueError):
        ssa.grn_forward(g, w.cfg, th[:-1], x)
    with pytest.raises(ValueError):
        ssa.grn_forward(g, w.cfg, th, x[:, :-1])
    f = ssa.grn_forward(g, w.cfg, th, x)
    with pytest.raises(ValueError):
        ssa.grn_backward(g, w.cfg, th, x, f, torch.zeros(3, dtype=torch.float64, device="cuda"))
    d = torch.zeros((w.net.n_out, g.B), dtype=torch.float64, device="cuda")
    dp = ssa.grn_backward(g, w.cfg, th, x, f, d)
    torch.cuda.synchronize()
    assert ssa.grn_device_status(g) == 0
    assert np.all(np.isfinite(dp.cpu().numpy()))
