"""ssa_backward_static (the backward with the library's static device scratch)
against ssa_backward with a caller-allocated work buffer: two calls in a row,
the second on a smaller batch, each equal bit for bit to the allocating entry
point's result (the same kernels read the same inputs)."""
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


def _pair(ssa, net, cfg, B, seed):
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=0)
    g = torch.Generator(device="cuda").manual_seed(seed)
    d = torch.randn(fwd.obs.numel(), dtype=torch.float64, device="cuda", generator=g)
    ref, ref_ppt = ssa.backward(h, cfg, th, x0, fwd, d, per_traj=True)
    dp = torch.full_like(ref, float("nan"))
    ppt = torch.full_like(ref_ppt, float("nan"))
    ssa.backward_static(h, cfg, th, x0, fwd, d, dp, ppt)
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    assert torch.equal(dp, ref)
    assert torch.equal(ppt, ref_ppt)
    return h


def test_static_backward_equals_allocating_backward(ssa):
    net = W.dimerization_2a()
    cfg = W.RunConfig(seed=3, n_steps=2000, obs_kind=W.OBS_BINS, n_bins=10, t_obs=400.0, temperature=0.5,
                      ckpt_every=128)
    _pair(ssa, net, cfg, 8192, 1)
    # the second call on a smaller batch reuses the scratch the first one filled
    _pair(ssa, net, cfg.replace(seed=4, n_steps=700), 300, 2)


def test_static_backward_oscillator_then_smaller(ssa):
    net = W.oscillator()
    cfg = W.RunConfig(seed=5, n_steps=3000, obs_kind=W.OBS_FINAL, temperature=0.5, ckpt_every=256)
    _pair(ssa, net, cfg, 4096, 3)
    _pair(ssa, net, cfg.replace(seed=6, n_steps=1000), 257, 4)


def test_static_backward_refuses_oversized_work(ssa):
    # 4,200 networks x 256 trajectories x 8 channels of FP64 partials exceed 32 MiB
    nets = W.random_network_batch(4200, seed=1, n_range=(4, 4), m_range=(8, 8))
    B = [256] * len(nets)
    cfg = W.RunConfig(seed=1, n_steps=10, obs_kind=W.OBS_FINAL, temperature=0.5, ckpt_every=8)
    h = ssa.Net(nets, B)
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = torch.tensor(np.concatenate([np.repeat(n.x0[:, None], b, 1).reshape(-1) for n, b in zip(nets, B)]),
                      dtype=torch.int32, device="cuda")
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=0)
    d = torch.zeros(fwd.obs.numel(), dtype=torch.float64, device="cuda")
    dp = torch.empty(h.param_total, dtype=torch.float32, device="cuda")
    with pytest.raises(ssa.SSAError, match="static array"):
        ssa.backward_static(h, cfg, th, x0, fwd, d, dp)
    torch.cuda.synchronize()
