"""The differentiable simulation as a torch.autograd.Function (SimulateST):
loss(simulate(theta)).backward() leaves dL/dtheta in theta.grad.

The loss is ordinary PyTorch code on the observation; the dL/dobs it hands
the Function's backward is captured with a tensor hook and given to the
oracle, which differentiates the same trajectories (same counter streams, the
GPU's near-tie log).  theta.grad is checked against the sum of the oracle's
per-trajectory gradients at the parity bar of test_gpu_parity.grad_bar, with
the oracle's conditioning of the sum.  Final-count observations keep every
trajectory away from bin edges, so the whole batch is compared.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import workloads as W

from test_gpu_parity import _ties_for_oracle, _x0, assert_grad_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


def _run(ssa, net, cfg, B, loss_of):
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    x0 = _x0([net], [B])
    theta = torch.tensor(net.theta0, device="cuda", requires_grad=True)
    rec, seen = {}, {}
    obs = ssa.simulate(theta, h, cfg, x0, tie_capacity=1 << 16, record=rec)
    assert obs.requires_grad and obs.dtype == torch.float64
    obs.register_hook(lambda g: seen.__setitem__("d_obs", g.detach().clone()))
    loss = loss_of(obs)
    loss.backward()
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    g = theta.grad.cpu().numpy().astype(np.float64)
    nob = len(net.obs_species)
    d = seen["d_obs"].cpu().numpy()[: nob * B].reshape(nob, B).T
    fwd = rec["forward"]
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(B),
                   ties=_ties_for_oracle(fwd.tie_records()), d_obs=d, kappa=True)
    assert r.n_bad.sum() == 0
    assert np.array_equal(fwd.x_final.cpu().numpy().reshape(net.n_species, B).T, r.x_final)
    assert_grad_parity(g, r.grad.sum(0), kappa=r.kappa.sum(0), T=cfg.temperature)
    return g, r


def test_simulate_st_dimer(ssa):
    """2A <-> A2: the mean and variance of the final A count against targets."""
    net = W.dimerization_2a()
    B = 4096
    cfg = W.RunConfig(seed=21, n_steps=2000, obs_kind=W.OBS_FINAL, temperature=0.5)

    def loss_of(obs):
        a = obs[:B]
        return (a.mean() - 45.0) ** 2 + (a.var(unbiased=False) - 25.0) ** 2

    g, _ = _run(ssa, net, cfg, B, loss_of)
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0


def test_simulate_st_oscillator(ssa):
    """The oscillator: the ensemble mean of the final R count against a target,
    plus a per-trajectory nonlinear term so that dL/dobs differs between
    trajectories."""
    net = W.oscillator()
    B = 512
    cfg = W.RunConfig(seed=22, n_steps=10000, obs_kind=W.OBS_FINAL, temperature=0.5, ckpt_every=1024)

    def loss_of(obs):
        r = obs[:B]
        return (r.mean() - 5.0) ** 2 + 1e-3 * torch.log1p(r).sum()

    g, _ = _run(ssa, net, cfg, B, loss_of)
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0


def test_simulate_st_matches_library_backward(ssa):
    """theta.grad through the Function equals ssa_backward on the same dL/dobs
    (the Function only marshals arguments)."""
    net = W.dimerization_abc()
    B = 1000
    cfg = W.RunConfig(seed=5, n_steps=300, obs_kind=W.OBS_BINS, n_bins=6, t_obs=3.0, temperature=0.5,
                      ckpt_every=64)
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    x0 = _x0([net], [B])
    theta = torch.tensor(net.theta0, device="cuda", requires_grad=True)
    w = torch.randn(cfg.n_bins * 3 * B, dtype=torch.float64, device="cuda")
    obs = ssa.simulate(theta, h, cfg, x0)
    (obs * w).sum().backward()
    fwd = ssa.forward(h, cfg, theta.detach(), x0, tie_capacity=0)
    dp = ssa.backward(h, cfg, theta.detach(), x0, fwd, w)
    torch.cuda.synchronize()
    assert torch.equal(theta.grad, dp)
