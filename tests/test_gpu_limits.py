"""Every execution mode at the largest network it accepts, with oracle parity
of counts, clocks, bin averages and per-trajectory gradients, and the first
size past each limit refused before anything runs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import workloads as W

from test_gpu_parity import _x0, assert_forward_parity, assert_grad_parity, edge_safe, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


def _net(N, M, seed):
    g = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    return W.random_network(g, name=f"limit_{N}x{M}", n_range=(N, N), m_range=(M, M))


# (mode, species, channels): the specialised lane kernels at the largest
# network the library's own choice gives them (64 x 32; an explicit request
# takes up to 64 x 64, whose topology takes minutes to compile), the generic
# lane kernels and the wave mode (64 lanes drawing two Philox blocks each)
LIMITS = [("spec", 64, 32), ("lane", 16, 32), ("wave", 64, 511)]


@pytest.mark.parametrize("mode,N,M", LIMITS, ids=[f"{m}_{n}x{k}" for m, n, k in LIMITS])
def test_largest_network_of_each_mode(ssa, mode, N, M):
    """Forward and per-trajectory gradient parity at the mode's size limit."""
    net = _net(N, M, seed=N * 1000 + M)
    assert net.n_species == N and net.n_reactions == M
    pilot = oracle.run(net, W.RunConfig(seed=1, n_steps=150, purpose=2), net.theta0, net.x0,
                       traj_ids=np.arange(8))
    cfg = W.RunConfig(seed=4, n_steps=150, obs_kind=W.OBS_BINS, n_bins=4,
                      t_obs=float(np.min(pilot.t_final)) * 0.8, temperature=0.5, ckpt_every=64)
    B = 80
    d_obs = np.random.default_rng(2).normal(size=(cfg.n_bins, len(net.obs_species), B))
    gpu, r, ids, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs, exec_mode=mode)
    assert_forward_parity(gpu, r, ids, cfg)
    keep = edge_safe(gpu, r, ids)
    assert keep.all()
    assert_grad_parity(gpu["ppt"], r.grad, keep, kappa=r.kappa, T=cfg.temperature)


@pytest.mark.parametrize("mode,N,M", [("spec", 65, 20), ("spec", 20, 65), ("lane", 17, 10), ("lane", 10, 33),
                                      ("wave", 65, 20), ("wave", 20, 512)])
def test_first_size_past_each_limit_is_refused(ssa, mode, N, M):
    net = _net(N, M, seed=N * 1000 + M)
    with pytest.raises(ssa.SSAError):
        ssa.Net([net], [8], exec_mode=mode)


def test_auto_mode_keeps_large_networks_off_the_specialised_kernels(ssa):
    """The library's own choice: the specialised kernels up to 32 channels
    (seen through the grid observation, which only they run)."""
    cfg = W.RunConfig(seed=1, n_steps=20, obs_kind=W.OBS_GRID, n_bins=4, t_obs=0.01)
    for M, spec in ((32, True), (33, False)):
        net = _net(8, M, seed=M)
        h = ssa.Net([net], [64], t_obs=[cfg.t_obs])
        th = torch.tensor(net.theta0, device="cuda")
        if spec:
            ssa.forward(h, cfg, th, _x0([net], [64]), tie_capacity=0)
        else:
            with pytest.raises(ssa.SSAError, match="specialised"):
                ssa.forward(h, cfg, th, _x0([net], [64]), tie_capacity=0)
