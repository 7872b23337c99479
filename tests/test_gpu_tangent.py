"""Forward-mode tangents (SSA_BWD_TANGENT) against the FP64 oracle's reverse
adjoint: the same straight-through derivative accumulated the other way.

- The tangent forward fires the same path as the ordinary forward: counts,
  step counts, clocks and observations bit-identical (same seeds).
- Per-trajectory gradients and their sums within the conditioning bar of
  test_gpu_parity (grad_bar), for bin and final observations, two- and
  three-channel networks, T = 0.5, 1 and 0.05.
- At the benchmarked dimer size (65,536 x 10,000, 20 bins, the moment loss) a
  sample of trajectories against the oracle one by one.
- Networks and settings outside the tangent limits are refused.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import losses
from paper_2602_19775_amd import workloads as W

from test_gpu_parity import (EDGE_WINDOW, _ties_for_oracle, _x0, assert_forward_parity, assert_grad_parity,
                             edge_safe, run_pair)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


CASES = {
    "dimer_bins": (W.dimerization_2a, dict(seed=1, n_steps=1500, obs_kind=W.OBS_BINS, n_bins=20, t_obs=300.0,
                                           temperature=0.5), 300),
    "dimer_bins_T1": (W.dimerization_2a, dict(seed=2, n_steps=800, obs_kind=W.OBS_BINS, n_bins=7, t_obs=100.0,
                                              temperature=1.0), 257),
    "abc_final_cold": (W.dimerization_abc, dict(seed=3, n_steps=250, obs_kind=W.OBS_FINAL, temperature=0.05), 400),
    "channel_bins": (W.ion_channel_coi, dict(seed=4, n_steps=20, obs_kind=W.OBS_BINS, n_bins=40, t_obs=8.0,
                                             temperature=0.3), 512),
}


@pytest.mark.parametrize("name", list(CASES))
def test_tangent_parity(ssa, name):
    make, kw, B = CASES[name]
    net = make()
    cfg = W.RunConfig(**kw)
    g = np.random.default_rng(7)
    bins = cfg.obs_kind == W.OBS_BINS
    nob = len(net.obs_species)
    d_obs = g.normal(size=(cfg.n_bins, nob, B)) if bins else g.normal(size=(nob, B))
    gpu, r, ids, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs, bwd_mode="tangent")
    assert_forward_parity(gpu, r, ids, cfg)
    ref, _, _, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs, bwd_mode="tape")
    for k in ("x_final", "t_final", "steps_done", "obs"):
        assert np.array_equal(gpu[k], ref[k]), k
    keep = edge_safe(gpu, r, ids)
    assert keep.all()
    T = cfg.temperature
    assert_grad_parity(gpu["ppt"], r.grad, keep, kappa=r.kappa, T=T)
    assert_grad_parity(gpu["ppt"].sum(0), r.grad.sum(0), kappa=r.kappa.sum(0), T=T)
    # the two accumulation orders of the library agree as they agree with the oracle
    assert_grad_parity(gpu["ppt"], ref["ppt"].astype(np.float64), kappa=r.kappa, T=T)
    tot = r.grad.sum(0)
    assert np.allclose(gpu["d_params"], tot, rtol=1e-5, atol=1e-5 * np.abs(tot).max())


def test_tangent_dimer_65536x10000(ssa):
    wl = W.dimer_fwdbwd_64k()
    net, B, cfg = wl.net, wl.n_traj, wl.cfg
    nb = cfg.n_bins
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    x0 = _x0([net], [B])
    target = torch.tensor(np.log(np.array(W.DIMER_TARGET_RATES)).astype(np.float32), device="cuda")
    tf = ssa.forward(h, cfg.replace(purpose=W.PURPOSE_TARGET), target, x0, keep_ckpt=False, tie_capacity=0)
    tm, tv = losses.bin_moments(tf.obs, nb, 1, B)
    tm, tv = tm.clone(), tv.clone()
    del tf
    th = torch.tensor(net.theta0, device="cuda")
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 16, bwd_mode="tangent")
    obs = fwd.obs.detach().requires_grad_(True)
    (d_obs,) = torch.autograd.grad(losses.moment_mse(obs, tm, tv, nb, 1, B), obs)
    dp, ppt = ssa.backward(h, cfg, th, x0, fwd, d_obs, per_traj=True)
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    g = np.random.default_rng(0)
    ids = np.unique(np.concatenate([[0, B - 1], g.choice(B, 62, replace=False)]))
    index = {int(q): k for k, q in enumerate(ids)}
    dnp = d_obs.cpu().numpy().reshape(nb, 1, B).transpose(2, 0, 1)
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=ids, ties=_ties_for_oracle(fwd.tie_records(), 0, index),
                   d_obs=dnp[ids], kappa=True, edge_window=EDGE_WINDOW)
    r.edge_window = EDGE_WINDOW
    gpu = {"x_final": fwd.x_final.cpu().numpy().reshape(2, B).T, "t_final": fwd.t_final.cpu().numpy(),
           "steps_done": fwd.steps_done.cpu().numpy(),
           "obs": fwd.obs.cpu().numpy().reshape(nb, 1, B).transpose(2, 0, 1)}
    assert_forward_parity(gpu, r, ids, cfg)
    pp = ppt.cpu().numpy().reshape(net.n_params, B).T
    assert_grad_parity(pp[ids], r.grad, kappa=r.kappa, T=cfg.temperature)
    assert_grad_parity(pp[ids].sum(0), r.grad.sum(0), kappa=r.kappa.sum(0), T=cfg.temperature)
    total = pp.astype(np.float64).sum(0)
    mag = np.abs(pp.astype(np.float64)).sum(0)
    assert np.all(np.abs(dp.cpu().numpy() - total) <= 1e-5 * np.abs(total) + 1e-6 * mag)


def test_tangent_refused_outside_its_limits(ssa):
    def refused(net, cfg, B=64):
        h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
        with pytest.raises(ssa.SSAError):
            ssa.forward(h, cfg, torch.tensor(net.theta0, device="cuda"), _x0([net], [B]), bwd_mode="tangent")
    refused(W.oscillator(), W.RunConfig(n_steps=50, obs_kind=W.OBS_FINAL))                 # 16 channels
    dim = W.dimerization_2a()
    refused(dim, W.RunConfig(n_steps=50, obs_kind=W.OBS_GRID, n_bins=5, t_obs=10.0))       # grid observation
    refused(dim, W.RunConfig(n_steps=50, t_end=5.0, obs_kind=W.OBS_FINAL))                 # t_end
    refused(dim, W.RunConfig(n_steps=50, obs_kind=W.OBS_TAIL, n_bins=10))                  # tail observation
