"""Parity at the benchmarked sizes, in the launch configuration bench.py times.

The GPU runs the whole workload; the oracle recomputes a sample of
trajectories one by one (same global trajectory ids, so the same random
streams), with the GPU's near-tie log.  dL/dobs comes from the workload's own
loss on the GPU's observation, as in the benchmark.

- counts and step counts bit-exact, clocks within 1e-5 relative;
- per-trajectory gradients at the bar of test_gpu_parity.grad_bar, every
  sampled trajectory (bin observations: the oracle takes the GPU's side of bin
  edges that event times fall close to, from the forward's edge log);
- the sample's summed gradient within 1e-5;
- the reduced d_params equal the FP64 sum of the (FP32) per-trajectory
  gradients, up to their rounding.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import losses
from paper_2602_19775_amd import workloads as W

from test_gpu_parity import (EDGE_WINDOW, _ties_for_oracle, _x0, assert_forward_parity, assert_grad_parity,
                             edge_safe)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


def _single_network(ssa, wl, loss_of, sample):
    net, B, cfg = wl.net, wl.n_traj, wl.cfg
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    if loss_of is None:
        d_obs = None
    else:
        tf = ssa.forward(h, cfg.replace(purpose=W.PURPOSE_TARGET), loss_of["target_theta"], x0, keep_ckpt=False,
                         tie_capacity=0)
        loss_fn = loss_of["make"](tf.obs)
        del tf
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 22)
    if loss_of is None:
        # a seeded dL/dobs of the workload's observation layout
        g = np.random.default_rng(17)
        d_obs = torch.tensor(g.normal(size=fwd.obs.numel()), device="cuda")
    else:
        obs = fwd.obs.detach().requires_grad_(True)
        (d_obs,) = torch.autograd.grad(loss_fn(obs), obs)
    dp, ppt = ssa.backward(h, cfg, th, x0, fwd, d_obs, per_traj=True)
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    nb, nob, N = max(cfg.n_bins, 1), len(net.obs_species), net.n_species
    if cfg.obs_kind == W.OBS_FINAL:
        nb = 1
    ids = np.asarray(sample)
    gpu = {"x_final": fwd.x_final.cpu().numpy().reshape(N, B).T,
           "t_final": fwd.t_final.cpu().numpy(), "steps_done": fwd.steps_done.cpu().numpy(),
           "obs": fwd.obs.cpu().numpy()[: nb * nob * B].reshape(nb, nob, B).transpose(2, 0, 1)}
    if cfg.obs_kind == W.OBS_FINAL:
        gpu["obs"] = gpu["obs"][:, 0, :]
    ppt = ppt.cpu().numpy().reshape(net.n_params, B).T
    dnp = d_obs.cpu().numpy()[: nb * nob * B].reshape(nb, nob, B).transpose(2, 0, 1)
    if cfg.obs_kind == W.OBS_FINAL:
        dnp = dnp[:, 0, :]
    index = {int(q): k for k, q in enumerate(ids)}
    ew = EDGE_WINDOW if cfg.obs_kind == W.OBS_BINS else 0.0
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=ids, ties=_ties_for_oracle(fwd.tie_records(), 0, index),
                   d_obs=dnp[ids], kappa=True, edge_window=ew)
    r.edge_window = ew
    assert_forward_parity(gpu, r, ids, cfg)
    keep = edge_safe(gpu, r, ids)
    assert keep.all()
    T = cfg.temperature
    assert_grad_parity(ppt[ids], r.grad, keep, kappa=r.kappa, T=T)
    assert_grad_parity(ppt[ids][keep].sum(0), r.grad[keep].sum(0), kappa=r.kappa[keep].sum(0), T=T)
    gs, rs = ppt[ids].sum(0), r.grad.sum(0)
    assert np.linalg.norm(gs - rs) <= 1e-5 * np.linalg.norm(rs)
    # the per-trajectory gradients are handed out in FP32: their sum carries
    # that rounding, relative to the sum of magnitudes
    total = ppt.astype(np.float64).sum(0)
    mag = np.abs(ppt.astype(np.float64)).sum(0)
    assert np.all(np.abs(dp.cpu().numpy() - total) <= 1e-5 * np.abs(total) + 1e-6 * mag)
    rel = np.linalg.norm(ppt[ids][keep] - r.grad[keep], axis=1) / np.linalg.norm(r.grad[keep], axis=1)
    print(f"\n{wl.name}: compared {int(keep.sum())} of {len(ids)} sampled trajectories, per-trajectory "
          f"relative error median {np.median(rel):.2e} max {rel.max():.2e}")
    return keep


def test_dimer_65536x10000(ssa):
    wl = W.dimer_fwdbwd_64k()
    B, nb = wl.n_traj, wl.cfg.n_bins

    def make(tobs):
        tm, tv = losses.bin_moments(tobs, nb, 1, B)
        tm, tv = tm.clone(), tv.clone()
        return lambda obs: losses.moment_mse(obs, tm, tv, nb, 1, B)
    target = torch.tensor(np.log(np.array(W.DIMER_TARGET_RATES)).astype(np.float32), device="cuda")
    g = np.random.default_rng(0)
    sample = np.unique(np.concatenate([[0, B - 1], g.choice(B, 62, replace=False)]))
    _single_network(ssa, wl, {"make": make, "target_theta": target}, sample)


def test_oscillator_65536x200000(ssa):
    """The benchmark's loss (autocorrelation of the 256 bin averages).  Over
    200,000 events nearly every trajectory has an event time within its FP32
    clock's drift of one of the 255 inner bin edges, where the derivative of a
    bin average jumps; the oracle takes the GPU's side of those edges from the
    forward's edge log, so all 24 sampled trajectories are compared one by
    one."""
    wl = W.oscillator_fwdbwd_64k()
    B, nb = wl.n_traj, wl.cfg.n_bins

    def make(tobs):
        tac = losses.mean_autocorrelation(tobs, nb, B, 64).clone()
        return lambda obs: losses.autocorrelation_mse(obs, tac, nb, B, 64)
    target = torch.tensor(wl.extra["target_net"].theta0, device="cuda")
    g = np.random.default_rng(1)
    sample = np.unique(np.concatenate([[0, 4097, 33333, B - 1], g.choice(B, 20, replace=False)]))
    _single_network(ssa, wl, {"make": make, "target_theta": target}, sample)


def test_oscillator_65536x200000_final_counts(ssa):
    """The oscillator at its full size and length with the final counts of R
    observed (no bin edges, so every sampled trajectory is compared) and a
    seeded dL/dobs: the straight-through adjoint per trajectory over 200,000
    steps."""
    wl = W.oscillator_fwdbwd_64k()
    wl.cfg = wl.cfg.replace(obs_kind=W.OBS_FINAL, n_bins=0)
    g = np.random.default_rng(2)
    sample = np.unique(np.concatenate([[0, 1, 65535], g.choice(wl.n_traj, 13, replace=False)]))
    _single_network(ssa, wl, None, sample)


def test_uneven_batch_4096x256x5000(ssa):
    """The uneven batch as benchmarked: 4 bins over each network's own window,
    the loss of ensemble means per network, species and bin.  The wave-mode
    forward logs the side of every bin edge an event time falls close to, and
    the oracle takes it, so every sampled trajectory is compared."""
    bw = W.uneven_batch()
    nets, Bs, cfg = bw.nets, bw.n_traj, bw.cfg
    nb = cfg.n_bins
    h = ssa.Net(nets, Bs, t_obs=bw.t_obs)
    th = torch.tensor(bw.theta(), device="cuda")
    x0 = torch.tensor(bw.x0_packed(), device="cuda")
    rows = sum(len(n.obs_species) for n in nets) * nb
    Bn = Bs[0]
    tf = ssa.forward(h, cfg.replace(purpose=W.PURPOSE_TARGET),
                     torch.tensor(np.concatenate([n.theta0 for n in bw.target_nets]), device="cuda"), x0,
                     keep_ckpt=False, tie_capacity=0)
    tmean = tf.obs[: rows * Bn].view(rows, Bn).mean(dim=1).clone()
    del tf
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 23)
    obs = fwd.obs.detach().requires_grad_(True)
    loss = ((obs[: rows * Bn].view(rows, Bn).mean(dim=1) - tmean) ** 2).mean()
    (d_obs,) = torch.autograd.grad(loss, obs)
    dp, ppt = ssa.backward(h, cfg, th, x0, fwd, d_obs, per_traj=True)
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    ties = fwd.tie_records()
    xf, tfin, sd = fwd.x_final.cpu().numpy(), fwd.t_final.cpu().numpy(), fwd.steps_done.cpu().numpy()
    ob, dob, pp = fwd.obs.cpu().numpy(), d_obs.cpu().numpy(), ppt.cpu().numpy()
    g = np.random.default_rng(5)
    picks = np.unique(np.concatenate([[0, len(nets) - 1], g.choice(len(nets), 14, replace=False)]))
    for n in picks:
        net = nets[n]
        ncfg = cfg.replace(t_obs=bw.t_obs[n])
        L = h.layout(int(n), cfg.obs_kind, nb)
        nob, N, P = len(net.obs_species), net.n_species, net.n_params
        ids = np.array([0, 1, 129, Bn - 1])
        index = {int(L.traj_offset + q): k for k, q in enumerate(ids)}
        ov = [(index[int(t["traj"])], int(t["step"]), int(t["kind"]), int(t["chosen"]))
              for t in ties if int(t["traj"]) in index]
        blk = lambda a: a[L.obs_offset: L.obs_offset + nb * nob * Bn].reshape(nb, nob, Bn).transpose(2, 0, 1)
        r = oracle.run(net, ncfg, net.theta0, net.x0, traj_ids=L.traj_offset + ids, ties=ov, d_obs=blk(dob)[ids],
                       kappa=True, edge_window=EDGE_WINDOW)
        r.edge_window = EDGE_WINDOW
        gpu = {"x_final": xf[L.state_offset: L.state_offset + N * Bn].reshape(N, Bn).T,
               "t_final": tfin[L.traj_offset: L.traj_offset + Bn],
               "steps_done": sd[L.traj_offset: L.traj_offset + Bn],
               "obs": blk(ob)}
        assert_forward_parity(gpu, r, ids, ncfg)
        keep = edge_safe(gpu, r, ids)
        assert keep.all(), (n, keep)
        gq = pp[L.ppt_offset: L.ppt_offset + P * Bn].reshape(P, Bn).T
        assert_grad_parity(gq[ids], r.grad, keep, kappa=r.kappa, T=cfg.temperature)
        tot = gq.astype(np.float64).sum(0)
        mag = np.abs(gq.astype(np.float64)).sum(0)
        dpn = dp.cpu().numpy()[L.param_offset: L.param_offset + P]
        assert np.all(np.abs(dpn - tot) <= 1e-5 * np.abs(tot) + 1e-6 * mag)
