"""Parity of the wave-mode kernels (one trajectory per group of lanes, one
persistent launch for a whole batch of networks) with the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
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


@pytest.fixture(params=[1, 0], ids=["split", "one_launch"])
def wave_mode(request):
    """Wave mode, one launch per lane-group width or one launch for the batch."""
    return request.param


def run_batch(ssa, nets, B, cfg, d_obs_fn=None, bwd_mode="auto", t_obs=None, wave_split=-1):
    h = ssa.Net(nets, B, t_obs=t_obs, exec_mode="wave", wave_split=wave_split)
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, B)
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 16, bwd_mode=bwd_mode)
    d_obs = None
    ppt = None
    if d_obs_fn is not None:
        d_obs = d_obs_fn(h)
        dp, ppt = ssa.backward(h, cfg, th, x0, fwd, torch.tensor(d_obs, device="cuda"), per_traj=True)
        ppt = ppt.cpu().numpy()
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    return h, fwd, d_obs, ppt


def check_batch(h, fwd, nets, B, cfg, d_obs=None, ppt=None):
    ties = fwd.tie_records()
    xf = fwd.x_final.cpu().numpy()
    sd = fwd.steps_done.cpu().numpy()
    tf = fwd.t_final.cpu().numpy()
    obs = fwd.obs.cpu().numpy()
    bins = cfg.obs_kind == W.OBS_BINS
    for n, (net, b) in enumerate(zip(nets, B)):
        L = h.layout(n, cfg.obs_kind, cfg.n_bins)
        nob = len(net.obs_species)
        ov = _ties_for_oracle([t for t in ties if L.traj_offset <= t["traj"] < L.traj_offset + b], L.traj_offset)
        dob = None
        if d_obs is not None:
            blk = d_obs[L.obs_offset: L.obs_offset + (cfg.n_bins if bins else 1) * nob * b]
            dob = (blk.reshape(cfg.n_bins, nob, b).transpose(2, 0, 1) if bins else blk.reshape(nob, b).T)
        ew = EDGE_WINDOW if bins else 0.0       # the wave forward logs the side of close bin edges
        r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=L.traj_offset + np.arange(b), ties=ov, d_obs=dob,
                       kappa=dob is not None, edge_window=ew)
        r.edge_window = ew
        ob = obs[L.obs_offset: L.obs_offset + (cfg.n_bins if bins else 1) * nob * b]
        gpu = {"x_final": xf[L.state_offset: L.state_offset + net.n_species * b].reshape(net.n_species, b).T,
               "t_final": tf[L.traj_offset: L.traj_offset + b],
               "steps_done": sd[L.traj_offset: L.traj_offset + b],
               "obs": ob.reshape(cfg.n_bins, nob, b).transpose(2, 0, 1) if bins else ob.reshape(nob, b).T}
        ids = np.arange(b)
        assert_forward_parity(gpu, r, ids, cfg)
        if ppt is not None:
            g = ppt[L.ppt_offset: L.ppt_offset + net.n_params * b].reshape(net.n_params, b).T
            keep = edge_safe(gpu, r, ids)
            assert keep.all()
            assert_grad_parity(g, r.grad, keep, kappa=r.kappa, T=cfg.temperature)


def test_wave_small_batch_forward(ssa, wave_mode):
    nets = W.random_network_batch(6, seed=5, n_range=(4, 16), m_range=(8, 32))
    B = [64, 37, 128, 1, 90, 65]
    cfg = W.RunConfig(seed=9, n_steps=400, obs_kind=W.OBS_FINAL)
    h, fwd, _, _ = run_batch(ssa, nets, B, cfg, wave_split=wave_mode)
    check_batch(h, fwd, nets, B, cfg)


def test_wave_large_networks_forward(ssa, wave_mode):
    nets = W.random_network_batch(5, seed=21, n_range=(40, 64), m_range=(200, 256))
    B = [17, 8, 33, 5, 12]
    cfg = W.RunConfig(seed=4, n_steps=300, obs_kind=W.OBS_FINAL)
    h, fwd, _, _ = run_batch(ssa, nets, B, cfg, wave_split=wave_mode)
    check_batch(h, fwd, nets, B, cfg)


@pytest.mark.parametrize("mode", ["tape", "recompute"])
def test_wave_gradients_random_batch(ssa, wave_mode, mode):
    nets = W.random_network_batch(4, seed=13, n_range=(4, 24), m_range=(8, 100))
    B = [40, 23, 64, 9]
    pilot = [oracle.run(n, W.RunConfig(seed=1, n_steps=300, purpose=2), n.theta0, n.x0,
                        traj_ids=np.arange(8)) for n in nets]
    t_obs = [float(np.min(r.t_final)) * 0.8 for r in pilot]
    cfg = W.RunConfig(seed=3, n_steps=300, obs_kind=W.OBS_BINS, n_bins=4, t_obs=1.0, temperature=0.5,
                      ckpt_every=64)
    g = np.random.default_rng(8)

    def d_obs_fn(h):
        return g.normal(size=h.obs_total(cfg.obs_kind, cfg.n_bins))

    h, fwd, d_obs, ppt = run_batch(ssa, nets, B, cfg, d_obs_fn, bwd_mode=mode, t_obs=t_obs,
                                   wave_split=wave_mode)
    check_batch_windows(h, fwd, nets, B, cfg, t_obs, d_obs, ppt)


def check_batch_windows(h, fwd, nets, B, cfg, t_obs, d_obs, ppt, layouts=None):
    """check_batch with a per-network observation window (the oracle runs
    network by network, each with its own window).  `layouts` gives each
    checked network's offsets when they are not networks 0, 1, ... of h."""
    ties = fwd.tie_records()
    xf = fwd.x_final.cpu().numpy()
    sd = fwd.steps_done.cpu().numpy()
    tf = fwd.t_final.cpu().numpy()
    obs = fwd.obs.cpu().numpy()
    for n, (net, b) in enumerate(zip(nets, B)):
        c = cfg.replace(t_obs=t_obs[n])
        L = layouts[n] if layouts is not None else h.layout(n, c.obs_kind, c.n_bins)
        nob = len(net.obs_species)
        ov = _ties_for_oracle([t for t in ties if L.traj_offset <= t["traj"] < L.traj_offset + b], L.traj_offset)
        blk = d_obs[L.obs_offset: L.obs_offset + c.n_bins * nob * b]
        dob = blk.reshape(c.n_bins, nob, b).transpose(2, 0, 1)
        r = oracle.run(net, c, net.theta0, net.x0, traj_ids=L.traj_offset + np.arange(b), ties=ov, d_obs=dob,
                       kappa=True, edge_window=EDGE_WINDOW)
        r.edge_window = EDGE_WINDOW
        ob = obs[L.obs_offset: L.obs_offset + c.n_bins * nob * b]
        gpu = {"x_final": xf[L.state_offset: L.state_offset + net.n_species * b].reshape(net.n_species, b).T,
               "t_final": tf[L.traj_offset: L.traj_offset + b],
               "steps_done": sd[L.traj_offset: L.traj_offset + b],
               "obs": ob.reshape(c.n_bins, nob, b).transpose(2, 0, 1)}
        ids = np.arange(b)
        assert_forward_parity(gpu, r, ids, c)
        gg = ppt[L.ppt_offset: L.ppt_offset + net.n_params * b].reshape(net.n_params, b).T
        keep = edge_safe(gpu, r, ids)
        assert keep.all()
        assert_grad_parity(gg, r.grad, keep, kappa=r.kappa, T=c.temperature)


def test_wave_dimer_gradients(ssa, wave_mode):
    net = W.dimerization_2a()
    B = 200
    cfg = W.RunConfig(seed=1, n_steps=1500, obs_kind=W.OBS_BINS, n_bins=20, t_obs=300.0,
                      temperature=0.5, ckpt_every=64)
    g = np.random.default_rng(2)
    d_obs = g.normal(size=(cfg.n_bins, 1, B))
    gpu, r, ids, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs, exec_mode="wave")
    assert_forward_parity(gpu, r, ids, cfg)
    keep = edge_safe(gpu, r, ids)
    assert_grad_parity(gpu["ppt"], r.grad, keep, kappa=r.kappa, T=cfg.temperature)


def test_wave_backward_deterministic(ssa, wave_mode):
    nets = W.random_network_batch(3, seed=2, n_range=(8, 32), m_range=(40, 120))
    B = [50, 50, 50]
    cfg = W.RunConfig(seed=5, n_steps=200, obs_kind=W.OBS_FINAL, ckpt_every=32)
    h = ssa.Net(nets, B, exec_mode="wave", wave_split=wave_mode)
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, B)
    d = torch.randn(h.obs_total(cfg.obs_kind, 0), dtype=torch.float64, device="cuda")
    outs = []
    for _ in range(2):
        f = ssa.forward(h, cfg, th, x0)
        dp, ppt = ssa.backward(h, cfg, th, x0, f, d, per_traj=True)
        outs.append((f.x_final.clone(), dp.clone(), ppt.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("lanes,m_range", [(8, (20, 60)), (16, (40, 120)), (32, (90, 250)), (64, (300, 500))],
                         ids=["w8", "w16", "w32", "w64"])
def test_wave_narrow_groups_gradients(ssa, wave_mode, lanes, m_range):
    """Groups capped at `lanes` lanes: networks that need more Philox blocks
    than lanes draw two per lane (8 channel slots), several trajectories per
    wavefront.  The fired channels are those of the default width; clocks and
    gradients agree with the oracle at the usual bars."""
    nets = W.random_network_batch(4, seed=31 + lanes, n_range=(4, 40), m_range=m_range)
    B = [24, 9, 33, 16]
    pilot = [oracle.run(n, W.RunConfig(seed=1, n_steps=200, purpose=2), n.theta0, n.x0,
                        traj_ids=np.arange(8)) for n in nets]
    t_obs = [float(np.min(r.t_final)) * 0.8 for r in pilot]
    cfg = W.RunConfig(seed=6, n_steps=200, obs_kind=W.OBS_BINS, n_bins=4, t_obs=1.0, temperature=0.5,
                      ckpt_every=64)
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, B)
    h = ssa.Net(nets, B, t_obs=t_obs, exec_mode="wave", wave_split=wave_mode, wave_lanes=lanes)
    d_obs = np.random.default_rng(3).normal(size=h.obs_total(cfg.obs_kind, cfg.n_bins))
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 16)
    dp, ppt = ssa.backward(h, cfg, th, x0, fwd, torch.tensor(d_obs, device="cuda"), per_traj=True)
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    check_batch_windows(h, fwd, nets, B, cfg, t_obs, d_obs, ppt.cpu().numpy())
    h0 = ssa.Net(nets, B, t_obs=t_obs, exec_mode="wave", wave_split=wave_mode)
    f0 = ssa.forward(h0, cfg, th, x0, tie_capacity=1 << 16)
    torch.cuda.synchronize()
    assert torch.equal(fwd.steps_done, f0.steps_done)
    assert torch.equal(fwd.x_final, f0.x_final)
    assert torch.allclose(fwd.t_final, f0.t_final, rtol=1e-6, atol=0)


def test_wave_lanes_values(ssa):
    nets = W.random_network_batch(2, seed=3, n_range=(4, 8), m_range=(100, 110))
    with pytest.raises(ssa.SSAError):
        ssa.Net(nets, [8, 8], exec_mode="wave", wave_lanes=12)
    ssa.Net(nets, [8, 8], exec_mode="wave", wave_lanes=8)         # 26+ blocks > 2 x 8: the library's width
    ssa.Net(nets, [8, 8], exec_mode="wave", wave_lanes=16)        # two blocks on each of 16 lanes


def test_wave_over_256_channels_recompute(ssa, wave_mode):
    """Channel indices past 255 in the backward's recovered choices (the
    recompute path keeps a segment's channels in LDS; the tape path is run
    by the width test above)."""
    nets = W.random_network_batch(3, seed=77, n_range=(10, 40), m_range=(260, 500))
    assert all(n.n_reactions > 256 for n in nets)
    B = [20, 13, 31]
    pilot = [oracle.run(n, W.RunConfig(seed=1, n_steps=150, purpose=2), n.theta0, n.x0,
                        traj_ids=np.arange(8)) for n in nets]
    t_obs = [float(np.min(r.t_final)) * 0.8 for r in pilot]
    cfg = W.RunConfig(seed=2, n_steps=150, obs_kind=W.OBS_BINS, n_bins=3, t_obs=1.0, temperature=0.5,
                      ckpt_every=64)
    g = np.random.default_rng(5)

    def d_obs_fn(h):
        return g.normal(size=h.obs_total(cfg.obs_kind, cfg.n_bins))

    h, fwd, d_obs, ppt = run_batch(ssa, nets, B, cfg, d_obs_fn, bwd_mode="recompute", t_obs=t_obs,
                                   wave_split=wave_mode)
    check_batch_windows(h, fwd, nets, B, cfg, t_obs, d_obs, ppt)


def test_wave_empty_network_in_batch(ssa, wave_mode):
    """A network with no trajectories between two others: the persistent
    queue skips it, the others match the oracle, and its parameters get a zero
    gradient."""
    nets = W.random_network_batch(3, seed=41, n_range=(4, 20), m_range=(20, 90))
    B = [16, 0, 9]
    pilot = [oracle.run(n, W.RunConfig(seed=1, n_steps=200, purpose=2), n.theta0, n.x0,
                        traj_ids=np.arange(8)) for n in nets]
    t_obs = [float(np.min(r.t_final)) * 0.8 for r in pilot]
    cfg = W.RunConfig(seed=8, n_steps=200, obs_kind=W.OBS_BINS, n_bins=4, t_obs=1.0, temperature=0.5,
                      ckpt_every=64)
    g = np.random.default_rng(9)

    def d_obs_fn(h):
        return g.normal(size=h.obs_total(cfg.obs_kind, cfg.n_bins))

    h, fwd, d_obs, ppt = run_batch(ssa, nets, B, cfg, d_obs_fn, bwd_mode="tape", t_obs=t_obs,
                                   wave_split=wave_mode)
    keep = [n for n, b in enumerate(B) if b > 0]
    # the oracle checks network by network; the empty one has nothing to compare
    check_batch_windows(h, fwd, [nets[n] for n in keep], [B[n] for n in keep], cfg, [t_obs[n] for n in keep],
                        d_obs, ppt, layouts=[h.layout(n, cfg.obs_kind, cfg.n_bins) for n in keep])
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    dp, _ = ssa.backward(h, cfg, th, _x0(nets, B), fwd, torch.tensor(d_obs, device="cuda"), per_traj=True)
    off = sum(n.n_params for n in nets[:1])
    assert np.all(dp.cpu().numpy()[off:off + nets[1].n_params] == 0.0)
