"""The trajectory-major observation layout, the shared dL/dobs of a loss of
ensemble means (Sec. 4.1, Sec. 4.4) and the library's ensemble mean, through
the C ABI.

- Forward and backward in the trajectory-major layout against the FP64 oracle
  with the same bars as the point-major parity tests, and bit for bit against
  the point-major run of the same seeds (the layout moves values, it changes
  no arithmetic).
- A shared dL/dobs block against the oracle fed that block for every
  trajectory, and bit for bit against the point-major backward given the
  block broadcast over the trajectories.
- ssa_obs_mean on observation values the oracle produced, in both layouts,
  against numpy's FP64 mean; fixed summation order (repeat calls agree bit for
  bit); ragged trajectory counts, several networks, a network without
  trajectories."""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import workloads as W

from test_gpu_parity import (_ties_for_oracle, _x0, assert_forward_parity, assert_grad_parity, edge_safe,
                              run_pair)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


CASES = {
    # A + B <-> C on a 24-point grid (the inference's observation), ragged batch
    "abc_grid": (lambda: W.dimerization_abc(),
                 W.RunConfig(seed=5, n_steps=250, obs_kind=W.OBS_GRID, n_bins=24, t_obs=4.5, temperature=0.5,
                             ckpt_every=64), 3000),
    # the ion channel's bin averages: most bins follow the absorbing state
    "channel_bins": (lambda: W.ion_channel_coi(n_channels=3),
                     W.RunConfig(seed=6, n_steps=20, obs_kind=W.OBS_BINS, n_bins=60, t_obs=8.0, temperature=0.2,
                                 ckpt_every=8), 2500),
    # bin averages of three observed species (paths run past t_obs)
    "abc_bins": (lambda: W.dimerization_abc(),
                 W.RunConfig(seed=8, n_steps=200, obs_kind=W.OBS_BINS, n_bins=40, t_obs=3.0, temperature=0.5,
                             ckpt_every=32), 2200),
    # final counts of the dimerisation
    "dimer_final": (lambda: W.dimerization_2a(),
                    W.RunConfig(seed=7, n_steps=300, obs_kind=W.OBS_FINAL, temperature=0.5, ckpt_every=64), 1000),
}


def _d_obs(cfg, nob, B, seed, shared):
    g = np.random.default_rng(seed)
    npts = cfg.n_bins if cfg.obs_kind != W.OBS_FINAL else 1
    if shared:
        v = g.normal(size=(npts, nob, 1))
        d = np.repeat(v, B, axis=2)
    else:
        d = g.normal(size=(npts, nob, B))
    return d if cfg.obs_kind != W.OBS_FINAL else d[0]


def _parity(gpu, r, ids, cfg):
    assert_forward_parity(gpu, r, ids, cfg)
    keep = edge_safe(gpu, r, ids)
    assert keep.mean() > 0.5
    assert_grad_parity(gpu["ppt"][ids], r.grad, keep, kappa=r.kappa, T=cfg.temperature)
    assert_grad_parity(gpu["ppt"][ids][keep].sum(0), r.grad[keep].sum(0), kappa=r.kappa[keep].sum(0),
                       T=cfg.temperature)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("shared", [False, True], ids=["per_traj_dobs", "shared_dobs"])
def test_traj_major_parity(ssa, case, shared):
    mk, cfg, B = CASES[case]
    net = mk()
    nob = len(net.obs_species)
    d_obs = _d_obs(cfg, nob, B, 11, shared)
    g = np.random.default_rng(3)
    sample = np.unique(np.concatenate([[0, 63, 64, B - 1], g.choice(B, 36, replace=False)]))
    tm_cfg = cfg.replace(obs_layout=W.OBS_TRAJ_MAJOR, dobs_shared=shared)
    gpu, r, ids, _ = run_pair(ssa, net, tm_cfg, B, d_obs=d_obs, bwd_mode="tape", sample=sample)
    _parity(gpu, r, ids, tm_cfg)
    # the point-major run of the same seeds with the per-trajectory d_obs
    ref, _, _, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs, bwd_mode="tape", sample=sample[:2])
    assert np.array_equal(gpu["obs"], ref["obs"])
    assert np.array_equal(gpu["x_final"], ref["x_final"])
    if shared and cfg.obs_kind == W.OBS_BINS:
        # whole bins enter through prefix sums of the shared block: the same
        # terms in another order and in FP64
        # (two GPU layouts, not oracle parity: within 1e-5 of each row's scale)
        gd = np.abs(gpu["ppt"].astype(np.float64) - ref["ppt"])
        assert np.all(gd <= 1e-5 * np.abs(ref["ppt"]).max(axis=1, keepdims=True))
        tot = ref["ppt"].astype(np.float64).sum(0)
        assert np.allclose(gpu["d_params"], ref["d_params"], rtol=1e-5,
                           atol=1e-6 * np.abs(ref["ppt"].astype(np.float64)).sum(0).max())
    else:
        assert np.array_equal(gpu["ppt"], ref["ppt"])
        assert np.array_equal(gpu["d_params"], ref["d_params"])


def test_shared_dobs_two_networks(ssa):
    """Two topologies in one handle, each with its own shared bin dL/dobs
    block (the prefix sums are laid out per network): per-trajectory
    gradients against the oracle fed each network's block."""
    nets = [W.ion_channel_coi(n_channels=3), W.dimerization_abc()]
    Bs = [700, 450]
    cfg = W.RunConfig(seed=12, n_steps=60, obs_kind=W.OBS_BINS, n_bins=30, t_obs=5.0, temperature=0.4,
                      ckpt_every=16, obs_layout=W.OBS_TRAJ_MAJOR, dobs_shared=True)
    h = ssa.Net(nets, Bs, t_obs=[5.0, 5.0])
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, Bs)
    g = np.random.default_rng(5)
    blocks = [g.normal(size=(cfg.n_bins, len(n.obs_species))) for n in nets]
    d = torch.tensor(np.concatenate([b.reshape(-1) for b in blocks]), device="cuda")
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 16, bwd_mode="tape")
    dp, ppt = ssa.backward(h, cfg, th, x0, fwd, d, per_traj=True)
    torch.cuda.synchronize()
    ties = fwd.tie_records()
    ppt = ppt.cpu().numpy()
    tf = fwd.t_final.cpu().numpy()
    for k, (net, B) in enumerate(zip(nets, Bs)):
        L = h.layout(k, cfg.obs_kind, cfg.n_bins)
        assert L.mean_offset == sum(cfg.n_bins * len(n.obs_species) for n in nets[:k])
        ids = np.arange(0, B, 7)
        index = {int(q): j for j, q in enumerate(ids)}
        ov = _ties_for_oracle([t for t in ties if L.traj_offset <= t["traj"] < L.traj_offset + B], L.traj_offset,
                              index)
        dn = np.broadcast_to(blocks[k][None], (len(ids),) + blocks[k].shape).copy()
        r = oracle.run(net, cfg.replace(obs_layout=0, dobs_shared=False), net.theta0, net.x0,
                       traj_ids=L.traj_offset + ids, ties=ov, d_obs=dn, kappa=True)
        assert r.n_bad.sum() == 0
        drift = float(np.max(np.abs(tf[L.traj_offset + ids] - r.t_final)))
        keep = r.bin_edge_dist > 50 * max(drift, 1e-12)
        assert keep.mean() > 0.5
        gk = ppt[L.ppt_offset: L.ppt_offset + net.n_params * B].reshape(net.n_params, B).T[ids]
        assert_grad_parity(gk, r.grad, keep, kappa=r.kappa, T=cfg.temperature)


def test_layout_needs_the_specialised_mode(ssa):
    net = W.dimerization_abc()
    B = 64
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    for mode in ("lane", "wave"):
        h = ssa.Net([net], [B], t_obs=[4.0], exec_mode=mode)
        for kw in ({"obs_layout": W.OBS_TRAJ_MAJOR}, {"dobs_shared": True}):
            cfg = W.RunConfig(seed=1, n_steps=10, obs_kind=W.OBS_BINS, n_bins=4, t_obs=4.0, **kw)
            with pytest.raises(ssa.SSAError, match="specialised"):
                ssa.forward(h, cfg, th, x0)


def _oracle_obs(net, cfg, B, seed):
    """Per-trajectory observations of B trajectories from the oracle: [B][W]."""
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(B))
    o = np.asarray(r.obs, np.float64)
    return o.reshape(B, -1)


@pytest.mark.parametrize("layout", [W.OBS_POINT_MAJOR, W.OBS_TRAJ_MAJOR], ids=["point_major", "traj_major"])
def test_obs_mean_of_oracle_values(ssa, layout):
    """Three networks (ragged trajectory counts, the last with none), the
    oracle's bin averages uploaded in the layout under test; the means match
    numpy's to 1e-13, and the empty network's are 0."""
    nets = [W.ion_channel_coi(n_channels=3), W.dimerization_abc(), W.dimerization_2a()]
    Bs = [1000, 333, 0]
    cfg = W.RunConfig(seed=2, n_steps=30, obs_kind=W.OBS_BINS, n_bins=17, t_obs=6.0, obs_layout=layout)
    h = ssa.Net(nets, Bs, t_obs=[6.0, 6.0, 6.0])
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, Bs)
    fwd = ssa.forward(h, cfg, th, x0, keep_ckpt=False, tie_capacity=0)
    blocks, expect = [], []
    for k, (net, B) in enumerate(zip(nets[:2], Bs[:2])):
        v = _oracle_obs(net, cfg.replace(obs_layout=0), B, k)        # [B][W]
        expect.append(v.mean(axis=0))
        blocks.append(v if layout == W.OBS_TRAJ_MAJOR else v.T)
    obs = torch.tensor(np.concatenate([b.reshape(-1) for b in blocks]), device="cuda")
    m1 = ssa.obs_mean(h, fwd, obs=obs).cpu().numpy()
    m2 = ssa.obs_mean(h, fwd, obs=obs).cpu().numpy()
    assert np.array_equal(m1, m2)
    for k in range(len(expect)):
        off = h.layout(k, cfg.obs_kind, cfg.n_bins).mean_offset
        got = m1[off: off + expect[k].size]
        assert np.allclose(got, expect[k], rtol=1e-13, atol=1e-13 * np.abs(expect[k]).max())
    off = h.layout(2, cfg.obs_kind, cfg.n_bins).mean_offset
    assert off + cfg.n_bins == m1.size and np.all(m1[off:] == 0.0)


@pytest.mark.parametrize("layout", [W.OBS_POINT_MAJOR, W.OBS_TRAJ_MAJOR], ids=["point_major", "traj_major"])
def test_obs_mean_large_ragged(ssa, layout):
    """Many chunks and a ragged tail: 100,003 trajectories x 37 values of
    seeded data, against numpy's FP64 mean."""
    net = W.dimerization_abc()
    B, nb = 100_003, 37
    cfg = W.RunConfig(seed=0, n_steps=1, obs_kind=W.OBS_BINS, n_bins=nb, t_obs=1.0, obs_layout=layout)
    h = ssa.Net([net], [B], t_obs=[1.0], obs_species=[[0]])
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    fwd = ssa.forward(h, cfg, th, x0, keep_ckpt=False, tie_capacity=0)
    v = np.random.default_rng(8).normal(loc=3.0, size=(B, nb))
    host = v if layout == W.OBS_TRAJ_MAJOR else v.T
    m = ssa.obs_mean(h, fwd, obs=torch.tensor(np.ascontiguousarray(host).reshape(-1), device="cuda"))
    assert np.allclose(m.cpu().numpy(), v.mean(axis=0), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("bwd_mode,T", [("recompute", 0.5), ("tape", 1.0), ("recompute", 1.0), ("recompute", 0.2)])
def test_shared_bins_backward_variants(ssa, bwd_mode, T):
    """The shared-block bin backward in each choice source (tape, segment
    re-run) and temperature class (1/T = 2, 1, other), against the oracle."""
    net = W.ion_channel_coi(n_channels=4)
    B = 1500
    cfg = W.RunConfig(seed=21, n_steps=24, obs_kind=W.OBS_BINS, n_bins=50, t_obs=6.0, temperature=T,
                      ckpt_every=8, obs_layout=W.OBS_TRAJ_MAJOR, dobs_shared=True)
    d_obs = _d_obs(cfg, len(net.obs_species), B, 4, True)
    g = np.random.default_rng(6)
    sample = np.unique(np.concatenate([[0, B - 1], g.choice(B, 40, replace=False)]))
    gpu, r, ids, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs, bwd_mode=bwd_mode, sample=sample)
    _parity(gpu, r, ids, cfg)


@pytest.mark.parametrize("case", ["channel_bins", "abc_bins", "abc_grid"])
def test_ensemble_mean_forward(ssa, case):
    """The forward that keeps only the ensemble means of the bins or grid
    points: against the mean of the oracle's values over every trajectory
    (the same near-tie choices), against the trajectory-major forward of the
    same seeds reduced by ssa_obs_mean, repeatable bit for bit, and followed
    by the same backward as that forward."""
    mk, cfg, B = CASES[case]
    net = mk()
    nob = len(net.obs_species)
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    ens = cfg.replace(obs_layout=W.OBS_ENSEMBLE_MEAN, dobs_shared=True)
    f1 = ssa.forward(h, ens, th, x0, tie_capacity=1 << 16, bwd_mode="tape")
    m1 = f1.obs.cpu().numpy()[: cfg.n_bins * nob].reshape(cfg.n_bins, nob)
    f2 = ssa.forward(h, ens, th, x0, tie_capacity=1 << 16, bwd_mode="tape")
    assert np.array_equal(f2.obs.cpu().numpy(), f1.obs.cpu().numpy())
    # the oracle, every trajectory
    ties = f1.tie_records()
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(B), ties=_ties_for_oracle(ties))
    assert r.n_bad.sum() == 0
    assert np.array_equal(f1.x_final.cpu().numpy().reshape(net.n_species, B).T, r.x_final)
    drift = float(np.max(np.abs(f1.t_final.cpu().numpy() - r.t_final)))
    ref = np.asarray(r.obs, np.float64).reshape(B, cfg.n_bins, nob).mean(axis=0)
    big = float(np.abs(r.obs).max())
    # the per-trajectory bars of the parity tests (bins: a count jump times
    # the clock drift over the bin width; grid: relative to the counts' scale)
    atol = (4.0 * big * drift * cfg.n_bins / cfg.t_obs if cfg.obs_kind == W.OBS_BINS else 1e-5 * big) + 1e-12
    assert np.all(np.abs(m1 - ref) <= 1e-5 * np.abs(ref) + atol)
    # the trajectory-major forward of the same seeds, reduced by the library
    tm = cfg.replace(obs_layout=W.OBS_TRAJ_MAJOR, dobs_shared=True)
    f3 = ssa.forward(h, tm, th, x0, tie_capacity=1 << 16, bwd_mode="tape")
    m3 = ssa.obs_mean(h, f3).cpu().numpy().reshape(cfg.n_bins, nob)
    # partly covered bins and grid values are summed in fixed point: at most
    # 2^-33 absolute
    assert np.allclose(m1, m3, rtol=1e-12, atol=2.0 ** -32)
    # the backward reads checkpoints and tape only: the same after both forwards
    d = torch.tensor(np.random.default_rng(2).normal(size=cfg.n_bins * nob), device="cuda")
    g1 = ssa.backward(h, ens, th, x0, f1, d, per_traj=True)[1]
    g3 = ssa.backward(h, tm, th, x0, f3, d, per_traj=True)[1]
    assert torch.equal(g1, g3)


def test_ensemble_mean_forward_networks_and_limits(ssa):
    """Two topologies and an empty network in one handle; the combinations
    the ensemble-mean forward does not run are refused before any launch."""
    nets = [W.ion_channel_coi(n_channels=2), W.dimerization_abc(), W.dimerization_2a()]
    Bs = [777, 130, 0]
    cfg = W.RunConfig(seed=13, n_steps=40, obs_kind=W.OBS_BINS, n_bins=25, t_obs=5.0, temperature=0.5,
                      ckpt_every=16, obs_layout=W.OBS_ENSEMBLE_MEAN, dobs_shared=True)
    h = ssa.Net(nets, Bs, t_obs=[5.0, 5.0, 5.0])
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, Bs)
    f = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 16)
    m = f.obs.cpu().numpy()
    ft = ssa.forward(h, cfg.replace(obs_layout=W.OBS_TRAJ_MAJOR), th, x0, tie_capacity=1 << 16)
    mt = ssa.obs_mean(h, ft).cpu().numpy()
    assert m.size >= h.mean_total(cfg.obs_kind, cfg.n_bins)
    n = h.mean_total(cfg.obs_kind, cfg.n_bins)
    assert np.allclose(m[:n], mt[:n], rtol=1e-12, atol=2.0 ** -32)
    off = h.layout(2, cfg.obs_kind, cfg.n_bins).mean_offset
    assert np.all(m[off:n] == 0.0)
    with pytest.raises(ssa.SSAError, match="means already"):
        ssa.obs_mean(h, f)
    f0 = ssa.forward(h, cfg.replace(dobs_shared=False), th, x0, tie_capacity=0)
    with pytest.raises(ssa.SSAError, match="shared d_obs"):
        ssa.backward(h, cfg, th, x0, f0, torch.zeros(n, dtype=torch.float64, device="cuda"))
    for bad, msg in ((cfg.replace(obs_kind=W.OBS_FINAL), "bins or grid points only"),
                     (cfg.replace(selection=W.SELECT_INVERSE_CDF), "per-trajectory"),
                     (cfg.replace(n_bins=1001), "1000")):
        with pytest.raises(ssa.SSAError, match=msg):
            ssa.forward(h, bad, th, x0)
    hl = ssa.Net(nets[:1], Bs[:1], t_obs=[5.0], exec_mode="lane")
    with pytest.raises(ssa.SSAError, match="specialised"):
        ssa.forward(hl, cfg, th[: nets[0].n_params], _x0(nets[:1], Bs[:1]))
