"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars (taken from the method's requirements):
- copy numbers, step counts and fired channels: bit-exact, except at steps the
  GPU logged as near-ties where the oracle's own FP64 relative margin is
  <= 1e-6 (the oracle then adopts the GPU's choice and must agree after);
- clock, waiting times, propensities, bin averages: relative 1e-5;
- gradients, per trajectory and summed: ||g - g*||_2 <= 1e-5 ||g*||_2, and
  every component within 1e-5 of itself unless the terms it sums cancel, in
  which case within the FP32 rounding of the sum of their magnitudes
  (c(T) 2^-24 kappa_i, kappa from the oracle), and never looser than 1e-5 of
  the largest component (grad_bar).  Per-trajectory checks leave out
  trajectories with an event time too close to a bin edge (edge_safe): there
  the bin assignment of a derivative term may legitimately differ between an
  FP32 and an FP64 clock.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


# Relative bin-edge window of the specialised forward's edge log (its kind-2
# tie records): for an event time inside it, the oracle's adjoint takes the
# side of the edge the GPU's clock took, as it takes the GPU's choice at a
# near-tie.
EDGE_WINDOW = 4e-7


def _x0(nets, n_traj):
    parts = [np.repeat(n.x0[:, None], b, axis=1).reshape(-1) for n, b in zip(nets, n_traj)]
    return torch.tensor(np.concatenate(parts), dtype=torch.int32, device="cuda")


def _ties_for_oracle(recs, traj_offset=0, traj_index=None):
    """GPU tie records -> oracle overrides (local traj index, step, kind, val)."""
    out = []
    for t in recs:
        q = int(t["traj"]) - traj_offset
        if traj_index is not None:
            if q not in traj_index:
                continue
            q = traj_index[q]
        out.append((q, int(t["step"]), int(t["kind"]), int(t["chosen"])))
    return out


def run_pair(ssa, net, cfg, B, theta=None, d_obs=None, bwd_mode="auto", sample=None, per_traj=True,
             exec_mode="auto"):
    """GPU forward (+backward) over B trajectories and the oracle on `sample`
    trajectory ids (default: all).  d_obs is [n_bins][n_obs][B] (bins, grid)
    or [n_obs][B] (final counts) whatever cfg.obs_layout is; with
    cfg.dobs_shared every trajectory's column must be the same."""
    theta = net.theta0 if theta is None else theta
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs], exec_mode=exec_mode)
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    x0 = _x0([net], [B])
    fwd = ssa.forward(h, cfg, th, x0, keep_ckpt=d_obs is not None, tie_capacity=1 << 16,
                      bwd_mode=bwd_mode)
    bins = cfg.obs_kind in (W.OBS_BINS, W.OBS_GRID)     # [n_bins][n_obs][B] layouts
    nob = len(net.obs_species)
    gpu = {}
    tm = cfg.obs_layout == W.OBS_TRAJ_MAJOR
    if d_obs is not None:
        dl = np.asarray(d_obs, np.float64)
        if not bins:
            dl = dl[None]
        if cfg.dobs_shared:
            assert np.array_equal(dl, np.broadcast_to(dl[:, :, :1], dl.shape))
            dl = dl[:, :, 0]
        elif tm:
            dl = dl.transpose(2, 0, 1)
        dd = torch.tensor(np.ascontiguousarray(dl).reshape(-1), device="cuda")
        dp, ppt = ssa.backward(h, cfg, th, x0, fwd, dd, per_traj=True)
        gpu["d_params"] = dp.cpu().numpy()
        gpu["ppt"] = ppt.cpu().numpy().reshape(net.n_params, B).T
    torch.cuda.synchronize()
    assert ssa.device_status(h) == 0
    ties = fwd.tie_records()
    N = net.n_species
    gpu["x_final"] = fwd.x_final.cpu().numpy().reshape(N, B).T
    gpu["t_final"] = fwd.t_final.cpu().numpy()
    gpu["steps_done"] = fwd.steps_done.cpu().numpy()
    obs = fwd.obs.cpu().numpy()
    npts = cfg.n_bins if bins else 1
    if tm:
        o = obs[: npts * nob * B].reshape(B, npts, nob)
        gpu["obs"] = o if bins else o[:, 0, :]
    else:
        gpu["obs"] = (obs[: cfg.n_bins * nob * B].reshape(cfg.n_bins, nob, B).transpose(2, 0, 1) if bins
                      else obs[: nob * B].reshape(nob, B).T)
    gpu["ties"] = ties
    ids = np.arange(B) if sample is None else np.asarray(sample)
    index = {int(q): k for k, q in enumerate(ids)}
    ov = _ties_for_oracle(ties, 0, index)
    oracle_dobs = None
    if d_obs is not None:
        oracle_dobs = (np.transpose(d_obs, (2, 0, 1))[ids] if bins else np.asarray(d_obs).T[ids])
    ew = EDGE_WINDOW if cfg.obs_kind == W.OBS_BINS else 0.0      # every mode logs the side of close edges
    r = oracle.run(net, cfg, theta, net.x0, traj_ids=ids, ties=ov, d_obs=oracle_dobs,
                   kappa=oracle_dobs is not None, edge_window=ew)
    r.edge_window = ew
    return gpu, r, ids, h


def clock_drift(gpu, r, ids):
    """Largest |t_gpu - t_oracle| at the end of the paths: the FP32 waiting
    times make the GPU's event times drift from the FP64 ones by about this."""
    return float(np.max(np.abs(gpu["t_final"][ids] - r.t_final))) if len(ids) else 0.0


def edge_safe(gpu, r, ids, factor=50.0):
    """Trajectories whose event times all stay farther from every bin edge than
    `factor` times the clock drift: both sides put each time-derivative term
    in the same bin.  Every trajectory, when the oracle took the GPU's side of
    the edges from its edge log (r.edge_window > 0)."""
    if getattr(r, "edge_window", 0.0) > 0.0:
        return np.ones(len(ids), bool)
    return r.bin_edge_dist > factor * max(clock_drift(gpu, r, ids), 1e-12)


def assert_forward_parity(gpu, r, ids, cfg=None):
    assert r.n_bad.sum() == 0, "a GPU/oracle disagreement outside a logged near-tie"
    assert np.array_equal(gpu["steps_done"][ids], r.steps_done)
    assert np.array_equal(gpu["x_final"][ids], r.x_final)
    assert np.allclose(gpu["t_final"][ids], r.t_final, rtol=1e-5, atol=0)
    o = gpu["obs"][ids]
    # A bin average moves by (count jump) * (time shift) / (bin width) when an
    # event time shifts, so small bin values get an absolute allowance tied
    # to the measured clock drift.
    atol = 1e-12
    if cfg is not None and cfg.obs_kind == W.OBS_BINS:
        jump = max(1.0, float(np.abs(r.x_final).max()))
        atol = 4.0 * jump * max(clock_drift(gpu, r, ids), 1e-15) * cfg.n_bins / cfg.t_obs + 1e-12
    if cfg is not None and cfg.obs_kind == W.OBS_GRID:
        # an interpolated value moves by (count jump) * (clock shift) / (waiting
        # time) when the event times shift: relative to the counts' scale
        atol = 1e-5 * float(np.abs(r.obs).max()) + 1e-12
    err = np.abs(o - r.obs)
    bad = err > 1e-5 * np.abs(r.obs) + atol
    assert not bad.any(), (int(bad.sum()), float(err.max()), atol, np.argwhere(bad)[:3])


# Rounding constant of the GPU's gradient against the oracle's conditioning
# kappa: the adjoint algebra of a term takes about a dozen FP32 roundings, and
# the ratio-form soft sample y~ ~ (r_ref / r_j)^(1/T) carries a relative error
# of about 16 units of 2^-24 divided by T (-ln u within 5 units, a_j within 3,
# one reciprocal, each ratio formed twice).
def gpu_rounding_constant(T: float) -> float:
    return 32.0 + 32.0 / T


# worst ratio |g - g*| / (2^-24 kappa) seen by assert_grad_parity in this process
KAPPA_RATIO = {"max": 0.0, "n": 0}


def grad_bar(ref, kappa=None, T=None, rtol=1e-5):
    """Per-component bar of a gradient (rows = trajectories or sums):
    |g_i - g*_i| <= min(rtol ||g*||_inf, max(rtol |g*_i|, c(T) 2^-24 kappa_i)),
    i.e. within rtol of the component itself unless its terms cancel, and then
    within the FP32 rounding of the sum of their magnitudes, never looser than
    rtol of the row's largest component.  Without kappa (gene network), S18's
    floor of 1e-2 of the largest component replaces the rounding term."""
    ref = np.atleast_2d(ref)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    if kappa is None:
        floor = 1e-2 * rtol * scale
    else:
        floor = gpu_rounding_constant(T) * 2.0 ** -24 * np.atleast_2d(kappa)
    return np.minimum(rtol * scale, np.maximum(rtol * np.abs(ref), floor))


def assert_grad_parity(gpu_g, ref, keep=None, rtol=1e-5, kappa=None, T=None):
    """Gradient parity per row (a trajectory, or a sum of trajectories):
    every component within grad_bar, and ||g - g*||_2 <= rtol ||g*||_2."""
    g = np.atleast_2d(np.asarray(gpu_g, np.float64))
    r = np.atleast_2d(np.asarray(ref, np.float64))
    k = None if kappa is None else np.atleast_2d(np.asarray(kappa, np.float64))
    if keep is not None:
        g, r = g[keep], r[keep]
        k = None if k is None else k[keep]
    err = np.abs(g - r)
    bar = grad_bar(r, k, T, rtol)
    bad = err > bar
    assert not bad.any(), (np.argwhere(bad)[:5], g[bad][:5], r[bad][:5], bar[bad][:5])
    nrm = np.linalg.norm(g - r, axis=1)
    assert np.all(nrm <= rtol * np.linalg.norm(r, axis=1)), (nrm, np.linalg.norm(r, axis=1))
    if k is not None and k.size:
        ratio = err / np.where(k > 0, 2.0 ** -24 * k, np.inf)
        KAPPA_RATIO["max"] = max(KAPPA_RATIO["max"], float(ratio.max()))
        KAPPA_RATIO["n"] += int(g.shape[0])


# ---------------------------------------------------------------------------
def test_philox_matches_oracle(ssa):
    g = np.random.default_rng(5)
    ck = g.integers(0, 2 ** 32, size=(4096, 6), dtype=np.uint64).astype(np.uint32)
    ck[:4] = [[0, 0, 0, 0, 0, 0], [2 ** 32 - 1] * 6, [1, 2, 3, 4, 5, 6], [7, 0, 9, 1 << 24, 3, 0]]
    got = ssa.selftest_philox(ck)
    ref = np.array([oracle.philox4x32_10(c[:4], c[4:]) for c in ck], np.uint32)
    assert np.array_equal(got, ref)


def test_neglog_exhaustive_lattice(ssa):
    """The GPU's FP32 -ln(u) over all 2^23 lattice points vs FP64: relative
    error at most 3e-7 (about 2.5 units of 2^-23).  The near-tie window of
    the selection (2e-6) is twice the worst-case relative error of
    r_j = E_j / a_j built from this bound, one reciprocal and the propensity
    products."""
    n = 1 << 23
    e = ssa.selftest_neglog(0, n).cpu().numpy().astype(np.float64)
    m = np.arange(n, dtype=np.float64)
    ref = -np.log((2 * m + 1) * 2.0 ** -24)
    rel = np.abs(e - ref) / ref
    assert np.all(np.isfinite(e)) and np.all(e > 0)
    assert rel.max() <= 3e-7, (rel.max(), int(rel.argmax()))


def test_dimer_forward_t_end_1024(ssa):
    """2A<->A2, kf=1e-3, kb=0.1, A(0)=100, 1,024 trajectories to t_end=50: every
    trajectory, full length."""
    wl = W.dimer_forward_1k()
    gpu, r, ids, _ = run_pair(ssa, wl.net, wl.cfg, wl.n_traj)
    assert_forward_parity(gpu, r, ids, wl.cfg)
    assert np.all(gpu["x_final"][:, 0] + 2 * gpu["x_final"][:, 1] == 100)
    assert np.all(gpu["t_final"] <= 50.0)


def test_step_batch_matches_oracle_trace(ssa):
    net = W.oscillator()
    B, steps = 100, 40
    cfg = W.RunConfig(seed=3, n_steps=steps)
    h = ssa.Net([net], [B])
    th = torch.tensor(net.theta0, device="cuda")
    x = _x0([net], [B])
    t = torch.zeros(B, dtype=torch.float64, device="cuda")
    traces = [oracle.trace(net, cfg, net.theta0, net.x0, traj_id=i, cap=steps) for i in range(B)]
    for k in range(steps):
        chosen, tau, a = ssa.step_batch(h, cfg, th, x, t, k, want_a=True)
        ch = chosen.cpu().numpy()
        ta = tau.cpu().numpy()
        aa = a.cpu().numpy().reshape(net.n_reactions, B).T
        for i in range(B):
            tr = traces[i]
            if k < len(tr.j):
                if tr.margin[k] > 1e-6:
                    assert ch[i] == tr.j[k], (k, i)
                assert abs(ta[i] - tr.tau[k]) <= 1e-5 * tr.tau[k]
                assert np.allclose(aa[i], tr.a[k], rtol=1e-5, atol=0)
    xf = x.cpu().numpy().reshape(net.n_species, B).T
    for i in range(B):
        assert np.array_equal(xf[i], traces[i].X[-1])


@pytest.mark.parametrize("B", [1, 63, 64, 200])
def test_ragged_batches_and_edge_sizes(ssa, B):
    net = W.dimerization_abc()
    cfg = W.RunConfig(seed=11, n_steps=300, obs_kind=W.OBS_BINS, n_bins=3, t_obs=2.0)
    gpu, r, ids, _ = run_pair(ssa, net, cfg, B)
    assert_forward_parity(gpu, r, ids, cfg)


def test_zero_steps_and_absorbing(ssa):
    net = W.ion_channel_coi()
    cfg = W.RunConfig(seed=2, n_steps=0, obs_kind=W.OBS_BINS, n_bins=4, t_obs=3.0)
    gpu, r, ids, _ = run_pair(ssa, net, cfg, 70)
    assert_forward_parity(gpu, r, ids, cfg)
    assert np.all(gpu["steps_done"] == 0)
    cfg = cfg.replace(n_steps=500)
    gpu, r, ids, _ = run_pair(ssa, net, cfg, 130)
    assert_forward_parity(gpu, r, ids, cfg)
    assert np.all(gpu["x_final"][:, 2] == 2) and np.all(gpu["steps_done"] < 500)


@pytest.mark.parametrize("exec_mode", ["spec", "lane"])
@pytest.mark.parametrize("mode", ["tape", "recompute"])
def test_dimer_gradients_small(ssa, mode, exec_mode):
    net = W.dimerization_2a()
    B = 300
    cfg = W.RunConfig(seed=1, n_steps=1500, obs_kind=W.OBS_BINS, n_bins=20, t_obs=300.0,
                      temperature=0.5, ckpt_every=64)
    g = np.random.default_rng(2)
    d_obs = g.normal(size=(cfg.n_bins, 1, B))
    gpu, r, ids, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs, bwd_mode=mode, exec_mode=exec_mode)
    assert_forward_parity(gpu, r, ids, cfg)
    keep = edge_safe(gpu, r, ids)
    assert keep.mean() > 0.8
    assert_grad_parity(gpu["ppt"], r.grad, keep, kappa=r.kappa, T=cfg.temperature)
    assert_grad_parity(gpu["ppt"][keep].sum(0), r.grad[keep].sum(0), kappa=r.kappa[keep].sum(0),
                       T=cfg.temperature)
    # the reduction: d_params is the FP64 sum of the per-trajectory partials,
    # rounded once to FP32 (the per-trajectory values are FP32 roundings of them)
    ppt64 = gpu["ppt"].astype(np.float64)
    assert np.all(np.abs(gpu["d_params"] - ppt64.sum(0)) <=
                  2.0 ** -23 * np.abs(ppt64.sum(0)) + 2.0 ** -24 * np.abs(ppt64).sum(0))
    tot = r.grad.sum(0)
    assert np.allclose(gpu["d_params"], tot, rtol=1e-5, atol=1e-5 * np.abs(tot).max())


def test_oscillator_gradients_small(ssa):
    net = W.oscillator()
    B = 128
    cfg = W.RunConfig(seed=4, n_steps=3000, obs_kind=W.OBS_FINAL, temperature=0.5, ckpt_every=256)
    pilot = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(16))
    t_obs = float(np.percentile(pilot.t_final, 1)) * 0.9
    cfg = cfg.replace(obs_kind=W.OBS_BINS, n_bins=16, t_obs=t_obs)
    g = np.random.default_rng(3)
    d_obs = g.normal(size=(cfg.n_bins, 1, B))
    gpu, r, ids, _ = run_pair(ssa, net, cfg, B, d_obs=d_obs)
    assert_forward_parity(gpu, r, ids, cfg)
    keep = edge_safe(gpu, r, ids)
    assert keep.mean() > 0.8
    assert_grad_parity(gpu["ppt"], r.grad, keep, kappa=r.kappa, T=cfg.temperature)
    assert_grad_parity(gpu["ppt"][keep].sum(0), r.grad[keep].sum(0), kappa=r.kappa[keep].sum(0),
                       T=cfg.temperature)


@pytest.mark.parametrize("exec_mode", ["spec", "lane"])
def test_random_networks_batch_forward(ssa, exec_mode):
    nets = W.random_network_batch(6, seed=5, n_range=(4, 16), m_range=(8, 32))
    B = [64, 37, 128, 1, 90, 65]
    cfg = W.RunConfig(seed=9, n_steps=400, obs_kind=W.OBS_FINAL)
    h = ssa.Net(nets, B, exec_mode=exec_mode)
    th = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, B)
    fwd = ssa.forward(h, cfg, th, x0, tie_capacity=1 << 12)
    torch.cuda.synchronize()
    ties = fwd.tie_records()
    xf = fwd.x_final.cpu().numpy()
    sd = fwd.steps_done.cpu().numpy()
    for n, (net, b) in enumerate(zip(nets, B)):
        L = h.layout(n)
        ov = _ties_for_oracle([t for t in ties if L.traj_offset <= t["traj"] < L.traj_offset + b],
                              L.traj_offset)
        r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=L.traj_offset + np.arange(b), ties=ov)
        assert r.n_bad.sum() == 0
        got = xf[L.state_offset: L.state_offset + net.n_species * b].reshape(net.n_species, b).T
        assert np.array_equal(got, r.x_final), n
        assert np.array_equal(sd[L.traj_offset: L.traj_offset + b], r.steps_done)


def test_forward_backward_deterministic(ssa):
    net = W.dimerization_2a()
    B = 512
    cfg = W.RunConfig(seed=7, n_steps=800, obs_kind=W.OBS_BINS, n_bins=5, t_obs=150.0, ckpt_every=128)
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    d = torch.randn(cfg.n_bins * B, dtype=torch.float64, device="cuda")
    outs = []
    for _ in range(2):
        f = ssa.forward(h, cfg, th, x0)
        dp = ssa.backward(h, cfg, th, x0, f, d)
        outs.append((f.obs.clone(), f.x_final.clone(), dp.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)
