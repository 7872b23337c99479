"""Scheduling: the autotuner's plan choice and cache, and whole optimisation
steps captured into a HIP graph and replayed (device-side epoch)."""
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


def test_autotune_chooses_and_caches(ssa, tmp_path):
    from paper_2602_19775_amd import autotune as A
    net = W.dimerization_2a()
    B = 8192
    cfg = W.RunConfig(seed=1, n_steps=3000, obs_kind=W.OBS_BINS, n_bins=20, t_obs=600.0, temperature=0.5)
    theta = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    cache = A.Cache(str(tmp_path / "tune.json"))
    lines = []
    plan = A.tune([net], [B], cfg, theta, x0, [cfg.t_obs], probe_steps=256, repeats=2, cache=cache,
                  log=lines.append)
    assert plan in A.candidate_plans(cfg.n_steps)
    entry = A.Cache(cache.path).data[A.signature([net], [B], cfg)]
    timed = {k: v for k, v in entry["timings_ms"].items() if v is not None}
    assert len(timed) >= 6                      # spec, lane and wave plans all run the dimer
    assert min(timed.values()) == pytest.approx(
        timed[plan.name])
    # a second call is a cache hit: nothing is timed
    def boom(*a, **k):
        raise AssertionError("timed a cached batch")
    orig = A._time_plan
    A._time_plan = boom
    try:
        assert A.tune([net], [B], cfg, theta, x0, [cfg.t_obs], cache=A.Cache(cache.path)) == plan
    finally:
        A._time_plan = orig
    # the chosen plan runs and agrees with the library's default plan on the counts
    h = plan.net([net], [B], [cfg.t_obs])
    f = ssa.forward(h, plan.config(cfg), theta, x0, bwd_mode=plan.bwd_mode)
    h0 = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    f0 = ssa.forward(h0, cfg, theta, x0)
    # trajectories with a selection or stop near-tie (not bin-edge records)
    ties = {int(t["traj"]) for t in f.tie_records() if t["kind"] != 2} | \
           {int(t["traj"]) for t in f0.tie_records() if t["kind"] != 2}
    xa = f.x_final.cpu().numpy().reshape(2, B)
    xb = f0.x_final.cpu().numpy().reshape(2, B)
    same = np.ones(B, bool)
    same[list(ties)] = False
    assert np.array_equal(xa[:, same], xb[:, same])


def _sgd_step(ssa, h, cfg, theta, x0, bufs, d_params, epoch, loss_fn, lr):
    ssa.forward(h, cfg, theta, x0, buffers=bufs, tie_capacity=0, d_epoch=epoch)
    obs = bufs.obs.detach().requires_grad_(True)
    loss = loss_fn(obs)
    (d_obs,) = torch.autograd.grad(loss, obs)
    ssa.backward(h, cfg, theta, x0, bufs, d_obs, d_params=d_params)
    theta.sub_(lr * d_params)
    epoch.add_(1)


def _check_graph_against_eager(ssa, h, cfg, theta0, x0, loss_fn, lr, n_replays=4):
    from paper_2602_19775_amd.graph import CapturedStep
    dev = theta0.device

    def fresh():
        theta = theta0.clone()
        epoch = torch.zeros(1, dtype=torch.int32, device=dev)
        bufs = ssa.forward(h, cfg, theta, x0, tie_capacity=0, d_epoch=epoch)
        d_params = torch.empty(h.param_total, dtype=torch.float32, device=dev)
        return theta, epoch, bufs, d_params

    # eager reference
    theta, epoch, bufs, d_params = fresh()
    ref = []
    for _ in range(n_replays):
        _sgd_step(ssa, h, cfg, theta, x0, bufs, d_params, epoch, loss_fn, lr)
        torch.cuda.synchronize()
        ref.append((bufs.obs.clone(), d_params.clone(), theta.clone()))
    # captured: warm-up steps run eagerly, then the state is reset and replayed
    theta, epoch, bufs, d_params = fresh()
    cap = CapturedStep(lambda: _sgd_step(ssa, h, cfg, theta, x0, bufs, d_params, epoch, loss_fn, lr))
    theta.copy_(theta0)
    epoch.zero_()
    torch.cuda.synchronize()
    noise = torch.randn(1 << 20, device=dev)
    for k in range(n_replays):
        cap.replay()
        torch.cuda.synchronize()
        assert torch.equal(bufs.obs, ref[k][0]), k
        assert torch.equal(d_params, ref[k][1]), k
        assert torch.equal(theta, ref[k][2]), k
        noise = noise * 1.0001 + float(k)       # eager work between replays
        torch.cuda.synchronize()
    assert int(epoch.item()) == n_replays
    assert ssa.device_status(h) == 0


def test_autotune_uneven_batch(ssa, tmp_path):
    """The tuner on a reduced uneven batch (the first 48 networks of the
    4,096-network generator, 64 trajectories each, their own 4-bin windows):
    only wave plans run it (more than 16 topologies, channels beyond the
    generic lane tables), every width and launch split among them, and the
    chosen plan fires the channels of the library's default plan."""
    from paper_2602_19775_amd import autotune as A
    bw = W.uneven_batch(n_networks=48, traj_per_network=64, n_steps=400)
    nets, Bs = bw.nets, bw.n_traj
    cfg = bw.cfg.replace(t_obs=bw.t_obs[0])
    theta = torch.tensor(bw.theta(), device="cuda")
    x0 = torch.tensor(bw.x0_packed(), device="cuda")
    cache = A.Cache(str(tmp_path / "tune.json"))
    lines = []
    plan = A.tune(nets, Bs, cfg, theta, x0, bw.t_obs, probe_steps=128, repeats=1, cache=cache, log=lines.append)
    timed = {k: v for k, v in A.Cache(cache.path).data[A.signature(nets, Bs, cfg)]["timings_ms"].items()
             if v is not None}
    assert plan.exec_mode == "wave" and plan.name in timed
    assert all(k.startswith("wave/") for k in timed), timed
    assert {"wave/split1/tape/K256", "wave/split0/tape/K256", "wave/split1/w32/tape/K256",
            "wave/split0/w16/tape/K256"} <= set(timed), lines
    h = plan.net(nets, Bs, bw.t_obs)
    f = ssa.forward(h, plan.config(cfg), theta, x0, bwd_mode=plan.bwd_mode)
    f0 = ssa.forward(ssa.Net(nets, Bs, t_obs=bw.t_obs), cfg, theta, x0)
    torch.cuda.synchronize()
    assert torch.equal(f.steps_done, f0.steps_done)
    assert torch.equal(f.x_final, f0.x_final)


def test_graph_replay_dimer_specialised(ssa):
    from paper_2602_19775_amd import losses
    net = W.dimerization_2a()
    B = 4096
    cfg = W.RunConfig(seed=3, n_steps=800, obs_kind=W.OBS_BINS, n_bins=10, t_obs=150.0, temperature=0.5,
                      ckpt_every=128)
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    theta0 = torch.tensor(net.theta0, device="cuda")
    x0 = _x0([net], [B])
    tm = torch.linspace(60.0, 80.0, cfg.n_bins, dtype=torch.float64, device="cuda")[:, None]
    tv = torch.full((cfg.n_bins, 1), 20.0, dtype=torch.float64, device="cuda")

    def loss_fn(obs):
        return losses.moment_mse(obs, tm, tv, cfg.n_bins, 1, B)
    _check_graph_against_eager(ssa, h, cfg, theta0, x0, loss_fn, lr=1e-4)


def test_graph_replay_wave_batch(ssa):
    nets = W.random_network_batch(3, seed=31, n_range=(6, 20), m_range=(20, 80))
    B = [96, 64, 130]
    cfg = W.RunConfig(seed=2, n_steps=300, obs_kind=W.OBS_FINAL, temperature=0.5, ckpt_every=64)
    h = ssa.Net(nets, B, exec_mode="wave")
    theta0 = torch.tensor(np.concatenate([n.theta0 for n in nets]), device="cuda")
    x0 = _x0(nets, B)

    def loss_fn(obs):
        return (obs * obs).sum() * 1e-6
    _check_graph_against_eager(ssa, h, cfg, theta0, x0, loss_fn, lr=1e-3)
