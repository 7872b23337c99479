"""Host-side logic that needs no GPU: the autotuner's plan space, batch
signature and cache, and the benchmark's single-GPU contract."""
import json
import os
import subprocess
import sys

import numpy as np
import torch

from paper_2602_19775_amd import autotune as A
from paper_2602_19775_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_candidate_plans():
    plans = A.candidate_plans(10000)
    assert len(plans) == len(set(plans))
    assert {p.exec_mode for p in plans} == {"spec", "lane", "wave"}
    assert all(p.ckpt_every <= 64 for p in plans if p.bwd_mode == "recompute")
    assert {p.wave_split for p in plans if p.exec_mode == "wave"} == {0, 1}
    assert {p.wave_lanes for p in plans if p.exec_mode == "wave"} == {0, 16, 32}
    assert all(p.wave_lanes == 0 for p in plans if p.exec_mode != "wave")
    assert len({p.name for p in plans}) == len(plans)
    short = A.candidate_plans(100)
    assert max(p.ckpt_every for p in short) == 64


def test_signature_separates_batches():
    net = W.dimerization_2a()
    cfg = W.RunConfig(n_steps=10000, obs_kind=W.OBS_BINS, n_bins=20)
    s = A.signature([net], [1024], cfg)
    assert s == A.signature([net], [1024], cfg)
    assert s == A.signature([net], [1024], cfg.replace(n_steps=9000))       # same power-of-two bucket
    assert s != A.signature([net], [2048], cfg)
    assert s != A.signature([net], [1024], cfg.replace(n_steps=40000))
    assert s != A.signature([net], [1024], cfg.replace(obs_kind=W.OBS_FINAL, n_bins=0))
    assert s != A.signature([W.isomerization()], [1024], cfg)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = A.Cache(path)
    assert c.get("k") is None
    p = A.Plan("wave", 1, "recompute", 64)
    c.put("k", p, {"wave/split1/recompute/K64": 1.5, "spec/split-1/tape/K256": None})
    assert A.Cache(path).get("k") == p
    assert json.load(open(path))["k"]["timings_ms"]["spec/split-1/tape/K256"] is None
    q = A.Plan("wave", 0, "tape", 256, 16)
    c.put("k2", q, {q.name: 2.0})
    assert A.Cache(path).get("k2") == q and q.name == "wave/split0/w16/tape/K256"
    # an entry written before the plan had a width reads as the library's width
    data = json.load(open(path))
    del data["k2"]["plan"]["wave_lanes"]
    json.dump(data, open(path, "w"))
    assert A.Cache(path).get("k2") == A.Plan("wave", 0, "tape", 256)
    with open(path, "w") as f:
        f.write("{not json")
    assert A.Cache(path).get("k") is None


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_moment_mse_gradient_matches_autograd():
    from paper_2602_19775_amd import losses
    g = torch.Generator().manual_seed(3)
    nb, no, B = 5, 2, 37
    obs = (torch.rand(nb * no * B + 7, generator=g, dtype=torch.float64) * 50).requires_grad_(True)
    tm = torch.rand(nb, no, generator=g, dtype=torch.float64) * 50
    tv = torch.rand(nb, no, generator=g, dtype=torch.float64) * 200
    l1 = losses.moment_mse(obs, tm, tv, nb, no, B)
    (g1,) = torch.autograd.grad(l1, obs)
    l2 = losses.moment_mse_autograd(obs, tm, tv, nb, no, B)
    (g2,) = torch.autograd.grad(l2, obs)
    assert abs(l1.item() - l2.item()) <= 1e-12 * abs(l2.item())
    assert torch.allclose(g1, g2, rtol=1e-10, atol=1e-14)
    assert torch.all(g1[nb * no * B:] == 0)


def test_autocorrelation_fft_matches_lag_sums():
    from paper_2602_19775_amd import losses
    g = torch.Generator().manual_seed(4)
    nb, B, lag = 40, 9, 12
    obs = (torch.rand(nb * B, generator=g, dtype=torch.float64) * 30).requires_grad_(True)
    r1 = losses.mean_autocorrelation(obs, nb, B, lag)
    r2 = losses.mean_autocorrelation_direct(obs, nb, B, lag)
    assert torch.allclose(r1, r2, rtol=0, atol=1e-13)
    w = torch.rand(lag, generator=g, dtype=torch.float64)
    (g1,) = torch.autograd.grad((r1 * w).sum(), obs)
    (g2,) = torch.autograd.grad((r2 * w).sum(), obs)
    assert torch.allclose(g1, g2, rtol=0, atol=1e-13)


def test_start_point_rate_loss_gradient_written_out():
    """The start-point map's loss gradient with respect to the tail
    observations, written out, equals torch autograd of the same loss."""
    import torch
    from paper_2602_19775_amd.startpoint import rate_loss
    g = torch.Generator().manual_seed(3)
    S, R = 7, 5
    obs = torch.rand(4 * S * R, generator=g, dtype=torch.float64) * 50 + 1.0
    obs.view(4, S, R)[3] = torch.rand(S, R, generator=g, dtype=torch.float64) * 0.3 + 0.05
    xs = torch.rand(S, 3, generator=g, dtype=torch.float64) * 40
    tr = torch.randn(S, 3, generator=g, dtype=torch.float64) * 10
    d = torch.zeros_like(obs)
    loss = rate_loss(obs, xs, tr, S, R, d)
    o = obs.clone().requires_grad_(True)
    ref = rate_loss(o, xs, tr, S, R)
    ref.sum().backward()
    assert torch.allclose(loss, ref.detach(), rtol=1e-14, atol=0)
    assert torch.allclose(d, o.grad, rtol=1e-12, atol=1e-15)


def test_uneven_windows_file():
    """The uneven batch's per-network observation windows (written by the oracle
    pilot script): one positive finite value per network, in network order."""
    from paper_2602_19775_amd import workloads as W
    t = np.asarray(W.uneven_t_obs(4096))
    assert t.shape == (4096,) and np.all(np.isfinite(t)) and np.all(t > 0)
    b = W.uneven_batch(16)
    assert b.cfg.obs_kind == W.OBS_BINS and b.cfg.n_bins == 4 and b.t_obs == list(t[:16])
