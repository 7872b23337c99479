"""Parity of the relaxed (soft) gene-network forward of Eq. 4 and its exact
backward with the FP64 oracle (the first phase of the two-phase training of
Sec. 3.5).

Split parity as for the hard path: the oracle runs on the GPU's hidden
pre-activations.  The relaxed map is smooth, so the GPU's FP32 soft sample and
the oracle's FP64 one give levels and gradients that differ by rounding only.
Per step, each weight of the sample carries a relative error of a few FP32
ulps (one reciprocal and the ratio, plus exp2 and log2 at a general T, the
log error scaled by 1/T), about eps_step = 8 (1 + 1/T) 2^-24; the GPU keeps
the levels in FP64.  Errors that added up linearly over n steps would reach
n eps_step, but they are of both signs and the decay channels contract the
levels, so the levels agree within 1e-5 of their scale and each trajectory's
compact gradient within 1e-5 of its largest component (the tolerance the
exact path is held to), which the test asserts; it prints the measured
errors beside the linear bound n eps_step.

At T -> 0 the relaxed sample becomes the hard choice (the race winner's
weight is exactly 1), so the relaxed forward at T = 1e-8 reproduces the hard
forward on every trajectory without a logged selection near-tie.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import workloads as W

from test_gpu_grn import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


def eps_step(T):
    return 8.0 * (1.0 + 1.0 / T) * 2.0 ** -24


def run_relaxed(ssa, w, d_obs=None):
    g = ssa.Grn(w.net, w.n_images, w.n_rep)
    cfg = w.cfg.replace(relaxed=True)
    th = torch.tensor(w.theta, device="cuda")
    x = torch.tensor(w.images, device="cuda")
    f = ssa.grn_forward(g, cfg, th, x, tie_capacity=0)
    out = {"u": f.u_hid.cpu().numpy(), "obs": f.obs.cpu().numpy().T, "x_final": f.x_final.cpu().numpy().T,
           "t_final": f.t_final.cpu().numpy(), "steps_done": f.steps_done.cpu().numpy()}
    if d_obs is not None:
        d = torch.tensor(np.ascontiguousarray(d_obs.T), device="cuda")
        dp, comp = ssa.grn_backward(g, cfg, th, x, f, d, per_traj=True)
        out["d_params"] = dp.cpu().numpy()
        out["comp"] = comp.cpu().numpy()
    torch.cuda.synchronize()
    assert ssa.grn_device_status(g) == 0
    return out


@pytest.mark.parametrize("T", [1.0, 0.5, 0.7])
def test_relaxed_parity(ssa, T):
    n_steps = 300
    w = workload(6, 4, n_steps, n_in=196, n_out=10, T=T, seed=1)
    B = w.n_images * w.n_rep
    g = np.random.default_rng(4)
    d_obs = g.normal(size=(B, w.net.n_out))
    gpu = run_relaxed(ssa, w, d_obs)
    ids = np.arange(B)
    r = oracle.grn_soft_run(w.net, w.cfg, w.theta, gpu["u"].astype(np.float64), ids // w.n_rep, traj_ids=ids,
                            d_obs=d_obs)
    assert np.all(gpu["steps_done"] == n_steps)
    scale_obs = max(1.0, np.abs(r.obs).max())
    err_obs = np.abs(gpu["obs"] - r.obs).max() / scale_obs
    assert err_obs <= 1e-5, err_obs
    assert np.array_equal(gpu["x_final"][:, 256:], np.rint(gpu["obs"]).astype(np.int32))
    assert np.allclose(gpu["t_final"], r.t_final, rtol=1e-5, atol=0)
    scale = np.abs(r.grad_c).max(axis=1, keepdims=True)
    err_g = np.abs(gpu["comp"] - r.grad_c) / scale
    assert err_g.max() <= 1e-5, err_g.max()
    full = oracle.grn_full_gradient(w.net, r.grad_c, w.images, ids // w.n_rep)
    assert np.abs(gpu["d_params"] - full).max() <= 1e-5 * np.abs(full).max()
    print(f"\nrelaxed T={T}: max |obs - obs*| / scale = {err_obs:.2e}, max gradient error / row scale = "
          f"{err_g.max():.2e} (bar 1e-5; linear rounding bound n eps_step = {n_steps * eps_step(T):.1e})")


def test_relaxed_is_deterministic(ssa):
    w = workload(4, 3, 200, n_in=64, n_out=4, T=0.8, seed=2)
    d_obs = np.random.default_rng(1).normal(size=(12, 4))
    a = run_relaxed(ssa, w, d_obs)
    b = run_relaxed(ssa, w, d_obs)
    for k in ("obs", "t_final", "d_params", "comp"):
        assert np.array_equal(a[k], b[k]), k


def test_relaxed_cold_limit_is_the_hard_path(ssa):
    """At T = 1e-8 every weight but the race winner's underflows, except at
    selection near-ties: the relaxed forward then fires the hard path."""
    w = workload(8, 8, 400, n_in=196, n_out=10, T=1e-8, seed=3)
    g = ssa.Grn(w.net, w.n_images, w.n_rep)
    th = torch.tensor(w.theta, device="cuda")
    x = torch.tensor(w.images, device="cuda")
    hard = ssa.grn_forward(g, w.cfg, th, x, tie_capacity=1 << 14)
    ties = hard.tie_records()
    hx, ht = hard.x_final.cpu().numpy().T.copy(), hard.t_final.cpu().numpy().copy()
    soft = ssa.grn_forward(g, w.cfg.replace(relaxed=True), th, x, tie_capacity=0, keep_tape=False)
    sx, so, st = soft.x_final.cpu().numpy().T, soft.obs.cpu().numpy().T, soft.t_final.cpu().numpy()
    torch.cuda.synchronize()
    B = w.n_images * w.n_rep
    clean = np.ones(B, bool)
    clean[np.unique(ties["traj"][ties["kind"] == 0]).astype(np.int64)] = False
    assert clean.sum() >= B // 2
    assert np.array_equal(sx[clean], hx[clean])
    assert np.array_equal(so[clean], hx[clean][:, 256:].astype(np.float64))
    assert np.allclose(st[clean], ht[clean], rtol=1e-5, atol=0)


def test_relaxed_refused_where_it_does_not_apply(ssa):
    net = W.dimerization_2a()
    h = ssa.Net([net], [64])
    x0 = torch.tensor(np.repeat(net.x0[:, None], 64, axis=1).reshape(-1), dtype=torch.int32, device="cuda")
    th = torch.tensor(net.theta0, device="cuda")
    with pytest.raises(ssa.SSAError, match="gene-network"):
        ssa.forward(h, W.RunConfig(n_steps=10, relaxed=True), th, x0, tie_capacity=0)
    w = workload(2, 2, 10, n_in=64, n_out=4, seed=0)
    g = ssa.Grn(w.net, w.n_images, w.n_rep)
    with pytest.raises(ssa.SSAError, match="Gumbel"):
        ssa.grn_forward(g, w.cfg.replace(relaxed=True, selection=W.SELECT_INVERSE_CDF),
                        torch.tensor(w.theta, device="cuda"), torch.tensor(w.images, device="cuda"))
