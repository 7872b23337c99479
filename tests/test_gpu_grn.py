"""Parity of the gene-network classifier path with the FP64 oracle.

Split parity: (i) the GPU's hidden pre-activations u = b + bf16(x) bf16(W)^T,
summed in FP32 on the matrix cores, against the oracle's exact FP64
contraction of the same bf16 operands, within the FP32 summation bound;
(ii) the oracle simulates on the GPU's u, and counts (bit-exact), clocks and
gradients (per trajectory and reduced) are compared.  The GPU logs selection
near-ties within 2e-6 (its FP32 error budget: -ln(u) <= 3e-7, production
rates <= 3e-7, reciprocal 1 ulp); the oracle adopts the GPU's choice there if
its own FP64 margin is within the same window."""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import workloads as W

from test_gpu_parity import _ties_for_oracle, assert_grad_parity

pytestmark = pytest.mark.gpu

TIE_WINDOW = 2e-6


@pytest.fixture(scope="module")
def ssa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa as m
    m.lib()
    return m


def run_gpu(ssa, w, d_obs=None, per_traj=True, x0=None):
    g = ssa.Grn(w.net, w.n_images, w.n_rep)
    th = torch.tensor(w.theta, device="cuda")
    x = torch.tensor(w.images, device="cuda")
    x0t = None if x0 is None else torch.tensor(np.ascontiguousarray(x0.T), device="cuda")
    f = ssa.grn_forward(g, w.cfg, th, x, x0t, tie_capacity=1 << 16)
    out = {"u": f.u_hid.cpu().numpy(), "x_final": f.x_final.cpu().numpy().T,
           "t_final": f.t_final.cpu().numpy(), "steps_done": f.steps_done.cpu().numpy(),
           "obs": f.obs.cpu().numpy().T, "ties": f.tie_records()}
    if d_obs is not None:
        d = torch.tensor(np.ascontiguousarray(d_obs.T), device="cuda")
        dp, comp = ssa.grn_backward(g, w.cfg, th, x, f, d, per_traj=True)
        out["d_params"] = dp.cpu().numpy()
        out["comp"] = comp.cpu().numpy() if per_traj else None
    torch.cuda.synchronize()
    assert ssa.grn_device_status(g) == 0
    return out


def oracle_for(w, gpu, ids, d_obs=None, x0=None):
    idx = {int(q): i for i, q in enumerate(ids)}
    ov = _ties_for_oracle(gpu["ties"], 0, idx)
    return oracle.grn_run(w.net, w.cfg, w.theta, gpu["u"].astype(np.float64), ids // w.n_rep,
                          x0=None if x0 is None else x0[ids], traj_ids=ids, ties=ov,
                          d_obs=None if d_obs is None else d_obs[ids], tie_threshold=TIE_WINDOW)


def assert_forward(gpu, r, ids):
    assert (r.n_bad == 0).all(), r.n_bad
    np.testing.assert_array_equal(gpu["steps_done"][ids], r.steps_done)
    np.testing.assert_array_equal(gpu["x_final"][ids], r.x_final)
    np.testing.assert_array_equal(gpu["obs"][ids], r.obs)
    t = r.t_final
    assert np.all(np.abs(gpu["t_final"][ids] - t) <= 1e-5 * np.maximum(t, 1e-300))


def workload(n_images, n_rep, n_steps, n_in=784, n_out=10, T=1.0, seed=0):
    net = W.GrnNet(n_in=n_in, n_out=n_out)
    side = max(8, int(np.ceil(np.sqrt(n_in))))
    imgs, labels = W.grn_images(n_images, seed=seed, side=side)
    imgs = np.ascontiguousarray(imgs[:, :n_in])     # other sizes: flattened images, cropped
    cfg = W.RunConfig(seed=seed + 3, n_steps=n_steps, obs_kind=W.OBS_FINAL, temperature=T)
    return W.GrnWorkload(f"grn_test_{n_in}x256x{n_out}", net, n_images, n_rep, cfg,
                         W.grn_init_params(net, seed), imgs, labels)


def test_hidden_input_contraction_bound(ssa):
    """Full 784 -> 256 contraction over 512 images on bf16 matrix cores."""
    w = W.grn_classifier()
    gpu = run_gpu(ssa, w.__class__(w.name, w.net, w.n_images, 1, w.cfg.replace(n_steps=1), w.theta,
                                   w.images, w.labels))
    exact = oracle.grn_hidden_input(w.net, w.theta, w.images)
    p = w.net.split(w.theta)
    Wb = np.abs(oracle.bf16(p["W"]).astype(np.float64))
    xb = np.abs(oracle.bf16(w.images).astype(np.float64))
    mag = xb @ Wb.T + np.abs(p["b"])[None, :]
    bound = (w.net.n_in + 2) * 2.0 ** -24 * mag
    err = np.abs(gpu["u"] - exact)
    assert (err <= bound).all(), (err.max(), bound[err > bound][:4])


def test_forward_backward_parity(ssa):
    w = workload(n_images=8, n_rep=4, n_steps=2000)
    g = np.random.default_rng(1)
    d_obs = g.normal(size=(w.n_traj, w.net.n_out))
    gpu = run_gpu(ssa, w, d_obs)
    ids = np.arange(w.n_traj)
    r = oracle_for(w, gpu, ids, d_obs)
    assert_forward(gpu, r, ids)
    for q in ids:
        assert_grad_parity(gpu["comp"][q], r.grad_c[q])
    full = oracle.grn_full_gradient(w.net, r.grad_c, w.images, ids // w.n_rep)
    assert_grad_parity(gpu["d_params"], full)


@pytest.mark.parametrize("n_out,T,n_in,n_images,n_rep,n_steps",
                         [(3, 0.5, 100, 5, 3, 300), (16, 0.7, 64, 17, 2, 129), (1, 1.0, 33, 3, 1, 128)])
def test_shapes_and_temperatures(ssa, n_out, T, n_in, n_images, n_rep, n_steps):
    """Output-gene buckets 4/16, every temperature path, ragged contraction
    tiles and depths, tapes ending inside a 128-step block."""
    w = workload(n_images=n_images, n_rep=n_rep, n_steps=n_steps, n_in=n_in, n_out=n_out, T=T, seed=2)
    g = np.random.default_rng(4)
    d_obs = g.normal(size=(w.n_traj, n_out))
    gpu = run_gpu(ssa, w, d_obs)
    exact = oracle.grn_hidden_input(w.net, w.theta, w.images)
    assert np.abs(gpu["u"] - exact).max() <= (n_in + 2) * 2.0 ** -24 * (np.abs(exact).max() + 10.0)
    ids = np.arange(w.n_traj)
    r = oracle_for(w, gpu, ids, d_obs)
    assert_forward(gpu, r, ids)
    for q in ids:
        assert_grad_parity(gpu["comp"][q], r.grad_c[q])
    full = oracle.grn_full_gradient(w.net, r.grad_c, w.images, ids // w.n_rep)
    assert_grad_parity(gpu["d_params"], full)


def test_nonzero_initial_counts_and_zero_steps(ssa):
    w = workload(n_images=4, n_rep=2, n_steps=500, n_in=49, n_out=5, seed=6)
    g = np.random.default_rng(7)
    x0 = g.integers(0, 6, size=(w.n_traj, w.net.n_species)).astype(np.int32)
    d_obs = g.normal(size=(w.n_traj, 5))
    gpu = run_gpu(ssa, w, d_obs, x0=x0)
    ids = np.arange(w.n_traj)
    r = oracle_for(w, gpu, ids, d_obs, x0=x0)
    assert_forward(gpu, r, ids)
    for q in ids:
        assert_grad_parity(gpu["comp"][q], r.grad_c[q])
    # no steps: final state = initial state, zero gradient
    w0 = w.__class__(w.name, w.net, w.n_images, w.n_rep, w.cfg.replace(n_steps=0), w.theta, w.images,
                     w.labels)
    gpu0 = run_gpu(ssa, w0, d_obs, x0=x0)
    np.testing.assert_array_equal(gpu0["x_final"], x0)
    assert (gpu0["steps_done"] == 0).all() and (gpu0["t_final"] == 0).all()
    assert (gpu0["d_params"] == 0).all() and (gpu0["comp"] == 0).all()


def test_full_size_sampled(ssa):
    """512 images x 32 trajectories x 2,000 steps (the benchmarked launch):
    sampled trajectories against the oracle; the reductions against FP64 sums
    of the GPU's own per-trajectory partials."""
    w = W.grn_classifier()
    g = np.random.default_rng(11)
    d_obs = g.normal(size=(w.n_traj, w.net.n_out)) / w.n_traj
    gpu = run_gpu(ssa, w, d_obs)
    ids = np.sort(g.choice(w.n_traj, size=48, replace=False))
    ids[:2] = [0, w.n_traj - 1]
    ids = np.unique(ids)
    r = oracle_for(w, gpu, ids, d_obs)
    assert_forward(gpu, r, ids)
    for i, q in enumerate(ids):
        assert_grad_parity(gpu["comp"][q], r.grad_c[i])
    comp = gpu["comp"]
    H = w.net.n_hid
    rest = comp.sum(axis=0)
    G_img = comp[:, :H].reshape(w.n_images, w.n_rep, H).sum(axis=1)
    x = oracle.bf16(w.images).astype(np.float64)
    dW = G_img.T @ x
    want = np.concatenate([dW.reshape(-1), rest]).astype(np.float32)
    assert_grad_parity(gpu["d_params"], want, rtol=1e-6)


def test_backward_deterministic(ssa):
    w = workload(n_images=6, n_rep=5, n_steps=700, seed=9)
    g = np.random.default_rng(3)
    d_obs = g.normal(size=(w.n_traj, w.net.n_out))
    a = run_gpu(ssa, w, d_obs)
    b = run_gpu(ssa, w, d_obs)
    for k in ("u", "x_final", "t_final", "d_params", "comp"):
        assert np.array_equal(a[k], b[k]), k
