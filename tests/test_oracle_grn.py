"""Pins of the oracle's gene-regulatory network classifier (Sec. 4.3, Fig. 4A).

What fixes each part independently of the oracle's own code:

* bfloat16 rounding: torch's float32 -> bfloat16 conversion (round to nearest
  even), on random values and on exact halfway cases;
* the input contraction: a float64 matmul of torch-rounded operands;
* regulated production and first-order decay, each channel kind on its own:
  with U = 0 every gene is an independent birth-death process from zero, whose
  count at time t is Poisson with mean beta sigmoid(E)/delta (1 - e^{-delta t})
  (a textbook solution of the chemical master equation);
* the output layer's regulation by hidden genes: at stationarity
  E[O_o] = beta/delta_o E[sigmoid(c_o + sum_h U_oh H_h)] with H_h independent
  Poisson (mean beta sigmoid(u_h)/delta_h), summed exactly;
* the first step's choice: categorical with probabilities a_j/a0 (Gumbel-max
  theorem, Sec. 3.2);
* the adjoint: torch float64 autograd of the literal stop-gradient graph of
  Eq. (5) replayed on the oracle's choices and noise, and central differences
  of the frozen surrogate.
"""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from paper_2602_19775_amd import workloads as W


def _tiny(n_hid=5, n_out=3, side=8, seed=0):
    net = W.GrnNet(n_in=side * side, n_hid=n_hid, n_out=n_out)
    theta = W.grn_init_params(net, seed)
    imgs, labels = W.grn_images(6, seed=seed, side=side)
    return net, theta, imgs, labels


def _set(net, theta, **blocks):
    th = theta.copy()
    o = net.offsets()
    ends = {"W": o["b"], "b": o["U"], "U": o["c"], "c": o["psi"], "psi": net.n_params}
    for k, v in blocks.items():
        th[o[k]:ends[k]] = np.asarray(v, np.float64).reshape(-1)
    return th.astype(np.float32)


def test_bf16_rounding_matches_torch(orc):
    g = np.random.default_rng(0)
    x = (g.standard_normal(20000) * np.exp(g.uniform(-30, 30, 20000))).astype(np.float32)
    # exact halfway cases: low 16 bits 0x8000, both parities of the kept part
    hw = ((g.integers(0x3F00, 0x4100, 2000).astype(np.uint32) << 16) | 0x8000).view(np.float32)
    x = np.concatenate([x, hw, -hw, np.float32([0.0, -0.0, 1.0, 3.4e38, 1e-40])])
    mine = orc.bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mine.view(np.uint32), ref.view(np.uint32))


def test_hidden_input_is_the_bf16_contraction(orc):
    net, theta, imgs, _ = _tiny(n_hid=7)
    u = orc.grn_hidden_input(net, theta, imgs)
    p = net.split(theta)
    Wb = torch.from_numpy(p["W"]).to(torch.bfloat16).to(torch.float64)
    xb = torch.from_numpy(imgs).to(torch.bfloat16).to(torch.float64)
    ref = (xb @ Wb.T + torch.from_numpy(p["b"]).to(torch.float64)).numpy()
    assert np.abs(u - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    # the rounding matters: with FP32 W the result differs
    raw = imgs.astype(np.float64) @ p["W"].astype(np.float64).T + p["b"]
    assert np.abs(raw - u).max() > 1e-6


def test_uncoupled_genes_are_poisson_at_t(orc):
    """U = 0: every gene is a birth-death process started at 0."""
    net, theta, imgs, _ = _tiny(n_hid=3, n_out=2)
    delta = np.array([0.5, 1.0, 2.0, 0.7, 1.3])
    u = np.array([[-1.0, 0.0, 1.5]])
    c = np.array([-0.5, 2.0])
    th = _set(net, theta, U=np.zeros((2, 3)), c=c, psi=np.log(delta - net.delta_min))
    t_end = 3.0
    n = 6000
    cfg = W.RunConfig(seed=11, n_steps=2 ** 31 - 1, t_end=t_end, temperature=1.0)
    r = orc.grn_run(net, cfg, th, u, np.zeros(n, np.int64))
    sig = 1.0 / (1.0 + np.exp(-np.concatenate([u[0], c])))
    lam = net.beta * sig / delta * (1.0 - np.exp(-delta * t_end))
    X = r.x_final.astype(np.float64)
    for s in range(5):
        m, v = X[:, s].mean(), X[:, s].var()
        assert abs(m - lam[s]) < 4.5 * math.sqrt(lam[s] / n), (s, m, lam[s])
        assert abs(v - lam[s]) < 4.5 * math.sqrt((lam[s] + 2 * lam[s] ** 2) / n), (s, v, lam[s])
    # full law of one gene: chi-square against Poisson(lam)
    s = 2
    kmax = int(lam[s] + 6 * math.sqrt(lam[s]))
    obs = np.bincount(np.minimum(X[:, s].astype(int), kmax), minlength=kmax + 1)
    pk = stats.poisson.pmf(np.arange(kmax + 1), lam[s])
    pk[-1] = 1.0 - pk[:-1].sum()
    assert stats.chisquare(obs, n * pk).pvalue > 1e-4
    assert (r.t_final <= t_end).all()


def _stationary_output_mean(net, u, U, c, delta_h, delta_o):
    lam = net.beta / (1.0 + np.exp(-u)) / delta_h
    ks = np.arange(0, 80)
    p0 = stats.poisson.pmf(ks, lam[0])
    p1 = stats.poisson.pmf(ks, lam[1])
    H0, H1 = np.meshgrid(ks, ks, indexing="ij")
    w = p0[:, None] * p1[None, :]
    out = []
    for o in range(len(c)):
        v = c[o] + U[o, 0] * H0 + U[o, 1] * H1
        out.append(net.beta / delta_o[o] * (w / (1.0 + np.exp(-v))).sum())
    return np.array(out)


def test_output_regulation_stationary_mean(orc):
    """Output genes regulated by the hidden counts through U (rows = outputs)."""
    net, theta, imgs, _ = _tiny(n_hid=2, n_out=2)
    u = np.array([0.3, -0.8])
    U = np.array([[0.4, -0.3], [-0.6, 0.25]])
    c = np.array([0.1, -0.2])
    delta = np.array([1.0, 1.5, 1.0, 0.6])
    th = _set(net, theta, U=U, c=c, psi=np.log(delta - net.delta_min))
    n = 4000
    cfg = W.RunConfig(seed=5, n_steps=2 ** 31 - 1, t_end=30.0, temperature=1.0)
    r = orc.grn_run(net, cfg, th, u[None, :], np.zeros(n, np.int64))
    want = _stationary_output_mean(net, u, U, c, delta[:2], delta[2:])
    O = r.obs
    se = O.std(axis=0) / math.sqrt(n)
    assert (np.abs(O.mean(axis=0) - want) < 4.5 * se).all(), (O.mean(axis=0), want, se)
    # the check separates U from its transpose-like mistake (rows swapped)
    wrong = _stationary_output_mean(net, u, U[::-1], c, delta[:2], delta[2:])
    assert (np.abs(wrong - want) > 10 * se).any()


def test_first_step_is_categorical(orc):
    net, theta, imgs, _ = _tiny(n_hid=4, n_out=3)
    u = np.array([[-0.5, 0.2, 1.0, -2.0]])
    c = np.array([0.3, -1.0, 0.0])
    th = _set(net, theta, c=c)
    n = 40000
    cfg = W.RunConfig(seed=8, n_steps=1, temperature=1.0)
    r = orc.grn_run(net, cfg, th, u, np.zeros(n, np.int64))
    which = np.argmax(r.x_final, axis=1)          # the one gene produced (all start at 0)
    assert (r.x_final.sum(axis=1) == 1).all()
    a = net.beta / (1.0 + np.exp(-np.concatenate([u[0], c])))   # decays are 0 at X = 0
    counts = np.bincount(which, minlength=7)
    assert stats.chisquare(counts, n * a / a.sum()).pvalue > 1e-4


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def _change_matrix(net):
    H, O = net.n_hid, net.n_out
    V = np.zeros((net.n_reactions, net.n_species))
    for h in range(H):
        V[h, h] = 1.0
        V[H + h, h] = -1.0
    for o in range(O):
        V[2 * H + o, H + o] = 1.0
        V[2 * H + O + o, H + o] = -1.0
    return torch.from_numpy(V)


def _literal_graph(net, cfg, theta, img, jk, E, frozen=None, w_off=None, masks=None):
    """Final output counts of the straight-through surrogate.

    theta: float64 tensor.  Stop-gradient terms are y~.detach() (Eq. 5) or, if
    `frozen` is given, those fixed values (the frozen surrogate, which also
    keeps the base point's set of active channels, `masks`).  The bfloat16
    rounding of W passes the gradient straight through (w_off: a fixed rounding
    offset for the frozen surrogate)."""
    H, O = net.n_hid, net.n_out
    o = net.offsets()
    W_ = theta[o["W"]:o["b"]].reshape(H, net.n_in)
    if w_off is None:
        w_off = (W_.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64) - W_.detach())
    W_eff = W_ + w_off
    b = theta[o["b"]:o["U"]]
    U = theta[o["U"]:o["c"]].reshape(O, H)
    c = theta[o["c"]:o["psi"]]
    delta = net.delta_min + torch.exp(theta[o["psi"]:])
    x = torch.from_numpy(img.astype(np.float64))
    u = W_eff @ x + b
    V = _change_matrix(net)
    X = torch.zeros(net.n_species, dtype=torch.float64)
    T = cfg.temperature
    ys, acts = [], []
    for k in range(len(jk)):
        # X is integral in exact arithmetic; its value is taken exactly (the
        # rounding residue of y + y~ - y~ would switch empty decays on) while
        # the derivative flows through X unchanged
        Xv = X.detach().round() + (X - X.detach()) if frozen is None else X
        a = torch.cat([net.beta * torch.sigmoid(u), delta[:H] * Xv[:H],
                       net.beta * torch.sigmoid(c + U @ Xv[:H]), delta[H:] * Xv[H:]])
        act = a.detach() > 0 if frozen is None else masks[k]
        acts.append(act)
        z = torch.where(act, (torch.log(torch.where(act, a, torch.ones_like(a))) -
                              torch.log(torch.from_numpy(E[k]))) / T,
                        torch.full_like(a, -math.inf))
        yt = torch.softmax(z, dim=0)
        ys.append(yt.detach())
        y = torch.zeros_like(yt)
        y[jk[k]] = 1.0
        stop = yt.detach() if frozen is None else frozen[k]
        X = X + (y + yt - stop) @ V
    return X[H:], (ys, acts)


def _replay_inputs(orc, net, cfg, theta, u_row, tid, n_steps):
    jk, _ = orc.grn_trace(net, cfg, theta, u_row, traj_id=tid, cap=n_steps)
    E = np.stack([-np.log(orc.step_uniforms(cfg.seed, cfg.purpose, cfg.epoch, tid, k,
                                            net.n_reactions + 1)[1:]) for k in range(len(jk))])
    return jk, E


def test_adjoint_matches_autograd_of_stopgrad_graph(orc):
    net, theta, imgs, _ = _tiny(n_hid=5, n_out=3)
    g = np.random.default_rng(3)
    # move biases and decays off their initial values so every block matters
    p = net.split(theta)
    theta = _set(net, theta, b=g.normal(0, 0.5, 5), c=g.normal(0, 0.5, 3),
                 U=p["U"] * 3.0, psi=g.normal(-0.5, 0.3, 8))
    cfg = W.RunConfig(seed=2, n_steps=60, temperature=0.7)
    image_of = np.array([0, 0, 1, 2, 2, 5])
    u = orc.grn_hidden_input(net, theta, imgs)
    d_obs = g.normal(size=(len(image_of), net.n_out))
    r = orc.grn_run(net, cfg, theta, u, image_of, d_obs=d_obs)
    full = orc.grn_full_gradient(net, r.grad_c, imgs, image_of)
    total = np.zeros(net.n_params)
    for q, m in enumerate(image_of):
        th = torch.tensor(theta.astype(np.float64), requires_grad=True)
        jk, E = _replay_inputs(orc, net, cfg, theta, u[m], q, cfg.n_steps)
        assert len(jk) == cfg.n_steps
        Xo, _ = _literal_graph(net, cfg, th, imgs[m], jk, E)
        assert np.abs(Xo.detach().numpy() - r.obs[q]).max() < 1e-9   # integral up to rounding
        (Xo * torch.from_numpy(d_obs[q])).sum().backward()
        gq = th.grad.numpy()
        total += gq
        # per trajectory: compact blocks and dW = du x^T
        H = net.n_hid
        o = net.offsets()
        gc = r.grad_c[q]
        xb = torch.from_numpy(imgs[m]).to(torch.bfloat16).to(torch.float64).numpy()
        mine = np.concatenate([np.outer(gc[:H], xb).reshape(-1), gc])
        assert np.abs(mine - gq).max() <= 1e-10 * max(np.abs(gq).max(), 1e-30), q
    assert np.abs(full - total).max() <= 1e-10 * np.abs(total).max()


def test_autograd_is_derivative_of_frozen_surrogate(orc):
    """Central differences (Richardson) of the frozen surrogate reproduce the
    stop-gradient autograd, coordinate by coordinate in every block."""
    net, theta, imgs, _ = _tiny(n_hid=4, n_out=2)
    g = np.random.default_rng(9)
    theta = _set(net, theta, b=g.normal(0, 0.5, 4), c=g.normal(0, 0.5, 2),
                 psi=g.normal(-0.5, 0.3, 6))
    cfg = W.RunConfig(seed=4, n_steps=40, temperature=0.8)
    u = orc.grn_hidden_input(net, theta, imgs)
    jk, E = _replay_inputs(orc, net, cfg, theta, u[1], 7, cfg.n_steps)
    d = torch.from_numpy(g.normal(size=net.n_out))
    th0 = torch.tensor(theta.astype(np.float64), requires_grad=True)
    Xo, (ys, acts) = _literal_graph(net, cfg, th0, imgs[1], jk, E)
    (Xo * d).sum().backward()
    auto = th0.grad.numpy()

    o = net.offsets()
    W0 = torch.tensor(theta[o["W"]:o["b"]].astype(np.float64)).reshape(net.n_hid, net.n_in)
    w_off = W0.to(torch.float32).to(torch.bfloat16).to(torch.float64) - W0

    def F(th):
        with torch.no_grad():
            X, _ = _literal_graph(net, cfg, th, imgs[1], jk, E, frozen=ys, w_off=w_off, masks=acts)
            return float((X * d).sum())

    for idx in [o["W"] + 3, o["W"] + 2 * net.n_in + 17, o["b"] + 1, o["U"] + 5, o["c"] + 1, o["psi"] + 2,
                o["psi"] + net.n_hid]:
        def central(h):
            tp = torch.tensor(theta.astype(np.float64))
            tm = tp.clone()
            tp[idx] += h
            tm[idx] -= h
            return (F(tp) - F(tm)) / (2 * h)
        h = 1e-3
        fd = (4 * central(h / 2) - central(h)) / 3
        assert abs(fd - auto[idx]) <= 1e-7 * max(abs(auto).max(), 1e-12), (idx, fd, auto[idx])
