"""Pins of the oracle's relaxed (soft) forward of the gene network (Eq. 4,
the first phase of the two-phase training of Sec. 3.5) and of its adjoint.

What fixes each part independently of the oracle's own code:

* the forward at T -> 0: the soft sample tends to the one-hot argmax of Eq. 3,
  so the relaxed path tends to the hard direct-method path of the same noise
  (`orc_grn_run`, pinned on its own in test_oracle_grn.py);
* the forward at T -> infinity: the soft sample is uniform over the channels
  with a_j > 0, so from the empty state one step moves every gene by
  1 / (n_hid + n_out) (closed form; decays of empty genes are excluded);
* the adjoint: central differences (Richardson) of the relaxed map itself,
  coordinate by coordinate in every parameter block and in the hidden
  pre-activations, and torch float64 autograd of the relaxed map written out
  in this file.
"""
import math

import numpy as np
import torch

from paper_2602_19775_amd import workloads as W

from test_oracle_grn import _change_matrix, _set, _tiny


def _moved(net, theta, g):
    p = net.split(theta)
    return _set(net, theta, b=g.normal(0, 0.5, net.n_hid), c=g.normal(0, 0.5, net.n_out),
                U=p["U"] * 3.0, psi=g.normal(-0.5, 0.3, net.n_hid + net.n_out))


def test_soft_forward_tends_to_the_hard_path(orc):
    net, theta, imgs, _ = _tiny(n_hid=5, n_out=3)
    theta = _moved(net, theta, np.random.default_rng(1))
    cfg = W.RunConfig(seed=6, n_steps=50, temperature=1e-6)
    image_of = np.arange(16) % 6
    u = orc.grn_hidden_input(net, theta, imgs)
    hard = orc.grn_run(net, cfg, theta, u, image_of)
    soft = orc.grn_soft_run(net, cfg, theta, u, image_of)
    # a gap g between the two best scores leaves exp(-g/T) off the one-hot
    clear = hard.min_margin > 1e-3
    assert clear.sum() >= 8
    assert np.all(hard.steps_done == cfg.n_steps)
    assert np.abs(soft.x_final[clear] - hard.x_final[clear]).max() < 1e-9
    assert np.allclose(soft.t_final[clear], hard.t_final[clear], rtol=1e-12)
    # a warm relaxation leaves the lattice
    warm = orc.grn_soft_run(net, cfg.replace(temperature=1.0), theta, u, image_of)
    assert np.abs(warm.x_final - np.round(warm.x_final)).max() > 1e-3


def test_soft_forward_hot_limit_is_uniform(orc):
    net, theta, imgs, _ = _tiny(n_hid=6, n_out=4)
    cfg = W.RunConfig(seed=2, n_steps=1, temperature=1e9)
    u = orc.grn_hidden_input(net, theta, imgs)
    r = orc.grn_soft_run(net, cfg, theta, u, np.arange(6))
    # from X = 0 only the 10 production channels are active
    assert np.allclose(r.x_final, 1.0 / 10.0, rtol=1e-8, atol=0)
    # a second step: every gene can now decay too; all 20 channels are active
    # and each gene gains 1/20 by production and loses 1/20 by decay
    X, _ = orc.grn_soft_trace(net, cfg.replace(n_steps=2), theta, u[0], cap=2)
    assert np.allclose(X[1], 0.1, rtol=1e-8) and np.allclose(X[2], 0.1, rtol=1e-8)


def _relaxed_graph(net, cfg, theta, u_row, E, T):
    """Final output levels of the relaxed map of Eq. 4, written out in torch:
    X <- X + softmax((ln a + G)/T) V over the channels with a > 0.
    theta: float64 tensor (U, c, psi used); u_row: float64 tensor."""
    H, O = net.n_hid, net.n_out
    o = net.offsets()
    U = theta[o["U"]:o["c"]].reshape(O, H)
    c = theta[o["c"]:o["psi"]]
    delta = net.delta_min + torch.exp(theta[o["psi"]:])
    V = _change_matrix(net)
    X = torch.zeros(net.n_species, dtype=torch.float64)
    for k in range(E.shape[0]):
        a = torch.cat([net.beta * torch.sigmoid(u_row), delta[:H] * torch.clamp(X[:H], min=0.0),
                       net.beta * torch.sigmoid(c + U @ X[:H]), delta[H:] * torch.clamp(X[H:], min=0.0)])
        act = a.detach() > 0
        z = torch.where(act, (torch.log(torch.where(act, a, torch.ones_like(a))) -
                              torch.log(torch.from_numpy(E[k]))) / T, torch.full_like(a, -math.inf))
        X = X + torch.softmax(z, dim=0) @ V
    return X[H:]


def test_soft_adjoint_matches_autograd_of_the_relaxed_map(orc):
    net, theta, imgs, _ = _tiny(n_hid=5, n_out=3)
    g = np.random.default_rng(3)
    theta = _moved(net, theta, g)
    cfg = W.RunConfig(seed=2, n_steps=60, temperature=0.7)
    image_of = np.array([0, 0, 1, 2, 5])
    u = orc.grn_hidden_input(net, theta, imgs)
    d_obs = g.normal(size=(len(image_of), net.n_out))
    r = orc.grn_soft_run(net, cfg, theta, u, image_of, d_obs=d_obs)
    H, O = net.n_hid, net.n_out
    o = net.offsets()
    for q, m in enumerate(image_of):
        E = np.stack([-np.log(orc.step_uniforms(cfg.seed, cfg.purpose, cfg.epoch, q, k,
                                                net.n_reactions + 1)[1:]) for k in range(cfg.n_steps)])
        th = torch.tensor(theta.astype(np.float64), requires_grad=True)
        ur = torch.tensor(u[m], requires_grad=True)
        Xo = _relaxed_graph(net, cfg, th, ur, E, cfg.temperature)
        assert np.abs(Xo.detach().numpy() - r.obs[q]).max() < 1e-10
        (Xo * torch.from_numpy(d_obs[q])).sum().backward()
        ref = np.concatenate([ur.grad.numpy(), th.grad.numpy()[o["U"]:]])
        gc = r.grad_c[q]
        assert gc.shape == ref.shape == (H + O * H + O + H + O,)
        assert np.abs(gc - ref).max() <= 1e-10 * np.abs(ref).max(), q


def test_soft_adjoint_matches_central_differences(orc):
    """Richardson central differences of the oracle's own relaxed forward
    reproduce its adjoint in every block: hidden pre-activations, U, c, psi."""
    net, theta, imgs, _ = _tiny(n_hid=4, n_out=2)
    g = np.random.default_rng(9)
    theta = _moved(net, theta, g)
    cfg = W.RunConfig(seed=4, n_steps=40, temperature=0.8)
    u = orc.grn_hidden_input(net, theta, imgs)
    m, tid = 1, 7
    d = g.normal(size=net.n_out)
    r = orc.grn_soft_run(net, cfg, theta, u[m:m + 1], [0], traj_ids=[tid], d_obs=d[None, :])
    gc = r.grad_c[0]
    H, O = net.n_hid, net.n_out
    o = net.offsets()
    scale = np.abs(gc).max()
    assert scale > 0

    def F(th, ur):
        s = orc.grn_soft_run(net, cfg, th, ur[None, :], [0], traj_ids=[tid], theta64=True)
        return float(s.obs[0] @ d)

    th64 = theta.astype(np.float64)
    checks = [("u", h) for h in range(H)] + [("th", o["U"] + i) for i in (0, 3, O * H - 1)] + \
             [("th", o["c"] + i) for i in range(O)] + [("th", o["psi"] + i) for i in range(H + O)]
    for kind, idx in checks:
        def central(h):
            base = u[m] if kind == "u" else th64
            p_, m_ = base.copy(), base.copy()
            p_[idx] += h
            m_[idx] -= h
            if kind == "u":
                return (F(th64, p_) - F(th64, m_)) / (2 * h)
            return (F(p_, u[m]) - F(m_, u[m])) / (2 * h)
        fd = (4 * central(5e-4) - central(1e-3)) / 3
        k = idx if kind == "u" else H + (idx - o["U"])
        assert abs(fd - gc[k]) <= 1e-6 * scale, (kind, idx, fd, gc[k])
