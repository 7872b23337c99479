"""Pins of the oracle's forward simulation against exact results.

- The chemical master equation (Eq. 1) of 2A <-> A2 with A(0)=100 is a 51-state
  chain; its transient law, the expected event count and the exact bin averages
  of E[A(t)] follow from matrix exponentials of the generator.
- Textbook special cases: A -> 0 (binomial), 0 <-> A from 0 (Poisson),
  A <-> B (binomial).
- The Gumbel-max theorem of Sec. 3.2: selection frequencies a_j/a0 and
  tau ~ Exp(a0).
- Invariants: A + 2 A2 = 100; promoter conservation in the oscillator;
  absorption of the closed/open/inactivated channel scheme (Sec. 4.4).
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from paper_2602_19775_amd import workloads as W


def _chi2_ok(counts, probs, min_expected=5.0, alpha=1e-4):
    counts = np.asarray(counts, np.float64)
    probs = np.asarray(probs, np.float64)
    n = counts.sum()
    exp_ = probs * n
    # merge cells with small expectation into one
    order = np.argsort(exp_)
    small = exp_ < min_expected
    obs_m = list(counts[~small]) + ([counts[small].sum()] if small.any() else [])
    exp_m = list(exp_[~small]) + ([exp_[small].sum()] if small.any() else [])
    exp_m = np.asarray(exp_m)
    exp_m *= n / exp_m.sum()
    stat, p = scipy.stats.chisquare(obs_m, exp_m)
    return p > alpha, p


def dimer_generator(kf, kb, a_total=100):
    n2 = np.arange(a_total // 2 + 1)
    A = a_total - 2 * n2
    up = kf * A * (A - 1) / 2.0
    down = kb * n2
    S = len(n2)
    Q = np.zeros((S, S))
    for i in range(S):
        if i + 1 < S:
            Q[i, i + 1] = up[i]
        if i > 0:
            Q[i, i - 1] = down[i]
        Q[i, i] = -(up[i] + down[i])
    return Q, A.astype(np.float64), up + down


def augmented_integral(Q, p0, f, t):
    """[p(t), int_0^t p(s).f ds] via the exponential of the augmented generator."""
    S = Q.shape[0]
    G = np.zeros((S + 1, S + 1))
    G[:S, :S] = Q
    G[:S, S] = f
    v = np.concatenate([p0, [0.0]]) @ scipy.linalg.expm(G * t)
    return v[:S], v[S]


def test_cme_dimer_expected_event_count(orc):
    kf, kb = 1e-3, 0.1
    Q, A, a0 = dimer_generator(kf, kb)
    p0 = np.zeros(Q.shape[0]); p0[0] = 1.0
    _, expected_steps = augmented_integral(Q, p0, a0, 50.0)
    assert abs(expected_steps - 193.59) < 0.01      # value derived when the workload was specified
    w = W.dimer_forward_1k()
    n = 20000
    r = orc.run(w.net, w.cfg, w.theta, w.net.x0, traj_ids=np.arange(n))
    m = r.steps_done.mean()
    se = r.steps_done.std() / math.sqrt(n)
    assert abs(m - expected_steps) < 4.5 * se, (m, expected_steps, se)
    assert np.all(r.t_final <= 50.0)
    assert np.all(r.x_final[:, 0] + 2 * r.x_final[:, 1] == 100)


def test_cme_dimer_bin_averages(orc):
    """Exact bin averages of E[A(t)] on [0, 50] vs the oracle's O1 observable."""
    kf, kb = 1e-3, 0.1
    Q, A, _ = dimer_generator(kf, kb)
    p0 = np.zeros(Q.shape[0]); p0[0] = 1.0
    nb, t_obs = 10, 50.0
    edges = np.linspace(0, t_obs, nb + 1)
    cum = np.array([augmented_integral(Q, p0, A, t)[1] for t in edges])
    exact = np.diff(cum) / (t_obs / nb)
    net = W.dimerization_2a(kf, kb, 100)
    cfg = W.RunConfig(t_end=60.0, obs_kind=W.OBS_BINS, n_bins=nb, t_obs=t_obs)
    n = 20000
    r = orc.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(n))
    obs = r.obs[:, :, 0]
    m, se = obs.mean(0), obs.std(0) / math.sqrt(n)
    assert np.all(np.abs(m - exact) < 5 * se + 1e-12), (m, exact, se)
    # first bin is almost deterministic near A=100: check tightly too
    assert abs(m[0] - exact[0]) < 0.05


def test_cme_dimer_transient_distribution(orc):
    kf, kb = 1e-3, 0.1
    Q, A, _ = dimer_generator(kf, kb)
    p0 = np.zeros(Q.shape[0]); p0[0] = 1.0
    p = p0 @ scipy.linalg.expm(Q * 20.0)
    net = W.dimerization_2a(kf, kb, 100)
    cfg = W.RunConfig(t_end=20.0, obs_kind=W.OBS_FINAL)
    n = 40000
    r = orc.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(n), obs_species=[1])
    counts = np.bincount(r.x_final[:, 1], minlength=len(p))[:len(p)]
    ok, pv = _chi2_ok(counts, p)
    assert ok, pv
    # stationary moments quoted for this workload
    pinf = scipy.linalg.null_space(Q.T)[:, 0]
    pinf /= pinf.sum()
    assert abs(pinf @ A - 61.9274) < 1e-3
    assert abs(pinf @ A ** 2 - (pinf @ A) ** 2 - 34.1831) < 1e-3


def test_decay_binomial_and_bins(orc):
    k, a0, T = 0.2, 50, 3.0
    net = W.decay(k, a0)
    n = 40000
    r = orc.run(net, W.RunConfig(t_end=T), net.theta0, net.x0, traj_ids=np.arange(n))
    probs = scipy.stats.binom.pmf(np.arange(a0 + 1), a0, math.exp(-k * T))
    ok, pv = _chi2_ok(np.bincount(r.x_final[:, 0], minlength=a0 + 1), probs)
    assert ok, pv
    nb = 6
    cfg = W.RunConfig(t_end=T + 1, obs_kind=W.OBS_BINS, n_bins=nb, t_obs=T)
    r = orc.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(n))
    e = np.linspace(0, T, nb + 1)
    exact = a0 * (np.exp(-k * e[:-1]) - np.exp(-k * e[1:])) / (k * (T / nb))
    obs = r.obs[:, :, 0]
    assert np.all(np.abs(obs.mean(0) - exact) < 5 * obs.std(0) / math.sqrt(n))


def test_birth_death_poisson(orc):
    kb_, kd, T = 20.0, 0.5, 6.0
    net = W.birth_death(kb_, kd, 0)
    n = 40000
    r = orc.run(net, W.RunConfig(t_end=T), net.theta0, net.x0, traj_ids=np.arange(n))
    lam = kb_ / kd * (1 - math.exp(-kd * T))
    top = int(lam + 12 * math.sqrt(lam))
    probs = scipy.stats.poisson.pmf(np.arange(top + 1), lam)
    probs[-1] += 1 - probs.sum()
    c = np.bincount(np.minimum(r.x_final[:, 0], top), minlength=top + 1)
    ok, pv = _chi2_ok(c, probs)
    assert ok, pv


def test_isomerization_binomial(orc):
    kab, kba, nmol, T = 0.3, 0.7, 40, 2.0
    net = W.isomerization(kab, kba, nmol)
    n = 40000
    r = orc.run(net, W.RunConfig(t_end=T), net.theta0, net.x0, traj_ids=np.arange(n))
    pi_a = kba / (kab + kba)
    pa = pi_a + (1 - pi_a) * math.exp(-(kab + kba) * T)
    probs = scipy.stats.binom.pmf(np.arange(nmol + 1), nmol, pa)
    ok, pv = _chi2_ok(np.bincount(r.x_final[:, 0], minlength=nmol + 1), probs)
    assert ok, pv
    assert np.all(r.x_final.sum(1) == nmol)


def _parallel_sources(rates):
    M = len(rates)
    sp = [f"S{j}" for j in range(M)]
    return W._net("sources", sp, [((), j, {sp[j]: +1}) for j in range(M)], M, np.log(rates),
                  [0] * M, sp[:1])


def test_gumbel_max_selects_categorically(orc):
    """Sec. 3.2: argmax(ln a_j + G_j) is a draw from a_j/a0; tau ~ Exp(a0)."""
    rates = np.array([0.5, 1.0, 2.0, 4.0, 0.25, 7.25])
    net = _parallel_sources(rates)
    n = 200000
    r = orc.run(net, W.RunConfig(n_steps=1), net.theta0, net.x0, traj_ids=np.arange(n))
    assert np.all(r.steps_done == 1)
    j = np.argmax(r.x_final, axis=1)
    probs = np.exp(net.theta0.astype(np.float64))
    probs /= probs.sum()
    ok, pv = _chi2_ok(np.bincount(j, minlength=len(rates)), probs)
    assert ok, pv
    a0 = np.exp(net.theta0.astype(np.float64)).sum()
    ks = scipy.stats.kstest(r.t_final, "expon", args=(0, 1 / a0))
    assert ks.pvalue > 1e-4


def test_exponential_race_equals_gumbel_max(orc):
    """The oracle's argmin E_j/a_j picks exactly argmax_j [ln a_j + G_j] with
    G_j = -ln(-ln u_j) (Sec. 3.2), and its margin is the gap of the two best."""
    net = W.oscillator()
    cfg = W.RunConfig(n_steps=3000)
    tr = orc.trace(net, cfg, net.theta0, net.x0, traj_id=5, cap=3000)
    assert len(tr.j) == 3000
    with np.errstate(divide="ignore"):
        score = np.log(tr.a) - np.log(-np.log(tr.u[:, 1:]))
    assert np.array_equal(np.argmax(score, axis=1), tr.j)
    srt = np.sort(score, axis=1)
    gap = srt[:, -1] - srt[:, -2]
    finite = np.isfinite(gap)
    # score gap g <-> ratio margin exp(g) - 1
    assert np.allclose(np.expm1(gap[finite]), tr.margin[finite], rtol=1e-6, atol=1e-12)
    # tau = -ln(u_0)/a0
    assert np.allclose(tr.tau, -np.log(tr.u[:, 0]) / tr.a.sum(1), rtol=1e-14)
    assert np.allclose(np.diff(tr.t), tr.tau, rtol=1e-12)


def test_invariants_along_paths(orc):
    net = W.dimerization_2a()
    tr = orc.trace(net, W.RunConfig(n_steps=5000), net.theta0, net.x0, traj_id=3, cap=5000)
    assert np.all(tr.X[:, 0] + 2 * tr.X[:, 1] == 100) and np.all(tr.X >= 0)
    osc = W.oscillator()
    tr = orc.trace(osc, W.RunConfig(n_steps=20000), osc.theta0, osc.x0, traj_id=9, cap=20000)
    assert np.all(tr.X >= 0)
    assert np.all(tr.X[:, 0] + tr.X[:, 1] == 1) and np.all(tr.X[:, 2] + tr.X[:, 3] == 1)
    # each step changes the state by exactly the fired change vector
    assert np.array_equal(np.diff(tr.X, axis=0), osc.stoich[tr.j])


def test_absorbing_channel_freezes(orc):
    net = W.ion_channel_coi()
    n = 2000
    r = orc.run(net, W.RunConfig(n_steps=1000), net.theta0, net.x0, traj_ids=np.arange(n))
    assert np.all(r.x_final[:, 2] == 2) and np.all(r.x_final.sum(1) == 2)
    assert np.all(r.steps_done < 1000)
    # every path needs an even count of C<->O flips plus two inactivations
    assert np.all(r.steps_done >= 4)


def test_step_and_time_limits(orc):
    net = W.dimerization_2a()
    r = orc.run(net, W.RunConfig(n_steps=37, t_end=5.0), net.theta0, net.x0, traj_ids=np.arange(500))
    assert np.all(r.steps_done <= 37) and np.all(r.t_final <= 5.0)
    assert np.any(r.steps_done == 37) or np.all(r.t_final <= 5.0)


def test_inverse_cdf_selects_categorically(orc):
    """The standard direct method (Sec. 2): the first j whose cumulative
    propensity exceeds u a0 is a draw from a_j/a0, from its own uniform."""
    rates = np.array([0.5, 1.0, 2.0, 4.0, 0.25, 7.25])
    net = _parallel_sources(rates)
    n = 200000
    cfg = W.RunConfig(n_steps=1, selection=W.SELECT_INVERSE_CDF)
    r = orc.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(n))
    j = np.argmax(r.x_final, axis=1)
    probs = np.exp(net.theta0.astype(np.float64))
    probs /= probs.sum()
    ok, pv = _chi2_ok(np.bincount(j, minlength=len(rates)), probs)
    assert ok, pv


def test_inverse_cdf_reads_the_cumulative_sum(orc):
    """Along an oscillator path the chosen channel is the cumulative sum's
    crossing of u_1 a0, and the margin is the nearest interior boundary."""
    net = W.oscillator()
    cfg = W.RunConfig(n_steps=2000, selection=W.SELECT_INVERSE_CDF)
    tr = orc.trace(net, cfg, net.theta0, net.x0, traj_id=9, cap=2000)
    c = np.cumsum(tr.a, axis=1)
    a0 = c[:, -1]
    target = tr.u[:, 1] * a0
    j = np.argmax(c > target[:, None], axis=1)
    assert np.array_equal(j, tr.j)
    active = tr.a > 0
    last = active.shape[1] - 1 - np.argmax(active[:, ::-1], axis=1)
    d = np.abs(c - target[:, None]) / a0[:, None]
    d[~active] = np.inf
    d[np.arange(len(last)), last] = np.inf
    assert np.allclose(d.min(axis=1), tr.margin, rtol=1e-9, atol=1e-15)


def test_inverse_cdf_isomerization_binomial(orc):
    kab, kba, nmol, T = 0.3, 0.7, 40, 2.0
    net = W.isomerization(kab, kba, nmol)
    n = 40000
    r = orc.run(net, W.RunConfig(t_end=T, selection=W.SELECT_INVERSE_CDF), net.theta0, net.x0,
                traj_ids=np.arange(n))
    pi_a = kba / (kab + kba)
    pa = pi_a + (1 - pi_a) * math.exp(-(kab + kba) * T)
    probs = scipy.stats.binom.pmf(np.arange(nmol + 1), nmol, pa)
    ok, pv = _chi2_ok(np.bincount(r.x_final[:, 0], minlength=nmol + 1), probs)
    assert ok, pv


def test_inverse_cdf_has_no_backward(orc):
    net = W.dimerization_2a()
    cfg = W.RunConfig(n_steps=10, selection=W.SELECT_INVERSE_CDF)
    with pytest.raises(Exception):
        orc.run(net, cfg, net.theta0, net.x0[None, :], traj_ids=[0], d_obs=np.zeros((1, 1)))
