"""Seeded synthetic workloads: reaction networks, initial states and run settings.

This module only *describes* inputs.  It holds none of the method's arithmetic
(no propensities, no random streams of the simulation, no gradients): both the
HIP path and the CPU oracle read the same descriptions and each turns them into
its own internal tables.  Host-side choices (random network topologies, rates,
images) use numpy's PCG64 generator seeded explicitly; the simulation's own
random numbers are drawn by each side from its own Philox4x32-10 stream.

Networks follow the problem statement of Sec. 2 of the paper: N species with
integer copy numbers, M reaction channels with mass-action propensities
(order 0, 1, 2, or homodimerisation, Sec. 2) and integer change vectors v_j.
Rate constants are parameterised as theta = ln k (Sec. 4.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import os
from typing import List, Optional, Sequence

import numpy as np

# Observation kinds.
OBS_FINAL = 0   # final copy numbers of the observed species
OBS_BINS = 1    # exact time average of the piecewise-constant path over uniform bins (Sec. 4.4)
OBS_GRID = 2    # the path linearly interpolated between its event points at n_bins uniform
                # times t_obs g / (n_bins - 1), held after the last event (Sec. 4.1)
OBS_TAIL = 3    # the mean of each observed count over the last n_bins of the n_steps + 1
                # states of a run, then the mean of their times (the rate-of-change loss
                # of Sec. 4.2); a run that stops early holds its last state and clock

# Channel selection of the forward: the Gumbel-max (exponential race) of
# Sec. 3.2, or the standard direct method's inverse CDF (Sec. 2), which has
# no straight-through backward.
SELECT_GUMBEL_MAX = 0
SELECT_INVERSE_CDF = 1
# memory order of an observation block: [point][obs][trajectory] or [trajectory][point][obs];
# or only the ensemble means [point][obs] of each network
OBS_POINT_MAJOR = 0
OBS_TRAJ_MAJOR = 1
OBS_ENSEMBLE_MEAN = 2

# Random-stream purposes (high byte of the fourth Philox counter word).
PURPOSE_SIMULATE = 0
PURPOSE_TARGET = 1
PURPOSE_PILOT = 2


@dataclass
class Network:
    """One reaction network.

    reactant[j] = (s1, s2): reactant species of channel j, -1 for none.
      (-1, -1) -> order 0, a = k
      (s, -1)  -> order 1, a = k X_s
      (s, s')  -> order 2, a = k X_s X_s'       (s != s')
      (s, s)   -> homodimer, a = k X_s (X_s - 1) / 2
    rate_index[j]: which entry of theta (= ln k) channel j uses (allows tied rates).
    stoich[j, :]: the change vector v_j.
    """
    name: str
    species: List[str]
    reactant: np.ndarray        # [M, 2] int32
    rate_index: np.ndarray      # [M] int32
    stoich: np.ndarray          # [M, N] int32
    n_params: int
    theta0: np.ndarray          # [P] float32, ln k
    x0: np.ndarray              # [N] int32
    obs_species: np.ndarray     # [n_obs] int32
    param_names: Optional[List[str]] = None

    @property
    def n_species(self) -> int:
        return len(self.species)

    @property
    def n_reactions(self) -> int:
        return int(self.reactant.shape[0])

    def validate(self) -> None:
        M, N = self.n_reactions, self.n_species
        assert self.reactant.shape == (M, 2) and self.stoich.shape == (M, N)
        assert self.rate_index.shape == (M,)
        assert np.all((self.reactant >= -1) & (self.reactant < N))
        # a lone second reactant is not a valid encoding
        assert not np.any((self.reactant[:, 0] < 0) & (self.reactant[:, 1] >= 0))
        assert np.all((self.rate_index >= 0) & (self.rate_index < self.n_params))
        assert np.all(np.abs(self.stoich) <= 2)
        assert self.theta0.shape == (self.n_params,)
        assert self.x0.shape == (N,) and np.all(self.x0 >= 0)
        assert np.all((self.obs_species >= 0) & (self.obs_species < N))


def _net(name, species, reactions, n_params, theta0, x0, obs, param_names=None) -> Network:
    """reactions: list of (reactant tuple, rate slot, {species: delta})."""
    idx = {s: i for i, s in enumerate(species)}
    M, N = len(reactions), len(species)
    reactant = -np.ones((M, 2), np.int32)
    rate_index = np.zeros(M, np.int32)
    stoich = np.zeros((M, N), np.int32)
    for j, (rs, slot, delta) in enumerate(reactions):
        for q, s in enumerate(rs):
            reactant[j, q] = idx[s]
        rate_index[j] = slot
        for s, d in delta.items():
            stoich[j, idx[s]] += d
    net = Network(name, list(species), reactant, rate_index, stoich, n_params,
                  np.asarray(theta0, np.float32), np.asarray(x0, np.int32),
                  np.asarray([idx[s] for s in obs], np.int32), param_names)
    net.validate()
    return net


# --------------------------------------------------------------------------
# Networks named in the paper or used as textbook pins
# --------------------------------------------------------------------------

def dimerization_2a(kf: float = 1.0e-3, kb: float = 0.1, a0: int = 100) -> Network:
    """Reversible homodimerisation 2A <-> A2 with mass-action kinetics (Sec. 2:
    homodimer propensity k X (X-1)/2).  A + 2*A2 is conserved."""
    return _net("dimerization_2A", ["A", "A2"],
                [(("A", "A"), 0, {"A": -2, "A2": +1}),
                 (("A2",), 1, {"A": +2, "A2": -1})],
                2, np.log([kf, kb]), [a0, 0], ["A"], ["ln_kf", "ln_kb"])


def dimerization_abc(k1: float = 0.01, k2: float = 0.32, x0=(100, 90, 0)) -> Network:
    """A + B <-> C of Sec. 4.1 (Eq. 8): a1 = k1 X_A X_B, a2 = k2 X_C."""
    return _net("dimerization_ABC", ["A", "B", "C"],
                [(("A", "B"), 0, {"A": -1, "B": -1, "C": +1}),
                 (("C",), 1, {"A": +1, "B": +1, "C": -1})],
                2, np.log([k1, k2]), list(x0), ["A", "B", "C"], ["ln_k1", "ln_k2"])


def ion_channel_coi(k_open=0.75, k_close=0.103, k_inact=1.159, n_channels: int = 2) -> Network:
    """Closed/open/inactivated channel scheme of Sec. 4.4: C->O, O->C, O->I, with I
    absorbing.  All channels start closed."""
    return _net("ion_channel_COI", ["C", "O", "I"],
                [(("C",), 0, {"C": -1, "O": +1}),
                 (("O",), 1, {"O": -1, "C": +1}),
                 (("O",), 2, {"O": -1, "I": +1})],
                3, np.log([k_open, k_close, k_inact]), [n_channels, 0, 0], ["O"],
                ["ln_k_open", "ln_k_close", "ln_k_inact"])


def decay(k: float = 0.2, a0: int = 50) -> Network:
    """A -> 0.  Closed form: A(t) ~ Binomial(A0, exp(-k t))."""
    return _net("decay", ["A"], [(("A",), 0, {"A": -1})], 1, np.log([k]), [a0], ["A"])


def birth_death(k_birth: float = 20.0, k_death: float = 0.5, a0: int = 0) -> Network:
    """0 -> A, A -> 0.  Stationary law Poisson(k_birth / k_death)."""
    return _net("birth_death", ["A"],
                [((), 0, {"A": +1}), (("A",), 1, {"A": -1})],
                2, np.log([k_birth, k_death]), [a0], ["A"])


def isomerization(k_ab: float = 0.3, k_ba: float = 0.7, n: int = 40) -> Network:
    """A <-> B with A + B = n.  Stationary law A ~ Binomial(n, k_ba / (k_ab + k_ba))."""
    return _net("isomerization", ["A", "B"],
                [(("A",), 0, {"A": -1, "B": +1}), (("B",), 1, {"A": +1, "B": -1})],
                2, np.log([k_ab, k_ba]), [n, 0], ["A"])


OSC_SPECIES = ["D_A", "D_A'", "D_R", "D_R'", "M_A", "M_R", "A", "R", "C"]
OSC_PARAMS = ["gamma_A", "theta_A", "gamma_R", "theta_R", "alpha_A", "alpha'_A",
              "alpha_R", "alpha'_R", "beta_A", "beta_R", "delta_MA", "delta_MR",
              "delta_A", "delta_R", "gamma_C"]


# Nominal rates of the activator-repressor oscillator as published with the
# model (Vilar, Kueh, Barkai and Leibler, PNAS 2002, the paper's ref. 30), per
# hour and per molecule: promoter binding and release, transcription from the
# free and bound promoters, translation, mRNA and protein decay, complex
# formation.  The paper's five protein rates (Sec. 4.2) are these values.
OSC_NOMINAL_RATES = {
    "gamma_A": 1.0, "theta_A": 50.0, "gamma_R": 1.0, "theta_R": 100.0,
    "alpha_A": 50.0, "alpha'_A": 500.0, "alpha_R": 0.01, "alpha'_R": 50.0,
    "beta_A": 50.0, "beta_R": 5.0, "delta_MA": 10.0, "delta_MR": 0.5,
    "delta_A": 1.0, "delta_R": 0.2, "gamma_C": 2.0,
}


def oscillator(rates=None, rate_seed: Optional[int] = None, log10_range=(-2.0, 3.0)) -> Network:
    """Activator-repressor oscillator of Sec. 4.2: 9 species, 16 mass-action channels
    (promoter binding/unbinding, transcription from both promoter states,
    translation, mRNA and protein degradation, A+R->C, C->R).  The complex C
    releases R at the activator's degradation rate, so 16 channels use 15 rates.
    Rates: the given vector (OSC_PARAMS order), else log-uniform seeded ones if
    rate_seed is given, else the nominal ones (OSC_NOMINAL_RATES).  Starts with
    one free copy of each promoter and nothing else."""
    if rates is None:
        if rate_seed is None:
            rates = [OSC_NOMINAL_RATES[p] for p in OSC_PARAMS]
        else:
            g = np.random.default_rng(np.random.SeedSequence([rate_seed, 3]))
            rates = 10.0 ** g.uniform(log10_range[0], log10_range[1], size=15)
    rates = np.asarray(rates, np.float64)
    assert rates.shape == (15,)
    P = {n: i for i, n in enumerate(OSC_PARAMS)}
    R = [
        (("D_A", "A"), P["gamma_A"], {"D_A": -1, "A": -1, "D_A'": +1}),
        (("D_A'",), P["theta_A"], {"D_A'": -1, "D_A": +1, "A": +1}),
        (("D_R", "A"), P["gamma_R"], {"D_R": -1, "A": -1, "D_R'": +1}),
        (("D_R'",), P["theta_R"], {"D_R'": -1, "D_R": +1, "A": +1}),
        (("D_A",), P["alpha_A"], {"M_A": +1}),
        (("D_A'",), P["alpha'_A"], {"M_A": +1}),
        (("D_R",), P["alpha_R"], {"M_R": +1}),
        (("D_R'",), P["alpha'_R"], {"M_R": +1}),
        (("M_A",), P["beta_A"], {"A": +1}),
        (("M_R",), P["beta_R"], {"R": +1}),
        (("M_A",), P["delta_MA"], {"M_A": -1}),
        (("M_R",), P["delta_MR"], {"M_R": -1}),
        (("A",), P["delta_A"], {"A": -1}),
        (("R",), P["delta_R"], {"R": -1}),
        (("A", "R"), P["gamma_C"], {"A": -1, "R": -1, "C": +1}),
        (("C",), P["delta_A"], {"C": -1, "R": +1}),
    ]
    x0 = [1, 0, 1, 0, 0, 0, 0, 0, 0]
    return _net("oscillator", OSC_SPECIES, R, 15, np.log(rates), x0, ["R"], list(OSC_PARAMS))


# The five protein rates of the oscillator that the start-point-map inference
# of Sec. 4.2 recovers (their values there are the nominal ones).
OSC_PROTEIN_PARAMS = ("beta_A", "beta_R", "delta_A", "delta_R", "gamma_C")
OSC_PROTEIN_RATES = tuple(OSC_NOMINAL_RATES[p] for p in OSC_PROTEIN_PARAMS)


def start_point_oscillator(protein_rates=OSC_PROTEIN_RATES) -> Network:
    """The oscillator of the start-point-map inference (Sec. 4.2), observing
    the three proteins A, R and C, with the given protein rates (beta_A,
    beta_R, delta_A, delta_R, gamma_C) and the other rates nominal."""
    rates = np.array([OSC_NOMINAL_RATES[p] for p in OSC_PARAMS])
    for name, k in zip(OSC_PROTEIN_PARAMS, protein_rates):
        rates[OSC_PARAMS.index(name)] = k
    net = oscillator(rates)
    idx = {s_: i for i, s_ in enumerate(net.species)}
    net.obs_species = np.asarray([idx["A"], idx["R"], idx["C"]], np.int32)
    net.name = "start_point_oscillator"
    net.validate()
    return net


def random_network(g: np.random.Generator, name: str = "random",
                   n_range=(4, 64), m_range=(8, 256), log10_k=(-3.0, 2.0),
                   x0_mean: float = 50.0) -> Network:
    """One random mass-action network: orders 0-2 (order-2 channels are
    homodimers or heterodimers with equal odds), reactants consumed, 0-2
    product molecules on uniform species, change vectors in {-2..2}, never zero.
    One rate per channel, log-uniform; Poisson initial counts."""
    N = int(g.integers(n_range[0], n_range[1] + 1))
    M = int(g.integers(m_range[0], m_range[1] + 1))
    reactant = -np.ones((M, 2), np.int32)
    stoich = np.zeros((M, N), np.int32)
    for j in range(M):
        while True:
            order = int(g.integers(0, 3))
            r = -np.ones(2, np.int32)
            v = np.zeros(N, np.int32)
            if order >= 1:
                r[0] = g.integers(0, N)
            if order == 2:
                r[1] = r[0] if g.random() < 0.5 else g.integers(0, N)
            for s in r:
                if s >= 0:
                    v[s] -= 1
            for _ in range(int(g.integers(0, 3))):
                v[g.integers(0, N)] += 1
            if np.any(v != 0) and np.all(np.abs(v) <= 2):
                break
        reactant[j] = r
        stoich[j] = v
    theta0 = np.log(10.0 ** g.uniform(log10_k[0], log10_k[1], size=M))
    x0 = g.poisson(x0_mean, size=N).astype(np.int32)
    obs = np.arange(min(N, 4), dtype=np.int32)
    net = Network(name, [f"S{i}" for i in range(N)], reactant,
                  np.arange(M, dtype=np.int32), stoich, M,
                  theta0.astype(np.float32), x0, obs)
    net.validate()
    return net


def random_network_batch(n_networks: int, seed: int = 0, **kw) -> List[Network]:
    g = np.random.default_rng(np.random.SeedSequence([seed, 3]))
    return [random_network(g, name=f"random_{i}", **kw) for i in range(n_networks)]


# --------------------------------------------------------------------------
# Run settings
# --------------------------------------------------------------------------

@dataclass
class RunConfig:
    seed: int = 0
    purpose: int = PURPOSE_SIMULATE
    epoch: int = 0
    n_steps: int = 2 ** 31 - 1        # fired reactions per trajectory (upper bound)
    t_end: float = float("inf")       # fire only while t + tau <= t_end
    obs_kind: int = OBS_FINAL
    n_bins: int = 0
    t_obs: float = 0.0
    temperature: float = 0.5
    ckpt_every: int = 256
    selection: int = 0                # SELECT_GUMBEL_MAX or SELECT_INVERSE_CDF (forward only)
    obs_layout: int = 0               # OBS_POINT_MAJOR, OBS_TRAJ_MAJOR or OBS_ENSEMBLE_MEAN
    dobs_shared: bool = False         # d_obs is one block per network (a loss of ensemble means)
    relaxed: bool = False             # gene network: the relaxed forward of Eq. 4 and its backward

    def replace(self, **kw) -> "RunConfig":
        d = dict(self.__dict__)
        d.update(kw)
        return RunConfig(**d)


@dataclass
class Workload:
    """A network, its trajectory count and run settings, named by what it is."""
    name: str
    net: Network
    n_traj: int
    cfg: RunConfig
    theta: np.ndarray = None          # ln k used for the run (float32)
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.theta is None:
            self.theta = self.net.theta0.copy()

    def x0_soa(self) -> np.ndarray:
        """[N, B] int32, every trajectory starts from net.x0."""
        return np.repeat(self.net.x0[:, None], self.n_traj, axis=1).astype(np.int32)


def dimer_forward_1k() -> Workload:
    """2A<->A2, kf=1e-3, kb=0.1, A(0)=100, 1,024 trajectories to t_end=50, final state."""
    net = dimerization_2a(1.0e-3, 0.1, 100)
    return Workload("dimer_2A_1024traj_tend50", net, 1024,
                    RunConfig(seed=0, t_end=50.0, obs_kind=OBS_FINAL, n_steps=2 ** 31 - 1))


DIMER_TARGET_RATES = (2.0e-3, 0.05)


def dimer_fwdbwd_64k(n_traj: int = 65536, n_steps: int = 10000) -> Workload:
    """2A<->A2 at kf=1e-3, kb=0.1 with gradients: 65,536 trajectories x 10,000 steps,
    20 exact bin averages of A on [0, 2500], temperature 0.5, checkpoints every 256."""
    net = dimerization_2a(1.0e-3, 0.1, 100)
    cfg = RunConfig(seed=0, n_steps=n_steps, obs_kind=OBS_BINS, n_bins=20, t_obs=2500.0,
                    temperature=0.5, ckpt_every=256)
    return Workload(f"dimer_2A_{n_traj}traj_{n_steps}steps_20bins", net, n_traj, cfg)


# Observation window of the oscillator workload: 0.9 x the 1st percentile of the
# clock after 200,000 steps in a 64-trajectory pilot run of the FP64 oracle
# (pilot stream, seeded rates of rate_seed 0); tests/golden/oscillator_pilot.py
# recomputes it.
OSC_T_OBS = 124299.29021959605


def oscillator_fwdbwd_64k(n_traj: int = 65536, n_steps: int = 200000, t_obs: float = OSC_T_OBS) -> Workload:
    """Activator-repressor oscillator with 15 log-uniform seeded rates in
    [1e-2, 1e3] (rate_seed 0): 65,536 trajectories x 200,000 steps, 256 exact
    bin averages of R on [0, t_obs], temperature 0.5, checkpoints every 1,024
    steps.  Targets come from a second seeded rate vector (rate_seed 1)."""
    net = oscillator(rate_seed=0)
    cfg = RunConfig(seed=0, n_steps=n_steps, obs_kind=OBS_BINS, n_bins=256, t_obs=t_obs,
                    temperature=0.5, ckpt_every=1024)
    return Workload(f"oscillator_{n_traj}traj_{n_steps}steps_256bins", net, n_traj, cfg,
                    extra={"target_net": oscillator(rate_seed=1)})


@dataclass
class BatchWorkload:
    """Several networks run together in one launch."""
    name: str
    nets: List[Network]
    n_traj: List[int]
    cfg: RunConfig
    target_nets: List[Network] = None
    t_obs: List[float] = None         # per-network observation windows (bins)

    def theta(self) -> np.ndarray:
        return np.concatenate([n.theta0 for n in self.nets]).astype(np.float32)

    def x0_packed(self) -> np.ndarray:
        return np.concatenate([np.repeat(n.x0[:, None], b, axis=1).reshape(-1)
                               for n, b in zip(self.nets, self.n_traj)]).astype(np.int32)


# Observation windows of the uneven batch (seed 0, in network order), written by
# tests/golden/uneven_pilot.py from an FP64 oracle pilot run.
UNEVEN_T_OBS_FILE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                                 "uneven_t_obs.txt")


def uneven_t_obs(n_networks: int) -> List[float]:
    with open(UNEVEN_T_OBS_FILE) as f:
        vals = [float(line) for line in f if line.strip() and not line.startswith("#")]
    if n_networks > len(vals):
        raise ValueError(f"the pilot file holds {len(vals)} networks")
    return vals[:n_networks]


def uneven_batch(n_networks: int = 4096, traj_per_network: int = 256, n_steps: int = 5000,
                 seed: int = 0, obs_kind: int = OBS_BINS, n_bins: int = 4) -> BatchWorkload:
    """4,096 random mass-action networks (4-64 species, 8-256 channels, orders
    0-2, change vectors in {-2..2}, log-uniform rates in [1e-3, 1e2], Poisson(50)
    initial counts), 256 trajectories each, 5,000 steps, temperature 0.5,
    checkpoints every 256 steps.  Observation: exact averages of up to 4
    observed species over 4 bins of each network's own window t_obs (0.9 x the
    smallest clock after 5,000 steps in an oracle pilot, seed 0), or their
    final counts.  Targets use the same networks with every rate scaled by a
    seeded factor in [0.5, 2]."""
    nets = random_network_batch(n_networks, seed=seed)
    g = np.random.default_rng(np.random.SeedSequence([seed, 4]))
    targets = []
    for n in nets:
        t = Network(n.name, n.species, n.reactant, n.rate_index, n.stoich, n.n_params,
                    (n.theta0 + np.log(g.uniform(0.5, 2.0, size=n.n_params))).astype(np.float32),
                    n.x0, n.obs_species, n.param_names)
        targets.append(t)
    t_obs = None
    if obs_kind == OBS_BINS:
        if seed != 0:
            raise ValueError("the pilot windows cover the seed-0 batch")
        t_obs = uneven_t_obs(n_networks)
        cfg = RunConfig(seed=seed, n_steps=n_steps, obs_kind=OBS_BINS, n_bins=n_bins, temperature=0.5,
                        ckpt_every=256)
    else:
        cfg = RunConfig(seed=seed, n_steps=n_steps, obs_kind=OBS_FINAL, temperature=0.5, ckpt_every=256)
    kind = f"{n_bins}bins" if obs_kind == OBS_BINS else "final"
    return BatchWorkload(f"uneven_{n_networks}nets_{traj_per_network}traj_{n_steps}steps_{kind}", nets,
                         [traj_per_network] * n_networks, cfg, targets, t_obs)


# --------------------------------------------------------------------------
# Gene-regulatory network classifier (Sec. 4.3, Fig. 4A)
# --------------------------------------------------------------------------

@dataclass
class GrnNet:
    """Feed-forward gene network: n_in fixed input factors (an image's pixels),
    n_hid hidden genes, n_out output genes.  Every gene is produced at
    beta * P(ON) with P(ON) = sigmoid(bias + sum of weighted regulator levels)
    and decays at delta = delta_min + exp(psi).  Parameters, packed:
    [W (n_hid x n_in) | b (n_hid) | U (n_out x n_hid) | c (n_out) | psi (n_hid + n_out)]."""
    n_in: int = 784
    n_hid: int = 256
    n_out: int = 10
    beta: float = 10.0
    delta_min: float = 0.25

    @property
    def n_species(self) -> int:
        return self.n_hid + self.n_out

    @property
    def n_reactions(self) -> int:
        return 2 * (self.n_hid + self.n_out)

    @property
    def n_params(self) -> int:
        return self.n_hid * self.n_in + self.n_hid + self.n_out * self.n_hid + self.n_out + self.n_hid + self.n_out

    @property
    def n_compact(self) -> int:
        """Width of a trajectory's compact gradient [du | dU | dc | dpsi]."""
        return self.n_hid + self.n_out * self.n_hid + self.n_out + self.n_hid + self.n_out

    def offsets(self) -> dict:
        I, H, O = self.n_in, self.n_hid, self.n_out
        o = {"W": 0, "b": H * I}
        o["U"] = o["b"] + H
        o["c"] = o["U"] + O * H
        o["psi"] = o["c"] + O
        return o

    def split(self, theta: np.ndarray) -> dict:
        """Views of a packed parameter vector."""
        I, H, O = self.n_in, self.n_hid, self.n_out
        o = self.offsets()
        return {"W": theta[o["W"]:o["b"]].reshape(H, I), "b": theta[o["b"]:o["U"]],
                "U": theta[o["U"]:o["c"]].reshape(O, H), "c": theta[o["c"]:o["psi"]],
                "psi": theta[o["psi"]:]}


def grn_init_params(net: GrnNet, seed: int = 0, delta0: float = 1.0) -> np.ndarray:
    """Glorot-uniform W and U, zero biases, every decay rate delta0
    (psi = ln(delta0 - delta_min)).  float32."""
    g = np.random.default_rng(np.random.SeedSequence([seed, 5]))
    I, H, O = net.n_in, net.n_hid, net.n_out
    lim_w = np.sqrt(6.0 / (I + H))
    lim_u = np.sqrt(6.0 / (H + O))
    W = g.uniform(-lim_w, lim_w, size=(H, I))
    U = g.uniform(-lim_u, lim_u, size=(O, H))
    psi = np.full(H + O, np.log(delta0 - net.delta_min))
    return np.concatenate([W.reshape(-1), np.zeros(H), U.reshape(-1), np.zeros(O), psi]).astype(np.float32)


def grn_images(n_images: int, seed: int = 0, side: int = 28, n_classes: int = 10):
    """Synthetic stand-ins with the shape of handwritten-digit images: each of
    n_classes prototypes is a sum of 3 Gaussian blobs (centres uniform in
    [4, side-4]^2, widths uniform in [1.5, 3.5] px); an image is its class
    prototype plus N(0, 0.15^2) pixel noise, clipped to [0, 1] and quantised to
    levels p/256 (p integer), which bfloat16 represents exactly.
    Image m has class m mod n_classes.  Returns (float32 [n_images, side*side],
    int64 labels)."""
    g = np.random.default_rng(np.random.SeedSequence([seed, 3]))
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    protos = []
    for _ in range(n_classes):
        img = np.zeros((side, side))
        for _ in range(3):
            cy, cx = g.uniform(4.0, side - 4.0, size=2)
            s = g.uniform(1.5, 3.5)
            img += np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
        protos.append(np.clip(img, 0.0, 1.0))
    labels = np.arange(n_images) % n_classes
    imgs = np.stack([protos[c] for c in labels]) + g.normal(0.0, 0.15, size=(n_images, side, side))
    imgs = np.round(np.clip(imgs, 0.0, 1.0) * 256.0) / 256.0
    return imgs.reshape(n_images, side * side).astype(np.float32), labels.astype(np.int64)


@dataclass
class GrnWorkload:
    name: str
    net: GrnNet
    n_images: int
    n_rep: int                    # trajectories per image (trajectory q runs image q // n_rep)
    cfg: RunConfig
    theta: np.ndarray
    images: np.ndarray            # [n_images, n_in] float32
    labels: np.ndarray            # [n_images]

    @property
    def n_traj(self) -> int:
        return self.n_images * self.n_rep

    def image_of(self) -> np.ndarray:
        return np.arange(self.n_traj) // self.n_rep

    def x0_soa(self) -> np.ndarray:
        return np.zeros((self.net.n_species, self.n_traj), np.int32)


def grn_classifier(n_images: int = 512, n_rep: int = 32, n_steps: int = 2000, seed: int = 0,
                   net: GrnNet = None) -> GrnWorkload:
    """784 -> 256 -> 10 gene network on synthetic 28x28 images: 512 images x 32
    trajectories, 2,000 steps from zero counts, final output counts observed,
    temperature 1.0."""
    net = net or GrnNet()
    side = int(round(np.sqrt(net.n_in)))
    imgs, labels = grn_images(n_images, seed=seed, side=side)
    cfg = RunConfig(seed=seed, n_steps=n_steps, obs_kind=OBS_FINAL, temperature=1.0)
    return GrnWorkload(f"grn_{net.n_in}x{net.n_hid}x{net.n_out}_{n_images}img_{n_rep}rep_{n_steps}steps",
                       net, n_images, n_rep, cfg, grn_init_params(net, seed), imgs, labels)
