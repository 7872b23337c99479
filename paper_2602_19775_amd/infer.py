"""Rate inference on the library: the reversible dimerisation A + B <-> C
(Sec. 4.1) and the closed/open/inactivated ion channel (Sec. 4.4).

- **Target.** A target ensemble at the true rates (its own random stream),
  observed like the model: for the dimerisation, A, B and C linearly
  interpolated between event points onto a uniform time grid (the library's
  grid observation); for the channel, the open count's exact bin averages.
- **Model.** `n_traj` trajectories at theta = ln k. The loss is the mean over
  observation points and observed species of the squared difference of the
  ensemble means.
- **Gradient.** The library's straight-through backward (Eqs. 3-7, Fig. 1).
- **Optimiser.** RMSprop on theta (decay 0.9, eps 1e-7). The Gumbel-Softmax
  temperature is annealed geometrically over the epochs (Sec. 3.5: 1.0 to
  0.001 for the dimerisation, 0.05 to 0.0005 for the channel), the learning
  rate geometrically as well (the channel's in proportion to the
  temperature, Sec. 4.4).
- **Layout.** The observation is summed over the ensemble inside the
  forward, which stores only the means.  The backward reads the loss
  gradient as one block shared by all trajectories (every trajectory's
  dL/dobs is the same for a loss of ensemble means).
- **Graph.** One optimisation step is captured once into a HIP graph and
  replayed per epoch. The step is: forward, loss gradient, backward, RMSprop
  update, schedule update and epoch count. The epoch, the temperature and the
  learning rate live in device scalars that the kernels and the update read,
  so every replay draws fresh noise at the current temperature.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import ssa
from . import workloads as W
from .graph import CapturedStep

TRUE_RATES = (0.01, 0.32)          # k1, k2 of the paper's reference run
START_RATES = (0.125, 0.025)       # its initial guesses
K2_SWEEP = (0.01, 0.02, 0.04, 0.08, 0.16, 0.32, 0.64, 1.28)
X0 = (100, 90, 0)


@dataclass
class InferenceResult:
    k_true: np.ndarray
    k_learned: np.ndarray
    ape: np.ndarray                # absolute percentage error per rate
    loss_first: float
    loss_last: float
    epochs: int
    t_obs: float
    train_s: float                 # wall time of the replayed epochs
    steps_per_epoch: int           # fired reactions of one epoch's forward
    losses: np.ndarray


def grid_end(net: W.Network, n_traj: int, n_steps: int, seed: int) -> float:
    """Grid span: 0.9 x the 1st percentile of the clock after n_steps steps
    of the target ensemble (the grid stays inside every target path)."""
    h = ssa.Net([net], [n_traj])
    cfg = W.RunConfig(seed=seed, purpose=W.PURPOSE_TARGET, n_steps=n_steps, obs_kind=W.OBS_FINAL)
    th = torch.tensor(net.theta0, device="cuda")
    x0 = _x0(net, n_traj)
    f = ssa.forward(h, cfg, th, x0, keep_ckpt=False, tie_capacity=0)
    t = f.t_final.cpu().numpy()
    return 0.9 * float(np.percentile(t, 1.0))


def _x0(net: W.Network, n: int) -> torch.Tensor:
    return torch.tensor(np.repeat(net.x0[:, None], n, axis=1).reshape(-1), dtype=torch.int32, device="cuda")


class Trainer:
    """The captured optimisation step: a model ensemble started at
    `theta_start`, observed like the target ensemble drawn at the true rates
    of `true_net`; the loss is the mean over observation points and observed
    species of the squared difference of the two ensembles' means."""

    def __init__(self, true_net: W.Network, theta_start: Sequence[float], cfg: W.RunConfig, *,
                 n_traj: int, n_target: int, epochs: int, t0: float, t1: float, lr0: float,
                 lr1: Optional[float] = None, rho: float = 0.9, eps: float = 1e-7):
        """lr1=None anneals the learning rate in proportion to the temperature."""
        dev = torch.device("cuda")
        self.true_net = true_net
        self.k_true = np.exp(true_net.theta0.astype(np.float64))
        self.net = true_net
        self.t_obs = cfg.t_obs
        self.epochs = epochs
        self.n_pts = cfg.n_bins if cfg.obs_kind != W.OBS_FINAL else 1
        self.n_obs, self.B = len(true_net.obs_species), n_traj
        self.cfg = cfg.replace(temperature=t0, obs_layout=W.OBS_ENSEMBLE_MEAN, dobs_shared=True)
        P_, O_ = self.n_pts, self.n_obs
        # target ensemble means
        ht = ssa.Net([true_net], [n_target], t_obs=[self.t_obs])
        tf = ssa.forward(ht, self.cfg.replace(purpose=W.PURPOSE_TARGET),
                         torch.tensor(true_net.theta0, device=dev), _x0(true_net, n_target),
                         keep_ckpt=False, tie_capacity=0)
        self.target = self._means_of(ht, tf).view(P_, O_).clone()
        del tf, ht
        # model state and schedules (device scalars)
        self.h = ssa.Net([true_net], [n_traj], t_obs=[self.t_obs])
        self.theta0 = torch.tensor(np.asarray(theta_start, np.float32), device=dev)
        self.theta = self.theta0.clone()
        self.v = torch.zeros_like(self.theta)
        self.x0 = _x0(true_net, n_traj)
        self.epoch = torch.zeros(1, dtype=torch.int32, device=dev)
        self.temp0, self.lr0 = t0, lr0
        self.temp = torch.full((1,), t0, dtype=torch.float32, device=dev)
        self.lr = torch.full((1,), lr0, dtype=torch.float32, device=dev)
        n1 = max(epochs - 1, 1)
        self.r_temp = (t1 / t0) ** (1.0 / n1)
        self.r_lr = self.r_temp if lr1 is None else (lr1 / lr0) ** (1.0 / n1)
        self.rho, self.eps = rho, eps
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.d_obs = torch.zeros(P_ * O_, dtype=torch.float64, device=dev)      # shared by the trajectories
        self.mean = torch.zeros(P_ * O_, dtype=torch.float64, device=dev)
        self.d_params = torch.zeros(self.h.param_total, dtype=torch.float32, device=dev)
        self.bufs = ssa.forward(self.h, self.cfg, self.theta, self.x0, tie_capacity=0, d_epoch=self.epoch,
                                d_temperature=self.temp)
        self.graph: Optional[CapturedStep] = None

    def _means_of(self, h, fwd, out=None) -> torch.Tensor:
        if self.cfg.obs_layout == W.OBS_ENSEMBLE_MEAN:
            return fwd.obs[: self.n_pts * self.n_obs]
        return ssa.obs_mean(h, fwd, out=out)

    def means(self, fwd=None) -> torch.Tensor:
        """Ensemble means [points][species] of the model forward's observation."""
        m = self._means_of(self.h, self.bufs if fwd is None else fwd, out=self.mean)
        return m.view(self.n_pts, self.n_obs)

    def d_obs_of(self, e: torch.Tensor, out: torch.Tensor):
        """dL/dobs = 2 (mean - target) / (points * species * B), the same for
        every trajectory: one shared block [points][species]."""
        torch.mul(e.reshape(-1), 2.0 / (self.n_pts * self.n_obs * self.B), out=out)

    def step(self):
        """One optimisation step on the current stream (preallocated tensors only)."""
        ssa.forward(self.h, self.cfg, self.theta, self.x0, buffers=self.bufs, tie_capacity=0,
                    d_epoch=self.epoch, d_temperature=self.temp)
        e = self.means() - self.target
        self.loss.copy_(e.square().mean().reshape(1))
        self.d_obs_of(e, self.d_obs)
        ssa.backward(self.h, self.cfg, self.theta, self.x0, self.bufs, self.d_obs, d_params=self.d_params)
        g = self.d_params
        self.v.mul_(self.rho).addcmul_(g, g, value=1.0 - self.rho)
        self.theta.sub_(self.lr * g / (self.v.sqrt() + self.eps))
        self.temp.mul_(self.r_temp)
        self.lr.mul_(self.r_lr)
        self.epoch.add_(1)

    def reset(self):
        self.theta.copy_(self.theta0)
        self.v.zero_()
        self.temp.fill_(self.temp0)
        self.lr.fill_(self.lr0)
        self.epoch.zero_()

    def capture(self):
        self.graph = CapturedStep(self.step)
        self.reset()
        torch.cuda.synchronize()

    def run(self, epochs: Optional[int] = None) -> InferenceResult:
        if self.graph is None:
            self.capture()
        n = self.epochs if epochs is None else epochs
        losses = torch.zeros(n, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in range(n):
            self.graph.replay()
            losses[e : e + 1].copy_(self.loss)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert ssa.device_status(self.h) == 0
        k = np.exp(self.theta.double().cpu().numpy())
        ls = losses.cpu().numpy()
        return InferenceResult(self.k_true, k, 100.0 * np.abs(k - self.k_true) / self.k_true,
                               float(ls[0]), float(ls[-1]), n, self.t_obs, dt,
                               int(self.bufs.steps_done.sum().item()), ls)


def dimerization(k_true: Sequence[float] = TRUE_RATES, *, n_traj: int = 100_000, n_target: int = 100_000,
                 n_steps: int = 250, n_grid: int = 64, epochs: int = 250, t0: float = 1.0, t1: float = 1e-3,
                 lr0: float = 0.15, lr1: float = 1e-4, seed: int = 0, k_start: Sequence[float] = START_RATES,
                 ckpt_every: int = 64) -> Trainer:
    """A + B <-> C (Sec. 4.1): the grid observation of A, B and C on the
    target's span, 250 steps, temperature 1.0 -> 0.001."""
    true_net = W.dimerization_abc(*k_true, x0=X0)
    cfg = W.RunConfig(seed=seed, n_steps=n_steps, obs_kind=W.OBS_GRID, n_bins=n_grid,
                      t_obs=grid_end(true_net, n_target, n_steps, seed), ckpt_every=ckpt_every)
    return Trainer(true_net, np.log(np.asarray(k_start, np.float64)), cfg, n_traj=n_traj, n_target=n_target,
                   epochs=epochs, t0=t0, t1=t1, lr0=lr0, lr1=lr1)


COI_RATES = (0.75, 0.103, 1.159)   # k_open, k_close, k_inact (1/ms) of the synthetic channel
COI_START = (0.3, 0.3, 0.3)


def ion_channel(k_true: Sequence[float] = COI_RATES, *, n_channels: int = 2, n_traj: int = 262_144,
                n_target: int = 262_144, n_steps: int = 20, n_bins: int = 800, t_obs: float = 8.0,
                epochs: int = 400, t0: float = 0.05, t1: float = 5e-4, lr0: float = 0.05, seed: int = 0,
                k_start: Sequence[float] = COI_START, ckpt_every: int = 32) -> Trainer:
    """Closed/open/inactivated channel (Sec. 4.4): N channels, 20 steps, exact
    bin averages of the open count on the recording grid (800 bins of
    0.01 ms), temperature 0.05 -> 0.0005 with the learning rate in
    proportion; the recorded sweeps are replaced by a target ensemble at
    known rates."""
    true_net = W.ion_channel_coi(*k_true, n_channels=n_channels)
    cfg = W.RunConfig(seed=seed, n_steps=n_steps, obs_kind=W.OBS_BINS, n_bins=n_bins, t_obs=t_obs,
                      ckpt_every=ckpt_every)
    return Trainer(true_net, np.log(np.asarray(k_start, np.float64)), cfg, n_traj=n_traj, n_target=n_target,
                   epochs=epochs, t0=t0, t1=t1, lr0=lr0, lr1=None)


def infer(k_true: Sequence[float] = TRUE_RATES, **kw) -> InferenceResult:
    return dimerization(k_true, **kw).run()


def sweep(k2_values: Sequence[float] = K2_SWEEP, k1: float = TRUE_RATES[0], **kw) -> List[InferenceResult]:
    """The robustness study of Sec. 4.1: k1 fixed, k2 over two orders of magnitude."""
    return [infer((k1, k2), **kw) for k2 in k2_values]
