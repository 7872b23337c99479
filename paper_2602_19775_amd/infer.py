"""Rate inference for the reversible dimerisation A + B <-> C (Sec. 4.1).

- **Target.** The ensemble-mean trajectories of A, B and C from `n_target`
  trajectories at the true rates (their own random stream), each path linearly
  interpolated between its event points onto a uniform time grid before the
  average is taken (the library's grid observation).
- **Model.** `n_traj` trajectories of `n_steps` steps at theta = ln k, observed
  the same way. The loss is the mean over grid points and species of the
  squared difference of the ensemble means.
- **Gradient.** The library's straight-through backward (Eqs. 3-7, Fig. 1).
- **Optimiser.** RMSprop on theta (decay 0.9, eps 1e-7). The Gumbel-Softmax
  temperature is annealed geometrically from 1.0 to 0.001 over the epochs
  (Sec. 3.5), and the learning rate geometrically from `lr0` to `lr1`.
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
    """The captured optimisation step for one target."""

    def __init__(self, k_true: Sequence[float], *, n_traj: int = 100_000, n_target: int = 100_000,
                 n_steps: int = 250, n_grid: int = 64, epochs: int = 250, t0: float = 1.0,
                 t1: float = 1e-3, lr0: float = 0.15, lr1: float = 1e-4, rho: float = 0.9,
                 eps: float = 1e-7, seed: int = 0, k_start: Sequence[float] = START_RATES,
                 ckpt_every: int = 64):
        dev = torch.device("cuda")
        self.k_true = np.asarray(k_true, np.float64)
        true_net = W.dimerization_abc(*k_true, x0=X0)
        self.net = W.dimerization_abc(*k_start, x0=X0)
        self.t_obs = grid_end(true_net, n_target, n_steps, seed)
        self.epochs = epochs
        self.n_grid, self.n_obs, self.B = n_grid, 3, n_traj
        self.cfg = W.RunConfig(seed=seed, n_steps=n_steps, obs_kind=W.OBS_GRID, n_bins=n_grid,
                               t_obs=self.t_obs, temperature=t0, ckpt_every=ckpt_every)
        # target ensemble means on the grid
        ht = ssa.Net([true_net], [n_target], t_obs=[self.t_obs])
        tf = ssa.forward(ht, self.cfg.replace(purpose=W.PURPOSE_TARGET),
                         torch.tensor(true_net.theta0, device=dev), _x0(true_net, n_target),
                         keep_ckpt=False, tie_capacity=0)
        self.target = tf.obs[: n_grid * 3 * n_target].view(n_grid, 3, n_target).mean(dim=2).clone()
        del tf, ht
        # model state and schedules (device scalars)
        self.h = ssa.Net([self.net], [n_traj], t_obs=[self.t_obs])
        self.theta0 = torch.tensor(np.log(np.asarray(k_start, np.float64)).astype(np.float32), device=dev)
        self.theta = self.theta0.clone()
        self.v = torch.zeros_like(self.theta)
        self.x0 = _x0(self.net, n_traj)
        self.epoch = torch.zeros(1, dtype=torch.int32, device=dev)
        self.temp0, self.lr0 = t0, lr0
        self.temp = torch.full((1,), t0, dtype=torch.float32, device=dev)
        self.lr = torch.full((1,), lr0, dtype=torch.float32, device=dev)
        n1 = max(epochs - 1, 1)
        self.r_temp = (t1 / t0) ** (1.0 / n1)
        self.r_lr = (lr1 / lr0) ** (1.0 / n1)
        self.rho, self.eps = rho, eps
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.d_obs = torch.zeros(n_grid * 3 * n_traj, dtype=torch.float64, device=dev)
        self.d_params = torch.zeros(self.h.param_total, dtype=torch.float32, device=dev)
        self.bufs = ssa.forward(self.h, self.cfg, self.theta, self.x0, tie_capacity=0, d_epoch=self.epoch,
                                d_temperature=self.temp)
        self.graph: Optional[CapturedStep] = None

    def step(self):
        """One optimisation step on the current stream (preallocated tensors only)."""
        G, O, B = self.n_grid, self.n_obs, self.B
        ssa.forward(self.h, self.cfg, self.theta, self.x0, buffers=self.bufs, tie_capacity=0,
                    d_epoch=self.epoch, d_temperature=self.temp)
        o = self.bufs.obs[: G * O * B].view(G, O, B)
        e = o.mean(dim=2) - self.target
        self.loss.copy_(e.square().mean().reshape(1))
        # dL/dobs = 2 (mean - target) / (G O B) for every trajectory
        self.d_obs.view(G, O, B).copy_((e * (2.0 / (G * O * B))).unsqueeze(2).expand(G, O, B))
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


def infer(k_true: Sequence[float] = TRUE_RATES, **kw) -> InferenceResult:
    return Trainer(k_true, **kw).run()


def sweep(k2_values: Sequence[float] = K2_SWEEP, k1: float = TRUE_RATES[0], **kw) -> List[InferenceResult]:
    """The robustness study of Sec. 4.1: k1 fixed, k2 over two orders of magnitude."""
    return [infer((k1, k2), **kw) for k2 in k2_values]
