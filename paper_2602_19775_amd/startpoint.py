"""Start-point-map inference of the oscillator's protein rates (Sec. 4.2).

- **Start points.** Reference paths at the true rates (their own random
  stream) run past a burn-in; a start point is taken every `stride` steps
  along each path.  The paper samples 262,144 start points along one path of
  2.4 million steps (about 33 periods of the oscillation); here `n_paths`
  independent paths (32 by default, each covering 73,728 steps, about one
  period, after a 300,000-step burn-in that spreads their phases) run side by
  side on the GPU, one chained forward per stride (the epoch counter gives
  each stride its own noise), which samples the same stationary path law.
- **Segments.** Each start point seeds `n_rep` replicate segments of `n_seg`
  steps (25 and 150 in the paper).  A segment's observation is the library's
  tail mean (SSA_OBS_TAIL): the mean count of A, R and C over its last
  `n_tail` states (100) and the mean time of those states.
- **Rate of change.** Per start point and protein: (mean over the replicates
  of the tail mean count - the start count) / (mean over the replicates of the
  tail mean time).  Targets come from segments at the true rates run every
  epoch on the same counters as the model's segments (common random numbers:
  at the true rates the two agree exactly, so the loss has no sampling floor);
  `crn=False` instead computes them once for every start point on a stream of
  their own.  By default the elapsed time is a normaliser of the rate, not
  differentiated (`time_grad`).
- **Loss.** Mean squared difference of the model's and the target's rates over
  a batch of start points and the three proteins.
- **Optimiser.** RMSprop (decay 0.9, eps 1e-7) on theta = ln k of the five
  protein parameters (beta_A, beta_R, delta_A, delta_R, gamma_C); the other
  rates stay at their true values.  Learning rate geometric from lr0 to lr1,
  fixed temperature (3e-6 in the paper).  The reported estimate is the median
  of theta over the last quarter of the epochs (a median Polyak-Ruppert
  average).
- **Graph.** One epoch (batch gather, forward, loss gradient, backward,
  update, schedule) is captured once into a HIP graph and replayed; the batch
  index, epoch and learning rate are device scalars.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import ssa
from . import workloads as W
from .graph import CapturedStep

PURPOSE_REFERENCE = 4          # random stream of the reference paths
PROTEIN = [W.OSC_PARAMS.index(p) for p in W.OSC_PROTEIN_PARAMS]


def rate_loss(obs: torch.Tensor, xs: torch.Tensor, tr: torch.Tensor, S: int, R: int,
              d_obs: Optional[torch.Tensor] = None, time_grad: bool = True) -> torch.Tensor:
    """The start-point map's loss and its gradient, written out.

    obs: tail observations [(3 + 1) * S * R] (A, R, C tail means, then the tail
    mean time; trajectory s * R + r is replicate r of start point s);
    xs: start counts [S, 3]; tr: target rates [S, 3].
    rate[o, s] = (mean_r obs[o, s, r] - xs[s, o]) / mean_r obs[3, s, r];
    loss = mean over (o, s) of (rate - tr)^2.  With d_obs given, dL/dobs is
    written into it (same layout as obs); time_grad=False leaves the elapsed
    time out of the gradient (a normaliser).  Returns the loss, shape [1]."""
    m = obs.view(4, S, R).mean(dim=2)
    dx = m[:3] - xs.T
    tau = m[3]
    e = dx / tau - tr.T
    if d_obs is not None:
        dr = e * (2.0 / (3 * S))
        dm = dr / tau / R
        dtau = -(dr * dx).sum(dim=0) / (tau * tau) / R
        d = d_obs.view(4, S, R)
        d[:3].copy_(dm.unsqueeze(2).expand(3, S, R))
        d[3].copy_(dtau.unsqueeze(1).expand(S, R) if time_grad else torch.zeros_like(d[3]))
    return e.square().mean().reshape(1)


def reference_start_points(net: W.Network, n_start: int, n_paths: int, stride: int, burn: int,
                           seed: int = 0) -> torch.Tensor:
    """[n_start, N] int32 start states (device): n_paths reference paths at
    the network's rates, burn-in steps, then one state every `stride` steps
    along each path (start point c * n_paths + p is path p after its c-th
    stride)."""
    assert n_start % n_paths == 0
    dev = torch.device("cuda")
    h = ssa.Net([net], [n_paths])
    th = torch.tensor(net.theta0, device=dev)
    x = torch.tensor(np.repeat(net.x0[:, None], n_paths, axis=1).reshape(-1), dtype=torch.int32, device=dev)
    cfg = W.RunConfig(seed=seed, purpose=PURPOSE_REFERENCE, epoch=0, n_steps=burn, obs_kind=W.OBS_FINAL)
    f = ssa.forward(h, cfg, th, x, keep_ckpt=False, tie_capacity=0)
    x = f.x_final.clone()
    out = torch.empty((n_start // n_paths, net.n_species, n_paths), dtype=torch.int32, device=dev)
    cfg = cfg.replace(n_steps=stride)
    for c in range(n_start // n_paths):
        f = ssa.forward(h, cfg.replace(epoch=c + 1), th, x, keep_ckpt=False, tie_capacity=0, buffers=f)
        x.copy_(f.x_final)
        out[c].copy_(f.x_final.view(net.n_species, n_paths))
    assert ssa.device_status(h) == 0
    return out.permute(0, 2, 1).reshape(n_start, net.n_species).contiguous()


@dataclass
class StartPointResult:
    k_true: np.ndarray             # the five protein rates
    k_start: np.ndarray
    k_learned: np.ndarray          # median of the last quarter of the epochs
    k_last: np.ndarray             # after the last epoch
    ape: np.ndarray                # absolute percentage error of k_learned
    loss_first: float
    loss_last: float
    epochs: int
    train_s: float
    steps_per_epoch: int
    losses: np.ndarray
    history: np.ndarray            # [epochs, 5] ln k after each epoch


class StartPointTrainer:
    """The captured start-point-map optimisation step (see the module
    docstring).  `true_net` holds the true rates; `k_start` the starting
    values of the five protein rates."""

    def __init__(self, true_net: W.Network, k_start: Sequence[float], *, n_start: int = 262_144,
                 n_paths: int = 32, stride: int = 9, burn: int = 300_000, n_seg: int = 150, n_tail: int = 100,
                 n_rep: int = 25, batch: int = 8192, epochs: int = 3000, temperature: float = 3e-6,
                 lr0: float = 0.1, lr1: float = 0.01, rho: float = 0.9, eps: float = 1e-7, seed: int = 0,
                 time_grad: bool = False, crn: bool = True):
        dev = torch.device("cuda")
        assert n_start % batch == 0
        self.true_net, self.epochs, self.time_grad, self.crn = true_net, epochs, time_grad, crn
        N, nob = true_net.n_species, len(true_net.obs_species)
        assert nob == 3
        self.S, self.R, self.B = batch, n_rep, batch * n_rep
        self.n_batches = n_start // batch
        self.k_true = np.exp(true_net.theta0.astype(np.float64))[PROTEIN]
        self.k_start = np.asarray(k_start, np.float64)
        osp = torch.tensor(true_net.obs_species, dtype=torch.long, device=dev)
        # start points and their per-batch replicate layouts
        starts = reference_start_points(true_net, n_start, n_paths, stride, burn, seed)
        self.xs_all = starts[:, osp].to(torch.float64).view(self.n_batches, batch, nob).contiguous()
        rep = starts.view(self.n_batches, batch, 1, N).expand(self.n_batches, batch, n_rep, N)
        self.x0_all = rep.reshape(self.n_batches, self.B, N).permute(0, 2, 1).reshape(self.n_batches, N * self.B)
        self.x0_all = self.x0_all.contiguous()
        del starts, rep
        self.cfg = W.RunConfig(seed=seed, n_steps=n_seg, obs_kind=W.OBS_TAIL, n_bins=n_tail,
                               temperature=temperature, ckpt_every=n_seg)
        self.h = ssa.Net([true_net], [self.B])
        # target rates of change at the true rates: once for every start point
        # on a stream of their own, or (crn) every epoch on the model's stream
        self.th_true = torch.tensor(true_net.theta0, device=dev)
        self.tr_all = None
        if not crn:
            self.tr_all = torch.empty((self.n_batches, batch, nob), dtype=torch.float64, device=dev)
            tf = None
            for b in range(self.n_batches):
                tf = ssa.forward(self.h, self.cfg.replace(purpose=W.PURPOSE_TARGET, epoch=b), self.th_true,
                                 self.x0_all[b], keep_ckpt=False, tie_capacity=0, buffers=tf)
                self.tr_all[b].copy_(self._rates(tf.obs, self.xs_all[b]).T)
            del tf
        # model state, schedules and buffers (device scalars for the graph)
        theta = true_net.theta0.astype(np.float64).copy()
        theta[PROTEIN] = np.log(self.k_start)
        self.theta0 = torch.tensor(theta.astype(np.float32), device=dev)
        self.theta = self.theta0.clone()
        self.mask = torch.zeros_like(self.theta)
        self.mask[PROTEIN] = 1.0
        self.pidx = torch.tensor(PROTEIN, dtype=torch.long, device=dev)
        self.v = torch.zeros_like(self.theta)
        self.lr0 = lr0
        self.lr = torch.full((1,), lr0, dtype=torch.float32, device=dev)
        self.r_lr = (lr1 / lr0) ** (1.0 / max(epochs - 1, 1))
        self.rho, self.eps = rho, eps
        self.epoch = torch.zeros(1, dtype=torch.int32, device=dev)
        self.x0 = self.x0_all[0].clone()
        self.xs = self.xs_all[0].clone()
        self.tr = torch.zeros((batch, nob), dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.d_obs = torch.zeros((nob + 1) * self.B, dtype=torch.float64, device=dev)
        self.d_params = torch.zeros(self.h.param_total, dtype=torch.float32, device=dev)
        self.bufs = ssa.forward(self.h, self.cfg, self.theta, self.x0, tie_capacity=0, d_epoch=self.epoch)
        self.tbufs = (ssa.forward(self.h, self.cfg, self.th_true, self.x0, keep_ckpt=False, tie_capacity=0,
                                  d_epoch=self.epoch) if crn else None)
        self.graph: Optional[CapturedStep] = None

    def _rates(self, obs: torch.Tensor, xs: torch.Tensor) -> torch.Tensor:
        """Rates of change [3, S] from tail observations [(3 + 1) * B] and
        start counts xs [S, 3]."""
        m = obs.view(4, self.S, self.R).mean(dim=2)
        return (m[:3] - xs.T) / m[3]

    def step(self):
        """One epoch on the current stream (preallocated tensors only)."""
        b = torch.remainder(self.epoch, self.n_batches).long()
        self.x0.copy_(self.x0_all.index_select(0, b).view(-1))
        self.xs.copy_(self.xs_all.index_select(0, b).view(self.S, 3))
        if self.crn:
            # the true rates on the same counters as the model's segments
            ssa.forward(self.h, self.cfg, self.th_true, self.x0, buffers=self.tbufs, keep_ckpt=False,
                        tie_capacity=0, d_epoch=self.epoch)
            self.tr.copy_(self._rates(self.tbufs.obs, self.xs).T)
        else:
            self.tr.copy_(self.tr_all.index_select(0, b).view(self.S, 3))
        ssa.forward(self.h, self.cfg, self.theta, self.x0, buffers=self.bufs, tie_capacity=0, d_epoch=self.epoch)
        self.loss.copy_(rate_loss(self.bufs.obs, self.xs, self.tr, self.S, self.R, self.d_obs, self.time_grad))
        ssa.backward(self.h, self.cfg, self.theta, self.x0, self.bufs, self.d_obs, d_params=self.d_params)
        g = self.d_params * self.mask
        self.v.mul_(self.rho).addcmul_(g, g, value=1.0 - self.rho)
        self.theta.sub_(self.lr * g / (self.v.sqrt() + self.eps))
        self.lr.mul_(self.r_lr)
        self.epoch.add_(1)

    def reset(self):
        self.theta.copy_(self.theta0)
        self.v.zero_()
        self.lr.fill_(self.lr0)
        self.epoch.zero_()

    def capture(self):
        self.graph = CapturedStep(self.step)
        self.reset()
        torch.cuda.synchronize()

    def run(self, epochs: Optional[int] = None) -> StartPointResult:
        if self.graph is None:
            self.capture()
        n = self.epochs if epochs is None else epochs
        losses = torch.zeros(n, dtype=torch.float64, device="cuda")
        hist = torch.zeros((n, len(PROTEIN)), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e in range(n):
            self.graph.replay()
            losses[e : e + 1].copy_(self.loss)
            hist[e].copy_(self.theta.index_select(0, self.pidx))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert ssa.device_status(self.h) == 0
        h = hist.double().cpu().numpy()
        k_med = np.exp(np.median(h[n - max(n // 4, 1):], axis=0))
        ls = losses.cpu().numpy()
        return StartPointResult(self.k_true, self.k_start, k_med, np.exp(h[-1]),
                                100.0 * np.abs(k_med - self.k_true) / self.k_true, float(ls[0]), float(ls[-1]),
                                n, dt, int(self.bufs.steps_done.sum().item()), ls, h)


def oscillator_start_points(k_start: Sequence[float] = None, **kw) -> StartPointTrainer:
    """The start-point-map protocol of Sec. 4.2 on the oscillator with the
    paper's protein rates (workloads.start_point_oscillator); k_start defaults
    to the true protein rates scaled by (2, 1/2, 2, 1/2, 2)."""
    net = W.start_point_oscillator()
    if k_start is None:
        k_start = np.asarray(W.OSC_PROTEIN_RATES) * np.array([2.0, 0.5, 2.0, 0.5, 2.0])
    return StartPointTrainer(net, k_start, **kw)
