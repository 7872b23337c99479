"""Two-phase training of the gene-network classifier (Sec. 3.5, Sec. 4.3).

- **Data.** A training set of synthetic images (workloads.grn_images) split
  into fixed minibatches of `batch` images; step s trains on minibatch
  s mod n_batches, gathered on the device, with `n_rep` trajectories per
  image.  A held-out set of images of the same prototypes measures accuracy.
- **Phase 1 (relaxed).** For the first `soft_frac` of the steps (16 of 80
  epochs in the paper) the forward is the relaxed map of Eq. 4 (real-valued
  levels moved by the soft sample's expected change) and the backward is the
  exact gradient of that map (`ssa_config.relaxed`).
- **Phase 2 (straight-through).** Hard forward (exact direct method) and the
  straight-through backward.
- **Loss.** Cross-entropy of the softmax over the final output levels of a
  trajectory against its image's label, averaged over trajectories; its
  gradient (softmax - one-hot) / B is written out.
- **Schedules.** Temperature geometric from t0 = 2 to t1 = 0.2 over all steps
  (Fig. 4D); RMSprop (decay 0.9, eps 1e-7) with a fixed learning rate of
  1e-2 (Sec. 3.5); the parameters are averaged over the last `avg_frac` of
  the steps (stochastic weight averaging, 16 of 80 epochs in the paper).
- **Graphs.** Each phase's step is captured into its own HIP graph and
  replayed; the step counter (the random stream's epoch), the minibatch index
  and the temperature are device scalars.
- **Accuracy.** The label of a held-out image is the argmax of its output
  levels averaged over `n_eval_rep` hard trajectories (Fig. 4E).
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import ssa
from . import workloads as W
from .graph import CapturedStep


@dataclass
class ClassifierResult:
    steps: int
    soft_steps: int
    losses: np.ndarray          # training loss of every step
    loss_soft_first: float      # mean over the first tenth of phase 1
    loss_soft_last: float       # mean over the last tenth of phase 1
    loss_hard_first: float
    loss_hard_last: float
    accuracy_start: float       # held-out accuracy of the initial parameters
    accuracy: float             # held-out accuracy of the averaged parameters
    train_s: float
    fired_per_step: float       # reactions fired per hard step


class TwoPhaseTrainer:
    """Relaxed-then-straight-through training of `net` on synthetic images."""

    def __init__(self, net: W.GrnNet, *, n_train: int = 512, batch: int = 128, n_rep: int = 8,
                 n_steps: int = 1000, steps: int = 200, soft_frac: float = 0.2, t0: float = 2.0,
                 t1: float = 0.2, lr: float = 1e-2, rho: float = 0.9, eps: float = 1e-7,
                 avg_frac: float = 0.2, n_test: int = 200, n_eval_rep: int = 16, side: int = 28, seed: int = 0):
        dev = torch.device("cuda")
        assert n_train % batch == 0 and 0.0 <= soft_frac <= 1.0
        self.net, self.steps = net, steps
        self.soft_steps = int(round(soft_frac * steps))
        self.avg_from = steps - max(int(round(avg_frac * steps)), 1)
        self.batch, self.n_rep, self.B = batch, n_rep, batch * n_rep
        self.n_batches = n_train // batch
        imgs, labels = W.grn_images(n_train + n_test, seed=seed, side=side)
        imgs = np.ascontiguousarray(imgs[:, : net.n_in])
        self.x_all = torch.tensor(imgs[:n_train], device=dev).view(self.n_batches, batch, net.n_in)
        self.y_all = torch.tensor(labels[:n_train], dtype=torch.long, device=dev).view(self.n_batches, batch)
        self.x_test = torch.tensor(imgs[n_train:], device=dev)
        self.y_test = labels[n_train:]
        self.n_eval_rep = n_eval_rep
        self.cfg = W.RunConfig(seed=seed, n_steps=n_steps, obs_kind=W.OBS_FINAL, temperature=t0)
        self.g = ssa.Grn(net, batch, n_rep)
        self.theta0 = torch.tensor(W.grn_init_params(net, seed), device=dev)
        self.theta = self.theta0.clone()
        self.avg = torch.zeros_like(self.theta, dtype=torch.float64)
        self.v = torch.zeros_like(self.theta)
        self.lr, self.rho, self.eps = lr, rho, eps
        self.t0 = t0
        self.r_temp = (t1 / t0) ** (1.0 / max(steps - 1, 1))
        self.step_no = torch.zeros(1, dtype=torch.int32, device=dev)
        self.temp = torch.full((1,), t0, dtype=torch.float32, device=dev)
        self.x = self.x_all[0].clone()
        self.y = self.y_all[0].repeat_interleave(n_rep)
        self.onehot = torch.zeros((net.n_out, self.B), dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.d_obs = torch.zeros((net.n_out, self.B), dtype=torch.float64, device=dev)
        self.d_params = torch.zeros(net.n_params, dtype=torch.float32, device=dev)
        self.soft_bufs = ssa.grn_forward(self.g, self.cfg.replace(relaxed=True), self.theta, self.x,
                                         tie_capacity=0, d_epoch=self.step_no, d_temperature=self.temp)
        self.hard_bufs = ssa.grn_forward(self.g, self.cfg, self.theta, self.x, tie_capacity=0,
                                         d_epoch=self.step_no, d_temperature=self.temp)
        _, wb = ssa.grn_buffer_sizes(self.g, self.soft_bufs.ccfg)
        _, wh = ssa.grn_buffer_sizes(self.g, self.hard_bufs.ccfg)
        self.work = torch.empty(max(wb, wh), dtype=torch.uint8, device=dev)
        self.graphs = {}

    def _step(self, relaxed: bool):
        """One optimisation step on the current stream (preallocated tensors only)."""
        b = torch.remainder(self.step_no, self.n_batches).long()
        self.x.copy_(self.x_all.index_select(0, b).view_as(self.x))
        self.y.copy_(self.y_all.index_select(0, b).view(-1).repeat_interleave(self.n_rep))
        cfg = self.cfg.replace(relaxed=relaxed)
        bufs = self.soft_bufs if relaxed else self.hard_bufs
        ssa.grn_forward(self.g, cfg, self.theta, self.x, tie_capacity=0, d_epoch=self.step_no,
                        d_temperature=self.temp, buffers=bufs)
        # cross-entropy of softmax over the output levels, gradient written out
        p = torch.softmax(bufs.obs, dim=0)
        self.onehot.zero_()
        self.onehot.scatter_(0, self.y.view(1, -1), 1.0)
        self.loss.copy_(-(self.onehot * torch.log_softmax(bufs.obs, dim=0)).sum().reshape(1) / self.B)
        torch.sub(p, self.onehot, out=self.d_obs)
        self.d_obs.mul_(1.0 / self.B)
        ssa.grn_backward(self.g, cfg, self.theta, self.x, bufs, self.d_obs, d_params=self.d_params,
                         work=self.work)
        gr = self.d_params
        self.v.mul_(self.rho).addcmul_(gr, gr, value=1.0 - self.rho)
        self.theta.sub_(self.lr * gr / (self.v.sqrt() + self.eps))
        self.temp.mul_(self.r_temp)
        self.step_no.add_(1)

    def reset(self):
        self.theta.copy_(self.theta0)
        self.v.zero_()
        self.temp.fill_(self.t0)
        self.step_no.zero_()
        self.avg.zero_()

    def capture(self):
        for relaxed in (True, False):
            self.graphs[relaxed] = CapturedStep(lambda r=relaxed: self._step(r))
        self.reset()
        torch.cuda.synchronize()

    def accuracy(self, theta: torch.Tensor) -> float:
        """Held-out accuracy: argmax of the output levels averaged over
        n_eval_rep hard trajectories per image (a separate stream)."""
        n = self.x_test.shape[0]
        ge = ssa.Grn(self.net, n, self.n_eval_rep)
        f = ssa.grn_forward(ge, self.cfg.replace(purpose=W.PURPOSE_TARGET), theta, self.x_test, keep_tape=False,
                            tie_capacity=0)
        mean = f.obs.view(self.net.n_out, n, self.n_eval_rep).mean(dim=2)
        pred = mean.argmax(dim=0).cpu().numpy()
        return float((pred == self.y_test).mean())

    def run(self) -> ClassifierResult:
        if not self.graphs:
            self.capture()
        acc0 = self.accuracy(self.theta0)
        losses = torch.zeros(self.steps, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(self.steps):
            self.graphs[s < self.soft_steps].replay()
            losses[s: s + 1].copy_(self.loss)
            if s >= self.avg_from:
                self.avg.add_(self.theta.double())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert ssa.grn_device_status(self.g) == 0
        avg = (self.avg / (self.steps - self.avg_from)).float()
        ls = losses.cpu().numpy()
        S = self.soft_steps
        tenth = lambda a: a[: max(len(a) // 10, 1)].mean() if len(a) else float("nan")
        last = lambda a: a[-max(len(a) // 10, 1):].mean() if len(a) else float("nan")
        return ClassifierResult(self.steps, S, ls, float(tenth(ls[:S])), float(last(ls[:S])),
                                float(tenth(ls[S:])), float(last(ls[S:])), acc0, self.accuracy(avg), dt,
                                float(self.hard_bufs.steps_done.double().sum().item()))
