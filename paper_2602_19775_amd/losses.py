"""Trajectory losses on the observation tensor (plain PyTorch, FP64).

The library returns observations; the loss and dL/dobs are ordinary autograd
outside it (the paper's losses are MSEs of ensemble statistics, Sec. 3.5)."""
from __future__ import annotations

import torch


def bin_moments(obs: torch.Tensor, n_bins: int, n_obs: int, B: int):
    """Per-bin ensemble mean and population variance of bin averages laid out
    [n_bins][n_obs][B] (the library's layout for one network)."""
    o = obs[: n_bins * n_obs * B].view(n_bins, n_obs, B)
    v, m = torch.var_mean(o, dim=2, correction=0)
    return m, v


def moment_mse(obs: torch.Tensor, target_m: torch.Tensor, target_v: torch.Tensor, n_bins: int,
               n_obs: int, B: int) -> torch.Tensor:
    """Mean squared error of per-bin means and variances against targets."""
    m, v = bin_moments(obs, n_bins, n_obs, B)
    return (((m - target_m) ** 2).sum() + ((v - target_v) ** 2).sum()) / (2 * m.numel())


def mean_autocorrelation(obs: torch.Tensor, n_bins: int, B: int, max_lag: int, eps: float = 1e-6):
    """Ensemble mean of each trajectory's normalised autocorrelation of its bin
    series (one observed species), lags 1..max_lag."""
    x = obs[: n_bins * B].view(n_bins, B)
    xc = x - x.mean(dim=0, keepdim=True)
    den = (xc * xc).sum(dim=0) + eps
    rho = torch.stack([(xc[:-l] * xc[l:]).sum(dim=0) / den for l in range(1, max_lag + 1)])
    return rho.mean(dim=1)


def autocorrelation_mse(obs: torch.Tensor, target: torch.Tensor, n_bins: int, B: int, max_lag: int = 64):
    return ((mean_autocorrelation(obs, n_bins, B, max_lag) - target) ** 2).mean()


def count_cross_entropy(obs: torch.Tensor, labels: torch.Tensor) -> torch.Tensor:
    """Cross-entropy of the softmax over final output-gene counts (Sec. 4.3),
    averaged over trajectories.  obs: [n_out, B] float64, labels: [B]."""
    logits = obs.t()
    return torch.nn.functional.cross_entropy(logits, labels)
