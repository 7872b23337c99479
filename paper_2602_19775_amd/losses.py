"""Trajectory losses on the observation tensor (plain PyTorch, FP64).

The library returns observations; the loss and dL/dobs are ordinary autograd
outside it (the paper's losses are MSEs of ensemble statistics, Sec. 3.5)."""
from __future__ import annotations

import torch


def bin_moments(obs: torch.Tensor, n_bins: int, n_obs: int, B: int):
    """Per-bin ensemble mean and population variance of bin averages laid out
    [n_bins][n_obs][B] (the library's layout for one network)."""
    o = obs[: n_bins * n_obs * B].view(n_bins, n_obs, B)
    m = o.mean(dim=2)
    v = ((o - m[:, :, None]) ** 2).mean(dim=2)
    return m, v


def moment_mse(obs: torch.Tensor, target_m: torch.Tensor, target_v: torch.Tensor, n_bins: int,
               n_obs: int, B: int) -> torch.Tensor:
    """Mean squared error of per-bin means and variances against targets."""
    m, v = bin_moments(obs, n_bins, n_obs, B)
    return (((m - target_m) ** 2).sum() + ((v - target_v) ** 2).sum()) / (2 * m.numel())
