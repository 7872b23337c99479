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


class _MomentMSE(torch.autograd.Function):
    """L = (sum (m - m*)^2 + sum (v - v*)^2) / (2 R) over the R = n_bins * n_obs
    rows, with the gradient written out: dL/dx_i = (e_m + 2 e_v (x_i - m)) / (R B)
    for a row's mean m, population variance v and errors e_m, e_v."""

    @staticmethod
    def forward(ctx, obs, target_mv, n_bins, n_obs, B):
        o = obs[: n_bins * n_obs * B].view(n_bins, n_obs, B)
        v, m = torch.var_mean(o, dim=2, correction=0)
        e = torch.stack((m, v)) - target_mv
        R = n_bins * n_obs
        ctx.save_for_backward(obs, m, e)
        ctx.dims = (n_bins, n_obs, B)
        return e.square().sum() / (2 * R)

    @staticmethod
    def backward(ctx, g):
        obs, m, e = ctx.saved_tensors
        n_bins, n_obs, B = ctx.dims
        n = n_bins * n_obs * B
        coef = e * (g / (n_bins * n_obs * B))
        o = obs[:n].view(n_bins, n_obs, B)
        d = torch.addcmul(coef[0].unsqueeze(2), coef[1].unsqueeze(2), o - m.unsqueeze(2), value=2.0)
        if obs.numel() != n:
            d = torch.cat((d.reshape(-1), obs.new_zeros(obs.numel() - n)))
        return d.reshape(obs.shape), None, None, None, None


def moment_mse(obs: torch.Tensor, target_m: torch.Tensor, target_v: torch.Tensor, n_bins: int,
               n_obs: int, B: int) -> torch.Tensor:
    """Mean squared error of per-bin means and variances against targets."""
    return _MomentMSE.apply(obs, torch.stack((target_m, target_v)), n_bins, n_obs, B)


def moment_mse_autograd(obs: torch.Tensor, target_m: torch.Tensor, target_v: torch.Tensor, n_bins: int,
                        n_obs: int, B: int) -> torch.Tensor:
    """The same loss through PyTorch's own differentiation (a check of the above)."""
    m, v = bin_moments(obs, n_bins, n_obs, B)
    return (((m - target_m) ** 2).sum() + ((v - target_v) ** 2).sum()) / (2 * m.numel())


def mean_autocorrelation(obs: torch.Tensor, n_bins: int, B: int, max_lag: int, eps: float = 1e-6):
    """Ensemble mean of each trajectory's normalised autocorrelation of its bin
    series (one observed species), lags 1..max_lag:
    rho_l = sum_t xc_t xc_{t+l} / (sum_t xc_t^2 + eps), xc the centred series.
    The lag sums come from one real FFT of the zero-padded series (long
    enough that the circular correlation equals the linear one up to max_lag)."""
    x = obs[: n_bins * B].view(n_bins, B)
    xc = x - x.mean(dim=0, keepdim=True)
    nfft = 1 << int(n_bins + max_lag - 1).bit_length()
    f = torch.fft.rfft(xc, n=nfft, dim=0)
    ac = torch.fft.irfft(f.real.square() + f.imag.square(), n=nfft, dim=0)
    rho = ac[1: max_lag + 1] / (ac[0] + eps)
    return rho.mean(dim=1)


def mean_autocorrelation_direct(obs: torch.Tensor, n_bins: int, B: int, max_lag: int, eps: float = 1e-6):
    """The same statistic from the lag sums written out (a check of the above)."""
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
