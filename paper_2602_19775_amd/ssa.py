"""Python binding of libssa (ctypes).  Argument marshalling only: every step of
the simulation and of its backward runs in the HIP kernels of libssa.so.
PyTorch provides device memory and the stream.

The library must be built (``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssa.so")

SSA_OK = 0
BWD_AUTO, BWD_TAPE, BWD_RECOMPUTE, BWD_TANGENT = 0, 1, 2, 3
_BWD = {"auto": BWD_AUTO, "tape": BWD_TAPE, "recompute": BWD_RECOMPUTE, "tangent": BWD_TANGENT}

_lib = None


class SSAError(RuntimeError):
    pass


class _Desc(C.Structure):
    _fields_ = [("n_networks", C.c_int32), ("n_species", C.c_void_p), ("n_reactions", C.c_void_p),
                ("n_params", C.c_void_p), ("n_traj", C.c_void_p), ("n_obs", C.c_void_p),
                ("reactant", C.c_void_p), ("rate_index", C.c_void_p), ("stoich", C.c_void_p),
                ("obs_species", C.c_void_p), ("t_obs", C.c_void_p), ("exec_mode", C.c_int32),
                ("wave_split", C.c_int32), ("wave_lanes", C.c_int32)]


class _Layout(C.Structure):
    _fields_ = [("traj_offset", C.c_int64), ("state_offset", C.c_int64), ("param_offset", C.c_int64),
                ("obs_offset", C.c_int64), ("ppt_offset", C.c_int64), ("mean_offset", C.c_int64)]


class _Cfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("purpose", C.c_uint32), ("epoch", C.c_uint32),
                ("d_epoch", C.c_void_p), ("traj_ids", C.c_void_p), ("n_steps", C.c_int32),
                ("t_end", C.c_double), ("obs_kind", C.c_int32), ("n_bins", C.c_int32),
                ("temperature", C.c_float), ("ckpt_every", C.c_int32), ("bwd_mode", C.c_int32),
                ("tie_capacity", C.c_int32), ("d_temperature", C.c_void_p), ("selection", C.c_int32),
                ("obs_layout", C.c_int32), ("dobs_shared", C.c_int32), ("relaxed", C.c_int32)]


TIE_DTYPE = np.dtype([("traj", np.uint32), ("step", np.uint32), ("chosen", np.int32),
                      ("second", np.int32), ("margin", np.float32), ("kind", np.int32)])

class _GrnDesc(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hid", C.c_int32), ("n_out", C.c_int32), ("n_images", C.c_int32),
                ("n_rep", C.c_int32), ("beta", C.c_float), ("delta_min", C.c_float)]


EXPORTS = ["ssa_config_default", "ssa_net_create", "ssa_net_destroy", "ssa_net_sizes", "ssa_net_layout",
           "ssa_buffer_sizes", "ssa_forward", "ssa_backward", "ssa_step_batch", "ssa_device_status",
           "ssa_status_string", "ssa_last_error", "ssa_selftest_philox", "ssa_selftest_neglog",
           "ssa_grn_create", "ssa_grn_destroy", "ssa_grn_buffer_sizes", "ssa_grn_forward",
           "ssa_grn_backward", "ssa_grn_device_status", "ssa_obs_mean", "ssa_backward_static"]


def lib():
    """Load libssa.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SSAError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        V = C.c_void_p
        L.ssa_config_default.argtypes = [C.POINTER(_Cfg)]
        L.ssa_net_create.argtypes = [C.POINTER(_Desc), C.POINTER(V)]
        L.ssa_net_destroy.argtypes = [V]
        L.ssa_net_sizes.argtypes = [V] + [C.POINTER(C.c_int64)] * 4
        L.ssa_net_layout.argtypes = [V, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_Layout)]
        L.ssa_buffer_sizes.argtypes = [V, C.POINTER(_Cfg), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.ssa_forward.argtypes = [V, C.POINTER(_Cfg), V, V, V, V, V, V, V, C.c_size_t, V, V, V,
                                  C.c_size_t, V]
        L.ssa_backward.argtypes = [V, C.POINTER(_Cfg), V, V, V, V, V, V, C.c_size_t, V, V, V, V,
                                   C.c_size_t, V]
        L.ssa_backward_static.argtypes = [V, C.POINTER(_Cfg), V, V, V, V, V, V, C.c_size_t, V, V, V, V]
        L.ssa_step_batch.argtypes = [V, C.POINTER(_Cfg), V, V, V, C.c_uint32, V, V, V, V]
        L.ssa_obs_mean.argtypes = [V, C.POINTER(_Cfg), V, V, V, C.c_size_t, V]
        L.ssa_device_status.argtypes = [V, V, C.POINTER(C.c_uint32)]
        L.ssa_status_string.argtypes = [C.c_int]
        L.ssa_status_string.restype = C.c_char_p
        L.ssa_last_error.restype = C.c_char_p
        L.ssa_selftest_philox.argtypes = [V, V, C.c_int64, V]
        L.ssa_selftest_neglog.argtypes = [C.c_uint32, C.c_int64, V, V]
        L.ssa_grn_create.argtypes = [C.POINTER(_GrnDesc), C.POINTER(V)]
        L.ssa_grn_destroy.argtypes = [V]
        L.ssa_grn_buffer_sizes.argtypes = [V, C.POINTER(_Cfg), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        L.ssa_grn_forward.argtypes = [V, C.POINTER(_Cfg), V, V, V, V, V, V, V, V, V, C.c_size_t, V, V, V]
        L.ssa_grn_backward.argtypes = [V, C.POINTER(_Cfg), V, V, V, V, V, V, V, C.c_size_t, V, V, V, V,
                                       C.c_size_t, V]
        L.ssa_grn_device_status.argtypes = [V, V, C.POINTER(C.c_uint32)]
        for name in EXPORTS:
            f = getattr(L, name)
            if name not in ("ssa_net_destroy", "ssa_grn_destroy", "ssa_config_default", "ssa_status_string",
                            "ssa_last_error"):
                f.restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != SSA_OK:
        L = lib()
        raise SSAError(f"{what}: {L.ssa_status_string(rc).decode()} ({L.ssa_last_error().decode()})")


def _need(ok: bool, what: str):
    """Argument check of the binding (kept under python -O: the kernels read
    every buffer at the size the handle and the run settings imply)."""
    if not ok:
        raise ValueError(what)


def _dev_tensor(t: torch.Tensor, dtype, n: int, name: str, exact: bool = True):
    _need(isinstance(t, torch.Tensor) and t.is_cuda, f"{name} must be a device tensor")
    _need(t.dtype == dtype, f"{name} must be {dtype}, not {t.dtype}")
    _need(t.is_contiguous(), f"{name} must be contiguous")
    _need(t.numel() == n if exact else t.numel() >= n,
          f"{name} has {t.numel()} elements, {'' if exact else 'at least '}{n} expected")



def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Net:
    """Device-resident tables of one or more networks (see include/ssa.h)."""

    EXEC = {"auto": 0, "spec": 1, "lane": 2, "wave": 3}

    def __init__(self, networks: Sequence[W.Network], n_traj: Sequence[int],
                 t_obs: Optional[Sequence[float]] = None, obs_species: Optional[Sequence] = None,
                 exec_mode: str = "auto", wave_split: int = -1, wave_lanes: int = 0):
        self.networks = list(networks)
        self.n_traj = [int(b) for b in n_traj]
        nn = len(self.networks)
        _need(len(self.n_traj) == nn, "one trajectory count per network")
        obs = [np.asarray(n.obs_species if obs_species is None else obs_species[i], np.int32)
               for i, n in enumerate(self.networks)]
        self._keep = [
            np.array([n.n_species for n in self.networks], np.int32),
            np.array([n.n_reactions for n in self.networks], np.int32),
            np.array([n.n_params for n in self.networks], np.int32),
            np.array(self.n_traj, np.int32),
            np.array([len(o) for o in obs], np.int32),
            np.ascontiguousarray(np.concatenate([n.reactant.reshape(-1) for n in self.networks]), np.int32),
            np.ascontiguousarray(np.concatenate([n.rate_index for n in self.networks]), np.int32),
            np.ascontiguousarray(np.concatenate([n.stoich.reshape(-1) for n in self.networks]), np.int8),
            np.ascontiguousarray(np.concatenate(obs) if sum(len(o) for o in obs) else np.zeros(1), np.int32),
            np.ascontiguousarray(t_obs if t_obs is not None else np.zeros(nn), np.float64),
        ]
        k = self._keep
        d = _Desc(nn, *[a.ctypes.data_as(C.c_void_p).value for a in k], self.EXEC[exec_mode], int(wave_split),
                  int(wave_lanes))
        self.exec_mode, self.wave_split, self.wave_lanes = exec_mode, wave_split, wave_lanes
        h = C.c_void_p()
        _check(lib().ssa_net_create(C.byref(d), C.byref(h)), "ssa_net_create")
        self.handle = h
        self.obs_species = obs
        tt, st, pt, nn_ = (C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64())
        _check(lib().ssa_net_sizes(h, C.byref(tt), C.byref(st), C.byref(pt), C.byref(nn_)), "ssa_net_sizes")
        self.traj_total, self.state_total, self.param_total = tt.value, st.value, pt.value

    def layout(self, n: int, obs_kind: int = W.OBS_FINAL, n_bins: int = 0) -> _Layout:
        L = _Layout()
        _check(lib().ssa_net_layout(self.handle, obs_kind, n_bins, n, C.byref(L)), "ssa_net_layout")
        return L

    def obs_total(self, obs_kind: int, n_bins: int) -> int:
        if obs_kind == W.OBS_TAIL:
            return sum((len(o) + 1) * b for o, b in zip(self.obs_species, self.n_traj))
        per = sum(len(o) * b for o, b in zip(self.obs_species, self.n_traj))
        return per * (n_bins if obs_kind in (W.OBS_BINS, W.OBS_GRID) else 1)

    def mean_total(self, obs_kind: int, n_bins: int) -> int:
        """Length of the ensemble-mean buffer (and of a shared d_obs)."""
        if obs_kind == W.OBS_TAIL:
            return sum(len(o) + 1 for o in self.obs_species)
        per = sum(len(o) for o in self.obs_species)
        return per * (n_bins if obs_kind in (W.OBS_BINS, W.OBS_GRID) else 1)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.ssa_net_destroy(h)
            self.handle = None


def make_cfg(cfg: W.RunConfig, tie_capacity: int = 0, bwd_mode: str = "auto",
             traj_ids: Optional[torch.Tensor] = None, d_epoch: Optional[torch.Tensor] = None,
             d_temperature: Optional[torch.Tensor] = None) -> _Cfg:
    n_steps = int(min(cfg.n_steps, 2 ** 31 - 1))
    return _Cfg(int(cfg.seed) & (2 ** 64 - 1), int(cfg.purpose), int(cfg.epoch), _ptr(d_epoch),
                _ptr(traj_ids), n_steps, float(cfg.t_end), int(cfg.obs_kind),
                int(cfg.n_bins if cfg.obs_kind in (W.OBS_BINS, W.OBS_GRID, W.OBS_TAIL) else 0),
                float(cfg.temperature),
                int(cfg.ckpt_every), _BWD[bwd_mode], int(tie_capacity), _ptr(d_temperature),
                int(cfg.selection), int(cfg.obs_layout), int(bool(cfg.dobs_shared)), int(bool(cfg.relaxed)))


@dataclass
class Forward:
    x_final: torch.Tensor      # int32 [state_total]
    t_final: torch.Tensor      # float64 [traj_total]
    steps_done: torch.Tensor   # int32 [traj_total]
    obs: torch.Tensor          # float64 [obs_total]
    ckpt: Optional[torch.Tensor]
    ties: Optional[torch.Tensor]
    n_ties: Optional[torch.Tensor]
    work: torch.Tensor
    ccfg: _Cfg

    def tie_records(self) -> np.ndarray:
        """Logged near-ties as a structured array (synchronises)."""
        if self.ties is None:
            return np.zeros(0, TIE_DTYPE)
        n = int(self.n_ties.item())
        cap = self.ties.numel() // TIE_DTYPE.itemsize
        if n > cap:
            raise SSAError(f"tie log overflow: {n} near-ties, capacity {cap}")
        return np.frombuffer(self.ties[: n * TIE_DTYPE.itemsize].cpu().numpy().tobytes(), TIE_DTYPE)


def buffer_sizes(net: Net, ccfg: _Cfg):
    ck, wk = C.c_size_t(), C.c_size_t()
    _check(lib().ssa_buffer_sizes(net.handle, C.byref(ccfg), C.byref(ck), C.byref(wk)), "ssa_buffer_sizes")
    return ck.value, wk.value


def forward(net: Net, cfg: W.RunConfig, theta: torch.Tensor, x0: torch.Tensor, *,
            keep_ckpt: bool = True, tie_capacity: int = 4096, bwd_mode: str = "auto",
            traj_ids: Optional[torch.Tensor] = None, d_epoch: Optional[torch.Tensor] = None,
            d_temperature: Optional[torch.Tensor] = None,
            buffers: Optional[Forward] = None, stream=None) -> Forward:
    """Runs ssa_forward.  theta: float32 [param_total], x0: int32 [state_total] (CUDA).
    d_epoch (int32 [1]) and d_temperature (float32 [1]), if given, are read on the
    device by this forward and by the backward that uses its buffers."""
    if d_temperature is not None:
        _dev_tensor(d_temperature, torch.float32, 1, "d_temperature")
    if d_epoch is not None:
        _dev_tensor(d_epoch, torch.int32, 1, "d_epoch")
    if traj_ids is not None:
        _dev_tensor(traj_ids, torch.int32, net.traj_total, "traj_ids")
    dev = theta.device
    _dev_tensor(theta, torch.float32, net.param_total, "theta")
    _dev_tensor(x0, torch.int32, net.state_total, "x0")
    ccfg = make_cfg(cfg, tie_capacity, bwd_mode, traj_ids, d_epoch, d_temperature)
    ck_bytes, wk_bytes = buffer_sizes(net, ccfg)
    if buffers is None:
        obs_n = max(net.mean_total(cfg.obs_kind, cfg.n_bins) if cfg.obs_layout == W.OBS_ENSEMBLE_MEAN
                    else net.obs_total(cfg.obs_kind, cfg.n_bins), 1)
        buffers = Forward(
            torch.empty(net.state_total, dtype=torch.int32, device=dev),
            torch.empty(net.traj_total, dtype=torch.float64, device=dev),
            torch.empty(net.traj_total, dtype=torch.int32, device=dev),
            torch.empty(obs_n, dtype=torch.float64, device=dev),
            torch.empty(max(ck_bytes, 1), dtype=torch.uint8, device=dev) if keep_ckpt and ck_bytes else None,
            torch.empty(max(tie_capacity, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
            if tie_capacity else None,
            torch.zeros(1, dtype=torch.int32, device=dev) if tie_capacity else None,
            torch.empty(wk_bytes, dtype=torch.uint8, device=dev),
            ccfg)
    else:
        obs_n = max(net.mean_total(cfg.obs_kind, cfg.n_bins) if cfg.obs_layout == W.OBS_ENSEMBLE_MEAN
                    else net.obs_total(cfg.obs_kind, cfg.n_bins), 1)
        _need(buffers.x_final.numel() >= net.state_total and buffers.t_final.numel() >= net.traj_total
              and buffers.steps_done.numel() >= net.traj_total and buffers.obs.numel() >= obs_n
              and buffers.work.numel() >= wk_bytes
              and (buffers.ckpt is None or not keep_ckpt or buffers.ckpt.numel() >= ck_bytes),
              "the buffers of another handle or run settings were passed")
        buffers.ccfg = ccfg
    b = buffers
    rc = lib().ssa_forward(net.handle, C.byref(ccfg), _ptr(theta), _ptr(x0), _ptr(b.x_final),
                           _ptr(b.t_final), _ptr(b.steps_done), _ptr(b.obs), _ptr(b.ckpt),
                           b.ckpt.numel() if b.ckpt is not None else 0, _ptr(b.ties), _ptr(b.n_ties),
                           _ptr(b.work), b.work.numel(), _stream(stream))
    _check(rc, "ssa_forward")
    return b


def _dobs_size(net: Net, c: "_Cfg") -> int:
    """Values of dL/dobs the backward reads for the forward's settings: one
    block of the ensemble-mean layout per network when it is shared (the only
    d_obs an ensemble-mean forward accepts), else the observation's."""
    if c.dobs_shared or c.obs_layout == W.OBS_ENSEMBLE_MEAN:
        return net.mean_total(c.obs_kind, c.n_bins)
    return net.obs_total(c.obs_kind, c.n_bins)


def backward(net: Net, cfg: W.RunConfig, theta: torch.Tensor, x0: torch.Tensor, fwd: Forward,
             d_obs: torch.Tensor, per_traj: bool = False, d_params: Optional[torch.Tensor] = None,
             stream=None):
    """Runs ssa_backward; returns d_params (float32 [param_total]) and, if asked,
    per-trajectory gradients (float32 [sum P_n*B_n])."""
    _need(fwd.ckpt is not None, "the forward kept no checkpoints")
    _dev_tensor(theta, torch.float32, net.param_total, "theta")
    _dev_tensor(x0, torch.int32, net.state_total, "x0")
    d_obs = d_obs.contiguous()
    _dev_tensor(d_obs, torch.float64, _dobs_size(net, fwd.ccfg), "d_obs", exact=False)
    if d_params is not None:
        _dev_tensor(d_params, torch.float32, net.param_total, "d_params", exact=False)
    if d_params is None:
        d_params = torch.empty(net.param_total, dtype=torch.float32, device=theta.device)
    ppt = None
    if per_traj:
        n = sum(nw.n_params * b for nw, b in zip(net.networks, net.n_traj))
        ppt = torch.empty(n, dtype=torch.float32, device=theta.device)
    rc = lib().ssa_backward(net.handle, C.byref(fwd.ccfg), _ptr(theta), _ptr(x0), _ptr(fwd.x_final),
                            _ptr(fwd.t_final), _ptr(fwd.steps_done), _ptr(fwd.ckpt), fwd.ckpt.numel(),
                            _ptr(d_obs), _ptr(d_params), _ptr(ppt), _ptr(fwd.work),
                            fwd.work.numel(), _stream(stream))
    _check(rc, "ssa_backward")
    return (d_params, ppt) if per_traj else d_params


def backward_static(net: Net, cfg: W.RunConfig, theta: torch.Tensor, x0: torch.Tensor, fwd: Forward,
                    d_obs: torch.Tensor, d_params: torch.Tensor, ppt: Optional[torch.Tensor] = None, stream=None):
    """Runs ssa_backward_static: ssa_backward with the library's static device
    scratch instead of a work buffer (the caller provides the outputs
    d_params float32 [param_total] and, optionally, ppt [sum P_n*B_n])."""
    _need(fwd.ckpt is not None, "the forward kept no checkpoints")
    _dev_tensor(theta, torch.float32, net.param_total, "theta")
    _dev_tensor(x0, torch.int32, net.state_total, "x0")
    _dev_tensor(d_obs, torch.float64, _dobs_size(net, fwd.ccfg), "d_obs", exact=False)
    _dev_tensor(d_params, torch.float32, net.param_total, "d_params", exact=False)
    if ppt is not None:
        _dev_tensor(ppt, torch.float32, sum(nw.n_params * b for nw, b in zip(net.networks, net.n_traj)), "ppt",
                    exact=False)
    rc = lib().ssa_backward_static(net.handle, C.byref(fwd.ccfg), _ptr(theta), _ptr(x0), _ptr(fwd.x_final),
                                   _ptr(fwd.t_final), _ptr(fwd.steps_done), _ptr(fwd.ckpt), fwd.ckpt.numel(),
                                   _ptr(d_obs), _ptr(d_params), _ptr(ppt), _stream(stream))
    _check(rc, "ssa_backward_static")
    return d_params


def obs_mean(net: Net, fwd: Forward, out: Optional[torch.Tensor] = None, obs: Optional[torch.Tensor] = None,
             stream=None) -> torch.Tensor:
    """Runs ssa_obs_mean on the observation of a forward (or on `obs`, laid
    out as that forward's observation): the ensemble means of every network,
    float64 [mean_total].  Uses the forward's work buffer."""
    c = fwd.ccfg
    obs = fwd.obs if obs is None else obs
    _dev_tensor(obs, torch.float64, net.mean_total(c.obs_kind, c.n_bins) if c.obs_layout == W.OBS_ENSEMBLE_MEAN
                else net.obs_total(c.obs_kind, c.n_bins), "obs", exact=False)
    n = max(net.mean_total(c.obs_kind, c.n_bins), 1)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=obs.device)
    _dev_tensor(out, torch.float64, n, "out", exact=False)
    rc = lib().ssa_obs_mean(net.handle, C.byref(c), _ptr(obs), _ptr(out), _ptr(fwd.work), fwd.work.numel(),
                            _stream(stream))
    _check(rc, "ssa_obs_mean")
    return out


def step_batch(net: Net, cfg: W.RunConfig, theta: torch.Tensor, x: torch.Tensor, t: torch.Tensor,
               step: int, want_a: bool = False, stream=None):
    """One direct-method step in place; returns (chosen, tau, a)."""
    ccfg = make_cfg(cfg)
    dev = theta.device
    _dev_tensor(theta, torch.float32, net.param_total, "theta")
    _dev_tensor(x, torch.int32, net.state_total, "x")
    _dev_tensor(t, torch.float64, net.traj_total, "t")
    chosen = torch.empty(net.traj_total, dtype=torch.int32, device=dev)
    tau = torch.empty(net.traj_total, dtype=torch.float32, device=dev)
    n_a = sum(nw.n_reactions * b for nw, b in zip(net.networks, net.n_traj))
    a = torch.empty(n_a, dtype=torch.float32, device=dev) if want_a else None
    rc = lib().ssa_step_batch(net.handle, C.byref(ccfg), _ptr(theta), _ptr(x), _ptr(t), step & 0xFFFFFFFF,
                              _ptr(chosen), _ptr(tau), _ptr(a), _stream(stream))
    _check(rc, "ssa_step_batch")
    return chosen, tau, a


def device_status(net: Net, stream=None) -> int:
    flags = C.c_uint32()
    rc = lib().ssa_device_status(net.handle, _stream(stream), C.byref(flags))
    _check(rc, "ssa_device_status")
    return flags.value


def selftest_philox(ctr_key: np.ndarray) -> np.ndarray:
    ck = torch.from_numpy(np.ascontiguousarray(ctr_key, np.uint32).view(np.int32)).cuda()
    out = torch.empty(ck.numel() // 6 * 4, dtype=torch.int32, device="cuda")
    _check(lib().ssa_selftest_philox(_ptr(ck), _ptr(out), ck.numel() // 6, _stream()), "selftest_philox")
    return out.cpu().numpy().view(np.uint32).reshape(-1, 4)


def selftest_neglog(first: int, count: int) -> torch.Tensor:
    out = torch.empty(count, dtype=torch.float32, device="cuda")
    _check(lib().ssa_selftest_neglog(first, count, _ptr(out), _stream()), "selftest_neglog")
    return out


# ---------------------------------------------------------------------------
class SimulateST(torch.autograd.Function):
    """obs = simulate(theta) with the straight-through backward of libssa:
    forward = ssa_forward (hard choices, checkpoints and choice tape kept),
    backward = ssa_backward on the incoming dL/dobs (float64), returning
    dL/dtheta (float32).  x0 is not differentiable."""

    @staticmethod
    def forward(ctx, theta, net, cfg, x0, bwd_mode, tie_capacity, record):
        fwd = forward(net, cfg, theta.detach().contiguous(), x0, keep_ckpt=True,
                      tie_capacity=tie_capacity, bwd_mode=bwd_mode)
        ctx.net, ctx.cfg, ctx.fwd = net, cfg, fwd
        ctx.save_for_backward(theta, x0)
        if record is not None:
            record["forward"] = fwd
        return fwd.obs

    @staticmethod
    def backward(ctx, d_obs):
        theta, x0 = ctx.saved_tensors
        d = backward(ctx.net, ctx.cfg, theta.detach().contiguous(), x0, ctx.fwd,
                     d_obs.to(torch.float64).contiguous())
        return d, None, None, None, None, None, None


def simulate(theta: torch.Tensor, net: Net, cfg: W.RunConfig, x0: torch.Tensor,
             bwd_mode: str = "auto", tie_capacity: int = 0, record: Optional[dict] = None) -> torch.Tensor:
    """Differentiable simulation: the observation (float64, the layout of
    ssa_forward's obs) as a function of theta.  record, if given, receives the
    forward's buffers under "forward" (final state, clock, near-tie log)."""
    return SimulateST.apply(theta, net, cfg, x0, bwd_mode, tie_capacity, record)


# ---------------------------------------------------------------------------
# Gene-regulatory network classifier
# ---------------------------------------------------------------------------
class Grn:
    """Handle of a gene-network classifier run shape (see include/ssa.h)."""

    def __init__(self, net: W.GrnNet, n_images: int, n_rep: int):
        self.net = net
        self.n_images, self.n_rep = int(n_images), int(n_rep)
        self.B = self.n_images * self.n_rep
        d = _GrnDesc(net.n_in, net.n_hid, net.n_out, self.n_images, self.n_rep, float(net.beta),
                     float(net.delta_min))
        h = C.c_void_p()
        _check(lib().ssa_grn_create(C.byref(d), C.byref(h)), "ssa_grn_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.ssa_grn_destroy(h)
            self.handle = None


@dataclass
class GrnForward:
    x0: torch.Tensor           # int32 [n_hid + n_out, B] (the forward's input)
    u_hid: torch.Tensor        # float32 [n_images, n_hid]
    x_final: torch.Tensor      # int32 [n_hid + n_out, B]
    t_final: torch.Tensor      # float64 [B]
    steps_done: torch.Tensor   # int32 [B]
    obs: torch.Tensor          # float64 [n_out, B]
    tape: Optional[torch.Tensor]
    ties: Optional[torch.Tensor]
    n_ties: Optional[torch.Tensor]
    ccfg: _Cfg

    tie_records = Forward.tie_records


def grn_buffer_sizes(g: Grn, ccfg: _Cfg):
    tb, wb = C.c_size_t(), C.c_size_t()
    _check(lib().ssa_grn_buffer_sizes(g.handle, C.byref(ccfg), C.byref(tb), C.byref(wb)), "ssa_grn_buffer_sizes")
    return tb.value, wb.value


def grn_forward(g: Grn, cfg: W.RunConfig, theta: torch.Tensor, x_img: torch.Tensor,
                x0: Optional[torch.Tensor] = None, *, keep_tape: bool = True, tie_capacity: int = 4096,
                traj_ids: Optional[torch.Tensor] = None, d_epoch: Optional[torch.Tensor] = None,
                d_temperature: Optional[torch.Tensor] = None,
                buffers: Optional[GrnForward] = None, stream=None) -> GrnForward:
    """Runs ssa_grn_forward.  theta float32 [P], x_img float32 [n_images, n_in] (CUDA).
    d_epoch / d_temperature: optional device scalars read by this forward and its backward."""
    dev = theta.device
    n = g.net
    _dev_tensor(theta, torch.float32, n.n_params, "theta")
    x_img = x_img.contiguous()
    _need(tuple(x_img.shape) == (g.n_images, n.n_in), f"x_img must be [{g.n_images}, {n.n_in}]")
    _dev_tensor(x_img, torch.float32, g.n_images * n.n_in, "x_img")
    if x0 is None:
        x0 = torch.zeros((n.n_species, g.B), dtype=torch.int32, device=dev)
    x0 = x0.contiguous()       # kept with the buffers: the backward reads it too
    _dev_tensor(x0, torch.int32, n.n_species * g.B, "x0")
    for name, t in (("traj_ids", traj_ids), ("d_epoch", d_epoch), ("d_temperature", d_temperature)):
        if t is not None:
            _dev_tensor(t, torch.float32 if name == "d_temperature" else torch.int32,
                        g.B if name == "traj_ids" else 1, name)
    ccfg = make_cfg(cfg, tie_capacity, "auto", traj_ids, d_epoch, d_temperature)
    tb, _ = grn_buffer_sizes(g, ccfg)
    if buffers is None:
        buffers = GrnForward(
            x0,
            torch.empty((g.n_images, n.n_hid), dtype=torch.float32, device=dev),
            torch.empty((n.n_species, g.B), dtype=torch.int32, device=dev),
            torch.empty(g.B, dtype=torch.float64, device=dev),
            torch.empty(g.B, dtype=torch.int32, device=dev),
            torch.empty((n.n_out, g.B), dtype=torch.float64, device=dev),
            torch.empty(max(tb, 1), dtype=torch.uint8, device=dev) if keep_tape else None,
            torch.empty(max(tie_capacity, 1) * TIE_DTYPE.itemsize, dtype=torch.uint8, device=dev)
            if tie_capacity else None,
            torch.zeros(1, dtype=torch.int32, device=dev) if tie_capacity else None,
            ccfg)
    else:
        buffers.ccfg = ccfg
        buffers.x0 = x0
    b = buffers
    rc = lib().ssa_grn_forward(g.handle, C.byref(ccfg), _ptr(theta), _ptr(x_img),
                               _ptr(x0), _ptr(b.u_hid), _ptr(b.x_final), _ptr(b.t_final),
                               _ptr(b.steps_done), _ptr(b.obs), _ptr(b.tape),
                               b.tape.numel() if b.tape is not None else 0, _ptr(b.ties), _ptr(b.n_ties),
                               _stream(stream))
    _check(rc, "ssa_grn_forward")
    return b


def grn_backward(g: Grn, cfg: W.RunConfig, theta: torch.Tensor, x_img: torch.Tensor, fwd: GrnForward,
                 d_obs: torch.Tensor, per_traj: bool = False, d_params: Optional[torch.Tensor] = None,
                 work: Optional[torch.Tensor] = None, stream=None):
    """Runs ssa_grn_backward; returns d_params float32 [P] and, if asked, the
    compact per-trajectory gradients float64 [B, C]."""
    _need(fwd.tape is not None, "the forward kept no tape")
    _dev_tensor(theta, torch.float32, g.net.n_params, "theta")
    x_img = x_img.contiguous()
    _dev_tensor(x_img, torch.float32, g.n_images * g.net.n_in, "x_img")
    d_obs = d_obs.contiguous()
    _dev_tensor(d_obs, torch.float64, g.net.n_out * g.B, "d_obs")
    dev = theta.device
    _, wb = grn_buffer_sizes(g, fwd.ccfg)
    if work is None:
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
    if d_params is None:
        d_params = torch.empty(g.net.n_params, dtype=torch.float32, device=dev)
    comp = torch.empty((g.B, g.net.n_compact), dtype=torch.float64, device=dev) if per_traj else None
    if d_params is not None:
        _dev_tensor(d_params, torch.float32, g.net.n_params, "d_params", exact=False)
    _dev_tensor(work, torch.uint8, wb, "work", exact=False)
    rc = lib().ssa_grn_backward(g.handle, C.byref(fwd.ccfg), _ptr(theta), _ptr(x_img),
                                _ptr(fwd.x0), _ptr(fwd.u_hid), _ptr(fwd.x_final), _ptr(fwd.steps_done), _ptr(fwd.tape),
                                fwd.tape.numel(), _ptr(d_obs), _ptr(d_params), _ptr(comp),
                                _ptr(work), work.numel(), _stream(stream))
    _check(rc, "ssa_grn_backward")
    return (d_params, comp) if per_traj else d_params


def grn_device_status(g: Grn, stream=None) -> int:
    flags = C.c_uint32()
    rc = lib().ssa_grn_device_status(g.handle, _stream(stream), C.byref(flags))
    _check(rc, "ssa_grn_device_status")
    return flags.value
