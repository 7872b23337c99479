"""Python access to the FP64 CPU oracle (``ssa_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg may use this module; the product path never does.
It imports nothing from the HIP package: callers hand it the seeded input
descriptions (networks, run settings) as plain objects and arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ssa_oracle.c")
SOURCES = [SRC, os.path.join(HERE, "ssa_oracle_grn.c")]
HEADER = os.path.join(HERE, "ssa_oracle.h")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or _stale():
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-Wno-unused-parameter",
                               *SOURCES, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + [HEADER])


class _Net(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32), ("n_params", C.c_int32),
                ("reactant", C.c_void_p), ("rate_index", C.c_void_p), ("stoich", C.c_void_p)]


class _Cfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("purpose", C.c_uint32), ("epoch", C.c_uint32),
                ("n_steps", C.c_int64), ("t_end", C.c_double), ("obs_kind", C.c_int32),
                ("n_bins", C.c_int32), ("t_obs", C.c_double), ("n_obs", C.c_int32),
                ("obs_species", C.c_void_p), ("temperature", C.c_double),
                ("tie_threshold", C.c_double), ("clock_tol", C.c_double), ("selection", C.c_int32),
                ("edge_window", C.c_double)]


class _Grn(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_hid", C.c_int32), ("n_out", C.c_int32),
                ("beta", C.c_double), ("delta_min", C.c_double)]


class _Ov(C.Structure):
    _fields_ = [("off", C.c_void_p), ("step", C.c_void_p), ("kind", C.c_void_p), ("val", C.c_void_p)]


class _Stats(C.Structure):
    _fields_ = [("min_margin", C.c_void_p), ("n_near", C.c_void_p), ("n_resync", C.c_void_p),
                ("n_bad", C.c_void_p), ("bin_edge_dist", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        L = C.CDLL(LIB)
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_step_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint32, C.c_int32, C.c_void_p]
        common = [C.POINTER(_Net), C.POINTER(_Cfg), C.c_void_p, C.c_int64, C.c_void_p,
                  C.c_void_p, C.POINTER(_Ov)]
        L.orc_forward.argtypes = common + [C.c_void_p] * 4 + [C.POINTER(_Stats), C.c_int]
        L.orc_forward.restype = C.c_int
        L.orc_adjoint.argtypes = common + [C.c_void_p] * 6 + [C.POINTER(_Stats), C.c_int]
        L.orc_adjoint.restype = C.c_int
        L.orc_adjoint_kappa.argtypes = common + [C.c_void_p] * 7 + [C.POINTER(_Stats), C.c_int]
        L.orc_adjoint_kappa.restype = C.c_int
        L.orc_trace.argtypes = [C.POINTER(_Net), C.POINTER(_Cfg), C.c_void_p, C.c_uint32,
                                C.c_void_p, C.c_int64] + [C.c_void_p] * 7
        L.orc_trace.restype = C.c_int64
        L.orc_bf16.argtypes = [C.c_float]
        L.orc_bf16.restype = C.c_float
        L.orc_grn_n_params.argtypes = [C.POINTER(_Grn)]
        L.orc_grn_n_params.restype = C.c_int64
        L.orc_grn_n_compact.argtypes = [C.POINTER(_Grn)]
        L.orc_grn_n_compact.restype = C.c_int64
        L.orc_grn_hidden_input.argtypes = [C.POINTER(_Grn), C.c_void_p, C.c_void_p, C.c_int64,
                                           C.c_void_p]
        L.orc_grn_run.argtypes = [C.POINTER(_Grn), C.POINTER(_Cfg), C.c_void_p, C.c_void_p,
                                  C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(_Ov),
                                  C.c_void_p] + [C.c_void_p] * 5 + [C.POINTER(_Stats), C.c_int]
        L.orc_grn_run.restype = C.c_int
        L.orc_grn_trace.argtypes = [C.POINTER(_Grn), C.POINTER(_Cfg), C.c_void_p, C.c_void_p,
                                    C.c_uint32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_grn_trace.restype = C.c_int64
        L.orc_grn_soft_run.argtypes = [C.POINTER(_Grn), C.POINTER(_Cfg), C.c_void_p, C.c_void_p, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.orc_grn_soft_run.restype = C.c_int
        L.orc_grn_soft_trace.argtypes = [C.POINTER(_Grn), C.POINTER(_Cfg), C.c_void_p, C.c_void_p, C.c_uint32,
                                         C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_grn_soft_trace.restype = C.c_int64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------
def philox4x32_10(counter: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.asarray(counter, np.uint32)
    k = np.asarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniform(x: int) -> float:
    return lib().orc_uniform(int(x) & 0xFFFFFFFF)


def step_uniforms(seed: int, purpose: int, epoch: int, traj: int, step: int, n_words: int) -> np.ndarray:
    u = np.zeros(n_words, np.float64)
    lib().orc_step_uniforms(seed, purpose, epoch, traj, step, n_words, _p(u))
    return u


@dataclass
class OracleResult:
    x_final: np.ndarray        # [n_traj, N]
    t_final: np.ndarray        # [n_traj]
    steps_done: np.ndarray     # [n_traj]
    obs: np.ndarray            # [n_traj, n_bins, n_obs] or [n_traj, n_obs]
    min_margin: np.ndarray
    n_near: np.ndarray
    n_resync: np.ndarray
    n_bad: np.ndarray
    bin_edge_dist: np.ndarray
    grad: Optional[np.ndarray] = None   # [n_traj, P]
    kappa: Optional[np.ndarray] = None  # [n_traj, P] conditioning of each gradient component


class _Keep:
    """Keeps numpy buffers alive while ctypes structures point at them."""

    def __init__(self):
        self.items = []

    def __call__(self, a):
        self.items.append(a)
        return a


def _structs(net, cfg, keep, tie_threshold, clock_tol, obs_species=None, edge_window=0.0):
    reactant = keep(np.ascontiguousarray(net.reactant, np.int32))
    rate_index = keep(np.ascontiguousarray(net.rate_index, np.int32))
    stoich = keep(np.ascontiguousarray(net.stoich, np.int32))
    n = _Net(net.n_species, net.n_reactions, net.n_params, _p(reactant).value,
             _p(rate_index).value, _p(stoich).value)
    obs_sp = keep(np.ascontiguousarray(net.obs_species if obs_species is None else obs_species,
                                       np.int32))
    c = _Cfg(cfg.seed, cfg.purpose, cfg.epoch, min(int(cfg.n_steps), 2 ** 62),
             float(cfg.t_end), cfg.obs_kind, cfg.n_bins, float(cfg.t_obs), len(obs_sp),
             _p(obs_sp).value, float(cfg.temperature), tie_threshold, clock_tol,
             int(getattr(cfg, "selection", 0)), float(edge_window))
    return n, c


def _overrides(n_traj, ties, keep):
    """ties: iterable of (local traj index, step, kind, val)."""
    if ties is None:
        return None
    t = np.asarray(list(ties), np.int64).reshape(-1, 4)
    order = np.lexsort((t[:, 1], t[:, 0])) if len(t) else np.zeros(0, np.int64)
    t = t[order]
    off = keep(np.searchsorted(t[:, 0], np.arange(n_traj + 1)).astype(np.int64))
    step = keep(np.ascontiguousarray(t[:, 1], np.int64))
    kind = keep(np.ascontiguousarray(t[:, 2], np.int32))
    val = keep(np.ascontiguousarray(t[:, 3], np.int32))
    return _Ov(_p(off).value, _p(step).value, _p(kind).value, _p(val).value)


def run(net, cfg, theta, x0: np.ndarray, traj_ids=None, ties=None, d_obs=None,
        tie_threshold: float = 1e-6, clock_tol: float = 1e-5, n_threads: int = 0,
        obs_species=None, kappa: bool = False, edge_window: float = 0.0) -> OracleResult:
    """Simulate (and, if d_obs is given, differentiate) a set of trajectories.

    x0: [n_traj, N] or [N] (broadcast).  traj_ids: global trajectory ids (the
    Philox counter), default 0..n_traj-1.  theta: ln k as float32 values.
    kappa: also return the conditioning of every gradient component (the sum
    over steps of the magnitudes of its terms, see orc_adjoint_kappa).
    edge_window: bins, with ties holding the GPU's kind-2 (bin-edge) records:
    the relative window within which the adjoint takes the GPU's side of a bin
    edge for an event time (0: the oracle's own clock decides)."""
    keep = _Keep()
    N = net.n_species
    x0 = np.asarray(x0, np.int32)
    if traj_ids is None:
        n_traj = x0.shape[0] if x0.ndim == 2 else 1
        traj_ids = np.arange(n_traj, dtype=np.uint32)
    traj_ids = keep(np.ascontiguousarray(traj_ids, np.uint32))
    n_traj = len(traj_ids)
    if x0.ndim == 1:
        x0 = np.repeat(x0[None, :], n_traj, axis=0)
    x0 = keep(np.ascontiguousarray(x0, np.int32))
    assert x0.shape == (n_traj, N)
    n, c = _structs(net, cfg, keep, tie_threshold, clock_tol, obs_species, edge_window)
    th = keep(np.ascontiguousarray(np.asarray(theta, np.float32).astype(np.float64)))
    ov = _overrides(n_traj, ties, keep)
    n_obs = c.n_obs
    obs_shape = ((n_traj, cfg.n_bins, n_obs) if cfg.obs_kind in (1, 2)
                 else (n_traj, n_obs + 1) if cfg.obs_kind == 3 else (n_traj, n_obs))
    res = OracleResult(np.zeros((n_traj, N), np.int32), np.zeros(n_traj), np.zeros(n_traj, np.int32),
                       np.zeros(obs_shape), np.zeros(n_traj), np.zeros(n_traj, np.int32),
                       np.zeros(n_traj, np.int32), np.zeros(n_traj, np.int32), np.zeros(n_traj))
    st = _Stats(_p(res.min_margin).value, _p(res.n_near).value, _p(res.n_resync).value,
                _p(res.n_bad).value, _p(res.bin_edge_dist).value)
    L = lib()
    ovp = C.byref(ov) if ov is not None else None
    if d_obs is None:
        rc = L.orc_forward(C.byref(n), C.byref(c), _p(th), n_traj, _p(traj_ids), _p(x0), ovp,
                           _p(res.x_final), _p(res.t_final), _p(res.steps_done), _p(res.obs),
                           C.byref(st), n_threads)
    else:
        d = keep(np.ascontiguousarray(np.broadcast_to(d_obs, obs_shape), np.float64))
        res.grad = np.zeros((n_traj, net.n_params))
        if kappa:
            res.kappa = np.zeros((n_traj, net.n_params))
            rc = L.orc_adjoint_kappa(C.byref(n), C.byref(c), _p(th), n_traj, _p(traj_ids), _p(x0), ovp,
                                     _p(d), _p(res.x_final), _p(res.t_final), _p(res.steps_done),
                                     _p(res.obs), _p(res.grad), _p(res.kappa), C.byref(st), n_threads)
        else:
            rc = L.orc_adjoint(C.byref(n), C.byref(c), _p(th), n_traj, _p(traj_ids), _p(x0), ovp,
                               _p(d), _p(res.x_final), _p(res.t_final), _p(res.steps_done),
                               _p(res.obs), _p(res.grad), C.byref(st), n_threads)
    if rc != 0:
        raise RuntimeError("oracle rejected its arguments")
    return res


@dataclass
class Trace:
    X: np.ndarray       # [n+1, N]
    t: np.ndarray       # [n+1]
    tau: np.ndarray     # [n]
    j: np.ndarray       # [n]
    a: np.ndarray       # [n, M]
    u: np.ndarray       # [n, M+1]
    margin: np.ndarray  # [n]


def trace(net, cfg, theta, x0, traj_id: int = 0, cap: int = 1000) -> Trace:
    keep = _Keep()
    n, c = _structs(net, cfg, keep, 1e-6, 1e-5)
    N, M = net.n_species, net.n_reactions
    th = keep(np.ascontiguousarray(np.asarray(theta, np.float32).astype(np.float64)))
    x = keep(np.ascontiguousarray(x0, np.int32))
    X = np.zeros((cap + 1, N), np.int32)
    t = np.zeros(cap + 1)
    tau = np.zeros(cap)
    j = np.zeros(cap, np.int32)
    a = np.zeros((cap, M))
    u = np.zeros((cap, M + 1))
    mg = np.zeros(cap)
    k = lib().orc_trace(C.byref(n), C.byref(c), _p(th), traj_id, _p(x), cap, _p(X), _p(t),
                        _p(tau), _p(j), _p(a), _p(u), _p(mg))
    if k < 0:
        raise RuntimeError("oracle rejected its arguments")
    return Trace(X[:k + 1], t[:k + 1], tau[:k], j[:k], a[:k], u[:k], mg[:k])


# ---------------------------------------------------------------------------
# Gene-regulatory network classifier
# ---------------------------------------------------------------------------
def _grn(net) -> _Grn:
    return _Grn(net.n_in, net.n_hid, net.n_out, float(net.beta), float(net.delta_min))


def bf16(x) -> np.ndarray:
    """The oracle's bfloat16 rounding (nearest even) of FP32 values, elementwise."""
    L = lib()
    x = np.asarray(x, np.float32)
    return np.array([L.orc_bf16(float(v)) for v in x.reshape(-1)], np.float32).reshape(x.shape)


def grn_hidden_input(net, theta, images) -> np.ndarray:
    """u [n_images, n_hid] = b + bf16(W) bf16(x), exact in FP64."""
    keep = _Keep()
    g = _grn(net)
    th = keep(np.ascontiguousarray(np.asarray(theta, np.float32).astype(np.float64)))
    x = keep(np.ascontiguousarray(np.asarray(images, np.float32).astype(np.float64)))
    n_img = x.shape[0]
    u = np.zeros((n_img, net.n_hid))
    lib().orc_grn_hidden_input(C.byref(g), _p(th), _p(x), n_img, _p(u))
    return u


@dataclass
class GrnResult:
    x_final: np.ndarray        # [n_traj, n_hid + n_out]
    t_final: np.ndarray
    steps_done: np.ndarray
    obs: np.ndarray            # [n_traj, n_out]
    min_margin: np.ndarray
    n_near: np.ndarray
    n_resync: np.ndarray
    n_bad: np.ndarray
    grad_c: Optional[np.ndarray] = None   # [n_traj, n_compact]


def grn_run(net, cfg, theta, u_hid, image_of, x0=None, traj_ids=None, ties=None, d_obs=None,
            tie_threshold: float = 1e-6, clock_tol: float = 1e-5, n_threads: int = 0) -> GrnResult:
    """Simulate (and with d_obs [n_traj, n_out], differentiate) GRN trajectories.
    u_hid: [n_images, n_hid] hidden pre-activations (the oracle's own from
    grn_hidden_input, or another implementation's, for split parity)."""
    keep = _Keep()
    g = _grn(net)
    image_of = keep(np.ascontiguousarray(image_of, np.int32))
    n_traj = len(image_of)
    N = net.n_hid + net.n_out
    if traj_ids is None:
        traj_ids = np.arange(n_traj, dtype=np.uint32)
    traj_ids = keep(np.ascontiguousarray(traj_ids, np.uint32))
    x0 = np.zeros((n_traj, N), np.int32) if x0 is None else np.asarray(x0, np.int32)
    x0 = keep(np.ascontiguousarray(np.broadcast_to(x0, (n_traj, N)), np.int32))
    u = keep(np.ascontiguousarray(u_hid, np.float64))
    th = keep(np.ascontiguousarray(np.asarray(theta, np.float32).astype(np.float64)))
    c = _Cfg(cfg.seed, cfg.purpose, cfg.epoch, min(int(cfg.n_steps), 2 ** 62), float(cfg.t_end),
             0, 0, 0.0, 0, None, float(cfg.temperature), tie_threshold, clock_tol)
    ov = _overrides(n_traj, ties, keep)
    res = GrnResult(np.zeros((n_traj, N), np.int32), np.zeros(n_traj), np.zeros(n_traj, np.int32),
                    np.zeros((n_traj, net.n_out)), np.zeros(n_traj), np.zeros(n_traj, np.int32),
                    np.zeros(n_traj, np.int32), np.zeros(n_traj, np.int32))
    st = _Stats(_p(res.min_margin).value, _p(res.n_near).value, _p(res.n_resync).value,
                _p(res.n_bad).value, None)
    dp = None
    if d_obs is not None:
        d = keep(np.ascontiguousarray(np.broadcast_to(d_obs, (n_traj, net.n_out)), np.float64))
        res.grad_c = np.zeros((n_traj, net.n_compact))
        dp = _p(d)
    rc = lib().orc_grn_run(C.byref(g), C.byref(c), _p(th), _p(u), n_traj, _p(traj_ids),
                           _p(image_of), _p(x0), C.byref(ov) if ov is not None else None, dp,
                           _p(res.x_final), _p(res.t_final), _p(res.steps_done), _p(res.obs),
                           _p(res.grad_c) if res.grad_c is not None else None, C.byref(st),
                           n_threads)
    if rc != 0:
        raise RuntimeError("oracle rejected its arguments")
    return res


def grn_full_gradient(net, res_grad_c, images, image_of) -> np.ndarray:
    """Assemble dL/dtheta [P] from the compact per-trajectory gradients:
    dW = sum_q du_q x_{image(q)}^T (x as the contraction sees it, bfloat16),
    the other blocks are sums over trajectories."""
    H, O = net.n_hid, net.n_out
    gc = np.asarray(res_grad_c, np.float64)
    du = gc[:, :H]
    x = bf16(np.asarray(images, np.float32)).astype(np.float64)[np.asarray(image_of)]
    dW = du.T @ x
    rest = gc.sum(axis=0)
    return np.concatenate([dW.reshape(-1), rest[:H], rest[H:H + O * H], rest[H + O * H:H + O * H + O],
                           rest[H + O * H + O:]])


def grn_trace(net, cfg, theta, u_row, traj_id: int = 0, x0=None, cap: int = 1000):
    """Fired channels [n] and clock [n+1] of one trajectory."""
    keep = _Keep()
    g = _grn(net)
    N = net.n_hid + net.n_out
    x = keep(np.ascontiguousarray(np.zeros(N, np.int32) if x0 is None else x0, np.int32))
    u = keep(np.ascontiguousarray(u_row, np.float64))
    th = keep(np.ascontiguousarray(np.asarray(theta, np.float32).astype(np.float64)))
    c = _Cfg(cfg.seed, cfg.purpose, cfg.epoch, min(int(cfg.n_steps), 2 ** 62), float(cfg.t_end),
             0, 0, 0.0, 0, None, float(cfg.temperature), 1e-6, 1e-5)
    j = np.zeros(cap, np.int32)
    t = np.zeros(cap + 1)
    n = lib().orc_grn_trace(C.byref(g), C.byref(c), _p(th), _p(u), traj_id, _p(x), cap, _p(j), _p(t))
    if n < 0:
        raise RuntimeError("oracle rejected its arguments")
    return j[:n], t[:n + 1]


@dataclass
class GrnSoftResult:
    x_final: np.ndarray        # [n_traj, n_hid + n_out] real
    t_final: np.ndarray
    obs: np.ndarray            # [n_traj, n_out]
    grad_c: Optional[np.ndarray] = None   # [n_traj, n_compact]


def _soft_cfg(cfg):
    if np.isfinite(cfg.t_end):
        raise ValueError("the relaxed forward runs a fixed number of steps (t_end must be infinite)")
    return _Cfg(cfg.seed, cfg.purpose, cfg.epoch, min(int(cfg.n_steps), 2 ** 62), float(cfg.t_end),
                0, 0, 0.0, 0, None, float(cfg.temperature), 1e-6, 1e-5)


def grn_soft_run(net, cfg, theta, u_hid, image_of, x0=None, traj_ids=None, d_obs=None,
                 n_threads: int = 0, theta64: bool = False) -> GrnSoftResult:
    """Relaxed forward (Eq. 4) of GRN trajectories and, with d_obs
    [n_traj, n_out], the gradient of sum d_obs * O_final through the whole
    relaxed map.  u_hid: [n_images, n_hid] hidden pre-activations.  theta is
    rounded to FP32 first (the values the library holds) unless theta64."""
    keep = _Keep()
    g = _grn(net)
    image_of = keep(np.ascontiguousarray(image_of, np.int32))
    n_traj = len(image_of)
    N = net.n_hid + net.n_out
    if traj_ids is None:
        traj_ids = np.arange(n_traj, dtype=np.uint32)
    traj_ids = keep(np.ascontiguousarray(traj_ids, np.uint32))
    x0 = np.zeros((n_traj, N)) if x0 is None else np.asarray(x0, np.float64)
    x0 = keep(np.ascontiguousarray(np.broadcast_to(x0, (n_traj, N)), np.float64))
    u = keep(np.ascontiguousarray(u_hid, np.float64))
    th = np.asarray(theta, np.float64) if theta64 else np.asarray(theta, np.float32).astype(np.float64)
    th = keep(np.ascontiguousarray(th))
    c = _soft_cfg(cfg)
    res = GrnSoftResult(np.zeros((n_traj, N)), np.zeros(n_traj), np.zeros((n_traj, net.n_out)))
    dp = None
    if d_obs is not None:
        d = keep(np.ascontiguousarray(np.broadcast_to(d_obs, (n_traj, net.n_out)), np.float64))
        res.grad_c = np.zeros((n_traj, net.n_compact))
        dp = _p(d)
    rc = lib().orc_grn_soft_run(C.byref(g), C.byref(c), _p(th), _p(u), n_traj, _p(traj_ids), _p(image_of),
                                _p(x0), dp, _p(res.x_final), _p(res.t_final), _p(res.obs),
                                _p(res.grad_c) if res.grad_c is not None else None, n_threads)
    if rc != 0:
        raise RuntimeError("oracle rejected its arguments")
    return res


def grn_soft_trace(net, cfg, theta, u_row, traj_id: int = 0, x0=None, cap: int = 1000):
    """The relaxed path of one trajectory: states [n+1, N] and clock [n+1]."""
    keep = _Keep()
    g = _grn(net)
    N = net.n_hid + net.n_out
    x = keep(np.ascontiguousarray(np.zeros(N) if x0 is None else x0, np.float64))
    u = keep(np.ascontiguousarray(u_row, np.float64))
    th = keep(np.ascontiguousarray(np.asarray(theta, np.float32).astype(np.float64)))
    c = _soft_cfg(cfg)
    X = np.zeros((cap + 1, N))
    t = np.zeros(cap + 1)
    n = lib().orc_grn_soft_trace(C.byref(g), C.byref(c), _p(th), _p(u), traj_id, _p(x), cap, _p(X), _p(t))
    if n < 0:
        raise RuntimeError("oracle rejected its arguments")
    return X[:n + 1], t[:n + 1]
