"""Autotuner of the execution plan of a batch of networks.

A plan is what `ssa.Net` and the run settings leave open:

- the execution mode: one trajectory per lane with topology-specialised
  kernels, one per lane with generic kernels, or one per group of lanes;
- for the lane-group mode, one persistent launch or one launch per width, and
  the widest group (lanes per trajectory; a network too large for one Philox
  block per lane of a narrower group draws two per lane);
- how the backward recovers the fired channels (choice tape or recompute);
- the checkpoint interval K.

The tuner times every plan that the library accepts for the batch. Each plan
gets a forward + backward on a shortened run of the same networks and
trajectory counts, and the fastest one is kept. Choices are cached in a JSON
file keyed by the device architecture and a signature of the batch: the
(species, channels, trajectories) triples, the step count rounded to a power of
two, and the observation kind and bin count.  Plans differ only in speed: every plan
computes the same results (the parity tests run all of them).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
from dataclasses import asdict, dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import ssa
from . import workloads as W

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ssa_mi355x", "autotune.json")


@dataclass(frozen=True)
class Plan:
    exec_mode: str = "auto"       # "spec" | "lane" | "wave" | "auto"
    wave_split: int = -1          # wave mode: 1 one launch per width, 0 one launch
    bwd_mode: str = "tape"        # "tape" | "recompute" | "tangent"
    ckpt_every: int = 256
    wave_lanes: int = 0           # wave mode: widest lane group (0: 64)

    @property
    def name(self) -> str:
        w = f"/w{self.wave_lanes}" if self.wave_lanes else ""
        return f"{self.exec_mode}/split{self.wave_split}{w}/{self.bwd_mode}/K{self.ckpt_every}"

    def net(self, nets, n_traj, t_obs=None) -> ssa.Net:
        return ssa.Net(nets, n_traj, t_obs=t_obs, exec_mode=self.exec_mode, wave_split=self.wave_split,
                       wave_lanes=self.wave_lanes)

    def config(self, cfg: W.RunConfig) -> W.RunConfig:
        return cfg.replace(ckpt_every=self.ckpt_every)


def candidate_plans(n_steps: int) -> List[Plan]:
    """Every plan the tuner tries (the library rejects the ones a batch cannot run)."""
    out = []
    ks = [k for k in (64, 256, 1024) if k <= max(64, n_steps)]
    for mode, splits in (("spec", [-1]), ("lane", [-1]), ("wave", [1, 0])):
        for split in splits:
            for k in ks:
                out.append(Plan(mode, split, "tape", k))
            out.append(Plan(mode, split, "recompute", 64))
    # narrower lane groups: more trajectories per wavefront, two Philox blocks
    # per lane for the networks that need them
    kw = 256 if 256 in ks else ks[-1]
    for lanes in (32, 16):
        for split in (1, 0):
            out.append(Plan("wave", split, "tape", kw, lanes))
    # forward-mode tangents (networks with few channels, specialised mode)
    out.append(Plan("spec", -1, "tangent", ks[-1]))
    return out


def signature(nets: Sequence[W.Network], n_traj: Sequence[int], cfg: W.RunConfig) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "none"
    h = hashlib.sha1()
    for n, b in zip(nets, n_traj):
        h.update(np.asarray([n.n_species, n.n_reactions, int(b)], np.int64).tobytes())
        h.update(np.ascontiguousarray(n.reactant, np.int32).tobytes())
        h.update(np.ascontiguousarray(n.stoich, np.int32).tobytes())
    steps = int(min(cfg.n_steps, 2 ** 31 - 1))
    bucket = 1 << max(0, int(math.ceil(math.log2(max(steps, 1)))))
    return f"{arch}|{h.hexdigest()[:16]}|n{len(nets)}|s{bucket}|o{cfg.obs_kind}|b{cfg.n_bins}"


class Cache:
    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        try:
            with open(path) as f:
                self.data: Dict[str, dict] = json.load(f)
        except (OSError, ValueError):
            self.data = {}

    def get(self, key: str) -> Optional[Plan]:
        d = self.data.get(key)
        return Plan(**d["plan"]) if d else None

    def put(self, key: str, plan: Plan, timings: dict):
        self.data[key] = {"plan": asdict(plan), "timings_ms": timings}
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _time_plan(plan: Plan, nets, n_traj, cfg, theta, x0, t_obs, d_obs_fn, repeats: int) -> float:
    h = plan.net(nets, n_traj, t_obs)
    c = plan.config(cfg)
    fwd = ssa.forward(h, c, theta, x0, tie_capacity=0, bwd_mode=plan.bwd_mode)
    d_obs = d_obs_fn(h, fwd)
    d_params = torch.empty(h.param_total, dtype=torch.float32, device=theta.device)
    ms = []
    for r in range(repeats + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ssa.forward(h, c, theta, x0, tie_capacity=0, bwd_mode=plan.bwd_mode, buffers=fwd)
        ssa.backward(h, c, theta, x0, fwd, d_obs, d_params=d_params)
        e1.record()
        torch.cuda.synchronize()
        if r:                                    # the first run warms caches and compiles
            ms.append(e0.elapsed_time(e1))
    if ssa.device_status(h) != 0:
        raise ssa.SSAError("device flags raised while tuning")
    return float(np.median(ms))


def tune(nets: Sequence[W.Network], n_traj: Sequence[int], cfg: W.RunConfig, theta: torch.Tensor,
         x0: torch.Tensor, t_obs: Optional[Sequence[float]] = None, *, probe_steps: int = 512,
         repeats: int = 3, cache: Optional[Cache] = None, plans: Optional[Sequence[Plan]] = None,
         retune: bool = False, log=None) -> Plan:
    """Best plan for a batch (cached).  The probe run keeps the networks,
    trajectory counts and observation, with at most `probe_steps` steps."""
    cache = cache if cache is not None else Cache()
    key = signature(nets, n_traj, cfg)
    if not retune:
        hit = cache.get(key)
        if hit is not None:
            return hit
    probe = cfg.replace(n_steps=int(min(cfg.n_steps, probe_steps)))

    def d_obs_fn(h, fwd):
        g = torch.Generator(device=theta.device).manual_seed(0)
        return torch.randn(fwd.obs.numel(), generator=g, dtype=torch.float64, device=theta.device)

    timings = {}
    best, best_ms = None, math.inf
    for plan in (plans if plans is not None else candidate_plans(int(min(cfg.n_steps, 2 ** 31 - 1)))):
        name = plan.name
        try:
            ms = _time_plan(plan, nets, n_traj, probe, theta, x0, t_obs, d_obs_fn, repeats)
        except ssa.SSAError as e:                # the library cannot run this plan for the batch
            timings[name] = None
            if log:
                log(f"{name}: rejected ({e})")
            continue
        timings[name] = ms
        if log:
            log(f"{name}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = plan, ms
    if best is None:
        raise ssa.SSAError("no execution plan accepted this batch")
    cache.put(key, best, timings)
    return best
