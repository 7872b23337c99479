#!/usr/bin/env python3
"""Throughput of the batched exact SSA step, forward and forward+backward, on one MI355X.

Workload: reversible dimerisation 2A <-> A2 (kf = 1e-3, kb = 0.1, A(0) = 100),
65,536 trajectories x 10,000 steps each, observation = exact bin averages of A
over 20 bins on [0, 2500], loss = MSE of per-bin ensemble mean and variance
against targets from a seeded run at kf = 2e-3, kb = 0.05, Gumbel-Softmax
temperature 0.5, checkpoints every 256 steps, gradients with respect to ln k.

One timed step = ssa_forward + loss (PyTorch FP64) + ssa_backward (+ the FP64
gradient reduction).  `value` counts fired reactions per second of that step;
the inputs are resident in HBM before timing starts.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSA steps/sec fwd and fwd+bwd on 1 MI355X; grad rel-err vs FP64 oracle"
PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes per clock x clock


def alu_slots_per_step(M: int, N: int, nnz_total: int, n_obs: int, backward: bool, inv_t_is_2=True) -> int:
    """Algorithmic VALU issue slots of one step of one trajectory (full-rate
    op = 1 slot, quarter-rate 32-bit multiply / reciprocal / log = 4 slots)."""
    nb = (M + 1 + 3) // 4
    rng = nb * 10 * (2 * 4 + 2)             # Philox4x32-10: two 32x32->64 products, two xor3 a round
    neglog = (M + 1) * (3 + 4 + 1)          # word -> lattice uniform, log, scale
    if not backward:
        prop = M * 5 + M                    # two conversions, subtract, two products; a0 sum
        tau = 4 + 1
        race = M * (4 + 1 + 3)              # reciprocal, product, compare/min/select
        upd = N + 1 + n_obs                 # state update, FP64 clock, FP64 bin integral
        return rng + neglog + prop + tau + race + upd
    prop = M * 7 + M                        # propensities and their two partial derivatives
    tau = 4 + 1 + 1                         # waiting time and the reversed FP64 clock
    soft = M * (5 + 5 + (1 if inv_t_is_2 else 8) + 1) + 4 + M   # ratios, rho, rho^(1/T), sum, normalise
    adj = 2 * nnz_total + M * (2 + 3 + 2 + 2 + 4)              # w_j, wbar, g_j, dtheta, coef, lambda
    return rng + neglog + prop + tau + soft + adj + N + 2 * n_obs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bwd-mode", default="tape", choices=["tape", "recompute"])
    ap.add_argument("--n-traj", type=int, default=65536)
    ap.add_argument("--n-steps", type=int, default=10000)
    ap.add_argument("--ckpt-every", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2602_19775_amd import losses, ssa
    from paper_2602_19775_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    dev = torch.device("cuda:0")

    if args.copy_bytes:
        n = args.copy_bytes // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": 3}))
        return

    wl = W.dimer_fwdbwd_64k(args.n_traj, args.n_steps)
    cfg = wl.cfg.replace(ckpt_every=args.ckpt_every)
    net, B = wl.net, wl.n_traj
    nb, nob = cfg.n_bins, len(net.obs_species)
    h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
    theta = torch.tensor(net.theta0, device=dev)
    x0 = torch.tensor(wl.x0_soa().reshape(-1), device=dev)

    # targets: a seeded run at the target rates (separate stream purpose), untimed
    tcfg = cfg.replace(purpose=W.PURPOSE_TARGET)
    theta_t = torch.tensor(np.log(np.array(W.DIMER_TARGET_RATES)).astype(np.float32), device=dev)
    tf = ssa.forward(h, tcfg, theta_t, x0, keep_ckpt=False, tie_capacity=0)
    tm, tv = losses.bin_moments(tf.obs, nb, nob, B)
    tm, tv = tm.clone(), tv.clone()
    del tf

    bufs = ssa.forward(h, cfg, theta, x0, tie_capacity=1 << 16, bwd_mode=args.bwd_mode)
    d_params = torch.empty(net.n_params, dtype=torch.float32, device=dev)

    def step(record=None):
        if record is not None:
            record[0].record()
        ssa.forward(h, cfg, theta, x0, buffers=bufs, tie_capacity=1 << 16, bwd_mode=args.bwd_mode)
        if record is not None:
            record[1].record()
        obs = bufs.obs.detach().requires_grad_(True)
        loss = losses.moment_mse(obs, tm, tv, nb, nob, B)
        (d_obs,) = torch.autograd.grad(loss, obs)
        if record is not None:
            record[2].record()
        ssa.backward(h, cfg, theta, x0, bufs, d_obs, d_params=d_params)
        if record is not None:
            record[3].record()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        loss = step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fired = int(bufs.steps_done.sum().item())
    ms_step = (t1 - t0) * 1e3 / args.steps
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    loss_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    bwd_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    value = fired / (ms_step * 1e-3)

    # forward-only rate of the same forward call
    for _ in range(args.warmup):
        ssa.forward(h, cfg, theta, x0, buffers=bufs, tie_capacity=1 << 16, bwd_mode=args.bwd_mode)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    for _ in range(args.steps):
        ssa.forward(h, cfg, theta, x0, buffers=bufs, tie_capacity=1 << 16, bwd_mode=args.bwd_mode)
    torch.cuda.synchronize()
    f1 = time.perf_counter()
    fwd_rate = fired * args.steps / (f1 - f0)
    n_ties = int(bufs.n_ties.item())
    assert ssa.device_status(h) == 0

    # gradient relative error against the oracle on a sample of trajectories
    import oracle
    obs = bufs.obs.detach().requires_grad_(True)
    loss = losses.moment_mse(obs, tm, tv, nb, nob, B)
    (d_obs,) = torch.autograd.grad(loss, obs)
    _, ppt = ssa.backward(h, cfg, theta, x0, bufs, d_obs, per_traj=True)
    sample = np.arange(0, B, max(1, B // 64))[:64]
    dob = d_obs.cpu().numpy().reshape(nb, nob, B).transpose(2, 0, 1)[sample]
    ties = bufs.tie_records()
    idx = {int(q): k for k, q in enumerate(sample)}
    ov = [(idx[int(t["traj"])], int(t["step"]), int(t["kind"]), int(t["chosen"]))
          for t in ties if int(t["traj"]) in idx]
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=sample, ties=ov, d_obs=dob)
    g_gpu = ppt.cpu().numpy().reshape(net.n_params, B).T[sample].astype(np.float64)
    xf = bufs.x_final.cpu().numpy().reshape(net.n_species, B).T[sample]
    counts_exact = bool(np.array_equal(xf, r.x_final)) and int(r.n_bad.sum()) == 0
    grad_rel_err = float(np.linalg.norm(g_gpu.sum(0) - r.grad.sum(0)) / np.linalg.norm(r.grad.sum(0)))

    # roofline of the dominant kernel (ALU-bound: algorithmic VALU issue slots)
    nnz = int(np.count_nonzero(net.stoich))
    per_step_b = alu_slots_per_step(net.n_reactions, net.n_species, nnz, nob, True)
    per_step_f = alu_slots_per_step(net.n_reactions, net.n_species, nnz, nob, False)
    if bwd_ms >= fwd_ms:
        dom, dom_ms, slots = "bwd_lane_kernel", bwd_ms, per_step_b
    else:
        dom, dom_ms, slots = "fwd_lane_kernel", fwd_ms, per_step_f
    achieved = fired * slots / (dom_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                "unit": "Tslot/s", "frac": achieved / PEAK_LANE_SLOTS, "traffic": None,
                "slots_per_step": slots, "kernel_ms": dom_ms}

    cpu = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        n_try = 32
        c0 = time.perf_counter()
        oracle.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(n_try), d_obs=np.zeros((n_try, nb, nob)),
                   n_threads=threads)
        dt = time.perf_counter() - c0
        n_cpu = int(min(B, max(n_try, n_try * args.cpu_seconds / max(dt, 1e-3))))
        c0 = time.perf_counter()
        rc = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(n_cpu),
                        d_obs=np.zeros((n_cpu, nb, nob)), n_threads=threads)
        dt = time.perf_counter() - c0
        cpu = {"value": float(rc.steps_done.sum() / dt), "unit": "steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{n_cpu} of the {B} trajectories, full {cfg.n_steps} steps, forward+adjoint in FP64"}

    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "n_traj": B, "steps_per_traj": cfg.n_steps, "n_bins": nb,
                   "t_obs": cfg.t_obs, "temperature": cfg.temperature, "ckpt_every": cfg.ckpt_every,
                   "bwd_mode": args.bwd_mode},
        "forward_steps_per_s": fwd_rate, "fwdbwd_over_forward": value / fwd_rate,
        "fwd_ms": fwd_ms, "loss_ms": loss_ms, "bwd_ms": bwd_ms,
        "grad_rel_err": grad_rel_err, "counts_bit_exact_sample": counts_exact, "near_ties": n_ties,
        "loss": float(loss.item()), "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
