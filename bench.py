#!/usr/bin/env python3
"""Throughput of the batched exact SSA step, forward and forward+backward, on one MI355X.

Default workload: the activator-repressor oscillator (9 species, 16 mass-action
channels, 15 seeded rates), 65,536 trajectories x 200,000 steps each (1.31e10
fired reactions a pass), observation = exact bin averages of R over 256 bins,
loss = MSE of the ensemble-mean normalised autocorrelation of R at lags 1-64
against a run with a second seeded rate vector, Gumbel-Softmax temperature
0.5, checkpoints every 1,024 steps, gradients with respect to ln k.  The
reversible dimerisation 2A <-> A2 (65,536 x 10,000 steps, 20 bins, moment MSE)
is reported beside it under other_workloads.

Other workloads (--workload): the dimer alone, an uneven batch of 4,096 random
networks in one launch, the 784 -> 256 -> 10 gene-network classifier (512
images x 32 trajectories x 2,000 steps, cross-entropy on the final output
counts), the two rate-inference trainers and the selection-variant study.

One timed step = ssa_forward + loss (PyTorch FP64) + ssa_backward (+ the FP64
gradient reduction).  `value` counts fired reactions per second of that step;
the inputs are resident in HBM before timing starts.  Prints one JSON line.
"""
import argparse
import dataclasses
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
HBM_PEAK = 8.0e12                        # MI355X HBM3E, bytes/s


def alu_ops_per_step(net, backward: bool, inv_t_is_2=True, tangent: bool = False) -> dict:
    """Algorithmic vector-ALU operations of one step of one trajectory of a
    mass-action network, by kind: mad = 32x32->64-bit product, bit3 = the
    three-input bit operation (a ^ b ^ c), int = 32-bit integer
    add/logic/shift, fp32 = FP32 add/mul/FMA/compare/select, cvt =
    int<->float conversion, log / rcp = transcendentals, f64 = FP64 add or FMA.
    Propensity work follows each channel's order: a zero-order channel's
    propensity is its rate, a first-order one costs one product and has a
    constant partial derivative, a second-order one costs two products and
    two partials (a homodimer also forms X - 1)."""
    M, N = net.n_reactions, net.n_species
    n_obs = len(net.obs_species)
    r = np.asarray(net.reactant)
    order = (r >= 0).sum(axis=1)
    n1, n2 = int((order == 1).sum()), int((order == 2).sum())
    homo = int(((r[:, 0] >= 0) & (r[:, 0] == r[:, 1])).sum())
    factors = n1 + 2 * n2                           # reactant factors (int -> float)
    nnz = int(np.count_nonzero(net.stoich))
    nb = (M + 1 + 3) // 4
    w = M + 1                                        # Philox words used
    ops = {"mad": 20 * nb,                           # Philox4x32-10: two products a round
           "bit3": 20 * nb,                          # and two three-input xors (one instruction each)
           "int": 2 * w,                             # word -> odd 24-bit integer
           "cvt": w + factors, "fp32": 2 * w,        # lattice u = int * 2^-24, E = log2(u) * -ln 2
           "log": w, "rcp": 0, "f64": 0}
    ops["int"] += homo                               # X - 1 of homodimers
    ops["fp32"] += factors + (M - 1) + 1             # propensities, a0, tau
    ops["rcp"] += 1 + M                              # 1/a0, 1/a_j
    if not backward:
        ops["cvt"] += 1 + n_obs                      # clock, bin value
        ops["int"] += nnz                            # state update (select of the fired change vector)
        ops["fp32"] += M + 3 * M                     # r_j, race compare/min/select
        ops["f64"] += 1 + n_obs                      # clock, bin integral
        if tangent:
            # forward-mode tangents for every channel rate q: the soft sample
            # (rho, its power, the sum), then per q the propensity tangents
            # (one product per reactant factor and the diagonal), d a0, dz,
            # the weighted mean, dy, d tau; the state, clock and bin tangents
            ops["rcp"] += M + 1
            ops["fp32"] += M + (M if inv_t_is_2 else 3 * M) + M
            if not inv_t_is_2:
                ops["log"] += M
            ops["fp32"] += M * (factors + M + M + 2 * M + 2 * M + 2 * M + 2)
            ops["fp32"] += nnz * M
            ops["cvt"] += 2 * N * M + 2 * n_obs * M
            ops["f64"] += N * M + M + 2 * n_obs * M
        return ops
    ops["cvt"] += 1 + 2 * n_obs                      # clock, time-path and bin terms
    ops["int"] += nnz                                # reversed state update
    ops["rcp"] += M + 1                              # 1/r_j, 1/sum
    ops["fp32"] += (2 * n2                           # partials of second-order channels
                    + M + M + (M if inv_t_is_2 else 0) + M + M      # r_j, rho, rho^(1/T), sum, normalise
                    + nnz + 2 * M + 3 * M + 2 * M + M              # w, w - w_ref and wbar, g, dtheta, coef
                    + factors)                                      # lambda updates
    if not inv_t_is_2:
        ops["log"] += M
        ops["fp32"] += 3 * M
    ops["f64"] += 2 + 2 * n_obs                      # reversed clock, time path, direct terms
    return ops


def measure_issue_costs():
    """Issue cost of each operation kind in full-rate lane slots (one FP32 FMA
    per lane per clock on every CU), measured on this GPU by the
    instruction-throughput probes of libssa_ubench.so."""
    import ctypes as C
    L = C.CDLL(os.path.join(ROOT, "paper_2602_19775_amd", "libssa_ubench.so"))
    L.ubench_run.restype = C.c_float
    L.ubench_run.argtypes = [C.c_int, C.c_int, C.c_int]
    blocks, iters = 2048, 4096
    lanes = blocks * 256
    t = {}
    for kind in range(8):
        ms = L.ubench_run(kind, iters, blocks)
        if ms <= 0:
            raise RuntimeError("instruction probe failed")
        t[kind] = ms * 1e-3 * PEAK_LANE_SLOTS / (lanes * 8 * iters)   # slots per chain step
    i32 = t[4] / 2                  # xor + add
    f32 = t[3]                      # fma
    return {"int": i32, "fp32": f32, "mad": t[0] - i32, "log": t[1] - f32, "rcp": t[2] - f32,
            "cvt": t[6] - i32, "f64": t[5], "bit3": t[7] - i32}


def gpu_rounding_constant(T: float) -> float:
    """Rounding constant of the GPU's gradient against the oracle's
    conditioning kappa (the same as the parity tests use)."""
    return 32.0 + 32.0 / T


def grad_error_detail(g_gpu, r, t_gpu, cfg) -> dict:
    """Per-trajectory gradient error of a sample against the oracle: the
    distribution of ||g - g*|| / ||g*|| over the trajectories (with bins and
    no edge log, those whose event times stay clear of every bin edge by 50
    times the clock drift), and
    the worst component against the parity bar
    min(1e-5 ||g*||_inf, max(1e-5 |g*_i|, c(T) 2^-24 kappa_i))."""
    drift = float(np.max(np.abs(t_gpu - r.t_final))) if len(t_gpu) else 0.0
    keep = np.ones(len(t_gpu), bool)
    if cfg.obs_kind != 0 and not getattr(r, "edge_window", 0.0) > 0.0:
        keep = r.bin_edge_dist > 50.0 * max(drift, 1e-12)
    g, ref, kap = g_gpu[keep], r.grad[keep], r.kappa[keep]
    out = {"sampled": int(len(t_gpu)), "compared": int(keep.sum()), "clock_drift": drift}
    if not keep.any():
        return out
    nrm = np.linalg.norm(ref, axis=1)
    ok = nrm > 0
    rel = np.linalg.norm(g - ref, axis=1)[ok] / nrm[ok]
    err = np.abs(g - ref)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    bar = np.minimum(1e-5 * scale, np.maximum(1e-5 * np.abs(ref),
                                              gpu_rounding_constant(cfg.temperature) * 2.0 ** -24 * kap))
    out.update({"rel_err_median": float(np.median(rel)) if rel.size else 0.0,
                "rel_err_p90": float(np.percentile(rel, 90)) if rel.size else 0.0,
                "rel_err_max": float(rel.max()) if rel.size else 0.0,
                "worst_component_over_bar": float((err / np.where(bar > 0, bar, np.inf)).max()),
                "worst_err_over_u_kappa": float((err / np.where(kap > 0, 2.0 ** -24 * kap, np.inf)).max())})
    return out


def host_info() -> dict:
    """The host's CPUs: its count, this process's affinity, the thread share
    (OMP_NUM_THREADS) and the lscpu model name."""
    import subprocess
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    model = ""
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"os_cpu_count": os.cpu_count(), "affinity_cpus": aff,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "model": model}


def cpu_threads() -> int:
    """Threads the oracle leg may use: every CPU this process may run on,
    within the host's thread share (OMP_NUM_THREADS) when one is set."""
    info = host_info()
    n = info["affinity_cpus"]
    if info["omp_num_threads"]:
        try:
            n = min(n, int(info["omp_num_threads"]))
        except ValueError:
            pass
    return max(1, n)


def cpu_baseline(run, n_total: int, n_try: int, seconds: float, what: str) -> dict:
    """The oracle timed on the host: run(ids, threads) simulates the
    trajectories `ids` and returns their fired steps.  A short calibration
    sizes a sample of about `seconds` of work on all threads; a sample of n_try
    trajectories is also timed on one thread."""
    threads = cpu_threads()
    n_cal = min(n_total, max(n_try, 2 * threads))
    c0 = time.perf_counter()
    run(np.arange(n_cal), threads)
    dt = time.perf_counter() - c0
    n_cpu = int(min(n_total, max(n_cal, n_cal * seconds / max(dt, 1e-3))))
    c0 = time.perf_counter()
    steps = float(run(np.arange(n_cpu), threads))
    dt = time.perf_counter() - c0
    c1 = time.perf_counter()
    steps1 = float(run(np.arange(n_try), 1))
    dt1 = time.perf_counter() - c1
    return {"value": steps / dt, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_cpu} {what}", "seconds": dt,
            "value_1core": steps1 / dt1, "sample_1core": f"{n_try} {what}",
            "host": host_info()}


# Library sources each workload's kernels are built from.
_SPEC_SOURCES = ["ssa_spec_body.hpp", "ssa_device.hpp", "ssa_plan.hpp", "ssa_jit.cpp", "ssa_jit.hpp",
                 "ssa_misc.hip", "ssa_misc.hpp", "ssa_api.cpp"]
WORKLOAD_SOURCES = {
    "dimer": _SPEC_SOURCES, "oscillator": _SPEC_SOURCES, "abc_infer": _SPEC_SOURCES, "coi_infer": _SPEC_SOURCES,
    "uneven": ["ssa_wave.hip", "ssa_wave.hpp", "ssa_device.hpp", "ssa_plan.hpp", "ssa_misc.hip", "ssa_misc.hpp",
               "ssa_api.cpp"],
    "grn": ["ssa_grn.hip", "ssa_grn.hpp", "ssa_grn_api.cpp", "ssa_device.hpp", "ssa_plan.hpp"],
}


def sources_sha1(workload: str = None) -> str:
    """Digest of the library sources a workload's kernels are built from (all
    of them when no workload is named); the profile summaries record the one
    their counters were taken with."""
    import hashlib
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_2602_19775_amd", "csrc")
    files = WORKLOAD_SOURCES[workload] if workload else [
        f for f in os.listdir(d) if f.endswith((".hip", ".hpp", ".cpp", ".h"))]
    for f in sorted(files):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str, kernel: str):
    """HBM bytes per launch of a workload's forward or backward from the
    FETCH_SIZE / WRITE_SIZE passes summarised under profiles/, scaled by the
    copy calibration; None when no summary covers it or the library sources
    changed since the counters were taken."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    sha = sources_sha1(workload)
    for f in sorted(os.listdir(d)):
        if not f.endswith(".md"):
            continue
        with open(os.path.join(d, f)) as fh:
            for line in fh:
                p = line.split()
                if len(p) == 5 and p[0] == "traffic_bytes_per_launch" and p[1] == workload and p[2] == kernel:
                    return float(p[3]) if p[4] == f"sources={sha}" else None
    return None


def progress(what: str):
    """A line on stderr as each phase of a benchmark ends (the JSON line is the
    only stdout)."""
    print(f"[bench] {what}", file=sys.stderr, flush=True)


def forward_reps(steps: int, fwd_s: float) -> int:
    """Repetitions of the forward-only timing: the step count, raised so that
    the timed forwards last at least half a second (a short forward timed
    over a few launches is at the mercy of one late launch), at most 200."""
    if fwd_s <= 0.0:
        return steps
    return int(min(max(steps, int(np.ceil(0.5 / fwd_s))), max(steps, 200)))


def spread(ms) -> dict:
    """Median, minimum and maximum of per-step times (ms)."""
    a = np.asarray(ms, dtype=np.float64)
    return {"median": float(np.median(a)), "min": float(a.min()), "max": float(a.max())}


def slots(ops: dict, cost: dict) -> float:
    return sum(n * cost[k] for k, n in ops.items())


def alu_ops_per_step_grn(n_hid: int, n_out: int, backward: bool, hidden_frac: float) -> dict:
    """Algorithmic vector-ALU operations of one gene-network step of one
    trajectory (same kinds as alu_ops_per_step).  hidden_frac: share of the
    steps that change a hidden gene (each updates the n_out output
    pre-activations and their production rates)."""
    M = 2 * (n_hid + n_out)
    nb = (M + 1 + 3) // 4
    w = M + 1
    ops = {"mad": 20 * nb, "bit3": 20 * nb, "int": 2 * w, "cvt": w, "fp32": 2 * w, "log": w, "rcp": 0, "f64": 0}
    ops["cvt"] += n_hid + n_out                      # decay propensities delta * count
    ops["fp32"] += n_hid + n_out + M                 # their products, a0 sum
    # a hidden event: v_o += U_oh in FP64 and beta sigmoid(v_o) (FP64 range
    # reduction, exp2, reciprocal)
    ev = {"f64": 4 * n_out, "cvt": 2 * n_out, "log": n_out, "rcp": n_out, "fp32": 3 * n_out}
    for k, v in ev.items():
        ops[k] += hidden_frac * v
    if not backward:
        ops["rcp"] += M + 1                          # 1/a_j, 1/a0
        ops["fp32"] += M + 3 * M + 1                 # r_j, race compare/min/select, tau
        ops["f64"] += 1                              # clock
        ops["int"] += 1
        return ops
    ops["rcp"] += M + n_hid + n_out                  # 1/E_j, 1/count of the decay terms
    ops["fp32"] += (2 * M                            # rho = r_ref a_j / E_j
                    + 2 * M                          # sums of rho and rho (w_j - w_ref)
                    + M + 3 * M                      # w_j - w_ref, g_j
                    + 2 * n_hid + n_hid + 2 * n_out  # production/decay sums, decay adjoint, dL/dv
                    + n_hid * n_out)                 # lambda_H += sum_o dL/dv_o U_oh
    ops["cvt"] += n_hid + n_out
    ops["f64"] += n_hid + 2 * n_out + hidden_frac * n_out   # lambda, dL/dc, dU on hidden events
    ops["int"] += 1
    return ops


def bench_grn(args, torch, dev):
    """Gene-network classifier: ssa_grn_forward (bf16 MFMA contraction +
    simulation) + cross-entropy (PyTorch FP64) + ssa_grn_backward (adjoint,
    FP64 reductions, dW on FP64 MFMA)."""
    from paper_2602_19775_amd import losses, ssa
    from paper_2602_19775_amd import workloads as W
    import oracle

    wl = W.grn_classifier(n_steps=args.n_steps or 2000)
    net, cfg = wl.net, wl.cfg
    g = ssa.Grn(net, wl.n_images, wl.n_rep)
    theta = torch.tensor(wl.theta, device=dev)
    x_img = torch.tensor(wl.images, device=dev)
    labels = torch.tensor(wl.labels, device=dev)[torch.arange(wl.n_traj, device=dev) // wl.n_rep]
    tie_cap = 1 << 20
    bufs = ssa.grn_forward(g, cfg, theta, x_img, tie_capacity=tie_cap)
    d_params = torch.empty(net.n_params, dtype=torch.float32, device=dev)
    _, wb = ssa.grn_buffer_sizes(g, bufs.ccfg)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)

    def step(record=None):
        if record is not None:
            record[0].record()
        ssa.grn_forward(g, cfg, theta, x_img, tie_capacity=tie_cap, buffers=bufs)
        if record is not None:
            record[1].record()
        obs = bufs.obs.detach().requires_grad_(True)
        loss = losses.count_cross_entropy(obs, labels)
        (d_obs,) = torch.autograd.grad(loss, obs)
        if record is not None:
            record[2].record()
        ssa.grn_backward(g, cfg, theta, x_img, bufs, d_obs, d_params=d_params, work=work)
        if record is not None:
            record[3].record()
        return loss

    for _ in range(args.warmup):
        step()
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
    step_stats = spread([e[0].elapsed_time(e[3]) for e in evs])
    value = fired / (ms_step * 1e-3)

    # forward-only rate of the plain forward (no choice tape)
    pbufs = ssa.grn_forward(g, cfg, theta, x_img, keep_tape=False, tie_capacity=tie_cap)
    for _ in range(args.warmup):
        ssa.grn_forward(g, cfg, theta, x_img, tie_capacity=tie_cap, buffers=pbufs)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    ssa.grn_forward(g, cfg, theta, x_img, tie_capacity=tie_cap, buffers=pbufs)
    torch.cuda.synchronize()
    n_fo = forward_reps(args.steps, time.perf_counter() - p0)
    fevs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n_fo)]
    f0 = time.perf_counter()
    for k in range(n_fo):
        fevs[k][0].record()
        ssa.grn_forward(g, cfg, theta, x_img, tie_capacity=tie_cap, buffers=pbufs)
        fevs[k][1].record()
    torch.cuda.synchronize()
    f1 = time.perf_counter()
    fwd_rate = int(pbufs.steps_done.sum().item()) * n_fo / (f1 - f0)
    fwd_only_stats = spread([e[0].elapsed_time(e[1]) for e in fevs])
    del pbufs

    n_ties = int(bufs.n_ties.item())
    assert ssa.grn_device_status(g) == 0

    graph = None
    if not args.no_graph:
        from paper_2602_19775_amd.graph import CapturedStep
        ep = torch.zeros(1, dtype=torch.int32, device=dev)
        gbufs = ssa.grn_forward(g, cfg, theta, x_img, tie_capacity=0, d_epoch=ep)
        gdp = torch.empty_like(d_params)
        gwork = torch.empty_like(work)

        def gstep():
            ssa.grn_forward(g, cfg, theta, x_img, tie_capacity=0, d_epoch=ep, buffers=gbufs)
            gobs = gbufs.obs.detach().requires_grad_(True)
            (gd,) = torch.autograd.grad(losses.count_cross_entropy(gobs, labels), gobs)
            ssa.grn_backward(g, cfg, theta, x_img, gbufs, gd, d_params=gdp, work=gwork)
            ep.add_(1)
        cap = CapturedStep(gstep, warmup=args.warmup)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.steps):
            cap.replay()
        torch.cuda.synchronize()
        g1 = time.perf_counter()
        graph = {"steps_per_s": fired * args.steps / (g1 - g0), "ms_per_step": (g1 - g0) * 1e3 / args.steps}
        del cap, gbufs, gwork

    # gradient relative error on a sample of trajectories: the oracle runs on
    # the GPU's hidden pre-activations (the bf16 contraction is checked on its
    # own by the parity tests)
    obs = bufs.obs.detach().requires_grad_(True)
    loss = losses.count_cross_entropy(obs, labels)
    (d_obs,) = torch.autograd.grad(loss, obs)
    _, comp = ssa.grn_backward(g, cfg, theta, x_img, bufs, d_obs, per_traj=True, work=work)
    sample = np.arange(0, wl.n_traj, wl.n_traj // 32)[:32]
    ties = bufs.tie_records()
    idx = {int(q): k for k, q in enumerate(sample)}
    ov = [(idx[int(t["traj"])], int(t["step"]), int(t["kind"]), int(t["chosen"]))
          for t in ties if int(t["traj"]) in idx]
    u_gpu = bufs.u_hid.cpu().numpy().astype(np.float64)
    dnp = d_obs.cpu().numpy().T[sample]
    r = oracle.grn_run(net, cfg, wl.theta, u_gpu, sample // wl.n_rep, traj_ids=sample, ties=ov, d_obs=dnp,
                       tie_threshold=2e-6)
    cg = comp[torch.from_numpy(sample).to(dev)].cpu().numpy()
    xf = bufs.x_final.cpu().numpy().T[sample]
    counts_exact = bool(np.array_equal(xf, r.x_final)) and int(r.n_bad.sum()) == 0
    grad_rel_err = float(np.linalg.norm(cg.sum(0) - r.grad_c.sum(0)) / np.linalg.norm(r.grad_c.sum(0)))
    # share of steps that change a hidden gene, from the oracle's traces
    hid = []
    for q in sample[:4]:
        jk, _ = oracle.grn_trace(net, cfg, wl.theta, u_gpu[q // wl.n_rep], traj_id=int(q), cap=cfg.n_steps)
        hid.append(np.mean(jk < 2 * net.n_hid))
    hidden_frac = float(np.mean(hid))

    cost = measure_issue_costs()
    ops_f = alu_ops_per_step_grn(net.n_hid, net.n_out, False, hidden_frac)
    ops_b = alu_ops_per_step_grn(net.n_hid, net.n_out, True, hidden_frac)
    dom, dom_ms, ops = ("backward", bwd_ms, ops_b) if bwd_ms >= fwd_ms else ("forward", fwd_ms, ops_f)
    per_step = slots(ops, cost)
    achieved = fired * per_step / (dom_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                "unit": "Tslot/s", "frac": achieved / PEAK_LANE_SLOTS, "traffic": profiled_traffic("grn", dom),
                "slots_per_step": per_step, "ops_per_step": ops, "issue_cost_slots": cost,
                "kernel_ms": dom_ms, "hidden_event_share": hidden_frac,
                "fwd_frac": fired * slots(ops_f, cost) / (fwd_ms * 1e-3) / PEAK_LANE_SLOTS}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(
            lambda ids, threads: oracle.grn_run(net, cfg, wl.theta, u_gpu, ids // wl.n_rep, traj_ids=ids,
                                                d_obs=np.zeros((len(ids), net.n_out)),
                                                n_threads=threads).steps_done.sum(),
            wl.n_traj, 32, args.cpu_seconds,
            f"of the {wl.n_traj} trajectories, full {cfg.n_steps} steps, "
            "forward+adjoint in FP64 on the GPU's hidden pre-activations")

    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "n_traj": wl.n_traj, "n_images": wl.n_images, "n_rep": wl.n_rep,
                   "steps_per_traj": cfg.n_steps, "n_params": net.n_params, "temperature": cfg.temperature},
        "forward_steps_per_s": fwd_rate, "fwdbwd_over_forward": value / fwd_rate, "graph_replay": graph,
        "fwd_ms": fwd_ms, "loss_ms": loss_ms, "bwd_ms": bwd_ms,
        "step_ms": step_stats, "forward_only_ms": fwd_only_stats, "forward_only_reps": n_fo,
        "grad_rel_err": grad_rel_err, "counts_bit_exact_sample": counts_exact, "near_ties": n_ties,
        "loss": float(loss.item()), "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def bench_infer(args, torch, dev):
    """Rate inference for A + B <-> C: 250 epochs of one captured optimisation
    step (forward with the grid observation, loss gradient, backward, RMSprop
    update) over 100,000 trajectories x 250 steps, from the paper's starting
    guess; value = fired steps of the replayed epochs / their wall time."""
    from paper_2602_19775_amd import infer, ssa
    from paper_2602_19775_amd import workloads as W
    import oracle

    coi = args.workload == "coi_infer"
    ep = {"epochs": args.epochs} if args.epochs else {}
    if coi:
        n_traj = args.n_traj if args.n_traj != 65536 else 262_144
        n_steps = args.n_steps or 20
        tr = infer.ion_channel(n_traj=n_traj, n_target=n_traj, n_steps=n_steps, **ep)
        k_start = infer.COI_START
    else:
        n_traj = args.n_traj if args.n_traj != 65536 else 100_000
        n_steps = args.n_steps or 250
        tr = infer.dimerization(infer.TRUE_RATES, n_traj=n_traj, n_target=n_traj, n_steps=n_steps, **ep)
        k_start = infer.START_RATES
    tr.capture()
    res = tr.run()
    value = res.steps_per_epoch * res.epochs / res.train_s

    # kernel times of one step at the learned rates and the final temperature
    T_end = float(tr.temp.item()) / tr.r_temp      # the temperature of the last epoch
    cfg = tr.cfg.replace(temperature=T_end, epoch=res.epochs)
    bufs = ssa.forward(tr.h, cfg, tr.theta, tr.x0, tie_capacity=1 << 16)
    G, O, B = tr.n_pts, tr.n_obs, tr.B
    NS, NP = tr.net.n_species, tr.net.n_params
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    d_obs = torch.zeros(G * O, dtype=torch.float64, device=dev)      # shared by the trajectories
    for k in range(args.warmup + args.steps):
        e = evs[k - args.warmup] if k >= args.warmup else None
        if e:
            e[0].record()
        ssa.forward(tr.h, cfg, tr.theta, tr.x0, buffers=bufs, tie_capacity=1 << 16)
        if e:
            e[1].record()
        tr.d_obs_of(tr.means(bufs) - tr.target, d_obs)
        if e:
            e[2].record()
        ssa.backward(tr.h, cfg, tr.theta, tr.x0, bufs, d_obs, d_params=tr.d_params)
        if e:
            e[3].record()
    torch.cuda.synchronize()
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    loss_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    bwd_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    fired = int(bufs.steps_done.sum().item())
    pb = ssa.forward(tr.h, cfg, tr.theta, tr.x0, keep_ckpt=False, tie_capacity=0)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    for _ in range(args.steps):
        ssa.forward(tr.h, cfg, tr.theta, tr.x0, buffers=pb, tie_capacity=0)
    torch.cuda.synchronize()
    fwd_rate = int(pb.steps_done.sum().item()) * args.steps / (time.perf_counter() - f0)

    # parity sample: per-trajectory gradients at the learned rates against the
    # oracle, at temperatures across the annealing schedule (the FP32 soft
    # weights carry a relative error of about 1e-7 / T)
    n_sample = 32
    sample = np.arange(0, B, B // n_sample)[:n_sample]
    th = tr.theta.cpu().numpy()
    dnp = np.broadcast_to(d_obs.cpu().numpy().reshape(1, G, O), (len(sample), G, O)).copy()
    idx = {int(q): k for k, q in enumerate(sample)}
    err_by_T = {}
    counts_exact = True
    for T in sorted({1.0, 0.1, 0.01, round(tr.temp0, 9), round(T_end, 9)}, reverse=True):
        c2 = cfg.replace(temperature=float(T))
        b2 = ssa.forward(tr.h, c2, tr.theta, tr.x0, tie_capacity=1 << 16)
        _, ppt = ssa.backward(tr.h, c2, tr.theta, tr.x0, b2, d_obs, per_traj=True)
        ov = [(idx[int(t["traj"])], int(t["step"]), int(t["kind"]), int(t["chosen"]))
              for t in b2.tie_records() if int(t["traj"]) in idx]
        r = oracle.run(tr.net, c2, th, tr.net.x0, traj_ids=sample, ties=ov, d_obs=dnp)
        g_gpu = ppt.cpu().numpy().reshape(NP, B).T[sample].astype(np.float64)
        xf = b2.x_final.cpu().numpy().reshape(NS, B).T[sample]
        counts_exact = counts_exact and bool(np.array_equal(xf, r.x_final)) and int(r.n_bad.sum()) == 0
        err_by_T[f"{T:.3g}"] = float(np.linalg.norm(g_gpu.sum(0) - r.grad.sum(0)) / np.linalg.norm(r.grad.sum(0)))
    grad_rel_err = max(err_by_T.values())

    cost = measure_issue_costs()
    inv2 = abs(1.0 / T_end - 2.0) < 1e-12
    ops_f, ops_b = alu_ops_per_step(tr.net, False, inv2), alu_ops_per_step(tr.net, True, inv2)
    dom, dom_ms, ops = ("backward", bwd_ms, ops_b) if bwd_ms >= fwd_ms else ("forward", fwd_ms, ops_f)
    # algorithmic HBM bytes of one launch: the observation buffer (written by
    # the forward, or its tiles' sums; the backward reads the shared dL/dobs
    # block only), the checkpoints and tape (written, then read), the
    # per-trajectory state and clock
    io = bufs.x_final.numel() * 4 * 2 + B * (8 + 4)
    ck = bufs.ckpt.numel() if bufs.ckpt is not None else 0
    ens = tr.cfg.obs_layout == W.OBS_ENSEMBLE_MEAN       # the forward stores one row of sums a 64-trajectory tile
    obs_bytes = -(-B // 64) * G * O * 8 if ens else G * O * B * 8
    alg_bytes = (obs_bytes if dom == "forward" else 0) + ck + io
    alu_s = fired * slots(ops, cost) / PEAK_LANE_SLOTS
    if alg_bytes / HBM_PEAK > alu_s:
        achieved = alg_bytes / (dom_ms * 1e-3)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK, "algorithmic_bytes": alg_bytes}
    else:
        achieved = fired * slots(ops, cost) / (dom_ms * 1e-3)
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                    "unit": "Tslot/s", "frac": achieved / PEAK_LANE_SLOTS, "algorithmic_bytes": alg_bytes}
    roofline.update({"traffic": profiled_traffic(args.workload, dom), "kernel_ms": dom_ms,
                     "fwd_frac": fired * slots(ops_f, cost) / (fwd_ms * 1e-3) / PEAK_LANE_SLOTS})
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(
            lambda ids, threads: oracle.run(tr.net, cfg, th, tr.net.x0, traj_ids=ids,
                                            d_obs=np.zeros((len(ids), G, O)), n_threads=threads).steps_done.sum(),
            B, 2048, args.cpu_seconds, f"of the {B} trajectories, {n_steps} steps, forward+adjoint in FP64")
    sweep = None
    if args.sweep and not coi:
        sweep = []
        for k2 in infer.K2_SWEEP:
            rr = infer.infer((infer.TRUE_RATES[0], k2), n_traj=n_traj, n_target=n_traj, n_steps=n_steps)
            sweep.append({"k_true": rr.k_true.tolist(), "k_learned": rr.k_learned.tolist(),
                          "ape_percent": rr.ape.tolist(), "loss_first": rr.loss_first, "loss_last": rr.loss_last})
    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": res.epochs,
        "warmup": 2, "ms_per_step": res.train_s * 1e3 / res.epochs, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"ion_channel_inference_{B}traj_{n_steps}steps_{G}bins_{res.epochs}epochs" if coi
                                else f"abc_inference_{B}traj_{n_steps}steps_{G}grid_{res.epochs}epochs"),
                   "n_traj": B, "steps_per_traj": n_steps, "n_obs_points": G, "t_obs": tr.t_obs,
                   "epochs": res.epochs, "temperature": [tr.temp0, T_end], "optimizer": "rmsprop"},
        "forward_steps_per_s": fwd_rate, "fwdbwd_over_forward": value / fwd_rate,
        "fwd_ms": fwd_ms, "bwd_ms": bwd_ms, "loss_ms": loss_ms, "grad_rel_err": grad_rel_err,
        "grad_rel_err_by_T": err_by_T,
        "counts_bit_exact_sample": counts_exact,
        "inference": {"k_true": res.k_true.tolist(), "k_start": list(k_start),
                      "k_learned": res.k_learned.tolist(), "ape_percent": res.ape.tolist(),
                      "loss_first": res.loss_first, "loss_last": res.loss_last, "train_s": res.train_s},
        "sweep": sweep, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def bench_selection(args, torch, dev):
    """Selection-variant study (the paper's standard Gillespie / Gumbel-Max /
    Gumbel-Softmax comparison): on the dimer and oscillator workloads, the
    plain forward with the inverse-CDF draw (one uniform for the channel), the
    plain forward with the Gumbel-max race (M uniforms), and one
    straight-through training step (Gumbel-max forward keeping its tape and
    checkpoints, then the Gumbel-Softmax backward).  Forward parity of the
    inverse-CDF runs is checked on a sample against the oracle."""
    from paper_2602_19775_amd import ssa
    from paper_2602_19775_amd import workloads as W
    import oracle

    rows = []
    for name, wl in (("dimer", W.dimer_fwdbwd_64k()), ("oscillator", W.oscillator_fwdbwd_64k(n_steps=args.n_steps or 200000))):
        net, B, cfg = wl.net, wl.n_traj, wl.cfg
        h = ssa.Net([net], [B], t_obs=[cfg.t_obs])
        th = torch.tensor(net.theta0, device=dev)
        x0 = torch.tensor(wl.x0_soa().reshape(-1), device=dev)
        row = {"workload": wl.name}

        def timed(fn, n):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(n):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / n

        n_rep = args.steps if name == "dimer" else max(1, args.steps // 5)
        for label, sel in (("inverse_cdf", W.SELECT_INVERSE_CDF), ("gumbel_max", W.SELECT_GUMBEL_MAX)):
            c = cfg.replace(selection=sel)
            # the oscillator's 256 bins log about 1.2e6 bin-edge events besides its near-ties
            b = ssa.forward(h, c, th, x0, keep_ckpt=False, tie_capacity=1 << 22)
            dt = timed(lambda: ssa.forward(h, c, th, x0, keep_ckpt=False, tie_capacity=1 << 22, buffers=b), n_rep)
            fired = int(b.steps_done.sum().item())
            row[label + "_forward_steps_per_s"] = fired / dt
            if sel == W.SELECT_INVERSE_CDF:
                sample = np.arange(0, B, B // 16)[:16]
                idx = {int(q): k for k, q in enumerate(sample)}
                ov = [(idx[int(t["traj"])], int(t["step"]), int(t["kind"]), int(t["chosen"]))
                      for t in b.tie_records() if int(t["traj"]) in idx]
                r = oracle.run(net, c, net.theta0, net.x0, traj_ids=sample, ties=ov)
                xf = b.x_final.cpu().numpy().reshape(net.n_species, B).T[sample]
                row["inverse_cdf_counts_bit_exact_sample"] = bool(np.array_equal(xf, r.x_final)) and int(r.n_bad.sum()) == 0
        bufs = ssa.forward(h, cfg, th, x0, tie_capacity=0)
        d_obs = torch.randn(bufs.obs.numel(), dtype=torch.float64, device=dev)
        d_params = torch.empty(h.param_total, dtype=torch.float32, device=dev)

        def st_step():
            ssa.forward(h, cfg, th, x0, buffers=bufs, tie_capacity=0)
            ssa.backward(h, cfg, th, x0, bufs, d_obs, d_params=d_params)
        dt = timed(st_step, n_rep)
        row["gumbel_softmax_st_fwdbwd_steps_per_s"] = int(bufs.steps_done.sum().item()) / dt
        rows.append(row)
    out = {"metric": METRIC, "study": "selection variants", "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "rows": rows}
    print(json.dumps(out))


def bench_mass_action(args, torch, dev, workload: str, light: bool = False) -> dict:
    """One timed step = ssa_forward + loss (PyTorch FP64) + ssa_backward for the
    dimer, oscillator or uneven-batch workload; returns the JSON record.
    light: no autotuning, graph replay or CPU baseline (a secondary line)."""
    from paper_2602_19775_amd import losses, ssa
    from paper_2602_19775_amd import workloads as W

    if workload in ("dimer", "oscillator"):
        if workload == "dimer":
            wl = W.dimer_fwdbwd_64k(args.n_traj, args.n_steps or 10000)
        else:
            wl = W.oscillator_fwdbwd_64k(args.n_traj, args.n_steps or 200000)
        cfg = wl.cfg.replace(ckpt_every=args.ckpt_every or wl.cfg.ckpt_every)
        nets, Bs, name = [wl.net], [wl.n_traj], wl.name
        h = ssa.Net(nets, Bs, t_obs=[cfg.t_obs])
        theta = torch.tensor(wl.net.theta0, device=dev)
        x0 = torch.tensor(wl.x0_soa().reshape(-1), device=dev)
        if workload == "dimer":
            theta_t = torch.tensor(np.log(np.array(W.DIMER_TARGET_RATES)).astype(np.float32), device=dev)
        else:
            theta_t = torch.tensor(wl.extra["target_net"].theta0, device=dev)
    else:
        bw = W.uneven_batch(n_steps=args.n_steps or 5000)
        # cfg.t_obs is the first network's window (the oracle's sample is drawn
        # from it); every network observes its own window
        cfg = bw.cfg.replace(ckpt_every=args.ckpt_every or bw.cfg.ckpt_every,
                             t_obs=bw.t_obs[0] if bw.t_obs else 0.0)
        nets, Bs, name = bw.nets, bw.n_traj, bw.name
        h = ssa.Net(nets, Bs, t_obs=bw.t_obs)
        theta = torch.tensor(bw.theta(), device=dev)
        x0 = torch.tensor(bw.x0_packed(), device=dev)
        theta_t = torch.tensor(np.concatenate([n.theta0 for n in bw.target_nets]), device=dev)
    plan = None
    bwd_mode = args.bwd_mode
    if bwd_mode == "auto":
        bwd_mode = "tangent" if workload == "dimer" else "tape"
    autotune_on = args.autotune if args.autotune is not None else workload == "uneven"
    if autotune_on and not light:
        from paper_2602_19775_amd import autotune
        t_obs_l = (bw.t_obs if workload == "uneven" else [cfg.t_obs] * len(nets)) \
            if cfg.obs_kind == W.OBS_BINS else None
        tune_log = []

        def tune_line(line):
            tune_log.append(line)
            progress("autotune " + line)
        plan = autotune.tune(nets, Bs, cfg, theta, x0, t_obs_l, log=tune_line)
        if not tune_log:
            progress("autotune: cached plan " + plan.name)
        h = plan.net(nets, Bs, t_obs_l)
        cfg = plan.config(cfg)
        bwd_mode = plan.bwd_mode
    net, B = nets[0], Bs[0]
    nb, nob = cfg.n_bins, len(net.obs_species)

    # targets: a seeded run at the target rates (separate stream purpose), untimed
    tcfg = cfg.replace(purpose=W.PURPOSE_TARGET)
    tf = ssa.forward(h, tcfg, theta_t, x0, keep_ckpt=False, tie_capacity=0)
    if workload == "dimer":
        tm, tv = losses.bin_moments(tf.obs, nb, nob, B)
        tm, tv = tm.clone(), tv.clone()

        def loss_fn(obs):
            return losses.moment_mse(obs, tm, tv, nb, nob, B)
    elif workload == "oscillator":
        tac = losses.mean_autocorrelation(tf.obs, nb, B, 64).clone()

        def loss_fn(obs):
            return losses.autocorrelation_mse(obs, tac, nb, B, 64)
    else:
        # per network [n_bins][n_obs][256] (or [n_obs][256] for final counts):
        # the ensemble mean of every observed species in every bin
        rows = sum(len(n.obs_species) for n in nets) * (nb if cfg.obs_kind == W.OBS_BINS else 1)
        tmean = tf.obs[: rows * B].view(rows, B).mean(dim=1).clone()

        def loss_fn(obs):
            return ((obs[: rows * B].view(rows, B).mean(dim=1) - tmean) ** 2).mean()
    del tf

    tie_cap = {"dimer": 1 << 16, "oscillator": 1 << 22, "uneven": 1 << 23}[workload]
    bufs = ssa.forward(h, cfg, theta, x0, tie_capacity=tie_cap, bwd_mode=bwd_mode)
    d_params = torch.empty(h.param_total, dtype=torch.float32, device=dev)

    def step(record=None):
        if record is not None:
            record[0].record()
        ssa.forward(h, cfg, theta, x0, buffers=bufs, tie_capacity=tie_cap, bwd_mode=bwd_mode)
        if record is not None:
            record[1].record()
        obs = bufs.obs.detach().requires_grad_(True)
        loss = loss_fn(obs)
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
    progress(f"{workload}: {args.warmup} warm-up steps done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        loss = step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fired = int(bufs.steps_done.sum().item())
    ms_step = (t1 - t0) * 1e3 / args.steps
    progress(f"{workload}: {args.steps} timed steps, {ms_step:.1f} ms each")
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    loss_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    bwd_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    step_stats = spread([e[0].elapsed_time(e[3]) for e in evs])
    value = fired / (ms_step * 1e-3)

    # forward-only rate of the plain forward (no checkpoints, no choice tape)
    pbufs = ssa.forward(h, cfg, theta, x0, keep_ckpt=False, tie_capacity=tie_cap, bwd_mode=bwd_mode)
    for _ in range(args.warmup):
        ssa.forward(h, cfg, theta, x0, buffers=pbufs, tie_capacity=tie_cap, bwd_mode=bwd_mode)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    ssa.forward(h, cfg, theta, x0, buffers=pbufs, tie_capacity=tie_cap, bwd_mode=bwd_mode)
    torch.cuda.synchronize()
    n_fo = forward_reps(args.steps, time.perf_counter() - p0)
    fevs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n_fo)]
    f0 = time.perf_counter()
    for k in range(n_fo):
        fevs[k][0].record()
        ssa.forward(h, cfg, theta, x0, buffers=pbufs, tie_capacity=tie_cap, bwd_mode=bwd_mode)
        fevs[k][1].record()
    torch.cuda.synchronize()
    f1 = time.perf_counter()
    fwd_rate = int(pbufs.steps_done.sum().item()) * n_fo / (f1 - f0)
    fwd_only_stats = spread([e[0].elapsed_time(e[1]) for e in fevs])
    del pbufs
    progress(f"{workload}: forward-only steps done")

    # the uneven batch as one persistent launch for every network (each then
    # runs on the lane-group class of the largest), beside the tuned plan
    one_launch = None
    if workload == "uneven" and not light and args.one_launch_steps > 0 and getattr(h, "wave_split", -1) != 0:
        h1 = ssa.Net(nets, Bs, t_obs=bw.t_obs, exec_mode="wave", wave_split=0)
        b1 = ssa.forward(h1, cfg, theta, x0, tie_capacity=0, bwd_mode=bwd_mode)
        dp1 = torch.empty_like(d_params)

        def step1():
            ssa.forward(h1, cfg, theta, x0, buffers=b1, tie_capacity=0, bwd_mode=bwd_mode)
            o1 = b1.obs.detach().requires_grad_(True)
            (g1,) = torch.autograd.grad(loss_fn(o1), o1)
            ssa.backward(h1, cfg, theta, x0, b1, g1, d_params=dp1)
        step1()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(args.one_launch_steps):
            step1()
        torch.cuda.synchronize()
        ms1 = (time.perf_counter() - s0) * 1e3 / args.one_launch_steps
        ref = d_params.double()
        one_launch = {"steps_per_s": int(b1.steps_done.sum().item()) / (ms1 * 1e-3), "ms_per_step": ms1,
                      "steps": args.one_launch_steps,
                      "counts_equal_tuned_plan": bool(torch.equal(b1.x_final, bufs.x_final)),
                      "grad_max_diff_over_max": float((dp1.double() - ref).abs().max() / ref.abs().max())}
        assert ssa.device_status(h1) == 0
        del b1, h1, dp1
        progress(f"{workload}: one-launch steps done, {ms1:.1f} ms each")
    n_ties = int(bufs.n_ties.item())
    assert ssa.device_status(h) == 0
    kinds = bufs.tie_records()["kind"]
    n_edge = int((kinds == 2).sum())

    # the same step captured into one HIP graph (the epoch advances on the
    # device, so every replay draws a fresh stream), replayed
    graph = None
    if not args.no_graph and not light:
        from paper_2602_19775_amd.graph import CapturedStep
        ep = torch.zeros(1, dtype=torch.int32, device=dev)
        gbufs = ssa.forward(h, cfg, theta, x0, tie_capacity=0, bwd_mode=bwd_mode, d_epoch=ep)
        gdp = torch.empty_like(d_params)

        def gstep():
            ssa.forward(h, cfg, theta, x0, buffers=gbufs, tie_capacity=0, bwd_mode=bwd_mode, d_epoch=ep)
            gobs = gbufs.obs.detach().requires_grad_(True)
            (gd,) = torch.autograd.grad(loss_fn(gobs), gobs)
            ssa.backward(h, cfg, theta, x0, gbufs, gd, d_params=gdp)
            ep.add_(1)
        cap = CapturedStep(gstep, warmup=args.warmup)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.steps):
            cap.replay()
        torch.cuda.synchronize()
        g1 = time.perf_counter()
        gfired = int(gbufs.steps_done.sum().item())
        graph = {"steps_per_s": gfired * args.steps / (g1 - g0), "ms_per_step": (g1 - g0) * 1e3 / args.steps}
        del cap, gbufs
        progress(f"{workload}: graph replays done")

    # gradient error against the oracle on a sample of trajectories (of the
    # first network of the batch): per-trajectory and summed, with the
    # oracle's conditioning of every component
    import oracle
    obs = bufs.obs.detach().requires_grad_(True)
    loss = loss_fn(obs)
    (d_obs,) = torch.autograd.grad(loss, obs)
    _, ppt = ssa.backward(h, cfg, theta, x0, bufs, d_obs, per_traj=True)
    n_sample = {"dimer": 64, "oscillator": 64, "uneven": 64}[workload]
    sample = np.arange(0, B, max(1, B // n_sample))[:n_sample]
    bins = cfg.obs_kind == W.OBS_BINS
    dnp = d_obs.cpu().numpy()
    dob = (dnp[: nb * nob * B].reshape(nb, nob, B).transpose(2, 0, 1)[sample] if bins
           else dnp[: nob * B].reshape(nob, B).T[sample])
    ties = bufs.tie_records()
    idx = {int(q): k for k, q in enumerate(sample)}
    ov = [(idx[int(t["traj"])], int(t["step"]), int(t["kind"]), int(t["chosen"]))
          for t in ties if int(t["traj"]) in idx]
    # bins in the specialised mode: the forward logs the side of every bin edge an
    # event time falls close to, and the oracle takes it (EDGE_WINDOW of the tests)
    ew = 4e-7 if bins else 0.0
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=sample, ties=ov, d_obs=dob, kappa=True, edge_window=ew)
    r.edge_window = ew
    g_gpu = ppt.cpu().numpy()[: net.n_params * B].reshape(net.n_params, B).T[sample].astype(np.float64)
    xf = bufs.x_final.cpu().numpy()[: net.n_species * B].reshape(net.n_species, B).T[sample]
    counts_exact = bool(np.array_equal(xf, r.x_final)) and int(r.n_bad.sum()) == 0
    grad_rel_err = float(np.linalg.norm(g_gpu.sum(0) - r.grad.sum(0)) / np.linalg.norm(r.grad.sum(0)))
    grad_detail = grad_error_detail(g_gpu, r, bufs.t_final.cpu().numpy()[sample], cfg)
    progress(f"{workload}: oracle sample compared")

    # roofline of the dominant kernel (ALU-bound): algorithmic operations of a
    # launch weighted by their measured issue cost, over the kernel's time,
    # against the full-rate issue limit of the vector ALUs
    inv2 = abs(1.0 / cfg.temperature - 2.0) < 1e-12
    cost = measure_issue_costs()
    wsum = float(sum(Bs))

    tangent = bwd_mode == "tangent"

    def avg_ops(backward):
        tot = {}
        for n_, b_ in zip(nets, Bs):
            o = alu_ops_per_step(n_, backward, inv2, tangent=tangent and not backward)
            for k_, v_ in o.items():
                tot[k_] = tot.get(k_, 0.0) + v_ * b_ / wsum
        return tot
    ops_b, ops_f = avg_ops(True), avg_ops(False)
    if bwd_ms >= fwd_ms:
        dom, dom_ms, ops = "backward", bwd_ms, ops_b
    else:
        dom, dom_ms, ops = "forward", fwd_ms, ops_f
    per_step = slots(ops, cost)
    achieved = fired * per_step / (dom_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": PEAK_LANE_SLOTS / 1e12,
                "unit": "Tslot/s", "frac": achieved / PEAK_LANE_SLOTS, "traffic": profiled_traffic(workload, dom),
                "slots_per_step": per_step, "ops_per_step": ops, "issue_cost_slots": cost,
                "kernel_ms": dom_ms,
                "fwd_frac": fired * slots(ops_f, cost) / (fwd_ms * 1e-3) / PEAK_LANE_SLOTS}

    cpu = None
    if not args.no_cpu_baseline and not light:
        zero = (lambda n: np.zeros((n, nb, nob))) if bins else (lambda n: np.zeros((n, nob)))
        cpu = cpu_baseline(
            lambda ids, threads: oracle.run(net, cfg, net.theta0, net.x0, traj_ids=ids, d_obs=zero(len(ids)),
                                            n_threads=threads).steps_done.sum(),
            B, {"dimer": 32, "oscillator": 4, "uneven": 16}[workload], args.cpu_seconds,
            f"of the {B} trajectories, full {cfg.n_steps} steps, forward+adjoint in FP64")

    return {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "n_traj": int(sum(Bs)), "n_networks": len(nets), "steps_per_traj": cfg.n_steps, "n_bins": nb,
                   "t_obs": cfg.t_obs, "temperature": cfg.temperature, "ckpt_every": cfg.ckpt_every,
                   "bwd_mode": bwd_mode,
                   "plan": None if plan is None else dataclasses.asdict(plan)},
        "forward_steps_per_s": fwd_rate, "graph_replay": graph, "fwdbwd_over_forward": value / fwd_rate,
        **({"one_persistent_launch": one_launch} if one_launch is not None else {}),
        "fwd_ms": fwd_ms, "loss_ms": loss_ms, "bwd_ms": bwd_ms,
        "step_ms": step_stats, "forward_only_ms": fwd_only_stats, "forward_only_reps": n_fo,
        "grad_rel_err": grad_rel_err, "grad_error": grad_detail, "counts_bit_exact_sample": counts_exact,
        "near_ties": n_ties - n_edge, "bin_edge_events": n_edge, "loss": float(loss.item()),
        "roofline": roofline, "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="oscillator",
                    choices=["dimer", "oscillator", "uneven", "grn", "abc_infer", "coi_infer", "selection"],
                    help="oscillator: 9 species / 16 channels, 65,536 x 200,000 steps (default); "
                         "dimer: 2A<->A2, 65,536 x 10,000 steps; "
                         "uneven: 4,096 random networks x 256 trajectories x 5,000 steps; "
                         "grn: 784->256->10 gene-network classifier, 512 images x 32 trajectories x 2,000 steps; "
                         "abc_infer: rate inference for A+B<->C, 100,000 x 250 steps, 250 captured epochs; "
                         "coi_infer: ion-channel rate inference, 262,144 x 20 steps, 800 bins, 400 captured epochs; "
                         "selection: inverse-CDF vs Gumbel-max forward vs Gumbel-Softmax training step (dimer, oscillator)")
    ap.add_argument("--sweep", action="store_true", help="abc_infer: also run the k2 sweep (8 targets)")
    ap.add_argument("--epochs", type=int, default=0,
                    help="abc_infer / coi_infer: replayed epochs (0: the protocol's; fewer for profiling)")
    ap.add_argument("--bwd-mode", default="auto", choices=["auto", "tape", "recompute", "tangent"],
                    help="auto: forward-mode tangents for the dimer (few channels), the tape otherwise")
    ap.add_argument("--n-traj", type=int, default=65536)
    ap.add_argument("--n-steps", type=int, default=0, help="steps per trajectory (0: the workload's)")
    ap.add_argument("--ckpt-every", type=int, default=0, help="checkpoint interval (0: the workload's)")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=None,
                    help="pick the execution plan with the autotuner (untimed; cached under ~/.cache); "
                         "default: on for the uneven batch, off otherwise")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay timing")
    ap.add_argument("--one-launch-steps", type=int, default=2,
                    help="uneven: also time this many steps with every network in one persistent launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="oscillator: skip the secondary dimer line (other_workloads)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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

    if args.workload == "grn":
        return bench_grn(args, torch, dev)
    if args.workload in ("abc_infer", "coi_infer"):
        return bench_infer(args, torch, dev)
    if args.workload == "selection":
        return bench_selection(args, torch, dev)

    if args.copy_bytes:
        n = args.copy_bytes // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "launches": 3}))
        return


    out = bench_mass_action(args, torch, dev, args.workload)
    if args.workload == "oscillator" and not args.no_extra:
        # the dimer workload as a secondary line: same contract, no CPU leg
        out["other_workloads"] = {"dimer": bench_mass_action(args, torch, dev, "dimer", light=True)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
