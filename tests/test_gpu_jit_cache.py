"""The on-disk cache of specialised code objects: the first plan of a topology
compiles and stores one object; a later process loads it instead of compiling
and runs to the same bits."""
import os
import subprocess
import sys
import time

import numpy as np
import pytest
import torch

from paper_2602_19775_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# a topology no other test plans, so the process's own module cache is cold
_SEED = 913_402


def _run(out_path: str) -> float:
    """Plans the topology in specialised lane mode, runs one forward and saves
    its outputs; returns the seconds the plan took."""
    from paper_2602_19775_amd import ssa
    g = np.random.default_rng(np.random.SeedSequence([_SEED, 7]))
    net = W.random_network(g, name="jit_cache_5x7", n_range=(5, 5), m_range=(7, 7))
    B = 128
    t0 = time.perf_counter()
    h = ssa.Net([net], [B], exec_mode="spec")
    plan_s = time.perf_counter() - t0
    cfg = W.RunConfig(seed=3, n_steps=200, obs_kind=W.OBS_FINAL)
    x0 = torch.tensor(np.repeat(net.x0[:, None], B, axis=1).reshape(-1), dtype=torch.int32, device="cuda")
    f = ssa.forward(h, cfg, torch.tensor(net.theta0, device="cuda"), x0, tie_capacity=0)
    torch.cuda.synchronize()
    np.savez(out_path, x=f.x_final.cpu().numpy(), t=f.t_final.cpu().numpy(), s=f.steps_done.cpu().numpy())
    return plan_s


def test_second_process_loads_the_stored_object(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cache = tmp_path / "jit"
    monkeypatch.setenv("SSA_JIT_CACHE_DIR", str(cache))
    first = _run(str(tmp_path / "a.npz"))
    stored = sorted(cache.iterdir())
    assert len(stored) == 1 and stored[0].suffix == ".co" and stored[0].stat().st_size > 0
    stamp = stored[0].stat().st_mtime_ns

    code = (f"import sys; sys.path[:0] = [{ROOT!r}, {HERE!r}]; import test_gpu_jit_cache as t; "
            f"print('plan_s', t._run({str(tmp_path / 'b.npz')!r}), flush=True)")
    env = dict(os.environ, SSA_JIT_CACHE_DIR=str(cache))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=100)
    assert r.returncode == 0, r.stderr[-2000:]
    second = float(r.stdout.split("plan_s")[-1])
    print(f"plan: {first:.2f} s compiling, {second:.2f} s from the stored object")

    assert sorted(cache.iterdir()) == stored and stored[0].stat().st_mtime_ns == stamp
    a, b = np.load(tmp_path / "a.npz"), np.load(tmp_path / "b.npz")
    for k in ("x", "t", "s"):
        np.testing.assert_array_equal(a[k], b[k])
    assert second < first
