"""A topology planned in a second process (compiled again there, or taken from
the compiler's own cache) runs to the same bits as in the first."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_2602_19775_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# a topology no other test plans
_SEED = 913_402


def _run(out_path: str) -> None:
    """Plans the topology in specialised lane mode, runs one forward and saves
    its outputs."""
    from paper_2602_19775_amd import ssa
    g = np.random.default_rng(np.random.SeedSequence([_SEED, 7]))
    net = W.random_network(g, name="processes_5x7", n_range=(5, 5), m_range=(7, 7))
    B = 128
    h = ssa.Net([net], [B], exec_mode="spec")
    cfg = W.RunConfig(seed=3, n_steps=200, obs_kind=W.OBS_FINAL)
    x0 = torch.tensor(np.repeat(net.x0[:, None], B, axis=1).reshape(-1), dtype=torch.int32, device="cuda")
    f = ssa.forward(h, cfg, torch.tensor(net.theta0, device="cuda"), x0, tie_capacity=0)
    torch.cuda.synchronize()
    np.savez(out_path, x=f.x_final.cpu().numpy(), t=f.t_final.cpu().numpy(), s=f.steps_done.cpu().numpy())


def test_second_process_runs_to_the_same_bits(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _run(str(tmp_path / "a.npz"))
    code = (f"import sys; sys.path[:0] = [{ROOT!r}, {HERE!r}]; import test_gpu_jit_processes as t; "
            f"t._run({str(tmp_path / 'b.npz')!r})")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=100)
    assert r.returncode == 0, r.stderr[-2000:]
    a, b = np.load(tmp_path / "a.npz"), np.load(tmp_path / "b.npz")
    for k in ("x", "t", "s"):
        np.testing.assert_array_equal(a[k], b[k])
    assert int(a["s"].min()) > 0
