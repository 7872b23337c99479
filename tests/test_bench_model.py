"""The benchmark's algorithmic operation model and its timing helper, checked
on the CPU against counts that follow from the method: Philox4x32-10 draws
four words a block, each of its ten rounds has two 32x32->64 products and two
three-input xors, and every channel word and the waiting time's word take one
logarithm."""
import numpy as np
import pytest

import bench
from paper_2602_19775_amd import workloads as W


@pytest.mark.parametrize("make,M", [(W.dimerization_2a, 2), (W.oscillator, 16), (W.dimerization_abc, 2)])
def test_philox_and_log_counts(make, M):
    net = make()
    assert net.n_reactions == M
    nb = -(-(M + 1) // 4)                    # blocks covering M + 1 words
    assert 4 * nb >= M + 1 > 4 * (nb - 1)
    for backward in (False, True):
        ops = bench.alu_ops_per_step(net, backward)
        assert ops["mad"] == 20 * nb and ops["bit3"] == 20 * nb
        assert ops["log"] == M + 1           # T = 1/2 needs no further logarithm
        # one reciprocal of a0 and one per channel forward; the backward adds
        # the soft sample's 1/r_j and 1/sum
        assert ops["rcp"] == (1 + M if not backward else 1 + M + M + 1)
        assert all(v >= 0 for v in ops.values())


def test_backward_costs_more_than_the_forward():
    net = W.oscillator()
    f, b = bench.alu_ops_per_step(net, False), bench.alu_ops_per_step(net, True)
    cost = {"int": 0.69, "fp32": 1.0, "mad": 1.7, "log": 2.0, "rcp": 2.0, "cvt": 1.0, "f64": 1.25, "bit3": 0.72}
    assert bench.slots(b, cost) > bench.slots(f, cost)


@pytest.mark.parametrize("steps", [1, 10, 300])
def test_forward_reps(steps):
    for fwd_s in (1e-4, 4.2e-3, 0.02, 0.22, 3.0):
        n = bench.forward_reps(steps, fwd_s)
        assert steps <= n <= max(steps, 200)
        # at least half a second of timed forwards unless the cap is reached
        assert n * fwd_s >= 0.5 or n == max(steps, 200) or n == steps and steps * fwd_s >= 0.5
    assert bench.forward_reps(steps, 0.0) == steps
