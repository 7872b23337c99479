"""The two-phase training of the gene-network classifier (Sec. 3.5, Sec. 4.3)
end to end on the library: relaxed forward and its exact backward for the
first fifth of the steps, then the straight-through estimator, each phase's
step captured into a HIP graph.

- A graph replay equals the same step run eagerly, bit for bit, in both
  phases (same parameters, optimiser state and device scalars before and
  after).
- A shortened run on synthetic digit-shaped images: the training loss falls
  in the relaxed phase and again in the straight-through phase, and the
  held-out accuracy of the averaged parameters (hard forward) rises from
  chance to at least 0.9.
"""
import numpy as np
import pytest
import torch

from paper_2602_19775_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import classify, ssa
    ssa.lib()
    return classify


def _state(tr):
    return [t.clone() for t in (tr.theta, tr.v, tr.temp, tr.step_no, tr.loss)]


def test_graph_replay_equals_eager_steps(cl):
    net = W.GrnNet(n_in=196, n_out=10)
    tr = cl.TwoPhaseTrainer(net, n_train=64, batch=32, n_rep=4, n_steps=300, steps=10, side=14)
    tr.capture()
    for relaxed in (True, False):
        tr.reset()
        for _ in range(3):
            tr._step(relaxed)
        torch.cuda.synchronize()
        eager = _state(tr)
        tr.reset()
        for _ in range(3):
            tr.graphs[relaxed].replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, _state(tr)):
            assert torch.equal(a, b), relaxed


def test_two_phase_training_learns(cl):
    net = W.GrnNet(n_in=784, n_out=10)
    tr = cl.TwoPhaseTrainer(net, n_train=512, batch=128, n_rep=8, n_steps=1000, steps=200, soft_frac=0.2)
    r = tr.run()
    print(f"\ntwo-phase: relaxed loss {r.loss_soft_first:.3f} -> {r.loss_soft_last:.4f}, "
          f"straight-through {r.loss_hard_first:.4f} -> {r.loss_hard_last:.5f}, "
          f"accuracy {r.accuracy_start:.3f} -> {r.accuracy:.3f} in {r.train_s:.2f} s")
    assert r.soft_steps == 40
    assert r.loss_soft_last < 0.2 * r.loss_soft_first
    assert r.loss_hard_last < r.loss_hard_first
    assert r.accuracy_start < 0.3 and r.accuracy >= 0.9
