"""The rate inference of A + B <-> C (Sec. 4.1) on the library: the captured
optimisation step replays exactly what the eager step computes, and a
shortened run recovers the rates it was generated with."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def infer():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import infer as m
    from paper_2602_19775_amd import ssa
    ssa.lib()
    return m


def test_captured_step_replays_the_eager_step(infer):
    tr = infer.Trainer(infer.TRUE_RATES, n_traj=8192, n_target=8192, n_grid=24, epochs=20)
    ref = []
    for _ in range(4):
        tr.step()
        torch.cuda.synchronize()
        ref.append((tr.theta.clone(), tr.d_params.clone(), tr.loss.clone(), tr.temp.clone()))
    tr.capture()                     # resets theta, the schedules and the epoch
    noise = torch.randn(1 << 18, device="cuda")
    for k in range(4):
        tr.graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(tr.theta, ref[k][0]), k
        assert torch.equal(tr.d_params, ref[k][1]), k
        assert torch.equal(tr.loss, ref[k][2]), k
        assert torch.equal(tr.temp, ref[k][3]), k
        noise = noise * 1.001 + 1.0  # eager work between replays
        torch.cuda.synchronize()
    assert int(tr.epoch.item()) == 4


def test_shortened_inference_recovers_the_rates(infer):
    r = infer.infer(infer.TRUE_RATES, n_traj=32768, n_target=65536, n_grid=48, epochs=200)
    assert r.loss_last < 1e-2 * r.loss_first
    assert np.all(r.ape < 3.0), (r.k_learned, r.ape)
