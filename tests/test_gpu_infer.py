"""Rate inference on the library (A + B <-> C of Sec. 4.1, the ion channel of
Sec. 4.4): the captured optimisation step replays exactly what the eager step
computes, and shortened runs recover the rates their targets were drawn at."""
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


@pytest.mark.parametrize("system", ["dimerization", "dimerization_benchmarked", "ion_channel"])
def test_captured_step_replays_the_eager_step(infer, system):
    if system == "dimerization":
        tr = infer.dimerization(infer.TRUE_RATES, n_traj=8192, n_target=8192, n_grid=24, epochs=20)
    elif system == "dimerization_benchmarked":      # the benchmark's batch and grid
        tr = infer.dimerization(infer.TRUE_RATES, epochs=20)
    else:
        tr = infer.ion_channel(n_traj=16384, n_target=16384, n_bins=200, epochs=20)
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


def test_ion_channel_inference_fits_the_open_count(infer):
    """The fit drives the loss to the ensembles' sampling noise and pins the
    opening and inactivation rates; the closing rate moves the mean open
    count only weakly (it trades off against the opening rate over the
    transient peak), so it is not held to a bound."""
    r = infer.ion_channel(n_traj=65536, n_target=262144, epochs=400).run()
    assert r.loss_last < 1e-2 * r.loss_first
    # sampling noise of the two ensemble means, per bin: p(1-p)-sized
    # variances over 65,536 and 262,144 trajectories
    assert r.loss_last < 20 * (0.5 / 65536 + 0.5 / 262144)
    assert r.ape[0] < 5.0 and r.ape[2] < 5.0, (r.k_learned, r.ape)
