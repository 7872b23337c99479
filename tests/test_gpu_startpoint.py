"""The start-point-map protocol of Sec. 4.2 on the library.

- The reference sampler chains library forwards; every start point equals the
  oracle's state after the same chained segments (same streams), bit for bit.
- The trainer's rates of change come from the tail observation, whose parity
  with the oracle tests/test_gpu_tail.py covers; its written-out loss
  gradient is checked on the CPU (tests/test_host.py).
- A captured epoch replays exactly what the eager epoch computes.
- With the targets on the model's counters (common random numbers), the loss
  and its gradient are exactly 0 at the true rates.
- The whole protocol at the paper's size, from rates off by factors of 2,
  recovers the five protein rates to within a few per cent (the paper reports
  1.2 %).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2602_19775_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_19775_amd import ssa, startpoint
    ssa.lib()
    return startpoint


def test_reference_start_points_match_the_oracle(sp):
    net = W.start_point_oscillator()
    n_paths, n_start, stride, burn = 256, 256 * 12, 9, 3000
    x = sp.reference_start_points(net, n_start, n_paths, stride, burn, seed=5).cpu().numpy()
    assert x.shape == (n_start, net.n_species) and np.all(x >= 0)
    sp_idx = {s: i for i, s in enumerate(net.species)}
    assert np.all(x[:, sp_idx["D_A"]] + x[:, sp_idx["D_A'"]] == 1)
    assert np.all(x[:, sp_idx["D_R"]] + x[:, sp_idx["D_R'"]] == 1)
    for p in (0, 77, 255):
        cfg = W.RunConfig(seed=5, purpose=sp.PURPOSE_REFERENCE, epoch=0, n_steps=burn)
        r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=[p])
        assert r.n_near[0] == 0
        state = r.x_final[0]
        for c in range(n_start // n_paths):
            r = oracle.run(net, cfg.replace(epoch=c + 1, n_steps=stride), net.theta0, state[None, :],
                           traj_ids=[p])
            state = r.x_final[0]
            if r.n_near[0]:
                break            # a near-tie may resolve either way: stop comparing this path
            assert np.array_equal(x[c * n_paths + p], state), (p, c)


def test_captured_epoch_equals_eager_epoch(sp):
    net = W.start_point_oscillator()
    k_start = np.asarray(W.OSC_PROTEIN_RATES) * 1.5
    tr = sp.StartPointTrainer(net, k_start, n_start=4096, n_paths=64, stride=9, burn=2000, batch=1024,
                              n_rep=5, epochs=6)
    tr.capture()
    tr.reset()
    for _ in range(3):
        tr.step()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (tr.theta, tr.v, tr.lr, tr.epoch, tr.loss)]
    tr.reset()
    for _ in range(3):
        tr.graph.replay()
    torch.cuda.synchronize()
    for a, b in zip(eager, (tr.theta, tr.v, tr.lr, tr.epoch, tr.loss)):
        assert torch.equal(a, b)


def test_common_random_numbers_target_is_exact_at_the_truth(sp):
    """Targets on the model's counters: at the true rates the model's segments
    are the targets' segments, so the loss and its gradient are exactly 0."""
    net = W.start_point_oscillator()
    tr = sp.StartPointTrainer(net, np.asarray(W.OSC_PROTEIN_RATES), n_start=4096, n_paths=64, stride=9,
                              burn=2000, batch=1024, n_rep=5, epochs=2)
    for _ in range(2):
        tr.step()
        torch.cuda.synchronize()
        assert float(tr.loss.item()) == 0.0
        assert torch.count_nonzero(tr.d_params).item() == 0
    assert np.allclose(tr.theta.cpu().numpy(), net.theta0)


def test_protocol_recovers_the_protein_rates(sp):
    """The protocol at the paper's size (262,144 start points, 8,192 a batch,
    25 replicates of 150 steps, T = 3e-6, 3,000 epochs of RMSprop from 0.1
    down to 1e-3) from rates off by factors of 2, targets on common random
    numbers and the elapsed time as the rates' normaliser: the loss falls more
    than a thousandfold and the five rates (median of the last quarter) come
    within 5 % of the truth on average."""
    tr = sp.oscillator_start_points(epochs=3000, temperature=3e-6, lr0=0.1, lr1=1e-3)
    r = tr.run()
    ape0 = 100.0 * np.abs(r.k_start - r.k_true) / r.k_true
    n = r.epochs // 10
    print(f"\nstart-point map: loss {r.losses[:n].mean():.4g} -> {r.losses[-n:].mean():.4g}, "
          f"MAPE {ape0.mean():.1f} % -> {r.ape.mean():.2f} %, rates {np.round(r.k_learned, 3).tolist()}, "
          f"{r.epochs} epochs in {r.train_s:.1f} s")
    assert r.losses[-n:].mean() < 1e-3 * r.losses[:n].mean()
    assert r.ape.mean() < 5.0
