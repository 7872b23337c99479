"""Observation window of the oscillator workload, from a pilot run of the FP64
oracle: t_obs = 0.9 x the 1st percentile of the clock after 200,000 steps over
64 trajectories of the pilot stream (purpose 2) at the seeded rates of
rate_seed 0.  Prints
the value stored as OSC_T_OBS in paper_2602_19775_amd/workloads.py."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle  # noqa: E402
from paper_2602_19775_amd import workloads as W  # noqa: E402

if __name__ == "__main__":
    net = W.oscillator(rate_seed=0)
    cfg = W.RunConfig(seed=0, purpose=W.PURPOSE_PILOT, n_steps=200000)
    r = oracle.run(net, cfg, net.theta0, net.x0, traj_ids=np.arange(64))
    print(repr(float(0.9 * np.percentile(r.t_final, 1))))
    print("steps", r.steps_done.min(), r.steps_done.max(), "t range", r.t_final.min(), r.t_final.max(),
          "final R", r.x_final[:, 7].min(), r.x_final[:, 7].max())
