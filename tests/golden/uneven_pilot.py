"""Observation windows of the uneven-batch workload, from a pilot run of the
FP64 oracle: for each of the 4,096 networks (seed 0), t_obs = 0.9 x the
smallest clock after 5,000 steps over 4 trajectories of the pilot stream
(purpose 2) at the network's rates (a path that stops early contributes its
stopping time).  Writes tests/golden/uneven_t_obs.txt, one value per network,
which paper_2602_19775_amd/workloads.py reads."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2602_19775_amd import workloads as W  # noqa: E402

if __name__ == "__main__":
    nets = W.random_network_batch(4096, seed=0)
    cfg = W.RunConfig(seed=0, purpose=W.PURPOSE_PILOT, n_steps=5000)
    out = []
    for n in nets:
        r = oracle.run(n, cfg, n.theta0, n.x0, traj_ids=np.arange(4))
        out.append(0.9 * float(r.t_final.min()))
    with open(os.path.join(HERE, "uneven_t_obs.txt"), "w") as f:
        f.write("# t_obs of the uneven batch (seed 0), one line per network; written by uneven_pilot.py\n")
        for v in out:
            f.write(repr(v) + "\n")
    print("networks", len(out), "t_obs range", min(out), max(out))
