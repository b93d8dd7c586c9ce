"""Write tests/golden/fp64_l12_trajectories.json: 20 trajectories of the FP64
workload at L=12, Nt=120 (theta = pi flux + N(0, 0.3^2), seed 1012; RNG
streams seed 1002; 20 leapfrog steps of length 1; CG 1e-10) computed by the
CPU oracle alone.  The chain carries theta from one trajectory to the next.
Takes about 40 minutes on one core.  Run: python tests/golden/make_fp64_l12_golden.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2508_16298_amd import inputs  # noqa: E402


def main(n_traj=20):
    wl = inputs.WORKLOADS["fp64_l12"]
    p = O.lat(wl.L, wl.Nt, wl.dtau, wl.t, wl.J, wl.K)
    th = wl.initial_theta()
    rows = []
    for k in range(n_traj):
        t0 = time.time()
        th, res, *_ = O.hmc_trajectory(p, th, seed=wl.seed, traj=k, n_steps=wl.n_steps,
                                       traj_len=wl.traj_len, tol=wl.tol)
        res = {key: (float(v) if isinstance(v, float) else int(v)) for key, v in res.items()}
        res["theta_sum"] = float(th.sum())
        res["theta_sumsq"] = float((th ** 2).sum())
        res["seconds"] = time.time() - t0
        rows.append(res)
        print(k, {key: res[key] for key in ("dH", "accepted", "cg_iters_total", "seconds")}, flush=True)
        out = {"workload": "fp64_l12", "source": "oracle/qed_oracle.c via oracle.hmc_trajectory",
               "L": wl.L, "Nt": wl.Nt, "seed": wl.seed, "theta": wl.theta, "sigma": wl.sigma,
               "theta_seed": wl.theta_seed, "n_steps": wl.n_steps, "traj_len": wl.traj_len,
               "tol": wl.tol, "trajectories": rows}
        with open(os.path.join(HERE, "fp64_l12_trajectories.json"), "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 20)
