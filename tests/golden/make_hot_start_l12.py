"""Write tests/golden/hot_start_l12_record.json from the CPU oracle alone: the
plain FP64 workload at L=12, Nt=120 from a hot start (angles i.i.d. uniform on
[0, 2 pi), seed 1002; RNG streams seed 1002; 20 leapfrog steps of length 1,
dt = 0.05; CG residual 1e-10).

Recorded:
  solve0        the first solve at the hot start: CG iterations, true residual,
                max |F_F|, rms F_F and max |F_B| of the forces there;
  first_steps   H before and after 1, 2 and 3 leapfrog steps of dt = 0.05
                (trajectory 0's momenta and source; no Metropolis), and the
                largest change of any angle;
  trajectories  the 20 chained trajectories (Methods, HQMC steps (i)-(iv)).

A hot start sits next to configurations with det M = 0, where the fermion
action is infinite: one leapfrog step already multiplies H by ~700, so every
trajectory is rejected and the chain stays at the hot start.  The trajectories
are therefore run in parallel processes, each from the hot start with its own
trajectory index; if one were accepted, the ones after it would be rerun in
order from the new angles (reported).  About two hours on six cores.

Run: python tests/golden/make_hot_start_l12.py [n_workers]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2508_16298_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "hot_start_l12_record.json")


def _wl():
    return inputs.WORKLOADS["fp64_l12_hot"]


def _traj(args):
    k, th = args
    wl = _wl()
    p = O.lat(wl.L, wl.Nt, wl.dtau, wl.t, wl.J, wl.K)
    t0 = time.time()
    th1, res, *_ = O.hmc_trajectory(p, th.copy(), seed=wl.seed, traj=k, n_steps=wl.n_steps,
                                    traj_len=wl.traj_len, tol=wl.tol)
    res = {key: (float(v) if isinstance(v, float) else int(v)) for key, v in res.items()}
    res["traj"] = k
    res["theta_sum"] = float(th1.sum())
    res["theta_sumsq"] = float((th1 ** 2).sum())
    res["seconds"] = time.time() - t0
    print("trajectory", k, {key: res[key] for key in ("dH", "accepted", "cg_iters_total", "seconds")},
          flush=True)
    return res, th1


def _first(args):
    what, k = args
    wl = _wl()
    p = O.lat(wl.L, wl.Nt, wl.dtau, wl.t, wl.J, wl.K)
    th = wl.initial_theta()
    mom, R = O.heatbath(p, wl.seed, 0)
    eta = O.apply_M(p, th, R, dagger=True).reshape(wl.Nt, wl.L, wl.L)
    if what == "solve0":
        X, st, it, rel = O.cg_solve(p, th, eta, tol=wl.tol)
        F = O.fermion_force(p, th, X)
        Fb = O.bosonic_force(p, th)
        out = {"status": int(st), "cg_iters": int(it), "true_resid": float(rel),
               "max_abs_F_F": float(np.abs(F).max()), "rms_F_F": float(np.sqrt((F ** 2).mean())),
               "max_abs_F_B": float(np.abs(Fb).max())}
    else:
        th1, _, hb, ha = O.leapfrog(p, th.copy(), mom.copy(), eta, k, traj_len=wl.traj_len / wl.n_steps * k,
                                    tol=wl.tol)
        out = {"steps": k, "dt": wl.traj_len / wl.n_steps, "H_before": float(hb), "H_after": float(ha),
               "max_abs_dtheta": float(np.abs(th1 - th).max())}
    print(what, k, out, flush=True)
    return what, out


def _write(out):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(out, f, indent=1)
    os.replace(tmp, OUT)


def main(workers=6, n_traj=20):
    wl = _wl()
    th0 = wl.initial_theta()
    t0 = time.time()
    out = {"workload": "fp64_l12_hot", "source": "oracle/qed_oracle.c via oracle (cg_solve, fermion_force, "
           "bosonic_force, leapfrog, hmc_trajectory)", "L": wl.L, "Nt": wl.Nt, "seed": wl.seed,
           "theta": "hot", "theta_seed": wl.theta_seed or wl.seed, "n_steps": wl.n_steps,
           "traj_len": wl.traj_len, "tol": wl.tol, "notes": [], "solve0": None, "first_steps": [],
           "trajectories": [], "complete": False}
    # the record is rewritten after every finished piece, so an interrupted run keeps what it has
    with mp.get_context("fork").Pool(workers) as pool:
        jobs = [("first", a) for a in (("solve0", 0), ("steps", 1), ("steps", 2), ("steps", 3))]
        jobs += [("traj", (k, th0)) for k in range(n_traj)]
        thetas = {}
        for kind, res in pool.imap_unordered(_job, jobs):
            if kind == "first":
                what, o = res
                if what == "solve0":
                    out["solve0"] = o
                else:
                    out["first_steps"] = sorted(out["first_steps"] + [o], key=lambda r: r["steps"])
            else:
                row, th1 = res
                thetas[row["traj"]] = th1
                out["trajectories"] = sorted(out["trajectories"] + [row], key=lambda r: r["traj"])
            out["wall_seconds"] = time.time() - t0
            _write(out)
    rows = out["trajectories"]
    # the parallel runs assumed every trajectory rejected; redo in order after an acceptance
    for k in range(n_traj):
        if rows[k]["accepted"]:
            out["notes"].append(f"trajectory {k} accepted: trajectories after it rerun in order")
            th = thetas[k]
            for j in range(k + 1, n_traj):
                rows[j], th = _traj((j, th))
                _write(out)
            break
    out["complete"] = True
    out["wall_seconds"] = time.time() - t0
    _write(out)
    print("wrote", OUT, flush=True)


def _job(job):
    kind, args = job
    return kind, (_first(args) if kind == "first" else _traj(args))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6)
