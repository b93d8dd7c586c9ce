"""Benchmark: seconds per HMC trajectory and the achieved bandwidth of the
fused M^dag M kernel, on one MI355X.

Workload (default): L=24, Nt=240, dtau=0.1, t=1, J=K=1, theta = pi flux plus
Gaussian noise (sigma 0.3, seed 1013; the stand-in for a thermalised
configuration -- a hot start at this size sits next to det M = 0 and its
molecular dynamics diverges within one step), 20 leapfrog steps of total
length 1, CG to true relative residual 1e-8, mixed precision (complex-FP32
matvecs and force, FP64 solution, reliable updates and reductions).  One
step = one trajectory: heat bath, 21 solves, 21 forces, leapfrog, Metropolis.

The timed set is stationary and does not depend on --warmup: a fixed number
of chained equilibration trajectories (--equilibrate, untimed) moves the
angles off the relaxing start, and every warm-up and timed trajectory then
starts from that same point with its own trajectory index (its own momenta,
source and Metropolis draw).  The first --compare timed trajectories, plus the
one with the largest |dH|, are rerun on the other paths from the same start
with the same indices: the plain FP64 GPU path and the mixed path with the
learned preconditioner (network trained at setup, untimed, on residuals of
the method's own solves); dH, decisions, iterations and seconds side by side.

Prints one JSON line.  The roofline block is for the dominant kernel of the
timed path, by default the fused CG iteration k_cg_iter (one launch per
iteration: recurrences, x update, M^dag M, inner products).  Its algorithmic
bytes per site are, in the mixed path, r, w, s, p read (4 x 8 B), two FP32
angles (8 B), x read and written (2 x 16 B, FP64) and r, s, p, w written
(4 x 8 B): 104 B per site (176 B in FP64).  Its duration comes from event
pairs around every 8th graph replay of 51 back-to-back iteration launches (a
replay holds nothing else) over the timed region; `traffic` is the
counter-measured HBM bytes per launch.  The metric's M^dag M bandwidth is
measured after the timed region on the standalone fused M^dag M kernel at
24 B per site (v in, out written, two FP32 angles; 48 B in FP64): the
start/end events of each of 200 dispatches (the events' own cost included;
rocprofv3's kernel-only duration is in profiles/).  The CPU baseline is the
plain FP64 oracle on a bounded sample (a fixed number of CG iterations plus
one force at the same lattice and angles), scaled to the trajectory's
measured CG iteration count.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector ALU peaks of the MI355X (256 CUs x 2.4 GHz): FP32 with packed
# instructions 157.3 TFLOP/s (the library builds without them, so half of it
# is the reachable rate), FP64 78.6 TFLOP/s
VALU_PEAK_FP32_TFLOPS = 157.3
VALU_PEAK_FP64_TFLOPS = 78.6

# HBM bytes per launch of the fused CG iteration from rocprofv3 counters
# (profiles/k_cg_iter_mixed_l24_hbm_counters.md): FETCH_SIZE and WRITE_SIZE in
# KiB, scaled by the copy-kernel calibration (x2.0 and x1.0).  Valid for the
# kernel as measured there; set to None whenever k_cg_iter changes.
CG_ITER_COUNTER_BYTES = {"fp32": (4652.0 * 2.0 + 6491.4 * 1.0) * 1024, "fp64": None}
# the same for the spectral preconditioner's tau-sum + inverse-DFT kernel at
# L=24, Nt=240 with a tau reach of 12 (profiles/k_pcs_tconv_idft_mixed_l24.md):
# 2009.0 KiB fetched, 1080.0 KiB written per live launch, x2.0 and x1.0
PC_SPEC_COUNTER_BYTES = {"fp32": (2009.0 * 2.0 + 1080.0 * 1.0) * 1024, "fp64": None}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed_l24")
    ap.add_argument("--prec", default=None, help="override: fp64 or mixed")
    ap.add_argument("--precond", default="paper", choices=["none", "paper", "learned"],
                    help="preconditioner of the timed path: the paper's G^dag G (default), none, or the "
                         "learned network (trained at setup on the method's own residuals)")
    ap.add_argument("--equilibrate", type=int, default=10,
                    help="chained trajectories from the workload's angles before the timed set (untimed)")
    ap.add_argument("--compare", type=int, default=3,
                    help="timed trajectories rerun on the other paths for the side-by-side comparison")
    ap.add_argument("--no-compare-learned", dest="compare_learned", action="store_false",
                    help="skip the learned-preconditioner path in the comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=800, help="oracle CG iterations in the CPU sample")
    ap.add_argument("--profile-every", type=int, default=8)
    ap.add_argument("--solve-only", type=int, default=0, metavar="MAXIT",
                    help="counter runs: one solve of MAXIT iterations plus 200 standalone M^dag M "
                         "launches on the workload instead of trajectories (same kernels and launch shapes)")
    ap.add_argument("--matvec-only", type=int, default=0, metavar="L",
                    help="only the standalone M^dag M at the large size with this L (for profiler runs)")
    ap.add_argument("--precond-only", type=int, default=0, metavar="L",
                    help="only the paper preconditioner z = G^dag G r at L, Nt = 10 L, FP32 (for profiler runs)")
    ap.add_argument("--train-only", type=int, default=0, metavar="L",
                    help="only 3 + 20 residual-form training steps of the network at L, Nt = 10 L (profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="counter calibration: 5 device copies of 256 MiB (torch copy kernel)")
    return ap.parse_args()


# Standalone M^dag M past the single-launch latency floor of L=24: the
# learned-preconditioner size and one size whose FP32 vectors (168 MB) exceed
# the 256 MB last-level cache together with input, output and phases.
MATVEC_LARGE = [(66, 660, 1005), (128, 1280, 1006)]


def matvec_large(n_calls=100, only_L=0):
    """Per-dispatch event timing of M^dag M (above 1024 cells per slice the
    tiled, tau-streamed kernel) at the large sizes, FP32 and FP64; GB/s
    against the algorithmic 24 / 48 B per site."""
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q
    rows = []
    for L, Nt, seed in MATVEC_LARGE:
        if only_L and L != only_L:
            continue
        theta = torch.from_numpy(inputs.noisy_pi_flux_theta(L, Nt, 0.3, seed)).cuda()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        N = L * L * Nt
        with Q.Lattice(L, Nt) as lat:
            for prec, cdt, bps, cls, tname in (("fp32", torch.complex64, 24, Q.K_MDAGM_FP32, "float"),
                                               ("fp64", torch.complex128, 48, Q.K_MDAGM_FP64, "double")):
                vin = torch.randn(Nt, L, L, dtype=cdt, device="cuda", generator=gen)
                vout = torch.empty_like(vin)
                lat.apply_MdagM(theta, vin, prec=prec, out=vout)
                lat.profile(1)
                for _ in range(n_calls):
                    lat.apply_MdagM(theta, vin, prec=prec, out=vout)
                n, ms = lat.profile_read(cls)
                lat.profile(0)
                us = 1e3 * ms / max(n, 1)
                gbs = bps * N / (us * 1e-6) / 1e9
                rows.append({"L": L, "Nt": Nt, "sites": N, "prec": prec,
                             "kernel": f"k_mdagm_tiled<{tname}>" if L * L // 4 > 1024 else f"k_mdagm<{tname}>",
                             "avg_launch_us": us, "alg_bytes_per_launch": bps * N, "gbs": gbs,
                             "frac_of_hbm_peak": gbs / HBM_PEAK_GBS, "launches": n})
                del vin, vout
        del theta
        torch.cuda.empty_cache()
    return rows


def run_train_only(L, n_steps=20):
    """Residual-form training steps of the learned preconditioner at L,
    Nt = 10 L (pi flux + noise angles, a Gaussian residual, the initial
    weights): 3 untimed, then n_steps timed between a host clock pair."""
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q
    Nt = 10 * L
    th = torch.from_numpy(inputs.noisy_pi_flux_theta(L, Nt, 0.3, 5000)).cuda()
    r = torch.from_numpy(inputs.gauss_cvec(L, Nt, 5001)).cuda()
    with Q.Lattice(L, Nt) as lat, Q.Net(lat) as net:
        net.set_params(inputs.net_init_weights(3))
        for _ in range(3):
            net.train_step_residual(th, r, lr=1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_steps):
            loss, _ = net.train_step_residual(th, r, lr=1e-3)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / n_steps * 1e3
    print(json.dumps({"train_only": {"L": L, "Nt": Nt, "steps": n_steps, "ms_per_step": ms, "loss": loss}}),
          flush=True)


def run_precond_only(L, n_calls=6):
    """The paper preconditioner applied n_calls times (after its build and one
    untimed call) to a seeded Gaussian vector at L, Nt = 10 L, FP32; the time
    per application from one event pair on the handle's stream."""
    import torch
    from paper_2508_16298_amd import qedhmc as Q
    Nt = 10 * L
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1005)
    with Q.Lattice(L, Nt) as lat:
        v = torch.randn(Nt, L, L, dtype=torch.complex64, device="cuda", generator=gen)
        z = torch.empty_like(v)
        lat.apply_precond(v, prec="fp32", out=z)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n_calls):
            lat.apply_precond(v, prec="fp32", out=z)
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / n_calls
    print(json.dumps({"precond_only": {"L": L, "Nt": Nt, "prec": "fp32", "us_per_apply": us,
                                       "passes_per_apply": 2, "calls": n_calls}}), flush=True)


def run_copy_calibration():
    """A plain copy of known size, for scaling the HBM byte counters
    (FETCH_SIZE, WRITE_SIZE) of the profiler: each launch reads and writes
    exactly 256 MiB."""
    import torch
    n = 64 * 2 ** 20
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                                           "launches": 5}}), flush=True)


def run_solve_only(a):
    """One mixed-precision solve of a fixed iteration count on the workload
    (with --precond: PCG with the paper's preconditioner, or plain CG, whose
    iteration is k_cg_iter in the trajectory's launch shape) and 200
    standalone M^dag M launches; prints the iteration count."""
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q
    wl = inputs.WORKLOADS[a.workload]
    prec = a.prec or wl.precision
    theta = torch.from_numpy(wl.initial_theta()).cuda()
    with Q.Lattice(wl.L, wl.Nt, dtau=wl.dtau, t=wl.t, J=wl.J, K=wl.K, seed=wl.seed) as lat:
        _, R = lat.heatbath(0)
        eta = lat.apply_M(theta, R, dagger=True)
        pc = "paper" if a.precond == "paper" else None
        x, st, it, rel = lat.cg_solve(theta, eta, tol=1e-30, maxit=a.solve_only, prec=prec, precond=pc)
        cdt = torch.complex64 if prec != "fp64" else torch.complex128
        vin = torch.from_numpy(inputs.gauss_cvec(wl.L, wl.Nt, 99)).to(cdt).cuda()
        vout = torch.empty_like(vin)
        for _ in range(200):
            lat.apply_MdagM(theta, vin, prec="fp32" if prec != "fp64" else "fp64", out=vout)
        torch.cuda.synchronize()
    print(json.dumps({"solve_only": {"workload": wl.name, "precond": a.precond, "iterations": it, "true_rel": rel,
                                     "matvec_launches": 200}}), flush=True)


def cpu_baseline(wl, th, total_cg_iters, n_solves, n_iter, pc=None):
    """Oracle (plain FP64 C, single thread) on a bounded sample of the same
    workload: n_iter CG iterations (PCG with the oracle's own G^dag G when
    the timed path uses the paper's preconditioner, whose stencil build is
    not counted) and one fermion force at the same lattice and angles (the
    timed trajectories' start), scaled to the trajectory's CG iteration and
    solve counts.  The oracle is single-threaded: a trajectory is a sequence
    of dependent solves and the oracle's CG runs on one core."""
    import oracle as O
    from paper_2508_16298_amd import inputs
    p = O.lat(wl.L, wl.Nt, wl.dtau, wl.t, wl.J, wl.K)
    R = inputs.gauss_cvec(wl.L, wl.Nt, wl.seed + 1)
    eta = O.apply_M(p, th, R, dagger=True)
    precond, kind = None, "CG"
    if pc == "paper":
        from oracle import precond as PC
        from paper_2508_16298_amd import qedhmc as Q
        taps = PC.build_stencil(8, 24, cap=Q.PC_TAU_REACH)[0]
        shape = (wl.Nt, wl.L, wl.L)
        precond, kind = (lambda r: PC.apply_P(taps, r.reshape(shape)).reshape(-1)), "PCG (G^dag G)"
        n_iter = max(4, n_iter // 40)
    t0 = time.perf_counter()
    X, st, it, rel = O.cg_solve(p, th, eta, tol=1e-30, maxit=n_iter, precond=precond)
    t_cg = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.fermion_force(p, th, X)
    O.bosonic_force(p, th)
    t_force = time.perf_counter() - t0
    per_iter = t_cg / max(it, 1)
    est = per_iter * total_cg_iters + t_force * n_solves
    hi = host_info()
    return {
        "value": est, "unit": "s/trajectory", "cores": 1, "kind": "oracle", "host": hi,
        "s_per_cg_iter": per_iter,
        "sample": (f"oracle FP64 {kind}, {it} iterations ({t_cg:.1f} s) + one fermion and gauge force "
                   f"({t_force:.2f} s) at L={wl.L} Nt={wl.Nt}, the timed trajectories' start angles; scaled to "
                   f"the GPU trajectory's {total_cg_iters:.0f} CG iterations and {n_solves} forces "
                   f"(extrapolation, single thread; host {hi['nproc']} cores, {hi['cpu_model']})"),
    }


def run_batched(a):
    """--workload batched_chains: 64 independent chains, L drawn from
    8/12/16/20 (seed 1004), Nt = 10 L, chain c with heat-bath seed 4000 + c,
    pi flux plus noise, mixed precision, 20 leapfrog steps, CG residual 1e-8;
    one step = one trajectory of every chain; value = sites x trajectories
    per second.  The roofline block is the batched CG iteration k_b_cg_iter at the
    autotuned tile shape, timed by the autotuner with events around 24
    back-to-back launches with every chain active (104 B per site of every
    chain, as k_cg_iter)."""
    import numpy as np
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q

    wl = inputs.WORKLOADS["batched_chains"]
    prec = a.prec or wl.precision
    sizes, ths, seeds = inputs.batched_chain_inputs()
    theta = torch.from_numpy(np.concatenate([t.reshape(-1) for t in ths])).cuda()
    b = Q.Batch(sizes, dtau=wl.dtau, t=wl.t, J=wl.J, K=wl.K, seeds=seeds)
    traj = 0
    for _ in range(a.warmup):
        b.trajectory(theta, traj, wl.n_steps, wl.traj_len, wl.tol, prec=prec)
        traj += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(a.steps):
        results.append(b.trajectory(theta, traj, wl.n_steps, wl.traj_len, wl.tol, prec=prec))
        traj += 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mc, nt, nb, us = b.tile("fp32" if prec != "fp64" else "fp64")
    shape_idx = {(1, 2): 0, (2, 2): 1, (1, 1): 2, (2, 1): 3}[(mc, nb)]
    N = sum(L * L * Nt for L, Nt in sizes)
    it_bytes = (104 if prec != "fp64" else 176) * N
    it_us = float(us[shape_idx])
    achieved = it_bytes / (it_us * 1e-6) / 1e9
    s_per = elapsed / a.steps
    per_chain_iters = [sum(r[c]["cg_iters_total"] for r in results) / a.steps for c in range(len(sizes))]
    out = {
        "metric": "lattice-site updates per s, 64 batched chains of uneven L (one update = one space-time "
                  "site advanced by one trajectory)",
        "value": N / s_per, "unit": "site-updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * s_per, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "c64+f64" if prec != "fp64" else "c128", "data": "synthetic",
        "config": {"workload": (f"batched_chains: {len(sizes)} chains, L in {sorted(set(L for L, _ in sizes))}, "
                                f"Nt = 10 L, {N} sites, theta pi flux + N(0, 0.3^2), {wl.n_steps} leapfrog "
                                f"steps, CG true residual {wl.tol}, {prec}"),
                   "chains": len(sizes), "sites": N, "precision": prec},
        "chain_traj_per_s": len(sizes) / s_per,
        "cg_iters_per_chain_traj": {"mean": float(np.mean(per_chain_iters)), "max": float(np.max(per_chain_iters))},
        "accept_rate": float(np.mean([r[c]["accepted"] for r in results for c in range(len(sizes))])),
        "tile": {"cells_per_thread": mc, "threads": nt, "exchange_buffers": nb,
                 "us_per_iter_candidates": [float(x) for x in us]},
        "roofline": {"bound": "hbm", "kernel": "k_b_cg_iter (batched fused CG iteration, all chains)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": it_bytes, "avg_launch_us": it_us, "timed_launches": "24, best of 2"},
    }
    b.close()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(wl, sizes, ths, per_chain_iters, a.cpu_iters)
    print(json.dumps(out), flush=True)


def run_se(a):
    """--workload se_l24: one measurement of the stochastic estimation per
    step (Methods, "Stochastic estimation of fermionic observables"): 40
    Philox probes, the multi-RHS solve X_p = (M^dag M)^-1 M^dag xi_p (mixed
    precision, true residual 1e-8, one gauge field for all 40 right-hand
    sides) and the FFT-averaged spin correlator over the 780 probe pairs, at
    L=24, Nt=240 on the angles of the trajectory workload.  value = seconds
    per measurement.  The roofline block is the solve phase: 104 B per site
    and right-hand side for every batched CG iteration (as k_cg_iter), over
    the solve's measured time (reliable updates and launch gaps included:
    a lower bound on the kernel's rate)."""
    import numpy as np
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q

    wl = inputs.WORKLOADS["se_l24"]
    n_rv = inputs.SE_PROBES
    prec = a.prec or wl.precision
    L, Nt = wl.L, wl.Nt
    N = L * L * Nt
    theta = torch.from_numpy(wl.initial_theta()).cuda()
    se = Q.Stochastic(L, Nt, n_rv, dtau=wl.dtau, t=wl.t, J=wl.J, K=wl.K, seed=wl.seed)
    xi = se._set()
    X = se._set()
    C = torch.empty((Nt, L, L), dtype=torch.complex128, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def measure(m):
        ev[0].record()
        se.probes(m, out=xi)
        _, st, it, rel = se.solve(theta, xi, tol=wl.tol, prec=prec, out=X)
        ev[1].record()
        se.spin_correlator(xi, X, out=C)
        ev[2].record()
        torch.cuda.synchronize()
        return st, it, rel, ev[0].elapsed_time(ev[1]) * 1e-3, ev[1].elapsed_time(ev[2]) * 1e-3

    for m in range(a.warmup):
        measure(m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows = [measure(1000 + m) for m in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s_per = elapsed / a.steps
    t_solve = float(np.mean([r[3] for r in rows]))
    t_corr = float(np.mean([r[4] for r in rows]))
    iters = np.array([r[1] for r in rows])
    # every launch of the batched iteration covers the right-hand sides still running
    it_sum = float(iters.sum(axis=1).mean())
    achieved = (104 if prec != "fp64" else 176) * N * it_sum / t_solve / 1e9
    npairs = n_rv * (n_rv - 1) // 2
    dft_flop = 8.0 * N * (2 * L + Nt)          # one 3-D DFT by direct sums along each axis
    corr_tflops = (2 * npairs + 1) * dft_flop / t_corr / 1e12
    Ch = C.cpu().numpy()
    out = {
        "metric": "s per stochastic-estimation measurement (40 probes, spin correlator) at L=24 Nt=240, "
                  "CG resid 1e-8",
        "value": s_per, "unit": "s/measurement", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * s_per, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "c64+f64" if prec != "fp64" else "c128", "data": "synthetic",
        "config": {"workload": (f"se_l24: L={L} Nt={Nt}, theta pi flux + N(0, 0.3^2) (seed 1013), {n_rv} "
                                f"probes (seed {wl.seed}), multi-RHS CG true residual {wl.tol} {prec}, "
                                f"spin correlator C_S(Delta) over {npairs} probe pairs"),
                   "L": L, "Nt": Nt, "sites": N, "probes": n_rv, "precision": prec},
        "solve_s": t_solve, "correlator_s": t_corr,
        "cg_iters_per_probe": {"mean": float(iters.mean()), "max": int(iters.max())},
        "max_true_resid": float(max(r[2].max() for r in rows)),
        "status": [int(r[0]) for r in rows],
        "C_S": {"Delta0": float(Ch[0, 0, 0].real), "Delta_x1": float(Ch[0, 0, 1].real),
                "Delta_tau1": float(Ch[1, 0, 0].real)},
        "correlator": {"kernels": "k_se_xy / k_se_t / k_se_accum (FP64 DFTs by direct sums)",
                       "dft_count": 2 * npairs + 1, "tflops": corr_tflops, "peak_fp64_tflops": 78.6},
        "roofline": {"bound": "hbm", "kernel": "k_b_cg_iter (multi-RHS CG iteration, 40 right-hand sides)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_launch": (104 if prec != "fp64" else 176) * N * n_rv,
                     "timing": "solve phase between events (includes updates and launch gaps)"},
    }
    se.close()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_se(wl, theta.cpu().numpy(), n_rv, it_sum, a.cpu_iters)
    print(json.dumps(out), flush=True)


def run_production(a):
    """--workload production_l24: the production loop at L=24, Nt=240 (mixed
    precision, CG residual 1e-8, the paper's preconditioner unless --precond
    none): --equilibrate thermalisation trajectories
    with step-size adaptation (3 leapfrog steps each, target acceptance 0.7,
    gain 0.5, from dt = 0.1), then --steps measured trajectories at the frozen step with
    S_tau, S_plaq and the flux correlator logged; value = seconds per measured
    trajectory.  The autocorrelation of the logged S_plaq series is reported
    (a short series: a pipeline check, not a physics estimate)."""
    import numpy as np
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q

    wl = inputs.WORKLOADS["mixed_l24"]
    prec = a.prec or wl.precision
    pc = "paper" if a.precond == "paper" else None
    theta = torch.from_numpy(wl.initial_theta()).cuda()
    with Q.Lattice(wl.L, wl.Nt, dtau=wl.dtau, t=wl.t, J=wl.J, K=wl.K, seed=wl.seed) as lat:
        t0 = time.perf_counter()
        st, rec_t, _, dt = lat.production(theta, 0, a.equilibrate, 0, 0.1, 0.7, 0.5, 3, tol=wl.tol, prec=prec,
                                          precond=pc, flux=False)
        t_therm = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st2, rec, Cf, _ = lat.production(theta, 10_000, 0, a.steps, dt, 0.7, 0.0, 3, tol=wl.tol, prec=prec,
                                         precond=pc)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        Cf = Cf.cpu().numpy()
    S_plaq = np.array([r["S_plaq"] for r in rec])
    ac = None
    if a.steps >= 8 and S_plaq.std() > 0:
        rho, ti, te = Q.autocorrelation(S_plaq, min(4, a.steps - 1))
        ac = {"rho": [float(x) for x in rho], "tau_int": ti, "tau_exp": te}
    s_per = elapsed / a.steps
    out = {
        "metric": "s per production trajectory (3 leapfrog steps, adapted dt) at L=24 Nt=240, CG resid 1e-8",
        "value": s_per, "unit": "s/trajectory", "n_gpus": 1, "steps": a.steps, "warmup": a.equilibrate,
        "ms_per_step": 1e3 * s_per, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "c64+f64" if prec != "fp64" else "c128", "data": "synthetic",
        "config": {"workload": (f"production_l24: L={wl.L} Nt={wl.Nt}, theta pi flux + N(0, 0.3^2), "
                                f"{a.equilibrate} thermalisation trajectories adapting dt from 0.1 to target "
                                f"acceptance 0.7, then {a.steps} at dt frozen, 3 leapfrog steps, {prec}, "
                                f"preconditioner {pc or 'none'}")},
        "status": [int(st), int(st2)],
        "dt_final": dt, "thermalisation_s": t_therm,
        "dt_history": [r["dt"] for r in rec_t],
        "accept_rate": float(np.mean([r["accepted"] for r in rec])),
        "cg_iters_per_traj": float(np.mean([r["cg_iters"] for r in rec])),
        "S_tau": [r["S_tau"] for r in rec], "S_plaq": S_plaq.tolist(),
        "C_flux_first": [float(x) for x in Cf[:6]], "autocorrelation_S_plaq": ac,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_se(wl, th, n_rv, it_sum, n_iter):
    """Oracle (plain FP64, one thread) on a bounded sample of the measurement:
    n_iter CG iterations of one probe and the FFT estimator (numpy) over 3
    probes; scaled to the measurement's total CG iterations (all probes) and
    780 probe pairs."""
    import numpy as np
    import oracle as O
    from oracle import se as SE
    p = O.lat(wl.L, wl.Nt, wl.dtau, wl.t, wl.J, wl.K)
    xi = O.probes(p, wl.seed, 0, 3)
    R = O.apply_M(p, th, xi[0], dagger=True)
    t0 = time.perf_counter()
    X, st, it, rel = O.cg_solve(p, th, R, tol=1e-30, maxit=n_iter)
    t_cg = (time.perf_counter() - t0) / max(it, 1)
    Xs = np.stack([X.reshape(wl.Nt, wl.L, wl.L)] * 3)
    t0 = time.perf_counter()
    SE.spin_correlator_se(p, xi, Xs)
    t_pair = (time.perf_counter() - t0) / 3
    npairs = n_rv * (n_rv - 1) // 2
    hi = host_info()
    return {"value": t_cg * it_sum + t_pair * npairs, "unit": "s/measurement", "cores": 1, "kind": "oracle",
            "host": hi,
            "sample": (f"oracle FP64 CG {it} iterations ({t_cg * it:.1f} s) on one probe and the numpy FFT "
                       f"estimator over 3 probe pairs ({3 * t_pair:.1f} s) at L={wl.L} Nt={wl.Nt}; scaled to "
                       f"{it_sum:.0f} CG iterations over all probes and {npairs} pairs (extrapolation, single "
                       f"thread; host {hi['nproc']} cores, {hi['cpu_model']})")}


def cpu_baseline_batched(wl, sizes, ths, per_chain_iters, n_iter):
    """Oracle (plain FP64 C, one thread) on a bounded sample: n_iter CG
    iterations and one fermion + gauge force on one chain of each lattice size
    in the batch; every chain's trajectory is then costed at its measured CG
    iteration count and N_md + 1 forces.  Reported in site-updates/s."""
    import oracle as O
    from paper_2508_16298_amd import inputs
    per_size = {}
    t_sample = 0.0
    for c, (L, Nt) in enumerate(sizes):
        if L in per_size:
            continue
        p = O.lat(L, Nt, wl.dtau, wl.t, wl.J, wl.K)
        th = ths[c]
        eta = O.apply_M(p, th, inputs.gauss_cvec(L, Nt, 77), dagger=True)
        t0 = time.perf_counter()
        X, st, it, rel = O.cg_solve(p, th, eta, tol=1e-30, maxit=n_iter)
        t1 = time.perf_counter()
        O.fermion_force(p, th, X)
        O.bosonic_force(p, th)
        t2 = time.perf_counter()
        per_size[L] = ((t1 - t0) / max(it, 1), t2 - t1)
        t_sample += t2 - t0
    est = sum(per_size[L][0] * per_chain_iters[c] + per_size[L][1] * (wl.n_steps + 1)
              for c, (L, Nt) in enumerate(sizes))
    N = sum(L * L * Nt for L, Nt in sizes)
    return {"value": N / est, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle FP64 CG, {n_iter} iterations + one fermion and gauge force per lattice size "
                       f"{sorted(per_size)} ({t_sample:.1f} s); every chain costed at its measured CG iterations "
                       f"and {wl.n_steps + 1} forces (extrapolation, single thread)")}


def run_learned(a):
    """--workload learned_l66: the learned preconditioner.  Training: the
    network (initial weights seed 1005) is trained with Adam (lr 1e-3, FP32)
    on triples (theta, eta, X) from mixed-precision CG solves (residual 1e-8)
    at L=24, Nt=240 -- theta pi flux + N(0, 0.3^2) noise (seeds 5000+k), eta =
    M^dag R -- cycling over the triples.  Evaluation at L=66, Nt=660 (theta pi
    flux + noise, seed 1005; eta = M^dag R from the heat bath), true residual
    1e-8: CG iterations and seconds for no preconditioner and the paper's
    (mixed precision, fused kernels) and for flexible CG with the trained
    network (BF16 MFMA, fallback the paper's; FP64 vectors).  value = seconds
    of the learned solve.  The roofline block is the BF16 MFMA conv layer
    (2 x 27 x 32 x 32 flop per site) timed by dispatch events during the
    learned solve."""
    import numpy as np
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q

    wl = inputs.WORKLOADS["learned_l66"]
    n_train_theta = int(os.environ.get("QEDHMC_NET_TRIPLES", "8"))
    n_steps = int(os.environ.get("QEDHMC_NET_STEPS", "1000"))
    Lt, Ntt = 24, 240
    out = {}
    t0 = time.perf_counter()
    with Q.Lattice(Lt, Ntt, dtau=wl.dtau, t=wl.t, J=wl.J, K=wl.K, seed=5000) as lt, Q.Net(lt) as net:
        # residuals r_k = eta - O x_k of the method's own (mixed) solves,
        # stopped after k = 0, 50, ..., 1250 iterations
        pool = []
        for k in range(n_train_theta):
            th = torch.from_numpy(inputs.noisy_pi_flux_theta(Lt, Ntt, 0.3, 5000 + k)).cuda()
            R = torch.from_numpy(inputs.gauss_cvec(Lt, Ntt, 5100 + k)).cuda()
            eta = lt.apply_M(th, R, dagger=True)
            pool.append((th, eta))
            for its in range(50, 1300, 50):
                x, st, it, rel = lt.cg_solve(th, eta, tol=1e-12, maxit=its, prec="fp32")
                pool.append((th, eta - lt.apply_MdagM(th, x, prec="fp64")))
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        net.set_params(inputs.net_init_weights(wl.seed))
        losses = []
        rng = np.random.default_rng(wl.seed)
        t1 = time.perf_counter()
        for s in range(n_steps):
            th, r = pool[int(rng.integers(len(pool)))]
            loss, _ = net.train_step_residual(th, r, lr=1e-3)
            losses.append(loss)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        params = net.get_params()
    out["training"] = {"lattice": f"L={Lt} Nt={Ntt}", "form": "residual |O z - r|^2 / |r|^2",
                       "residuals": len(pool), "thetas": n_train_theta, "steps": n_steps,
                       "loss_first": losses[0], "loss_last_avg": float(np.mean(losses[-50:])),
                       "data_s": t_data, "train_s": t_train, "ms_per_step": 1e3 * t_train / max(n_steps, 1)}
    L, Nt = wl.L, wl.Nt
    th_np = inputs.noisy_pi_flux_theta(L, Nt, 0.3, wl.seed)
    with Q.Lattice(L, Nt, dtau=wl.dtau, t=wl.t, J=wl.J, K=wl.K, seed=wl.seed) as lat, Q.Net(lat) as net:
        theta = torch.from_numpy(th_np).cuda()
        _, R = lat.heatbath(0)
        eta = lat.apply_M(theta, R, dagger=True)
        net.set_params(params)
        res = {}
        for name, pc in (("none", None), ("paper", "paper")):
            lat.cg_solve(theta, eta, tol=1e-3, maxit=20, prec="fp32", precond=pc)  # load kernels / build P
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st, it, rel = lat.cg_solve(theta, eta, tol=wl.tol, prec="fp32", precond=pc)
            torch.cuda.synchronize()
            res[name] = {"iterations": it, "s": time.perf_counter() - t, "true_rel": rel, "status": st}
        net.fcg_solve(theta, eta, tol=1e-2, maxit=3, arith="bf16", fallback="paper")
        lat.profile(1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st, it, rel, sw = net.fcg_solve(theta, eta, tol=wl.tol, arith="bf16", fallback="paper")
        torch.cuda.synchronize()
        res["learned"] = {"iterations": it, "s": time.perf_counter() - t, "true_rel": rel, "status": st,
                          "switched_at": sw}
        n_k, ms_k = lat.profile_read(Q.K_NET_MFMA)
        lat.profile(0)
    N = L * L * Nt
    flops = 2.0 * 27 * 32 * 32 * N
    avg_ms = ms_k / max(n_k, 1)
    achieved = flops / (avg_ms * 1e-3) / 1e12 if n_k else None
    line = {
        "metric": "seconds to true residual 1e-8 at L=66 Nt=660, flexible CG with the learned preconditioner",
        "value": res["learned"]["s"], "unit": "s/solve", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * res["learned"]["s"], "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "bf16 (network) + f64 (FCG)", "data": "synthetic",
        "config": {"workload": (f"learned_l66: L={L} Nt={Nt} ({N} sites), theta pi flux + N(0, 0.3^2) seed "
                                f"{wl.seed}, eta = M^dag R, tol {wl.tol}; network trained at L={Lt} Nt={Ntt}"),
                   "sites": N},
        "solves": res,
        **out,
        "roofline": {"bound": "mfma", "kernel": "k_conv_mfma<true> (one 32->32 3x3x3 layer, BF16 MFMA)",
                     "achieved": achieved, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": (achieved / 2500.0) if achieved else None, "traffic": None,
                     "alg_flops_per_launch": flops, "avg_launch_us": avg_ms * 1e3, "timed_launches": n_k},
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_learned(res["learned"]["iterations"], res["learned"]["switched_at"],
                                                    params, L, Nt)
    print(json.dumps(line), flush=True)


def cpu_baseline_learned(iters, switched, flat_params, L, Nt):
    """Oracle (FP64 numpy network, plain C M^dag M, numpy preconditioner
    twin) on a bounded sample: one network application, one M^dag M and one
    preconditioner application on an 8 x 8 x 80 lattice, scaled per site to
    the evaluation lattice and to the learned solve's iterations (network
    iterations until the switch, the paper's preconditioner after it)."""
    import numpy as np
    import oracle as O
    from oracle import net as NN
    from oracle import precond as PC
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q
    Ls, Nts = 8, 80
    th = inputs.noisy_pi_flux_theta(Ls, Nts, 0.3, 1)
    r = inputs.gauss_cvec(Ls, Nts, 2)
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in Q.Net.unpack(flat_params)]
    p = O.lat(Ls, Nts)
    t0 = time.perf_counter()
    NN.forward(params, th, r)
    t1 = time.perf_counter()
    O.apply_MdagM(p, th, r)
    t2 = time.perf_counter()
    taps, _ = PC.build_stencil(cap=Q.PC_TAU_REACH)
    t3 = time.perf_counter()
    PC.apply_P(taps, r)
    t4 = time.perf_counter()
    scale = (L * L * Nt) / (Ls * Ls * Nts)
    n_net = iters if switched < 0 else switched
    est = scale * (n_net * (t1 - t0) + iters * (t2 - t1) + (iters - n_net) * (t4 - t3))
    return {"value": est, "unit": "s/solve", "cores": 1, "kind": "oracle",
            "sample": (f"oracle FP64 network forward ({t1 - t0:.2f} s), M^dag M ({t2 - t1:.3f} s) and paper "
                       f"preconditioner ({t4 - t3:.2f} s) on L={Ls} Nt={Nts}, scaled per site to L={L} Nt={Nt} and "
                       f"to {iters} iterations ({n_net} with the network) (extrapolation)")}


def host_info():
    """Core count and CPU model of the host the CPU baseline ran on."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def train_learned(lat, net, theta, n_eta=4, steps=600, seed=1003):
    """Setup of the learned path (untimed): the network (initial weights
    seed `seed`) trained with Adam (lr 1e-3, FP32) in residual form on
    residuals r_k = eta - O x_k of the method's own mixed CG solves at the
    starting angles, stopped after k = 0, 50, ..., 1000 iterations, for
    n_eta sources eta = M^dag R; then bound as the handle's learned
    preconditioner (BF16 MFMA inference, the paper's preconditioner as
    fallback)."""
    import numpy as np
    import torch
    from paper_2508_16298_amd import inputs
    t0 = time.perf_counter()
    pool = []
    for k in range(n_eta):
        R = torch.from_numpy(inputs.gauss_cvec(lat.L, lat.Nt, seed + 100 + k)).cuda()
        eta = lat.apply_M(theta, R, dagger=True)
        pool.append(eta)
        for its in range(50, 1050, 50):
            x, _, _, _ = lat.cg_solve(theta, eta, tol=1e-12, maxit=its, prec="fp32")
            pool.append(eta - lat.apply_MdagM(theta, x, prec="fp64"))
    net.set_params(inputs.net_init_weights(seed))
    rng = np.random.default_rng(seed)
    losses = []
    for _ in range(steps):
        loss, _ = net.train_step_residual(theta, pool[int(rng.integers(len(pool)))], lr=1e-3)
        losses.append(loss)
    net.bind("bf16", "paper")
    # one learned solve, untimed: builds the paper's preconditioner (the
    # fallback) and captures the graphs the timed solves replay
    lat.cg_solve(theta, pool[0], tol=1e-8, prec="fp32", precond="learned")
    torch.cuda.synchronize()
    return {"form": "residual |O z - r|^2 / |r|^2 on the method's own CG residuals at the starting angles",
            "residuals": len(pool), "steps": steps, "loss_first": losses[0],
            "loss_last_avg": float(np.mean(losses[-50:])), "setup_s": time.perf_counter() - t0,
            "inference": "bf16 (MFMA)", "fallback": "paper"}


def run_set(lat, theta, th_start, indices, wl, prec, pc):
    """Trajectories with the given indices, each from th_start (restored
    before every one), timed one by one; returns (results, seconds)."""
    import torch
    out, secs = [], []
    for k in indices:
        theta.copy_(th_start)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lat.hmc_trajectory(theta, k, wl.n_steps, wl.traj_len, wl.tol, prec=prec, precond=pc)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        out.append(r)
    return out, secs


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {a.gpus} is not supported (this path has no "
              "multi-GPU sharding: it would shard along tau, with halo slices exchanged between neighbours)", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        return run_copy_calibration()
    if a.workload == "batched_chains":
        return run_batched(a)
    if a.workload == "learned_l66":
        return run_learned(a)
    if a.workload == "se_l24":
        return run_se(a)
    if a.workload == "production_l24":
        return run_production(a)
    if a.solve_only:
        return run_solve_only(a)
    if a.precond_only:
        return run_precond_only(a.precond_only)
    if a.train_only:
        return run_train_only(a.train_only)
    if a.matvec_only:
        print(json.dumps({"matvec_large": matvec_large(only_L=a.matvec_only)}), flush=True)
        return
    import numpy as np
    import torch
    from paper_2508_16298_amd import inputs
    from paper_2508_16298_amd import qedhmc as Q

    wl = inputs.WORKLOADS[a.workload]
    prec = a.prec or wl.precision
    th0 = wl.initial_theta()
    theta = torch.from_numpy(th0).cuda()
    lat = Q.Lattice(wl.L, wl.Nt, dtau=wl.dtau, t=wl.t, J=wl.J, K=wl.K, seed=wl.seed)
    pc = None if a.precond == "none" else a.precond

    # load every kernel once (code objects, LDS attributes) before timing
    v = torch.zeros((wl.Nt, wl.L, wl.L), dtype=torch.complex128, device="cuda")
    v[0, 0, 0] = 1.0
    lat.cg_solve(theta, v, tol=1e-3, maxit=50, prec=prec, precond="paper" if pc == "paper" else None)
    lat.fermion_force(theta, v, prec=prec)
    lat.bosonic_action_force(theta)
    torch.cuda.synchronize()

    # (1) equilibration: a fixed number of chained trajectories (indices
    # 0 .. E-1) from the workload's angles, untimed and independent of
    # --warmup; their end point is the start of every later trajectory
    t_eq = time.perf_counter()
    eq = [lat.hmc_trajectory(theta, k, wl.n_steps, wl.traj_len, wl.tol, prec=prec) for k in range(a.equilibrate)]
    th_start = theta.clone()
    t_eq = time.perf_counter() - t_eq
    net, training = None, None
    if pc == "learned":
        net = Q.Net(lat)
        training = train_learned(lat, net, th_start)

    # (2) warm-up and (3) timed trajectories: each from th_start with its
    # own trajectory index (its own momenta, source and Metropolis draw), so
    # the timed set is a fixed sample whatever --warmup is
    run_set(lat, theta, th_start, [1000 + k for k in range(a.warmup)], wl, prec, pc)
    timed_idx = [2000 + k for k in range(a.steps)]
    lat.profile(a.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, secs = run_set(lat, theta, th_start, timed_idx, wl, prec, pc)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {c: lat.profile_read(c) for c in (Q.K_CG_FP32, Q.K_CG_FP64, Q.K_NET_MFMA, Q.K_MDAGM_FP32,
                                             Q.K_MDAGM_FP64, Q.K_PCG_MV_FP32, Q.K_PCG_MV_FP64,
                                             Q.K_PC_SPEC_FP32, Q.K_PC_SPEC_FP64)}
    lat.profile(0)

    # (4) the same trajectories (same start, same indices) on the other
    # paths: the plain FP64 GPU path, and the mixed path with and without the
    # learned preconditioner; the timed trajectory with the largest |dH| is
    # always among the ones rerun in FP64
    m = min(a.steps, a.compare)
    worst = int(np.argmax([abs(r["dH"]) for r in results]))
    cmp_pos = list(range(m)) + ([worst] if worst >= m else [])
    cmp_idx = [timed_idx[i] for i in cmp_pos]

    def side_by_side(name, p_prec, p_pc):
        rs, ss = run_set(lat, theta, th_start, cmp_idx, wl, p_prec, p_pc)
        rows = []
        for i, r, s_ in zip(cmp_pos, rs, ss):
            rows.append({"traj": timed_idx[i], "dH": r["dH"], "dH_timed_path": results[i]["dH"],
                         "accepted": r["accepted"], "accepted_timed_path": results[i]["accepted"],
                         "cg_iters_total": r["cg_iters_total"], "s": s_, "s_timed_path": secs[i],
                         "status": r["status"], "max_true_resid": r["max_true_resid"],
                         "pc_fallbacks": r.get("pc_fallbacks", 0)})
        t_path = sum(ss[:m]) / m
        t_here = sum(secs[:m]) / m
        return {"path": name, "trajectories": rows, "s_per_traj_first": t_path, "timed_path_s_per_traj_first": t_here,
                "time_ratio_vs_timed_path": t_path / t_here, "first": m}

    paths = {}
    if m == 0:
        pass
    elif not (prec == "fp64" and pc is None):
        paths["fp64"] = side_by_side("plain FP64 GPU path (FP64 CG at the same tolerance)", "fp64", None)
    if m > 0 and a.compare_learned and pc != "learned" and prec != "fp64":
        try:
            with Q.Net(lat) as cnet:
                tr = train_learned(lat, cnet, th_start)
                paths["learned"] = side_by_side("mixed precision + learned preconditioner (flexible CG)", prec,
                                                "learned")
                paths["learned"]["training"] = tr
                cnet.unbind()
        except Q.QedhmcError as e:
            paths["learned"] = {"error": str(e)}
    if m > 0 and pc is not None and prec != "fp64":
        paths["mixed_plain"] = side_by_side("mixed precision, no preconditioner", prec, None)

    # standalone fused M^dag M on the same lattice (the metric's matvec)
    cdt = torch.complex64 if prec != "fp64" else torch.complex128
    vin = torch.from_numpy(inputs.gauss_cvec(wl.L, wl.Nt, 99)).to(cdt).cuda()
    vout = torch.empty_like(vin)
    mv_prec = "fp32" if prec != "fp64" else "fp64"
    lat.apply_MdagM(theta, vin, prec=mv_prec, out=vout)
    lat.profile(1)
    for _ in range(200):
        lat.apply_MdagM(theta, vin, prec=mv_prec, out=vout)
    n_mv, ms_mv = lat.profile_read(Q.K_MDAGM_FP32 if prec != "fp64" else Q.K_MDAGM_FP64)
    lat.profile(0)
    # the same 200 calls between one event pair on the handle's stream
    # (torch's current stream): includes the host's per-call cost and gaps
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(200):
        lat.apply_MdagM(theta, vin, prec=mv_prec, out=vout)
    ev1.record()
    torch.cuda.synchronize()
    b2b_us = 1e3 * ev0.elapsed_time(ev1) / 200

    # the paper preconditioner z = P r, 200 back-to-back applications on the
    # same lattice in the trajectory's launch shape, every launch of its
    # tau-sum + inverse-DFT kernel timed by its own dispatch events (the
    # trajectory's PCG replays captured graphs, which carry no events)
    pc_block = None
    if pc == "paper":
        zin = torch.from_numpy(inputs.gauss_cvec(wl.L, wl.Nt, 98)).to(cdt).cuda()
        zout = torch.empty_like(zin)
        lat.apply_precond(zin, prec=mv_prec, out=zout)
        lat.profile(1)
        for _ in range(200):
            lat.apply_precond(zin, prec=mv_prec, out=zout)
        pc_block = lat.profile_read(Q.K_PC_SPEC_FP32 if prec != "fp64" else Q.K_PC_SPEC_FP64)
        lat.profile(0)

    N = wl.L * wl.L * wl.Nt
    mv_bytes = (24 if prec != "fp64" else 48) * N
    mv_us = 1e3 * ms_mv / max(n_mv, 1)
    mv_gbs = mv_bytes / (mv_us * 1e-6) / 1e9 if n_mv else None
    # the dominant kernel of the timed path and its algorithmic work per launch
    if pc == "learned":
        kcls, work, unit, bound, peak, kname = (Q.K_NET_MFMA, 2.0 * 27 * 32 * 32 * N, "TFLOP/s", "mfma", 2500.0,
                                                "k_conv_mfma<true> (one 32->32 3x3x3 layer, BF16 MFMA)")
    elif pc == "paper":
        # the largest of the PCG iteration's three kernels: the tau sum over
        # 2R + 1 offsets (2 x 2 blocks: 2(2R + 1) complex FMAs per site) and
        # the inverse DFT (L/2 + L complex FMAs per site), 8 flops per complex
        # FMA; 43 flops per algorithmic HBM byte (16 B per site) at R = 12,
        # so vector-ALU bound by the roofline
        kcls = Q.K_PC_SPEC_FP32 if prec != "fp64" else Q.K_PC_SPEC_FP64
        work = 8.0 * (2 * (2 * Q.PC_TAU_REACH + 1) + wl.L // 2 + wl.L) * N
        unit, bound, peak = "TFLOP/s", "alu", (VALU_PEAK_FP32_TFLOPS if prec != "fp64" else VALU_PEAK_FP64_TFLOPS)
        kname = (f"k_pcs_tconv_idft<{'float' if prec != 'fp64' else 'double'}> (spectral paper preconditioner: "
                 f"tau sum + inverse 2D DFT; 200 applications of P back to back)")
    else:
        kcls = Q.K_CG_FP32 if prec != "fp64" else Q.K_CG_FP64
        work, unit, bound, peak = (104 if prec != "fp64" else 176) * N, "GB/s", "hbm", HBM_PEAK_GBS
        kname = f"k_cg_iter<{'float' if prec != 'fp64' else 'double'}> (one fused CG iteration)"
    n_k, ms_k = pc_block if pc == "paper" else prof[kcls]
    avg_ms = ms_k / max(n_k, 1)
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    achieved = work / (avg_ms * 1e-3) / scale if n_k else None
    s_per_traj = elapsed / a.steps
    cg_all = sum(r["cg_iters_total"] for r in results)
    n_solves = results[-1]["n_solves"]
    traffic = {None: CG_ITER_COUNTER_BYTES, "paper": PC_SPEC_COUNTER_BYTES}.get(pc, {}).get(
        "fp32" if prec != "fp64" else "fp64")

    out = {
        "metric": "s per HMC trajectory + M†M matvec HBM GB/s at L=24 Nτ=240, CG resid 1e-8",
        "value": s_per_traj,
        "unit": "s/trajectory",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * s_per_traj,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "c64+f64" if prec != "fp64" else "c128",
        "data": "synthetic",
        "config": {
            "workload": (f"{wl.name}: L={wl.L} Nt={wl.Nt} dtau={wl.dtau} t={wl.t} J={wl.J} K={wl.K}, "
                         f"theta {wl.theta}{' sigma %g' % wl.sigma if wl.sigma else ''} then {a.equilibrate} "
                         f"chained equilibration trajectories; every timed trajectory starts there with its own "
                         f"index; {wl.n_steps} leapfrog steps, length {wl.traj_len}, CG true residual {wl.tol}, "
                         f"{'mixed FP32/FP64' if prec != 'fp64' else 'FP64'}"),
            "L": wl.L, "Nt": wl.Nt, "sites": N, "n_steps": wl.n_steps, "tol": wl.tol,
            "precision": prec, "preconditioner": a.precond, "equilibration_trajectories": a.equilibrate,
            "timed_traj_indices": [timed_idx[0], timed_idx[-1]],
        },
        "s_per_traj_each": secs,
        "cg_iters_per_traj": cg_all / a.steps,
        "s_per_cg_iter": elapsed / max(cg_all, 1),
        "equilibration": {"trajectories": a.equilibrate, "s": t_eq,
                          "dH": [r["dH"] for r in eq], "accepted": [r["accepted"] for r in eq],
                          "cg_iters_total": [r["cg_iters_total"] for r in eq]},
        "matvec_gbs": mv_gbs,
        "matvec": {"kernel": f"k_mdagm<{'float' if prec != 'fp64' else 'double'}> (standalone fused M^dag M)",
                   "avg_launch_us": mv_us, "alg_bytes_per_launch": mv_bytes, "gbs": mv_gbs,
                   "frac_of_hbm_peak": (mv_gbs / HBM_PEAK_GBS) if mv_gbs else None, "launches": n_mv,
                   "timing": "start/end events of each dispatch (hipExtLaunchKernelGGL)",
                   "host_driven_back_to_back_us": b2b_us},
        "traj": [{"traj": timed_idx[i], **{k: r[k] for k in ("dH", "accepted", "cg_iters_total", "cg_iters_max",
                                                             "reliable_updates", "max_true_resid", "status",
                                                             "pc_fallbacks")}}
                 for i, r in enumerate(results)],
        "worst_dH_traj": timed_idx[worst],
        "paths": paths,
        "roofline": {
            "bound": bound,
            "kernel": kname,
            "achieved": achieved,
            "peak": peak,
            "unit": unit,
            "frac": (achieved / peak) if achieved else None,
            "traffic": traffic,
            "alg_work_per_launch": work,
            "avg_launch_us": avg_ms * 1e3,
            "timed_launches": n_k,
        },
    }
    if training:
        out["training"] = training
    if net is not None:
        net.close()
    lat.close()
    out["matvec_large"] = matvec_large()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, th_start.cpu().numpy(), cg_all / a.steps, n_solves, a.cpu_iters, pc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
