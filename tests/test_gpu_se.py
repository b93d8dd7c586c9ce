"""GPU parity of the stochastic estimation (Methods, "Stochastic estimation
of fermionic observables", Eq. Cij_est; Supplemental Material SIV) against
the oracle: probes, the multi-RHS solve (true residuals recomputed by the
oracle), the FFT-averaged spin correlator on identical inputs, and the whole
measurement end to end.  Bars: probes 1e-13 (Box-Muller through device and
host libm); correlator on identical probes and solutions 1e-12 of max |C|
(FP64 DFTs in a different summation order than numpy's FFT); end to end
from the GPU's own solves 1e3 x tol of max |C| (C is bilinear in X, whose
error is bounded by the residual times the condition number; the lattices
here are small and well conditioned)."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from oracle import se as SE
from paper_2508_16298_amd import inputs
from paper_2508_16298_amd import qedhmc as Q

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _theta(L, Nt, seed):
    return inputs.noisy_pi_flux_theta(L, Nt, 0.3, seed)


@pytest.mark.parametrize("L,Nt,n_rv", [(4, 6, 3), (6, 10, 5), (24, 240, 2)])
def test_probes_match_oracle(L, Nt, n_rv):
    p = O.lat(L, Nt)
    with Q.Stochastic(L, Nt, n_rv, seed=77) as se:
        xi = _host(se.probes(meas=5))
    ref = O.probes(p, seed=77, meas=5, n_rv=n_rv)
    assert np.abs(xi - ref).max() < 1e-13


@pytest.mark.parametrize("L,Nt,n_rv,pairs", [(2, 4, 3, None), (4, 6, 4, 2), (6, 10, 5, None), (12, 40, 4, 4),
                                             (8, 36, 6, 5)])
def test_spin_correlator_on_oracle_inputs(L, Nt, n_rv, pairs):
    """The GPU estimator on the oracle's probes and solutions; pairs forces
    the pair passes (ragged last pass) through QEDHMC_SE_PAIRS."""
    p = O.lat(L, Nt)
    th = _theta(L, Nt, 300 + L)
    xi = O.probes(p, seed=3, meas=1, n_rv=n_rv)
    X = SE.solve_probes(p, th, xi, tol=1e-12)
    ref = SE.spin_correlator_se(p, xi, X)
    if pairs:
        os.environ["QEDHMC_SE_PAIRS"] = str(pairs)
    try:
        with Q.Stochastic(L, Nt, n_rv) as se:
            print(f"spin correlator L={L} Nt={Nt} n_rv={n_rv} pairs/pass {pairs}", flush=True)
            C = _host(se.spin_correlator(_dev(xi), _dev(X)))
    finally:
        os.environ.pop("QEDHMC_SE_PAIRS", None)
    err = np.abs(C - ref).max() / np.abs(ref).max()
    print(f"  max rel err {err:.2e}", flush=True)
    assert err < 1e-12


def test_unit_vector_probes_on_the_gpu():
    """Probes sqrt(N) e_l through the GPU solve and estimator reproduce the
    exact identity of the unit-vector pin: T1 exact, N/(N-1) T2 at Delta != 0,
    T2(0) = 0 (the GPU's X within its residual)."""
    L, Nt = 2, 4
    p = O.lat(L, Nt)
    N = p.N
    th = inputs.hot_start_theta(L, Nt, 31)
    G = SE.green_exact(p, th)
    xi = (np.sqrt(N) * np.eye(N)).reshape(N, Nt, L, L).astype(np.complex128)
    with Q.Stochastic(L, Nt, N) as se:
        X, st, it, rel = se.solve(_dev(th), _dev(xi), tol=1e-12, prec="fp64")
        assert st == Q.OK and rel.max() <= 1e-12
        C = _host(se.spin_correlator(_dev(xi), X)).reshape(-1)
    exact = SE.spin_correlator_exact(p, th).reshape(-1)
    T1 = np.trace(G) / N
    want = (N / (N - 1)) * exact
    want[0] = T1
    assert np.abs(C - want).max() < 1e-9 * np.abs(want).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-8)])
def test_measurement_end_to_end(prec, tol):
    """Probes, multi-RHS solve and estimator on the GPU vs the oracle's whole
    measurement on the same seed: per-probe true residuals recomputed by the
    oracle, solutions against the single-RHS solver, correlator 1e3 x tol."""
    L, Nt, n_rv = 8, 40, 6
    p = O.lat(L, Nt)
    th = _theta(L, Nt, 41)
    xi_o = O.probes(p, seed=123, meas=9, n_rv=n_rv)
    X_o = SE.solve_probes(p, th, xi_o, tol=1e-13)
    ref = SE.spin_correlator_se(p, xi_o, X_o)
    thd = _dev(th)
    with Q.Stochastic(L, Nt, n_rv, seed=123) as se:
        xi = se.probes(meas=9)
        X, st, it, rel = se.solve(thd, xi, tol=tol, prec=prec)
        C = _host(se.spin_correlator(xi, X))
        Xh, xih = _host(X), _host(xi)
    print(f"{prec}: iterations {it.tolist()}, residuals {rel.max():.2e}", flush=True)
    assert st == Q.OK and rel.max() <= tol
    for k in range(n_rv):
        eta = O.apply_M(p, th, xih[k], dagger=True)
        true = np.linalg.norm(eta.reshape(-1) - O.apply_MdagM(p, th, Xh[k]).reshape(-1)) / np.linalg.norm(eta)
        assert true <= 1.05 * tol, (k, true)
    with Q.Lattice(L, Nt) as lat:
        for k in (0, n_rv - 1):
            eta = lat.apply_M(thd, _dev(xih[k]), dagger=True)
            xs, sts, its, rels = lat.cg_solve(thd, eta, tol=tol, prec=prec)
            d = O.apply_MdagM(p, th, Xh[k] - _host(xs))
            assert np.linalg.norm(d) <= (rel[k] + rels) * np.linalg.norm(_host(eta)) * 1.01
    err = np.abs(C - ref).max() / np.abs(ref).max()
    print(f"  correlator max rel err {err:.2e}", flush=True)
    assert err < 1e3 * tol


def test_full_size_measurement_is_consistent():
    """L=24, Nt=240 (the benchmark lattice) with 8 probes: every probe's true
    residual (oracle), and the GPU estimator against the oracle's estimator
    on the GPU's own probes and solutions (1e-12)."""
    L, Nt, n_rv = 24, 240, 8
    p = O.lat(L, Nt)
    wl = inputs.WORKLOADS["mixed_l24"]
    th = wl.initial_theta()
    with Q.Stochastic(L, Nt, n_rv, seed=2024) as se:
        xi = se.probes(meas=0)
        print("full-size multi-RHS solve", flush=True)
        X, st, it, rel = se.solve(_dev(th), xi, tol=1e-8, prec="fp32")
        C = _host(se.spin_correlator(xi, X))
        Xh, xih = _host(X), _host(xi)
    print(f"iterations {it.tolist()}, residuals {rel.max():.2e}", flush=True)
    assert st == Q.OK and rel.max() <= 1e-8
    for k in (0, n_rv - 1):
        eta = O.apply_M(p, th, xih[k], dagger=True)
        true = np.linalg.norm(eta.reshape(-1) - O.apply_MdagM(p, th, Xh[k]).reshape(-1)) / np.linalg.norm(eta)
        assert true <= 1.05e-8
    ref = SE.spin_correlator_se(p, xih, Xh)
    assert np.abs(C - ref).max() < 1e-12 * np.abs(ref).max()


def test_solve_reports_nonconvergence_and_rejects_bad_arguments():
    L, Nt, n_rv = 6, 10, 3
    th = _dev(inputs.hot_start_theta(L, Nt, 8))
    with Q.Stochastic(L, Nt, n_rv, seed=1) as se:
        xi = se.probes(meas=0)
        X, st, it, rel = se.solve(th, xi, tol=1e-12, maxit=3, prec="fp64")
        assert st == Q.ENOCONV and (it == 3).all()
        with pytest.raises(Q.QedhmcError):
            se.solve(th, xi, tol=0.0)
    with pytest.raises(Q.QedhmcError):
        Q.Stochastic(L, Nt, 1)
    with pytest.raises(Q.QedhmcError):
        Q.Stochastic(46, 4, 2)
