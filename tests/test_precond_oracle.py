"""Pins of the oracle twin of the paper's preconditioner (Methods, "CG method
and preconditioner"; Fig. 3).  The paper prints no entries or iteration
counts, so the stencil's values are parity unpinned against the paper; what
is pinned: G is non-singular (P = G^dag G Hermitian positive definite), the
band is 0 <= dtau <= 6 in G (+-6 in P), the dagger pass is the adjoint, the
factor reproduces O_pi on its pattern, and PCG keeps the solution while
cutting iterations."""
import functools

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from oracle import precond as PC
from paper_2508_16298_amd import inputs


@functools.lru_cache(maxsize=1)
def _taps():
    return PC.build_stencil(8, 24)


def test_ic0_reproduces_matrix_on_pattern():
    p = O.lat(4, 6)
    A = O.dense_MdagM(p, PC.pi_flux_theta(4, 6))
    Lf, shift = PC.ic0_forward(A)
    assert shift == 0.0
    assert np.allclose(np.triu(Lf, 1), 0)
    pat = np.abs(A) > 1e-12 * np.abs(A).max()
    R = Lf @ Lf.conj().T - A
    assert np.abs(R[pat]).max() < 1e-12 * np.abs(A).max()     # exact on the pattern (IC(0))
    assert np.abs(R).max() > 1e-6                               # ... and incomplete off it


def test_stencil_shape_and_band():
    taps, shift = _taps()
    for par in (0, 1):
        t = taps[par]
        assert 100 < len(t) < 400
        assert min(e[0] for e in t) == 0 and max(e[0] for e in t) <= 6
        assert all(abs(e[3]) >= 1e-3 for e in t)
        d0 = [e for e in t if e[0] == 0 and e[1] == 0 and e[2] == 0]
        assert len(d0) == 1 and d0[0][3].real > 0          # diagonal of L^{-1} is 1 / L_ii > 0


def test_G_nonsingular_P_hpd_band_and_adjoint():
    taps, _ = _taps()
    L, Nt = 8, 8
    G = PC.dense_G(taps, L, Nt)
    Vs = L * L
    tau = np.repeat(np.arange(Nt), Vs)
    d = (tau[:, None] - tau[None, :]) % Nt
    assert np.abs(G[d > 6]).max() == 0.0                        # band 0 <= dtau <= 6 (with wrap)
    smin = sla.svdvals(G).min()
    assert smin > 0.05, smin
    P = G.conj().T @ G
    ev = np.linalg.eigvalsh(P)
    assert ev.min() > 0
    v = inputs.gauss_cvec(L, Nt, 3)
    w = inputs.gauss_cvec(L, Nt, 4)
    lhs = np.vdot(w.reshape(-1), PC.apply_G(taps, v).reshape(-1))
    rhs = np.vdot(PC.apply_G(taps, w, dagger=True).reshape(-1), v.reshape(-1))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert np.abs(PC.apply_G(taps, v).reshape(-1) - G @ v.reshape(-1)).max() < 1e-12
    assert np.abs(PC.apply_G(taps, v, dagger=True).reshape(-1) - G.conj().T @ v.reshape(-1)).max() < 1e-12
    assert np.abs(PC.apply_P(taps, v).reshape(-1) - P @ v.reshape(-1)).max() < 1e-12


@pytest.mark.parametrize("which", ["pi", "noisy", "hot"])
def test_pcg_keeps_solution_and_cuts_iterations(which):
    taps, _ = _taps()
    L, Nt = 8, 24
    p = O.lat(L, Nt)
    th = {"pi": inputs.pi_flux_theta(L, Nt), "noisy": inputs.noisy_pi_flux_theta(L, Nt, 0.3, 5),
          "hot": inputs.hot_start_theta(L, Nt, 5)}[which]
    eta = O.apply_M(p, th, inputs.gauss_cvec(L, Nt, 7), dagger=True)
    X0, _, it0, _ = O.cg_solve(p, th, eta, tol=1e-10)
    X1, st, it1, rel = O.cg_solve(p, th, eta, tol=1e-10,
                                  precond=lambda r: PC.apply_P(taps, r.reshape(Nt, L, L)).reshape(-1))
    assert st == 0 and rel <= 1e-10
    assert it1 < 0.6 * it0, (it0, it1)
    assert np.linalg.norm(X1 - X0) <= 1e-6 * np.linalg.norm(X0)
