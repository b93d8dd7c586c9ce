"""Oracle of the stochastic estimation of fermionic observables (Methods,
"Stochastic estimation of fermionic observables", Eq. Cij_est and the FFT
translational average after it; Supplemental Material SIV for the spin
correlator).  TEST INFRASTRUCTURE ONLY: imported by tests/ and bench.py's CPU
baseline, never by the product library.

Arrays: vectors complex128 (Nt, L, L); probe sets (n_rv, Nt, L, L);
correlators C[dtau, dy, dx] of the space-time displacement Delta.

Definitions (G = M^{-1}, the fermion Green's function of a fixed gauge
configuration; both flavours share it):

  spin correlator  C_S(i, j) = Gbar(i, j) G(i, j),  Gbar(i, j) = delta_ij - G(j, i)
                   (SIV, C_S^{up down})
  translational average  C(Delta) = (1/N) sum_i C(i, i + Delta), i + Delta on
                   the periodic space-time torus (the two Green's functions of
                   a bilinear carry the antiperiodic sign twice).

So C_S(Delta) = delta_{Delta,0} T1 - T2(Delta), T1 = (1/N) sum_i G(i,i),
T2(Delta) = (1/N) sum_i G(i+Delta, i) G(i, i+Delta).

Estimator from probes xi_p (E[xi^* xi^T] = 1) and X_p = G xi_p, computed as
the paper does, X_p = (M^dag M)^{-1} M^dag xi_p:
  T1 ~ (1/(n_rv N)) sum_p sum_i X_{p,i} conj(xi_{p,i});
  T2 ~ average over ordered pairs p != q of (1/N) sum_i a_i b_{i+Delta} with
       a = X_p conj(xi_q), b = X_q conj(xi_p)  (Eq. Cij_est: G(i,j) from probe
       p, G(j,i) from probe q, so the estimate is unbiased);
  each term is a correlation, evaluated with FFTs:
       (1/N) sum_i a_i b_{i+Delta} = (1/N^2) sum_k A_{-k} B_k e^{+i k.Delta}.
Swapping p and q swaps a and b and mirrors Delta, so the ordered-pair average
is 1/(n_rv (n_rv - 1)) times the sum over p < q of the Delta and -Delta terms.
"""
import numpy as np

from . import apply_M, cg_solve, dense_M


def green_exact(p, theta):
    """G = M^{-1} by dense inversion (tiny lattices only)."""
    return np.linalg.inv(dense_M(p, theta))


def _shift_index(p):
    """j[d, i]: flat site i shifted by every displacement d (flat over (dtau, dy, dx))."""
    Nt, L = p.Nt, p.L
    t, y, x = np.meshgrid(np.arange(Nt), np.arange(L), np.arange(L), indexing="ij")
    t, y, x = t.reshape(-1), y.reshape(-1), x.reshape(-1)
    out = np.empty((p.N, p.N), dtype=np.int64)
    for d in range(p.N):
        dt, dy, dx = d // (L * L), (d // L) % L, d % L
        out[d] = ((t + dt) % Nt) * L * L + ((y + dy) % L) * L + (x + dx) % L
    return out


def spin_correlator_exact(p, theta):
    """C_S(Delta) from the dense Green's function (the plain definition)."""
    G = green_exact(p, theta)
    N = p.N
    j = _shift_index(p)
    i = np.arange(N)
    C = np.empty(N, dtype=np.complex128)
    for d in range(N):
        C[d] = -np.sum(G[j[d], i] * G[i, j[d]]) / N
    C[0] += np.trace(G) / N
    return C.reshape(p.Nt, p.L, p.L)


def solve_probes(p, theta, xi, tol=1e-12):
    """X_p = (M^dag M)^{-1} M^dag xi_p for every probe (the oracle's CG)."""
    X = np.empty_like(xi)
    for k in range(xi.shape[0]):
        R = apply_M(p, theta, xi[k], dagger=True)
        x, st, _, _ = cg_solve(p, theta, R, tol=tol)
        assert st == 0
        X[k] = x.reshape(p.Nt, p.L, p.L)
    return X


def _mirror(A):
    """A_{-k}: index k -> -k mod n on every axis."""
    for ax in range(A.ndim):
        A = np.roll(np.flip(A, axis=ax), 1, axis=ax)
    return A


def spin_correlator_se(p, xi, X):
    """The stochastic estimate of C_S(Delta) with FFT averaging."""
    n_rv = xi.shape[0]
    assert n_rv >= 2
    N = p.N
    T1 = np.sum(X * np.conj(xi)) / (n_rv * N)
    S = np.zeros((p.Nt, p.L, p.L), dtype=np.complex128)
    for a_ in range(n_rv):
        for b_ in range(a_ + 1, n_rv):
            A = np.fft.fftn(X[a_] * np.conj(xi[b_]))
            B = np.fft.fftn(X[b_] * np.conj(xi[a_]))
            S += _mirror(A) * B + A * _mirror(B)
    # sum_k S_k e^{+ik.Delta} = N ifftn(S)
    T2 = np.fft.ifftn(S) * N / (n_rv * (n_rv - 1) * N * N)
    C = -T2
    C[0, 0, 0] += T1
    return C


def spin_correlator_se_direct(p, xi, X):
    """The same estimate by the O(N^2) direct sums (brute force, tiny lattices)."""
    n_rv = xi.shape[0]
    N = p.N
    j = _shift_index(p)
    i = np.arange(N)
    Xf, xf = X.reshape(n_rv, N), xi.reshape(n_rv, N)
    T1 = 0.0
    for a_ in range(n_rv):
        T1 += np.sum(Xf[a_] * np.conj(xf[a_]))
    T1 /= n_rv * N
    T2 = np.zeros(N, dtype=np.complex128)
    for a_ in range(n_rv):
        for b_ in range(n_rv):
            if a_ == b_:
                continue
            a = Xf[a_] * np.conj(xf[b_])
            b = Xf[b_] * np.conj(xf[a_])
            for d in range(N):
                T2[d] += np.sum(a[i] * b[j[d]]) / N
    T2 /= n_rv * (n_rv - 1)
    C = -T2
    C[0] += T1
    return C.reshape(p.Nt, p.L, p.L)
