"""Oracle twin of the paper's preconditioner (Methods, "CG method and
preconditioner"; banded structure of Fig. 3).  TEST INFRASTRUCTURE ONLY.

The paper: incomplete Cholesky of O = M^dag M at a pi-flux configuration,
an approximate inverse of the factor, entries below 1e-3 truncated, the
result Otilde^{-1} = L^{-1} L^{-dagger} reused for every theta and (its bulk
entries) for every lattice size; bandwidth 6 in tau.  Taken literally
(reversed-order IC(0), the 20-term series 1 + (1-L) + (1-L)^2 + ... for
L^{-1}, truncation of the product) the result is not positive definite, so
the reading followed here, step by step:

1. O_pi = M^dag M on a small build lattice L0 x L0 x Nt0 at pi flux
   (theta_x = 0, theta_y = pi x: flux pi through every plaquette).
2. Forward IC(0) in the natural order n = tau*Vs + s: O_pi ~ L L^dag with L
   lower triangular on the sparsity pattern of O_pi, the entries with
   |O| > 1e-12 max|O| (a diagonal shift of the matrix when a pivot is not
   positive).
3. G = L^{-1} exactly, by triangular solves (the series is meant to
   approximate this).
4. From an interior site of a bulk slice, one per x parity (the pi-flux unit
   cell is two sites wide), keep the entries of G's row with
   0 <= dtau <= cap and |G| >= thresh, as taps (dtau, dx, dy, value).
5. On the target lattice G[(tau,s),(tau-dtau, s+ds)] = g_{x(s) mod 2}(dtau, ds),
   times -1 when tau - dtau wraps below 0 (M is antiperiodic in tau).
6. P = G^dag G, applied as two stencil passes; Hermitian positive definite
   whenever G is non-singular, and banded +-cap in tau.
"""
import numpy as np
import scipy.linalg as sla

from . import dense_MdagM, lat


def pi_flux_theta(L, Nt):
    th = np.zeros((2, Nt, L, L))
    th[1] = np.pi * np.arange(L)[None, None, :]
    return th


def ic0_forward(A):
    """Incomplete Cholesky IC(0), natural order, A ~ L L^dag with L lower
    triangular on the lower pattern of A.  Returns (L, shift) where shift is
    the diagonal shift (fraction of diag(A)) that made every pivot positive."""
    n = A.shape[0]
    pattern = np.abs(A) > 1e-12 * np.abs(A).max()
    shift = 0.0
    while True:
        As = A + shift * np.diag(np.diag(A))
        L = np.zeros_like(As)
        ok = True
        for k in range(n):
            # left-looking column k: L[k:, k] = (A[k:, k] - L[k:, :k] conj(L[k, :k])) / L[k, k]
            col = As[k:, k] - L[k:, :k] @ np.conj(L[k, :k])
            piv = col[0].real
            if not piv > 0:
                ok = False
                break
            d = np.sqrt(piv)
            col = col / d
            col[0] = d
            col[~pattern[k:, k]] = 0.0   # drop fill outside the pattern of A
            L[k:, k] = col
        if ok:
            return L, shift
        shift = 1e-3 if shift == 0.0 else 2 * shift
        if shift > 1.0:
            raise ValueError("IC(0) pivots stay non-positive")


def build_stencil(L0=8, Nt0=24, dtau=0.1, t=1.0, cap=6, thresh=1e-3, tau0=None):
    """Taps per x parity: list over parity p of arrays (dtau, dx, dy, g)."""
    p = lat(L0, Nt0, dtau, t)
    Vs = L0 * L0
    O = dense_MdagM(p, pi_flux_theta(L0, Nt0))
    Lf, shift = ic0_forward(O)
    G = sla.solve_triangular(Lf, np.eye(O.shape[0], dtype=complex), lower=True)
    tau0 = Nt0 // 2 + 4 if tau0 is None else tau0
    y0 = L0 // 2
    taps = []
    for par in (0, 1):
        x0 = L0 // 2 + par
        row = G[tau0 * Vs + y0 * L0 + x0]
        out = []
        for m in np.nonzero(np.abs(row) >= thresh)[0]:
            tm, sm = divmod(int(m), Vs)
            dt = tau0 - tm
            if not 0 <= dt <= cap:
                continue
            dx = (sm % L0 - x0 + L0 // 2) % L0 - L0 // 2
            dy = (sm // L0 - y0 + L0 // 2) % L0 - L0 // 2
            out.append((dt, dx, dy, row[m]))
        out.sort(key=lambda e: (e[0], e[2], e[1]))
        taps.append(out)
    return taps, shift


def apply_G(taps, v, dagger=False):
    """(G v) or (G^dag v) on a target lattice; v complex (Nt, L, L)."""
    Nt, L, _ = v.shape
    out = np.zeros_like(v)
    xpar = (np.arange(L) % 2)[None, None, :]
    tau = np.arange(Nt)[:, None, None]
    for par in (0, 1):
        for dt, dx, dy, g in taps[par]:
            if not dagger:
                # out[tau, y, x] += g * v[tau - dt, y + dy, x + dx] * sign, rows of parity par
                src = np.roll(v, shift=(dt, -dy, -dx), axis=(0, 1, 2))
                sign = np.where(tau - dt < 0, -1.0, 1.0)
                out += np.where(xpar == par, g * sign * src, 0.0)
            else:
                # out[tau, y, x] += conj(g) * v[tau + dt, y - dy, x - dx] * sign, the row
                # (tau + dt, y - dy, x - dx) being of parity par
                src = np.roll(v, shift=(-dt, dy, dx), axis=(0, 1, 2))
                rowpar = (np.arange(L)[None, None, :] - dx) % 2
                sign = np.where(tau + dt >= Nt, -1.0, 1.0)
                out += np.where(rowpar == par, np.conj(g) * sign * src, 0.0)
    return out


def apply_P(taps, r):
    """z = G^dag (G r) on flat or (Nt, L, L) complex vectors of a lattice whose
    shape is taken from r (flat vectors need `shape`)."""
    return apply_G(taps, apply_G(taps, r), dagger=True)


def dense_G(taps, L, Nt):
    """G as a dense matrix, scattered entry by entry from the taps (a second,
    loop-based reading of the definition used by apply_G)."""
    Vs = L * L
    N = Vs * Nt
    G = np.zeros((N, N), dtype=complex)
    for tau in range(Nt):
        for y in range(L):
            for x in range(L):
                row = tau * Vs + y * L + x
                for dt, dx, dy, g in taps[x % 2]:
                    ts = tau - dt
                    sign = -1.0 if ts < 0 else 1.0
                    col = (ts % Nt) * Vs + ((y + dy) % L) * L + (x + dx) % L
                    G[row, col] += sign * g
    return G
