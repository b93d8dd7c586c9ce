"""Plain FP64 CPU oracle for the HQMC hot path of lattice QED3.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product library.  It wraps
``qed_oracle.c`` (built into ``liboracle.so`` by ``build_oracle.py``) with
numpy arrays and adds the dense-matrix views used by the pins:

* vectors are complex128 arrays of shape (Nt, L, L) or flat (N,)
* theta is a float64 array of shape (2, Nt, L, L) (d, tau, y, x)

Each function names the passage of the paper it implements in the C source.
"""
import ctypes as C
import os

import numpy as np

from . import build_oracle

_LIB = None


class Lat(C.Structure):
    """Lattice and couplings (Methods, Model and partition function)."""
    _fields_ = [("L", C.c_int32), ("Nt", C.c_int32), ("dtau", C.c_double),
                ("t", C.c_double), ("J", C.c_double), ("K", C.c_double),
                ("noncompact", C.c_int32)]

    @property
    def Vs(self):
        return self.L * self.L

    @property
    def N(self):
        return self.L * self.L * self.Nt


class Traj(C.Structure):
    _fields_ = [("dH", C.c_double), ("H0", C.c_double), ("H1", C.c_double),
                ("SB0", C.c_double), ("SB1", C.c_double), ("SF0", C.c_double),
                ("SF1", C.c_double), ("K0", C.c_double), ("K1", C.c_double),
                ("u", C.c_double), ("accepted", C.c_int32), ("n_solves", C.c_int32),
                ("cg_iters_total", C.c_int32), ("cg_iters_max", C.c_int32),
                ("status", C.c_int32), ("max_true_resid", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PRECOND_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

_P = C.c_void_p


def lib():
    global _LIB
    if _LIB is None:
        path = build_oracle.LIB
        src = build_oracle.SRC
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            build_oracle.build()
        L = C.CDLL(path)
        LP = C.POINTER(Lat)
        L.oracle_bond_tables.argtypes = [C.c_int32, _P]
        L.oracle_apply_B.argtypes = [LP, _P, C.c_int32, _P, _P]
        L.oracle_apply_factor.argtypes = [LP, _P, C.c_int32, C.c_int32, C.c_double, _P]
        L.oracle_apply_M.argtypes = [LP, _P, _P, _P, C.c_int32]
        L.oracle_apply_MdagM.argtypes = [LP, _P, _P, _P]
        L.oracle_cg_solve.argtypes = [LP, _P, _P, _P, C.c_double, C.c_int32, _P, _P]
        L.oracle_cg_solve.restype = C.c_int32
        L.oracle_cg_solve_pc.argtypes = [LP, _P, _P, _P, C.c_double, C.c_int32,
                                         PRECOND_FN, _P, _P, _P]
        L.oracle_cg_solve_pc.restype = C.c_int32
        L.oracle_fermion_force.argtypes = [LP, _P, _P, _P]
        L.oracle_bosonic_action.argtypes = [LP, _P]
        L.oracle_bosonic_action.restype = C.c_double
        L.oracle_bosonic_force.argtypes = [LP, _P, _P]
        L.oracle_philox4x32_10.argtypes = [_P, _P, _P]
        L.oracle_heatbath.argtypes = [LP, C.c_uint64, C.c_uint64, _P, _P]
        L.oracle_metropolis_uniform.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_probes.argtypes = [LP, C.c_uint64, C.c_uint64, C.c_int32, _P]
        L.oracle_metropolis_uniform.restype = C.c_double
        L.oracle_hmc_trajectory.argtypes = [LP, _P, C.c_uint64, C.c_uint64, C.c_int32,
                                            C.c_double, C.c_double, C.c_int32,
                                            C.POINTER(Traj), _P, _P, _P]
        L.oracle_hmc_trajectory_pc.argtypes = [LP, _P, C.c_uint64, C.c_uint64, C.c_int32,
                                               C.c_double, C.c_double, C.c_int32,
                                               PRECOND_FN, _P, C.POINTER(Traj), _P, _P, _P]
        L.oracle_leapfrog.argtypes = [LP, _P, _P, _P, C.c_int32, C.c_double, C.c_double,
                                      C.c_int32, _P, _P]
        _LIB = L
    return _LIB


def lat(L, Nt, dtau=0.1, t=1.0, J=1.0, K=1.0, noncompact=False):
    """Lattice and couplings; noncompact selects the gauge action L_B^nc of
    Results, Eq. (3) instead of the compact L_B^c."""
    return Lat(L, Nt, dtau, t, J, K, 1 if noncompact else 0)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _cvec(v, p):
    v = np.ascontiguousarray(v, dtype=np.complex128)
    assert v.size == p.N, (v.shape, p.N)
    return v


def _th(theta, p):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    assert theta.size == 2 * p.N, (theta.shape, p.N)
    return theta


def bond_tables(L):
    """int32 [4][L*L/2][3] rows (i, j, d*Vs + s) per family f0..f3."""
    out = np.zeros((4, L * L // 2, 3), dtype=np.int32)
    lib().oracle_bond_tables(L, _ptr(out))
    return out


def apply_B(p, theta, tau, v):
    """B_tau v for one slice v of shape (L, L) or (Vs,)."""
    th = _th(theta, p)
    v = np.ascontiguousarray(v, dtype=np.complex128)
    out = np.empty_like(v)
    lib().oracle_apply_B(C.byref(p), _ptr(th), tau, _ptr(v), _ptr(out))
    return out


def apply_factor(p, theta, tau, f, a, v):
    th = _th(theta, p)
    out = np.array(v, dtype=np.complex128, copy=True, order="C")
    lib().oracle_apply_factor(C.byref(p), _ptr(th), tau, f, a, _ptr(out))
    return out


def apply_M(p, theta, v, dagger=False):
    th, v = _th(theta, p), _cvec(v, p)
    out = np.empty_like(v)
    lib().oracle_apply_M(C.byref(p), _ptr(th), _ptr(v), _ptr(out), int(bool(dagger)))
    return out


def apply_MdagM(p, theta, v):
    th, v = _th(theta, p), _cvec(v, p)
    out = np.empty_like(v)
    lib().oracle_apply_MdagM(C.byref(p), _ptr(th), _ptr(v), _ptr(out))
    return out


def cg_solve(p, theta, rhs, tol=1e-10, maxit=1_000_000, precond=None):
    """Returns (X, status, iters, true_rel_resid).  ``precond`` is an optional
    python callable z = precond(r) on flat complex arrays."""
    th, rhs = _th(theta, p), _cvec(rhs, p)
    X = np.zeros_like(rhs)
    it = C.c_int32(0)
    rel = C.c_double(0.0)
    if precond is None:
        st = lib().oracle_cg_solve(C.byref(p), _ptr(th), _ptr(rhs), _ptr(X), tol, maxit,
                                   C.byref(it), C.byref(rel))
    else:
        n = p.N

        def _cb(_ctx, rp, zp):
            r = np.ctypeslib.as_array(C.cast(rp, C.POINTER(C.c_double)), shape=(2 * n,))
            z = np.ctypeslib.as_array(C.cast(zp, C.POINTER(C.c_double)), shape=(2 * n,))
            zc = np.asarray(precond(r.view(np.complex128).copy()), dtype=np.complex128)
            z[:] = zc.reshape(-1).view(np.float64)

        cb = PRECOND_FN(_cb)
        st = lib().oracle_cg_solve_pc(C.byref(p), _ptr(th), _ptr(rhs), _ptr(X), tol, maxit,
                                      cb, None, C.byref(it), C.byref(rel))
    return X, int(st), int(it.value), float(rel.value)


def fermion_force(p, theta, X):
    """F = -dS_F/dtheta, shape of theta."""
    th, X = _th(theta, p), _cvec(X, p)
    F = np.zeros_like(th)
    lib().oracle_fermion_force(C.byref(p), _ptr(th), _ptr(X), _ptr(F))
    return F


def bosonic_action(p, theta):
    return float(lib().oracle_bosonic_action(C.byref(p), _ptr(_th(theta, p))))


def bosonic_force(p, theta):
    th = _th(theta, p)
    F = np.zeros_like(th)
    lib().oracle_bosonic_force(C.byref(p), _ptr(th), _ptr(F))
    return F


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def heatbath(p, seed, traj):
    mom = np.zeros((2, p.Nt, p.L, p.L), dtype=np.float64)
    R = np.zeros((p.Nt, p.L, p.L), dtype=np.complex128)
    lib().oracle_heatbath(C.byref(p), seed, traj, _ptr(mom), _ptr(R))
    return mom, R


def probes(p, seed, meas, n_rv):
    """Probe vectors of the stochastic estimation: complex128 (n_rv, Nt, L, L)."""
    assert n_rv * p.N < 2 ** 32
    xi = np.zeros((n_rv, p.Nt, p.L, p.L), dtype=np.complex128)
    lib().oracle_probes(C.byref(p), seed, meas, n_rv, _ptr(xi))
    return xi


def metropolis_uniform(seed, traj):
    return float(lib().oracle_metropolis_uniform(seed, traj))


def hmc_trajectory(p, theta, seed, traj, n_steps, traj_len=1.0, tol=1e-10,
                   maxit=1_000_000, precond=None):
    """One trajectory; returns (theta_out, result dict, mom0, R, eta)."""
    th = np.array(_th(theta, p), copy=True)
    res = Traj()
    mom = np.zeros_like(th)
    R = np.zeros(p.N, dtype=np.complex128)
    eta = np.zeros(p.N, dtype=np.complex128)
    if precond is None:
        lib().oracle_hmc_trajectory(C.byref(p), _ptr(th), seed, traj, n_steps, traj_len,
                                    tol, maxit, C.byref(res), _ptr(mom), _ptr(R), _ptr(eta))
    else:
        n = p.N

        def _cb(_ctx, rp, zp):
            r = np.ctypeslib.as_array(C.cast(rp, C.POINTER(C.c_double)), shape=(2 * n,))
            z = np.ctypeslib.as_array(C.cast(zp, C.POINTER(C.c_double)), shape=(2 * n,))
            zc = np.asarray(precond(r.view(np.complex128).copy()), dtype=np.complex128)
            z[:] = zc.reshape(-1).view(np.float64)

        cb = PRECOND_FN(_cb)
        lib().oracle_hmc_trajectory_pc(C.byref(p), _ptr(th), seed, traj, n_steps, traj_len,
                                       tol, maxit, cb, None, C.byref(res), _ptr(mom),
                                       _ptr(R), _ptr(eta))
    return th, res.as_dict(), mom, R, eta


def leapfrog(p, theta, mom, eta, n_steps, traj_len=1.0, tol=1e-12, maxit=1_000_000):
    """Leapfrog without Metropolis; returns (theta, mom, H_before, H_after)."""
    th = np.array(_th(theta, p), copy=True)
    m = np.array(np.ascontiguousarray(mom, dtype=np.float64), copy=True)
    eta = _cvec(eta, p)
    hb, ha = C.c_double(0), C.c_double(0)
    lib().oracle_leapfrog(C.byref(p), _ptr(th), _ptr(m), _ptr(eta), n_steps, traj_len,
                          tol, maxit, C.byref(hb), C.byref(ha))
    return th, m, hb.value, ha.value


# ---------------------------------------------------------------------------
# Dense views (tiny lattices only): columns are the matrix-free oracle applied
# to unit vectors, so the dense pins below check the matrix-free code itself.
# ---------------------------------------------------------------------------
def dense_B(p, theta, tau):
    Vs = p.Vs
    B = np.zeros((Vs, Vs), dtype=np.complex128)
    e = np.zeros(Vs, dtype=np.complex128)
    for k in range(Vs):
        e[:] = 0
        e[k] = 1
        B[:, k] = apply_B(p, theta, tau, e)
    return B


def dense_M(p, theta, dagger=False):
    N = p.N
    M = np.zeros((N, N), dtype=np.complex128)
    e = np.zeros(N, dtype=np.complex128)
    for k in range(N):
        e[:] = 0
        e[k] = 1
        M[:, k] = apply_M(p, theta, e, dagger)
    return M


def dense_MdagM(p, theta):
    N = p.N
    O = np.zeros((N, N), dtype=np.complex128)
    e = np.zeros(N, dtype=np.complex128)
    for k in range(N):
        e[:] = 0
        e[k] = 1
        O[:, k] = apply_MdagM(p, theta, e)
    return O
