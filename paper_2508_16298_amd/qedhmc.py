"""ctypes binding of libqedhmc (the C ABI in include/qedhmc.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of libqedhmc.so.  torch provides device memory and the current HIP
stream.  The library is loaded on first use and a missing or unloadable
library raises -- there is no CPU fallback.

Layouts (torch tensors on the GPU, contiguous)
  theta   float64     (2, Nt, L, L)   [d, tau, y, x]
  vector  complex128  (Nt, L, L)      FP64 path
          complex64   (Nt, L, L)      FP32 apply calls
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqedhmc.so")

OK, EINVAL, ENOCONV, EHIP, ENOMEM, EUNSUPPORTED = range(6)
(K_MDAGM_FP32, K_MDAGM_FP64, K_FORCE, K_CG_FP32, K_CG_FP64, K_PCG_MV_FP32, K_PCG_MV_FP64, K_NET_MFMA,
 K_NET_FP32, K_PC_SPEC_FP32, K_PC_SPEC_FP64) = range(11)
FP64, FP32 = 0, 1
COMPACT, NONCOMPACT = 0, 1
PC_NONE, PC_PAPER, PC_LEARNED = 0, 1, 2
_PC = {None: PC_NONE, "none": PC_NONE, "paper": PC_PAPER, "learned": PC_LEARNED, PC_NONE: PC_NONE,
       PC_PAPER: PC_PAPER, PC_LEARNED: PC_LEARNED}

_PREC = {"fp64": FP64, "fp32": FP32, "mixed": FP32, FP64: FP64, FP32: FP32}


class QedhmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qedhmc status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("L", C.c_int32), ("Nt", C.c_int32), ("dtau", C.c_double), ("t", C.c_double),
                ("J", C.c_double), ("K", C.c_double), ("seed", C.c_uint64), ("action", C.c_int32),
                ("reserved", C.c_int32)]


class TrajResult(C.Structure):
    _fields_ = [("dH", C.c_double), ("H0", C.c_double), ("H1", C.c_double), ("SB0", C.c_double),
                ("SB1", C.c_double), ("SF0", C.c_double), ("SF1", C.c_double), ("K0", C.c_double),
                ("K1", C.c_double), ("u", C.c_double), ("accepted", C.c_int32),
                ("n_solves", C.c_int32), ("cg_iters_total", C.c_int32),
                ("cg_iters_max", C.c_int32), ("status", C.c_int32),
                ("reliable_updates", C.c_int32), ("max_true_resid", C.c_double),
                ("pc_fallbacks", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ProdParams(C.Structure):
    _fields_ = [("first_traj", C.c_uint64), ("n_therm", C.c_int32), ("n_meas", C.c_int32),
                ("n_steps", C.c_int32), ("maxit", C.c_int32), ("dt0", C.c_double),
                ("target_accept", C.c_double), ("gain", C.c_double), ("tol", C.c_double),
                ("prec", C.c_int), ("pc", C.c_int)]


class ProdRecord(C.Structure):
    _fields_ = [("traj", C.c_uint64), ("dt", C.c_double), ("dH", C.c_double), ("S_tau", C.c_double),
                ("S_plaq", C.c_double), ("accepted", C.c_int32), ("cg_iters", C.c_int32),
                ("status", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None
_P = C.c_void_p


def load():
    """Load libqedhmc.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_2508_16298_amd.build")
    L = C.CDLL(LIB_PATH)
    st = C.c_int
    sig = {
        "qedhmc_init_lattice": [C.POINTER(Params), _P, C.POINTER(_P)],
        "qedhmc_destroy": [_P],
        "qedhmc_set_stream": [_P, _P],
        "qedhmc_get_bond_tables": [_P, _P],
        "qedhmc_apply_B": [_P, _P, C.c_int32, _P, _P, C.c_int],
        "qedhmc_apply_M": [_P, _P, _P, _P, C.c_int32, C.c_int],
        "qedhmc_apply_MdagM": [_P, _P, _P, _P, C.c_int],
        "qedhmc_apply_MdagM_noalloc": [C.POINTER(Params), _P, _P, _P, C.c_int, _P],
        "qedhmc_cg_solve": [_P, _P, _P, _P, C.c_double, C.c_int32, C.c_int, C.c_int,
                            C.POINTER(C.c_int32), C.POINTER(C.c_double)],
        "qedhmc_fermion_force": [_P, _P, _P, _P, C.c_int],
        "qedhmc_bosonic_action_force": [_P, _P, C.POINTER(C.c_double), _P],
        "qedhmc_heatbath": [_P, C.c_uint64, _P, _P],
        "qedhmc_precond_taps": [_P, C.c_int32, C.POINTER(C.c_int32), _P, C.c_int32],
        "qedhmc_apply_precond": [_P, _P, _P, C.c_int],
        "qedhmc_profile": [_P, C.c_int32],
        "qedhmc_profile_read": [_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
        "qedhmc_hmc_trajectory": [_P, _P, C.c_uint64, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                  C.c_int, C.c_int, C.POINTER(TrajResult)],
        "qedhmc_net_create": [_P, C.POINTER(_P)],
        "qedhmc_net_destroy": [_P],
        "qedhmc_net_set_params": [_P, _P, C.c_int64],
        "qedhmc_net_get_params": [_P, _P, C.c_int64],
        "qedhmc_net_reset_optimizer": [_P],
        "qedhmc_net_apply": [_P, _P, _P, _P, C.c_int],
        "qedhmc_net_train_step": [_P, _P, _P, _P, C.c_double, C.c_int, C.POINTER(C.c_double), _P],
        "qedhmc_net_train_step_residual": [_P, _P, _P, C.c_double, C.c_int, C.POINTER(C.c_double), _P],
        "qedhmc_set_learned_precond": [_P, _P, C.c_int, C.c_int],
        "qedhmc_checkpoint_save": [_P, _P, C.c_uint64, C.c_char_p],
        "qedhmc_checkpoint_info": [C.c_char_p, C.POINTER(Params), C.POINTER(C.c_uint64)],
        "qedhmc_checkpoint_load": [_P, C.c_char_p, _P, C.POINTER(C.c_uint64)],
        "qedhmc_fcg_solve": [_P, _P, _P, _P, C.c_double, C.c_int32, C.c_int, C.c_int, C.POINTER(C.c_int32),
                             C.POINTER(C.c_double), C.POINTER(C.c_int32)],
        "qedhmc_gauge_observables": [_P, _P, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "qedhmc_flux_correlator": [_P, _P, _P],
        "qedhmc_production": [_P, _P, C.POINTER(ProdParams), _P, _P, C.POINTER(C.c_double)],
        "qedhmc_autocorrelation": [_P, C.c_int32, C.c_int32, _P, C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "qedhmc_se_create": [C.POINTER(Params), C.c_int32, _P, C.POINTER(_P)],
        "qedhmc_se_destroy": [_P],
        "qedhmc_se_probes": [_P, C.c_uint64, _P],
        "qedhmc_se_solve": [_P, _P, _P, _P, C.c_double, C.c_int32, C.c_int, _P, _P],
        "qedhmc_se_spin_correlator": [_P, _P, _P, _P],
        "qedhmc_batch_create": [C.POINTER(Params), C.c_int32, _P, C.POINTER(_P)],
        "qedhmc_batch_destroy": [_P],
        "qedhmc_batch_layout": [_P, _P, _P],
        "qedhmc_batch_tile": [_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                              _P],
        "qedhmc_batch_cg_solve": [_P, _P, _P, _P, C.c_double, C.c_int32, C.c_int, _P, _P],
        "qedhmc_batch_trajectory": [_P, _P, C.c_uint64, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                    C.c_int, _P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = st
    L.qedhmc_net_param_count.argtypes = []
    L.qedhmc_net_param_count.restype = C.c_int64
    L.qedhmc_last_error.argtypes = []
    L.qedhmc_last_error.restype = C.c_char_p
    _lib = L
    return L


def last_error():
    return load().qedhmc_last_error().decode()


def _check(status, allow=(OK,)):
    if status not in allow:
        raise QedhmcError(status, last_error())
    return status


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream_handle():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def checkpoint_info(path):
    """(params dict, next_traj) from a checkpoint file's verified header (no device work)."""
    p = Params()
    nxt = C.c_uint64(0)
    _check(load().qedhmc_checkpoint_info(os.fsencode(path), C.byref(p), C.byref(nxt)))
    return {k: getattr(p, k) for k, _ in p._fields_}, nxt.value


def autocorrelation(series, kmax):
    """qedhmc_autocorrelation: (rho[0..kmax], tau_int, tau_exp) of a host series."""
    import numpy as np
    x = np.ascontiguousarray(series, dtype=np.float64)
    rho = np.zeros(int(kmax) + 1, dtype=np.float64)
    ti, te = C.c_double(0.0), C.c_double(0.0)
    _check(load().qedhmc_autocorrelation(x.ctypes.data_as(C.c_void_p), x.size, int(kmax),
                                         rho.ctypes.data_as(C.c_void_p), C.byref(ti), C.byref(te)))
    return rho, ti.value, te.value


NOALLOC_SCRATCH_BYTES = 16 << 20
PC_TAU_REACH = 12  # QEDHMC_PC_TAU_REACH: tau reach of the paper's preconditioner G as built


def apply_MdagM_noalloc(theta, v, out, L, Nt, dtau=0.1, t=1.0, J=1.0, K=1.0, noncompact=False,
                        prec="fp64"):
    """qedhmc_apply_MdagM_noalloc on torch's current stream: out = M^dag M v with
    no handle and no device allocation (caller-owned theta, v and out)."""
    import torch
    params = Params(int(L), int(Nt), dtau, t, J, K, 0, NONCOMPACT if noncompact else COMPACT, 0)
    n = int(L) * int(L) * int(Nt)
    dt = torch.complex128 if _PREC[prec] == FP64 else torch.complex64
    for a, d, m in ((theta, torch.float64, 2 * n), (v, dt, n), (out, dt, n)):
        assert a.is_cuda and a.dtype == d and a.is_contiguous() and a.numel() == m, (a.dtype, a.shape)
    _check(load().qedhmc_apply_MdagM_noalloc(C.byref(params), _ptr(theta), _ptr(v), _ptr(out), _PREC[prec],
                                             _stream_handle()))
    return out


class Lattice:
    """A qedhmc handle (qedhmc_init_lattice) bound to torch's current stream."""

    def __init__(self, L, Nt, dtau=0.1, t=1.0, J=1.0, K=1.0, seed=0, noncompact=False):
        import torch
        self.L, self.Nt = int(L), int(Nt)
        self.params = Params(self.L, self.Nt, dtau, t, J, K, seed, NONCOMPACT if noncompact else COMPACT, 0)
        self._torch = torch
        h = _P()
        _check(load().qedhmc_init_lattice(C.byref(self.params), _stream_handle(), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().qedhmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers -----------------------------------------------------------
    @property
    def N(self):
        return self.L * self.L * self.Nt

    def _sync_stream(self):
        _check(load().qedhmc_set_stream(self.h, _stream_handle()))

    def _vec(self, prec):
        dt = self._torch.complex128 if _PREC[prec] == FP64 else self._torch.complex64
        return self._torch.empty((self.Nt, self.L, self.L), dtype=dt, device="cuda")

    def _check_theta(self, theta):
        assert theta.is_cuda and theta.dtype == self._torch.float64 and theta.is_contiguous()
        assert theta.numel() == 2 * self.N, theta.shape

    def _check_vec(self, v, prec):
        dt = self._torch.complex128 if _PREC[prec] == FP64 else self._torch.complex64
        assert v.is_cuda and v.dtype == dt and v.is_contiguous(), (v.dtype, dt)
        assert v.numel() == self.N, v.shape

    # -- the C ABI ---------------------------------------------------------
    def get_bond_tables(self):
        import numpy as np
        out = np.zeros((4, self.L * self.L // 2, 3), dtype=np.int32)
        self._sync_stream()
        _check(load().qedhmc_get_bond_tables(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def apply_B(self, theta, tau, v, prec="fp64", out=None):
        self._check_theta(theta)
        dt = self._torch.complex128 if _PREC[prec] == FP64 else self._torch.complex64
        assert v.is_cuda and v.dtype == dt and v.numel() == self.L * self.L
        out = self._torch.empty_like(v) if out is None else out
        self._sync_stream()
        _check(load().qedhmc_apply_B(self.h, _ptr(theta), int(tau), _ptr(v), _ptr(out), _PREC[prec]))
        return out

    def apply_M(self, theta, v, dagger=False, prec="fp64", out=None):
        self._check_theta(theta)
        self._check_vec(v, prec)
        out = self._vec(prec) if out is None else out
        self._sync_stream()
        _check(load().qedhmc_apply_M(self.h, _ptr(theta), _ptr(v), _ptr(out), int(bool(dagger)),
                                     _PREC[prec]))
        return out

    def apply_MdagM(self, theta, v, prec="fp64", out=None):
        self._check_theta(theta)
        self._check_vec(v, prec)
        out = self._vec(prec) if out is None else out
        self._sync_stream()
        _check(load().qedhmc_apply_MdagM(self.h, _ptr(theta), _ptr(v), _ptr(out), _PREC[prec]))
        return out

    def precond_taps(self, parity):
        """The paper's preconditioner stencil of one x parity: float64 (n, 5) rows
        (dtau, dx, dy, Re g, Im g)."""
        import numpy as np
        n = C.c_int32(0)
        _check(load().qedhmc_precond_taps(self.h, int(parity), C.byref(n), None, 0))
        out = np.zeros((n.value, 5))
        _check(load().qedhmc_precond_taps(self.h, int(parity), C.byref(n), out.ctypes.data_as(C.c_void_p),
                                          n.value))
        return out

    def apply_precond(self, v, prec="fp64", out=None):
        self._check_vec(v, prec)
        out = self._vec(prec) if out is None else out
        self._sync_stream()
        _check(load().qedhmc_apply_precond(self.h, _ptr(v), _ptr(out), _PREC[prec]))
        return out

    def cg_solve(self, theta, rhs, tol=1e-10, maxit=1_000_000, prec="fp64", x=None, precond=None):
        """Returns (x, status, iters, true_rel_resid); status OK or ENOCONV.
        precond: None or "paper"."""
        self._check_theta(theta)
        self._check_vec(rhs, "fp64")
        x = self._vec("fp64") if x is None else x
        it = C.c_int32(0)
        rel = C.c_double(0.0)
        self._sync_stream()
        st = _check(load().qedhmc_cg_solve(self.h, _ptr(theta), _ptr(rhs), _ptr(x), float(tol), int(maxit),
                                           _PREC[prec], _PC[precond], C.byref(it), C.byref(rel)),
                    allow=(OK, ENOCONV))
        return x, st, it.value, rel.value

    def fermion_force(self, theta, X, prec="fp64", out=None):
        self._check_theta(theta)
        self._check_vec(X, "fp64")
        out = self._torch.empty_like(theta) if out is None else out
        self._sync_stream()
        _check(load().qedhmc_fermion_force(self.h, _ptr(theta), _ptr(X), _ptr(out), _PREC[prec]))
        return out

    def bosonic_action_force(self, theta, force=True):
        self._check_theta(theta)
        S = C.c_double(0.0)
        F = self._torch.empty_like(theta) if force else None
        self._sync_stream()
        _check(load().qedhmc_bosonic_action_force(self.h, _ptr(theta), C.byref(S),
                                                  _ptr(F) if force else None))
        return S.value, F

    def heatbath(self, traj):
        mom = self._torch.empty((2, self.Nt, self.L, self.L), dtype=self._torch.float64, device="cuda")
        R = self._vec("fp64")
        self._sync_stream()
        _check(load().qedhmc_heatbath(self.h, int(traj), _ptr(mom), _ptr(R)))
        return mom, R

    def hmc_trajectory(self, theta, traj, n_steps, traj_len=1.0, tol=1e-10, maxit=1_000_000,
                       prec="fp64", precond=None):
        """theta is updated in place (proposal on acceptance); returns the result dict.
        A trajectory with an unconverged solve (ENOCONV) is rejected and returns
        its dict with status 2."""
        self._check_theta(theta)
        res = TrajResult()
        self._sync_stream()
        _check(load().qedhmc_hmc_trajectory(self.h, _ptr(theta), int(traj), int(n_steps),
                                            float(traj_len), float(tol), int(maxit), _PREC[prec],
                                            _PC[precond], C.byref(res)), allow=(OK, ENOCONV))
        return res.as_dict()

    def gauge_observables(self, theta):
        """(S_tau, S_plaq) at theta."""
        self._check_theta(theta)
        a, b = C.c_double(0.0), C.c_double(0.0)
        self._sync_stream()
        _check(load().qedhmc_gauge_observables(self.h, _ptr(theta), C.byref(a), C.byref(b)))
        return a.value, b.value

    def flux_correlator(self, theta, out=None):
        self._check_theta(theta)
        out = self._torch.empty(self.Nt, dtype=self._torch.float64, device="cuda") if out is None else out
        self._sync_stream()
        _check(load().qedhmc_flux_correlator(self.h, _ptr(theta), _ptr(out)))
        return out

    def production(self, theta, first_traj, n_therm, n_meas, dt0, target_accept=0.7, gain=1.0, n_steps=3,
                   tol=1e-10, maxit=1_000_000, prec="fp64", precond=None, flux=True):
        """Chained trajectories with step-size adaptation during thermalisation
        (theta updated in place); returns (status, records, C_flux mean or None, dt_final)."""
        self._check_theta(theta)
        n = int(n_therm) + int(n_meas)
        pp = ProdParams(int(first_traj), int(n_therm), int(n_meas), int(n_steps), int(maxit), float(dt0),
                        float(target_accept), float(gain), float(tol), _PREC[prec], _PC[precond])
        recs = (ProdRecord * max(n, 1))()
        Cf = self._torch.empty(self.Nt, dtype=self._torch.float64, device="cuda") if flux else None
        dtf = C.c_double(0.0)
        self._sync_stream()
        st = _check(load().qedhmc_production(self.h, _ptr(theta), C.byref(pp), C.cast(recs, C.c_void_p),
                                             _ptr(Cf) if flux else None, C.byref(dtf)), allow=(OK, ENOCONV))
        return st, [recs[k].as_dict() for k in range(n)], Cf, dtf.value


    def checkpoint_save(self, theta, next_traj, path):
        """Write the chain state (parameters, theta, next trajectory index) to path."""
        self._check_theta(theta)
        self._sync_stream()
        _check(load().qedhmc_checkpoint_save(self.h, _ptr(theta), int(next_traj), os.fsencode(path)))

    def checkpoint_load(self, path, theta=None):
        """Read a checkpoint of this lattice into theta (allocated if None);
        returns (theta, next_traj)."""
        import torch
        if theta is None:
            theta = torch.empty((2, self.Nt, self.L, self.L), dtype=torch.float64, device="cuda")
        self._check_theta(theta)
        nxt = C.c_uint64(0)
        self._sync_stream()
        _check(load().qedhmc_checkpoint_load(self.h, os.fsencode(path), _ptr(theta), C.byref(nxt)))
        return theta, nxt.value

    def profile(self, every):
        """Time every every-th launch of the timed kernels with HIP events (0: off)."""
        self._sync_stream()
        _check(load().qedhmc_profile(self.h, int(every)))

    def profile_read(self, kernel_class):
        """(count, total_ms) of the timed launches of one kernel class."""
        n = C.c_int64(0)
        ms = C.c_double(0.0)
        _check(load().qedhmc_profile_read(self.h, int(kernel_class), C.byref(n), C.byref(ms)))
        return n.value, ms.value


class Batch:
    """Independent chains on lattices of different sizes, advanced together
    (qedhmc_batch_create); bound to torch's current stream at creation.

    Concatenated layouts: theta_all float64 (theta_off[-1],) with chain c at
    theta_off[c] in (2, Nt_c, L_c, L_c) order; vectors complex128
    (vec_off[-1],) with chain c at vec_off[c]."""

    def __init__(self, sizes, dtau=0.1, t=1.0, J=1.0, K=1.0, seeds=None, noncompact=False):
        import numpy as np
        import torch
        self._torch = torch
        self.sizes = [(int(L), int(Nt)) for L, Nt in sizes]
        n = len(self.sizes)
        seeds = list(range(n)) if seeds is None else [int(s) for s in seeds]
        act = NONCOMPACT if noncompact else COMPACT
        arr = (Params * n)(*[Params(L, Nt, dtau, t, J, K, sd, act, 0) for (L, Nt), sd in zip(self.sizes, seeds)])
        self.params = arr
        h = _P()
        _check(load().qedhmc_batch_create(arr, n, _stream_handle(), C.byref(h)))
        self.h = h
        self.theta_off = np.zeros(n + 1, dtype=np.int64)
        self.vec_off = np.zeros(n + 1, dtype=np.int64)
        _check(load().qedhmc_batch_layout(self.h, self.theta_off.ctypes.data_as(C.c_void_p),
                                          self.vec_off.ctypes.data_as(C.c_void_p)))

    @property
    def n(self):
        return len(self.sizes)

    def close(self):
        if getattr(self, "h", None):
            load().qedhmc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def theta_view(self, theta_all, c):
        L, Nt = self.sizes[c]
        return theta_all[self.theta_off[c]:self.theta_off[c + 1]].view(2, Nt, L, L)

    def vec_view(self, v_all, c):
        L, Nt = self.sizes[c]
        return v_all[self.vec_off[c]:self.vec_off[c + 1]].view(Nt, L, L)

    def tile(self, prec="fp32"):
        """(cells_per_thread, threads, exchange_buffers, us_per_iter[4]) chosen by the autotuner."""
        import numpy as np
        mc, nt, nb = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        us = np.zeros(4, dtype=np.float32)
        _check(load().qedhmc_batch_tile(self.h, _PREC[prec], C.byref(mc), C.byref(nt), C.byref(nb),
                                        us.ctypes.data_as(C.c_void_p)))
        return mc.value, nt.value, nb.value, us

    def _check_all(self, t, n, dtype):
        assert t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == n, (t.shape, t.dtype)

    def cg_solve(self, theta_all, rhs_all, tol=1e-10, maxit=1_000_000, prec="fp64", x_all=None):
        """Returns (x_all, status, iters[n], true_rel[n])."""
        import numpy as np
        torch = self._torch
        self._check_all(theta_all, int(self.theta_off[-1]), torch.float64)
        self._check_all(rhs_all, int(self.vec_off[-1]), torch.complex128)
        x_all = torch.empty_like(rhs_all) if x_all is None else x_all
        it = np.zeros(self.n, dtype=np.int32)
        rel = np.zeros(self.n)
        st = _check(load().qedhmc_batch_cg_solve(self.h, _ptr(theta_all), _ptr(rhs_all), _ptr(x_all),
                                                 float(tol), int(maxit), _PREC[prec],
                                                 it.ctypes.data_as(C.c_void_p),
                                                 rel.ctypes.data_as(C.c_void_p)),
                    allow=(OK, ENOCONV))
        return x_all, st, it, rel

    def trajectory(self, theta_all, traj, n_steps, traj_len=1.0, tol=1e-10, maxit=1_000_000, prec="fp64"):
        """theta_all updated per chain in place; returns a list of result dicts.
        A chain with an unconverged solve rejects its proposal (status 2)."""
        self._check_all(theta_all, int(self.theta_off[-1]), self._torch.float64)
        res = (TrajResult * self.n)()
        _check(load().qedhmc_batch_trajectory(self.h, _ptr(theta_all), int(traj), int(n_steps),
                                              float(traj_len), float(tol), int(maxit), _PREC[prec], res),
               allow=(OK, ENOCONV))
        return [r.as_dict() for r in res]


NET_FP32, NET_BF16 = 0, 1
_ARITH = {"fp32": NET_FP32, "bf16": NET_BF16, NET_FP32: NET_FP32, NET_BF16: NET_BF16}


class Stochastic:
    """Stochastic estimation of the spin correlator on one lattice with n_rv
    probes (qedhmc_se_create); bound to torch's current stream at creation.
    Probe sets and solutions are complex128 tensors (n_rv, Nt, L, L)."""

    def __init__(self, L, Nt, n_rv, dtau=0.1, t=1.0, J=1.0, K=1.0, seed=0, noncompact=False):
        import torch
        self._torch = torch
        self.L, self.Nt, self.n_rv = int(L), int(Nt), int(n_rv)
        self.params = Params(self.L, self.Nt, dtau, t, J, K, seed, NONCOMPACT if noncompact else COMPACT, 0)
        h = _P()
        _check(load().qedhmc_se_create(C.byref(self.params), self.n_rv, _stream_handle(), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().qedhmc_se_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _set(self):
        return self._torch.empty((self.n_rv, self.Nt, self.L, self.L), dtype=self._torch.complex128, device="cuda")

    def _check_set(self, v):
        assert v.is_cuda and v.dtype == self._torch.complex128 and v.is_contiguous()
        assert tuple(v.shape) == (self.n_rv, self.Nt, self.L, self.L), v.shape

    def probes(self, meas, out=None):
        out = self._set() if out is None else out
        self._check_set(out)
        _check(load().qedhmc_se_probes(self.h, int(meas), _ptr(out)))
        return out

    def solve(self, theta, xi, tol=1e-10, maxit=1_000_000, prec="fp64", out=None):
        """Returns (X, status, iters[n_rv], true_rel[n_rv]); status OK or ENOCONV."""
        import numpy as np
        assert theta.is_cuda and theta.dtype == self._torch.float64 and theta.is_contiguous()
        assert theta.numel() == 2 * self.L * self.L * self.Nt
        self._check_set(xi)
        X = self._set() if out is None else out
        self._check_set(X)
        it = np.zeros(self.n_rv, dtype=np.int32)
        rel = np.zeros(self.n_rv, dtype=np.float64)
        st = _check(load().qedhmc_se_solve(self.h, _ptr(theta), _ptr(xi), _ptr(X), float(tol), int(maxit),
                                           _PREC[prec], it.ctypes.data_as(C.c_void_p),
                                           rel.ctypes.data_as(C.c_void_p)), allow=(OK, ENOCONV))
        return X, st, it, rel

    def spin_correlator(self, xi, X, out=None):
        self._check_set(xi)
        self._check_set(X)
        out = (self._torch.empty((self.Nt, self.L, self.L), dtype=self._torch.complex128, device="cuda")
               if out is None else out)
        assert out.is_cuda and out.dtype == self._torch.complex128 and out.numel() == self.Nt * self.L * self.L
        _check(load().qedhmc_se_spin_correlator(self.h, _ptr(xi), _ptr(X), _ptr(out)))
        return out


class Net:
    """The learned preconditioner (qedhmc_net_*) bound to a Lattice.

    Parameters travel as a flat float32 array in the C layout (per layer
    W[Cout][Cin][27] then b[Cout]); ``pack``/``unpack`` convert from/to a list
    of (W, b) numpy pairs."""

    def __init__(self, lat):
        self.lat = lat
        h = _P()
        lat._sync_stream()
        _check(load().qedhmc_net_create(lat.h, C.byref(h)))
        self.h = h
        self.count = int(load().qedhmc_net_param_count())

    def close(self):
        if getattr(self, "h", None):
            load().qedhmc_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @staticmethod
    def pack(params):
        import numpy as np
        return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in params]).astype(np.float32)

    @staticmethod
    def unpack(flat, channels=(6, 32, 32, 32, 32, 32, 2)):
        out, o = [], 0
        for l in range(len(channels) - 1):
            ci, co = channels[l], channels[l + 1]
            W = flat[o:o + co * ci * 27].reshape(co, ci, 27)
            o += co * ci * 27
            b = flat[o:o + co]
            o += co
            out.append((W, b))
        return out

    def set_params(self, params):
        import numpy as np
        flat = params if isinstance(params, np.ndarray) else self.pack(params)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.count
        _check(load().qedhmc_net_set_params(self.h, flat.ctypes.data_as(C.c_void_p), self.count))

    def get_params(self):
        import numpy as np
        flat = np.zeros(self.count, dtype=np.float32)
        _check(load().qedhmc_net_get_params(self.h, flat.ctypes.data_as(C.c_void_p), self.count))
        return flat

    def reset_optimizer(self):
        _check(load().qedhmc_net_reset_optimizer(self.h))

    def apply(self, theta, r, arith="fp32", out=None):
        self.lat._check_theta(theta)
        self.lat._check_vec(r, "fp64")
        out = self.lat._vec("fp64") if out is None else out
        self.lat._sync_stream()
        _check(load().qedhmc_net_apply(self.h, _ptr(theta), _ptr(r), _ptr(out), _ARITH[arith]))
        return out

    def train_step(self, theta, r, e, lr=1e-3, arith="fp32", want_grad=False):
        """Returns (loss, grad) with grad the flat float32 gradient (or None)."""
        import numpy as np
        self.lat._check_theta(theta)
        self.lat._check_vec(r, "fp64")
        self.lat._check_vec(e, "fp64")
        loss = C.c_double(0.0)
        grad = np.zeros(self.count, dtype=np.float32) if want_grad else None
        self.lat._sync_stream()
        _check(load().qedhmc_net_train_step(self.h, _ptr(theta), _ptr(r), _ptr(e), float(lr), _ARITH[arith],
                                            C.byref(loss),
                                            grad.ctypes.data_as(C.c_void_p) if want_grad else None))
        return loss.value, grad

    def train_step_residual(self, theta, r, lr=1e-3, arith="fp32", want_grad=False):
        """Residual-form step (loss |O N(r) - r|^2 / |r|^2).  Returns (loss, grad)."""
        import numpy as np
        self.lat._check_theta(theta)
        self.lat._check_vec(r, "fp64")
        loss = C.c_double(0.0)
        grad = np.zeros(self.count, dtype=np.float32) if want_grad else None
        self.lat._sync_stream()
        _check(load().qedhmc_net_train_step_residual(self.h, _ptr(theta), _ptr(r), float(lr), _ARITH[arith],
                                                     C.byref(loss),
                                                     grad.ctypes.data_as(C.c_void_p) if want_grad else None))
        return loss.value, grad

    def bind(self, arith="bf16", fallback="paper"):
        """Make this network the lattice's learned preconditioner
        (precond="learned" in cg_solve and hmc_trajectory)."""
        _check(load().qedhmc_set_learned_precond(self.lat.h, self.h, _ARITH[arith], _PC[fallback]))
        return self

    def unbind(self):
        _check(load().qedhmc_set_learned_precond(self.lat.h, None, 0, 0))

    def fcg_solve(self, theta, rhs, tol=1e-10, maxit=100_000, arith="bf16", fallback="paper", x=None):
        """Returns (x, status, iters, true_rel, switched_at)."""
        self.lat._check_theta(theta)
        self.lat._check_vec(rhs, "fp64")
        x = self.lat._vec("fp64") if x is None else x
        it, rel, sw = C.c_int32(0), C.c_double(0.0), C.c_int32(0)
        self.lat._sync_stream()
        st = _check(load().qedhmc_fcg_solve(self.h, _ptr(theta), _ptr(rhs), _ptr(x), float(tol), int(maxit),
                                            _ARITH[arith], _PC[fallback], C.byref(it), C.byref(rel),
                                            C.byref(sw)), allow=(OK, ENOCONV))
        return x, st, it.value, rel.value, sw.value


def init_lattice(L, Nt, **kw):
    return Lattice(L, Nt, **kw)
