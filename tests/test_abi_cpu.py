"""The C-ABI library loads and exports every symbol include/qedhmc.h declares;
argument checks that need no device.  CPU only."""
import ctypes as C
import os
import re

import pytest

from paper_2508_16298_amd import qedhmc as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qedhmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qedhmc_[a-z_A-Z0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = Q.load()
    names = _declared()
    assert len(names) >= 13, names
    for n in names:
        assert hasattr(lib, n), n


def test_library_is_gfx950_hip():
    # the shared object carries a gfx950 code object
    data = open(Q.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_init_rejects_bad_gauge_action_without_touching_the_device():
    lib = Q.load()
    h = C.c_void_p(1234)
    for act, res in ((2, 0), (-1, 0), (0, 1)):
        p = Q.Params(4, 4, 0.1, 1.0, 1.0, 1.0, 0, act, res)
        assert lib.qedhmc_init_lattice(C.byref(p), None, C.byref(h)) == Q.EINVAL
        assert "gauge action" in Q.last_error()


@pytest.mark.parametrize("L,Nt", [(3, 4), (0, 4), (5, 1), (4, 0), (2050, 4), (2048, 1024)])
def test_init_rejects_bad_lattices_without_touching_the_device(L, Nt):
    lib = Q.load()
    p = Q.Params(L, Nt, 0.1, 1.0, 1.0, 1.0, 0)
    h = C.c_void_p(1234)
    st = lib.qedhmc_init_lattice(C.byref(p), None, C.byref(h))
    assert st == Q.EINVAL
    assert Q.last_error()


def test_null_arguments_are_rejected():
    lib = Q.load()
    assert lib.qedhmc_init_lattice(None, None, None) == Q.EINVAL
    assert lib.qedhmc_apply_M(None, None, None, None, 0, 0) == Q.EINVAL
    assert lib.qedhmc_cg_solve(None, None, None, None, 1e-8, 10, 0, 0, None, None) == Q.EINVAL
    assert lib.qedhmc_destroy(None) == Q.OK
    p = Q.Params(4, 4, 0.1, 1.0, -1.0, 1.0, 0)  # J <= 0
    h = C.c_void_p()
    assert lib.qedhmc_init_lattice(C.byref(p), None, C.byref(h)) == Q.EINVAL


def _fnv1a(b):
    h = 1469598103934665603
    for x in b:
        h ^= x
        h = (h * 1099511628211) % (1 << 64)
    return h


def _write_checkpoint(path, L, Nt, next_traj, theta, dtau=0.1, t=1.0, J=1.0, K=1.0, seed=7, action=0):
    import struct
    body = b"QEDHMCK1" + struct.pack("<Qqqdddd", 1, L, Nt, dtau, t, J, K)
    body += struct.pack("<QqQQ", seed, action, next_traj, theta.size) + theta.astype("<f8").tobytes()
    open(path, "wb").write(body + struct.pack("<Q", _fnv1a(body)))


def test_checkpoint_info_reads_the_documented_format(tmp_path):
    """A checkpoint written here byte by byte from the layout qedhmc.h states
    is read back by qedhmc_checkpoint_info; a flipped byte, a wrong magic, a
    wrong length or an odd L are refused (EINVAL)."""
    import numpy as np
    L, Nt = 4, 3
    th = np.random.default_rng(1).uniform(0, 6.28, size=(2, Nt, L, L))
    path = str(tmp_path / "chain.ckpt")
    _write_checkpoint(path, L, Nt, 12345, th, dtau=0.05, J=1.25, seed=99, action=1)
    prm, nxt = Q.checkpoint_info(path)
    assert (prm["L"], prm["Nt"], prm["seed"], prm["action"], nxt) == (L, Nt, 99, Q.NONCOMPACT, 12345)
    assert (prm["dtau"], prm["t"], prm["J"], prm["K"]) == (0.05, 1.0, 1.25, 1.0)
    raw = bytearray(open(path, "rb").read())
    for mutate in (lambda b: b.__setitem__(200, b[200] ^ 1),       # a theta byte
                   lambda b: b.__setitem__(0, ord("X")),           # magic
                   lambda b: b.__delitem__(slice(100, 108))):      # length
        bad = bytearray(raw)
        mutate(bad)
        open(path, "wb").write(bytes(bad))
        with pytest.raises(Q.QedhmcError) as e:
            Q.checkpoint_info(path)
        assert e.value.status == Q.EINVAL
    _write_checkpoint(path, 5, Nt, 0, np.zeros((2, Nt, 5, 5)))
    with pytest.raises(Q.QedhmcError):
        Q.checkpoint_info(path)
    _write_checkpoint(path, L, Nt, 0, th, action=2)  # not a gauge action
    with pytest.raises(Q.QedhmcError):
        Q.checkpoint_info(path)
    with pytest.raises(Q.QedhmcError):
        Q.checkpoint_info(str(tmp_path / "missing.ckpt"))


def test_library_autocorrelation_matches_the_oracle():
    """qedhmc_autocorrelation is host code of the library (no device): the
    same rho(k), tau_int and tau_exp as the oracle's analysis of an AR(1)
    series; a constant series is rejected."""
    import numpy as np
    from oracle import production as PR
    rng = np.random.default_rng(3)
    x = np.empty(5000)
    x[0] = rng.standard_normal()
    for t in range(1, x.size):
        x[t] = 0.6 * x[t - 1] + rng.standard_normal()
    rho, ti, te = Q.autocorrelation(x, 40)
    rho_o, ti_o, te_o = PR.autocorrelation(x, 40)
    assert np.abs(rho - rho_o).max() < 1e-12
    assert abs(ti - ti_o) < 1e-12 * ti_o and abs(te - te_o) < 1e-12 * te_o
    with pytest.raises(Q.QedhmcError):
        Q.autocorrelation(np.ones(10), 3)


def test_pc_tau_reach_matches_header():
    """The binding's PC_TAU_REACH (the oracle's cap in the GPU parity tests)
    is the library's QEDHMC_PC_TAU_REACH."""
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qedhmc.h")).read()
    m = re.search(r"#define QEDHMC_PC_TAU_REACH (\d+)", hdr)
    assert m and int(m.group(1)) == Q.PC_TAU_REACH
