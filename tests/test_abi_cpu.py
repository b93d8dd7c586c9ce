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
