"""The tiled, tau-streamed M^dag M (large slices) against the oracle, in
every region form: the whole periodic slice, full-x strips with a y halo and
square tiles with halos both ways, with ragged last tiles and ragged runs of
slices; forced on small lattices through the tuning variables, and in its
default use at L = 66, 128 and 172."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2508_16298_amd import inputs
from paper_2508_16298_amd import qedhmc as Q

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture
def tiled_env(monkeypatch):
    def set_(form="tiled", tc=0, cap=1024):
        monkeypatch.setenv("QEDHMC_MDAGM", form)
        monkeypatch.setenv("QEDHMC_TILE_TC", str(tc))
        monkeypatch.setenv("QEDHMC_TILE_THREADS", str(cap))
    return set_


TOL = {"fp64": 1e-12, "fp32": 3e-6}
CDT = {"fp64": torch.complex128, "fp32": torch.complex64}

# (L, Nt, slices per run, thread cap): whole slice (tiny, ragged runs), strips
# with a ragged last strip, squares (exact and ragged), Nt = 1
FORMS = [(2, 3, 1, 1024), (6, 10, 3, 1024), (32, 6, 4, 224), (24, 24, 5, 100), (30, 5, 2, 100), (4, 1, 0, 1024),
         (12, 120, 7, 1024)]


@pytest.mark.parametrize("L,Nt,tc,cap", FORMS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiled_mdagm_forms(L, Nt, tc, cap, prec, tiled_env):
    tiled_env("tiled", tc, cap)
    th = inputs.hot_start_theta(L, Nt, seed=900 + L)
    v = inputs.gauss_cvec(L, Nt, seed=910 + L)
    with Q.Lattice(L, Nt) as lat:
        out = _host(lat.apply_MdagM(_dev(th), _dev(v, CDT[prec]), prec=prec))
    err = _rel(out, O.apply_MdagM(O.lat(L, Nt), th, v))
    print(f"L={L} Nt={Nt} Tc={tc} cap={cap} {prec}: {err:.2e}", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("L,Nt", [(66, 6), (128, 4), (172, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiled_mdagm_default_large_slices(L, Nt, prec):
    """Default plan at large L: strips at L = 66 and 128, squares at 172."""
    th = inputs.noisy_pi_flux_theta(L, Nt, 0.3, seed=920 + L)
    v = inputs.gauss_cvec(L, Nt, seed=930 + L)
    with Q.Lattice(L, Nt) as lat:
        out = _host(lat.apply_MdagM(_dev(th), _dev(v, CDT[prec]), prec=prec))
    err = _rel(out, O.apply_MdagM(O.lat(L, Nt), th, v))
    print(f"L={L} Nt={Nt} {prec}: {err:.2e}", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("L,Nt,tc", [(128, 6, 0), (128, 5, 2)])
def test_tiled_x_exchange_by_wavefront_rotation(L, Nt, tc, monkeypatch):
    """At L = 128 every FP32 strip row is one wavefront and one x ring: the x
    exchanges go by wavefront rotation instead of LDS, and the halo rows skip
    the sweeps whose results are never used.  Same arithmetic on the same
    values for every stored site: bitwise equal to the LDS exchange, with and
    without the skipping, and to the oracle to the FP32 bar (default and
    forced ragged runs)."""
    th = inputs.noisy_pi_flux_theta(L, Nt, 0.3, seed=950 + Nt)
    v = _dev(inputs.gauss_cvec(L, Nt, seed=951 + Nt), CDT["fp32"])
    monkeypatch.setenv("QEDHMC_TILE_TC", str(tc))
    with Q.Lattice(L, Nt) as lat:
        thd = _dev(th)
        monkeypatch.setenv("QEDHMC_TILE_DPP", "0")
        a = lat.apply_MdagM(thd, v, prec="fp32")
        torch.cuda.synchronize()
        monkeypatch.setenv("QEDHMC_TILE_DPP", "1")
        monkeypatch.setenv("QEDHMC_TILE_SKIP", "0")
        c = lat.apply_MdagM(thd, v, prec="fp32")
        torch.cuda.synchronize()
        monkeypatch.setenv("QEDHMC_TILE_SKIP", "1")
        b = lat.apply_MdagM(thd, v, prec="fp32")
        torch.cuda.synchronize()
    assert torch.equal(a, c) and torch.equal(a, b)
    assert _rel(_host(b), O.apply_MdagM(O.lat(L, Nt), th, v.cpu().numpy().astype(np.complex128))) < TOL["fp32"]


@pytest.mark.parametrize("L,Nt,tc,cap", [(66, 6, 0, 1024), (172, 3, 2, 1024), (40, 5, 2, 100), (32, 6, 4, 224)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiled_halo_rows_skip_unused_sweeps(L, Nt, tc, cap, prec, tiled_env, monkeypatch):
    """Wavefronts whose region rows are all outside the rows a B application
    is needed on skip its sweeps (strips at L = 66 and 32, squares at 172 and
    40): every stored site is bitwise what the kernel gives when every row
    computes every sweep, and within the bar of the oracle."""
    tiled_env("tiled", tc, cap)
    th = inputs.noisy_pi_flux_theta(L, Nt, 0.3, seed=980 + L)
    v = inputs.gauss_cvec(L, Nt, seed=981 + L)
    with Q.Lattice(L, Nt) as lat:
        thd, vd = _dev(th), _dev(v, CDT[prec])
        monkeypatch.setenv("QEDHMC_TILE_SKIP", "0")
        a = lat.apply_MdagM(thd, vd, prec=prec)
        torch.cuda.synchronize()
        monkeypatch.setenv("QEDHMC_TILE_SKIP", "1")
        b = lat.apply_MdagM(thd, vd, prec=prec)
        torch.cuda.synchronize()
    err = _rel(_host(b), O.apply_MdagM(O.lat(L, Nt), th, v))
    print(f"L={L} Nt={Nt} {prec}: bitwise {torch.equal(a, b)}, oracle {err:.2e}", flush=True)
    assert torch.equal(a, b)
    assert err < TOL[prec]


def test_tiled_matches_whole_slice_kernel(tiled_env):
    """Both forms run at L = 48: the same operator to rounding."""
    L, Nt = 48, 16
    th = inputs.hot_start_theta(L, Nt, seed=940)
    v = _dev(inputs.gauss_cvec(L, Nt, seed=941))
    with Q.Lattice(L, Nt) as lat:
        tiled_env("slice")
        a = _host(lat.apply_MdagM(_dev(th), v))
        tiled_env("tiled")
        b = _host(lat.apply_MdagM(_dev(th), v))
    assert _rel(b, a) < 1e-13


def test_whole_slice_calls_reject_large_slices():
    """L = 68 passes the lattice checks; M^dag M runs tiled, the calls that
    hold a slice per workgroup report QEDHMC_EUNSUPPORTED."""
    L, Nt = 68, 2
    th = _dev(inputs.hot_start_theta(L, Nt, seed=950))
    v = inputs.gauss_cvec(L, Nt, seed=951)
    with Q.Lattice(L, Nt) as lat:
        out = _host(lat.apply_MdagM(th, _dev(v)))
        assert _rel(out, O.apply_MdagM(O.lat(L, Nt), _host(th), v)) < 1e-12
        with pytest.raises(Q.QedhmcError) as e:
            lat.apply_M(th, _dev(v))
        assert e.value.status == Q.EUNSUPPORTED
        with pytest.raises(Q.QedhmcError) as e:
            lat.fermion_force(th, _dev(v))
        assert e.value.status == Q.EUNSUPPORTED


@pytest.mark.parametrize("L,Nt,prec,tol,precond", [(68, 6, "fp64", 1e-10, None), (68, 6, "fp32", 1e-8, None),
                                                   (128, 4, "fp32", 1e-8, None), (66, 12, "fp32", 1e-8, "paper"),
                                                   (70, 10, "fp64", 1e-10, "paper")])
def test_cg_past_whole_slice_limit(L, Nt, prec, tol, precond):
    """CG and PCG on slices of more than 1024 cells run in the two-launch form
    with the tiled M^dag M writing one partial tuple per (slice, tile); past
    L = 66 this is the only form.  True residual recomputed by the oracle;
    the FP64 CG iteration count matches the oracle's."""
    p = O.lat(L, Nt)
    th = inputs.noisy_pi_flux_theta(L, Nt, 0.3, 960 + L)
    R = inputs.gauss_cvec(L, Nt, 961 + L)
    eta = O.apply_M(p, th, R, dagger=True).reshape(Nt, L, L)
    with Q.Lattice(L, Nt) as lat:
        x, st, it, rel = lat.cg_solve(_dev(th), _dev(eta), tol=tol, prec=prec, precond=precond)
        xg = _host(x)
    true = np.linalg.norm(eta.reshape(-1) - O.apply_MdagM(p, th, xg).reshape(-1)) / np.linalg.norm(eta)
    print(f"L={L} Nt={Nt} {prec} precond={precond}: {it} iterations, true residual {true:.2e}", flush=True)
    assert st == Q.OK and rel <= tol and true <= 1.05 * tol
    if prec == "fp64" and precond is None:
        _, _, ito, _ = O.cg_solve(p, th, eta, tol=tol)
        assert abs(it - ito) <= max(2, ito // 50), (it, ito)


@pytest.mark.parametrize("L,Nt,prec,precond", [(68, 6, "fp32", None), (68, 6, "fp64", None),
                                               (12, 40, "fp32", "paper"), (66, 12, "fp32", "paper")])
def test_two_launch_graph_replays_match_direct_launches(L, Nt, prec, precond):
    """Two-launch CG (slices of more than 1024 cells) and PCG replay their full
    chunks from captured graphs; over several solves on one handle (graphs
    replayed many times, reliable updates and host reads in between) they give
    bitwise the solution, iteration count and residual of the same solves
    launched directly."""
    p = O.lat(L, Nt)
    tol = 1e-10 if prec == "fp64" else 1e-8
    out = {}
    with Q.Lattice(L, Nt) as lat:
        for mode in ("graph", "direct", "graph"):
            if mode == "direct":
                os.environ["QEDHMC_NO_GRAPH"] = "1"
            try:
                res = []
                for seed in (31, 32):
                    th = inputs.noisy_pi_flux_theta(L, Nt, 0.3, seed)
                    eta = O.apply_M(p, th, inputs.gauss_cvec(L, Nt, seed + 50), dagger=True).reshape(Nt, L, L)
                    x, st, it, rel = lat.cg_solve(_dev(th), _dev(eta), tol=tol, prec=prec, precond=precond)
                    res.append((_host(x), st, it, rel))
            finally:
                os.environ.pop("QEDHMC_NO_GRAPH", None)
            out.setdefault(mode, []).append(res)
    ref = out["direct"][0]
    for run in out["graph"]:
        for (xg, sg, ig, rg), (xd, sd, id_, rd) in zip(run, ref):
            print(f"L={L} {prec} {precond}: graph {sg} {ig} {rg:.3e} direct {sd} {id_} {rd:.3e}", flush=True)
            assert sg == sd == Q.OK and ig == id_ and rg == rd
            assert np.array_equal(xg, xd)
