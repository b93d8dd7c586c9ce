"""The allocation-free M^dag M (qedhmc_apply_MdagM_noalloc) against the
handle's qedhmc_apply_MdagM, through the C ABI: the two share their kernels,
so the results must agree bitwise; two calls in a row with the second on a
smaller lattice (the static scratch keeps the first call's phases, so a
stale cache would show), in FP64 and FP32, the tiled form at L = 66, and the
size limit."""
import pytest
import torch

from paper_2508_16298_amd import inputs
from paper_2508_16298_amd import qedhmc as Q

pytestmark = pytest.mark.gpu


def _case(L, Nt, prec, seed):
    th = torch.from_numpy(inputs.hot_start_theta(L, Nt, seed)).cuda()
    v = torch.from_numpy(inputs.gauss_cvec(L, Nt, seed + 1)).cuda()
    if prec == "fp32":
        v = v.to(torch.complex64)
    return th, v


def _handle_result(L, Nt, th, v, prec):
    with Q.Lattice(L, Nt) as lat:
        out = lat.apply_MdagM(th, v, prec=prec)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_handle_call_on_two_calls_in_a_row(prec):
    sizes = [(24, 240, 31), (8, 16, 32)]   # the second call is smaller
    cases = [(L, Nt) + _case(L, Nt, prec, seed) for L, Nt, seed in sizes]
    outs = []
    for L, Nt, th, v in cases:
        out = torch.full_like(v, float("nan"))
        print(f"noalloc M^dag M L={L} Nt={Nt} {prec}", flush=True)
        Q.apply_MdagM_noalloc(th, v, out, L, Nt, prec=prec)
        torch.cuda.synchronize()
        outs.append(out.clone())
    for (L, Nt, th, v), got in zip(cases, outs):
        ref = _handle_result(L, Nt, th, v, prec)
        assert torch.equal(got, ref), (L, Nt, prec, (got - ref).abs().max().item())


def test_noalloc_tiled_form_and_repeat():
    # L = 66 runs the tiled M^dag M; a short Nt keeps the phase cache within the scratch
    L, Nt = 66, 24
    th, v = _case(L, Nt, "fp32", 41)
    out = torch.empty_like(v)
    for _ in range(2):
        print(f"noalloc M^dag M L={L} Nt={Nt} fp32 (tiled)", flush=True)
        Q.apply_MdagM_noalloc(th, v, out, L, Nt, prec="fp32")
        torch.cuda.synchronize()
        assert torch.equal(out, _handle_result(L, Nt, th, v, "fp32"))


def test_noalloc_rejects_lattices_beyond_its_scratch():
    L, Nt = 66, 240          # 2 L^2 Nt complex FP64 values: 33 MB > 16 MiB
    assert 2 * L * L * Nt * 16 > Q.NOALLOC_SCRATCH_BYTES
    th = torch.zeros(2 * L * L * Nt, dtype=torch.float64, device="cuda")
    v = torch.zeros(Nt * L * L, dtype=torch.complex128, device="cuda")
    out = torch.full_like(v, 7.0)
    with pytest.raises(Q.QedhmcError) as e:
        Q.apply_MdagM_noalloc(th, v, out, L, Nt, prec="fp64")
    assert e.value.status == Q.EINVAL and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
