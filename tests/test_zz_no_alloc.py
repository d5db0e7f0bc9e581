"""bl_adjoint_noalloc (the allocation-free adjoint, for callers that cannot allocate) through
the C ABI, against bl_adjoint on the same plan and inputs: two calls in a row on one GPU's
shared scratch array, the second with a smaller plan and fewer nodes, each within the
parity tolerance of the precision (1e-12 FP64, 1e-6 FP32 with compensated sums).  Also the
refusal of a grid larger than the fixed scratch and the oracle's adjoint as a third check."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32c": 1e-6}


def _run(spec, prec):
    import torch
    from paper_2502_07155_amd import Plan
    d, M, L, m, N = spec
    p = W.custom_problem(d, M, L, m, N, seed=900 + M + N, precision="f32" if prec != "f64" else "f64",
                         with_targets=True)
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    plan = Plan(d, M, L, m, precision=prec)
    plan.set_nodes(torch.from_numpy(p.x).to(rdt).cuda())
    g = torch.from_numpy(p.y).to(cdt).cuda()
    ref = plan.adjoint(g).cpu().numpy().astype(np.complex128)
    out = torch.full((M,) * d, float("nan"), dtype=cdt, device="cuda")
    lib = plan._lib
    st = lib.bl_adjoint_noalloc(plan.handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert st == 0, lib.bl_last_error().decode()
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)
    plan.close()
    orc = O.adjoint_shannon(p.y.astype(np.complex128), p.x.astype(np.float64), M, L, m)
    return got, ref, orc


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_noalloc_adjoint_matches_adjoint_twice_second_smaller(prec):
    first = (2, 128, 256, 5, 6000)
    second = (2, 32, 64, 3, 700)
    for spec in (first, second):
        got, ref, orc = _run(spec, prec)
        assert np.all(np.isfinite(got)), spec
        assert O.rel_err_inf(got, ref) <= TOL[prec], spec
        assert O.rel_err_inf(got, orc) <= (1e-12 if prec == "f64" else 1e-5), spec


def test_noalloc_adjoint_refuses_grid_above_its_scratch():
    import torch
    from paper_2502_07155_amd import Plan
    plan = Plan(2, 1024, 4096, 4, precision="f32")   # 4096^2 float complex = 128 MiB
    x = torch.zeros((10, 2), dtype=torch.float32, device="cuda")
    plan.set_nodes(x)
    g = torch.zeros(10, dtype=torch.complex64, device="cuda")
    out = torch.zeros((1024, 1024), dtype=torch.complex64, device="cuda")
    st = plan._lib.bl_adjoint_noalloc(plan.handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert st == 6   # BL_EUNSUPPORTED
    assert b"scratch" in plan._lib.bl_last_error()
    plan.close()
