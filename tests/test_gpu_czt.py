"""Steps 1-2 and the adjoint for L that is not a power of two (and d = 1 lines longer than
the LDS transform): the chirp-z passes against the oracle, forward (samples theta and
short sums) and adjoint, in every precision.  Tolerances as in the other parity tests:
normwise max error / max |reference| of 1e-12 (FP64), 1e-5 (FP32), 1e-6 (FP32 with FP64
twiddles and compensated sums, and FP32 with FP64 passes)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f32c": 1e-6, "f32d": 1e-6}
THETA_TOL = {"f64": 1e-13, "f32": 1e-6, "f32c": 1e-6, "f32d": 1e-7}
PRECS = ["f64", "f32", "f32c", "f32d"]

# (d, M, L, m, N): L = 40 .. 12000 with M = L/2 (several prime factors: 40 = 2^3 5,
# 120 = 2^3 3 5, 2000 = 2^4 5^3, 12000 = 2^5 3 5^3), d = 1 lines that need the split
# path (P = 32768, 65536), and d = 2, 3 grids whose lines share a workgroup.
CASES = [
    (1, 20, 40, 5, 700),
    (1, 60, 120, 6, 900),
    (1, 500, 1000, 4, 1500),
    (1, 1000, 2000, 5, 2500),
    (1, 6000, 12000, 6, 3000),
    (1, 8192, 16384, 6, 3000),
    (1, 16384, 32768, 4, 3000),
    (1, 30, 34, 3, 500),
    (2, 48, 96, 4, 3000),
    (2, 80, 160, 5, 4000),
    (2, 400, 1000, 3, 5000),
    (3, 24, 48, 3, 3000),
    (3, 30, 40, 2, 2000),
]


def _dev(a, prec, cplx):
    import torch
    if cplx:
        dt = torch.complex128 if prec == "f64" else torch.complex64
    else:
        dt = torch.float64 if prec == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()


def _host(t):
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"d{c[0]}_M{c[1]}_L{c[2]}")
@pytest.mark.parametrize("prec", PRECS)
def test_chirp_z_forward_and_adjoint(case, prec):
    from paper_2502_07155_amd import Plan
    d, M, L, m, N = case
    p = W.custom_problem(d, M, L, m, N, seed=2000 + d * 7 + L, with_targets=True,
                         precision="f32" if prec != "f64" else "f64")
    plan = Plan(d, M, L, m, precision=prec)
    plan.set_nodes(_dev(p.x, prec, False))
    f = _host(plan.forward(_dev(p.fhat, prec, True)))
    theta = _host(plan.theta())
    fo, _, tho = O.forward_shannon(p.fhat, p.x, L, m, return_stages=True)
    a = _host(plan.adjoint(_dev(p.y, prec, True)))
    ao = O.adjoint_shannon(p.y, p.x, M, L, m)
    et, ef, ea = O.rel_err_inf(theta, tho), O.rel_err_inf(f, fo), O.rel_err_inf(a, ao)
    print(f"case d={d} M={M} L={L} m={m} N={N} {prec}: theta {et:.2e} f {ef:.2e} adjoint {ea:.2e}")
    assert et <= THETA_TOL[prec]
    assert ef <= TOL[prec]
    assert ea <= (TOL[prec] if prec != "f32" else 1e-5)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_chirp_z_classical_nfft(prec):
    """Algorithm 2.1 (phihat deconvolution, periodic window sums) at L = 120, 2 x 60."""
    from paper_2502_07155_amd import Plan
    for d, M, L, m, N in ((1, 60, 120, 5, 800), (2, 60, 120, 4, 3000)):
        p = W.custom_problem(d, M, L, m, N, seed=2100 + d, with_targets=True,
                             precision="f32" if prec != "f64" else "f64")
        plan = Plan(d, M, L, m, precision=prec, method="nfft")
        plan.set_nodes(_dev(p.x, prec, False))
        f = _host(plan.forward(_dev(p.fhat, prec, True)))
        assert O.rel_err_inf(f, O.forward_nfft(p.fhat, p.x, L, m)) <= TOL[prec]
        a = _host(plan.adjoint(_dev(p.y, prec, True)))
        assert O.rel_err_inf(a, O.adjoint_nfft(p.y, p.x, M, L, m)) <= TOL[prec]
        plan.close()


def test_chirp_z_refused_where_lines_exceed_lds():
    """d = 2 with L + M - 1 above the LDS transform: short sums still run, the transforms
    report BL_EUNSUPPORTED."""
    import torch
    from paper_2502_07155_amd import Plan
    from paper_2502_07155_amd._lib import BLNFFTError
    M, L = 4000, 6000   # P = 16384 > 8192 double points
    plan = Plan(2, M, L, 3, precision="f64")
    plan.set_nodes(torch.zeros((4, 2), dtype=torch.float64, device="cuda"))
    with pytest.raises(BLNFFTError) as e:
        plan.forward(torch.zeros((M, M), dtype=torch.complex128, device="cuda"))
    assert e.value.status == 6
    f = plan.interpolate(torch.zeros((L, L), dtype=torch.complex128, device="cuda"))
    assert torch.all(f == 0)
    plan.close()
