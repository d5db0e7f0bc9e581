"""Differentiation through torch.autograd: the hand-written backward (adjoint spreading +
forward FFT for grad fhat, psi' short sums for grad x) against the FP64 oracle and
against central finite differences evaluated with the FP64 GPU transform."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _setup(p, prec):
    import torch
    from paper_2502_07155_amd import Plan
    rdt = torch.float64 if prec == "f64" else torch.float32
    cdt = torch.complex128 if prec == "f64" else torch.complex64
    plan = Plan(p.d, p.M, p.L, p.m, precision=prec)
    fhat = torch.from_numpy(p.fhat).to(cdt).cuda().requires_grad_(True)
    x = torch.from_numpy(p.x).to(rdt).cuda().requires_grad_(True)
    y = torch.from_numpy(p.y).to(cdt).cuda()
    return plan, fhat, x, y


def _loss(plan, fhat, x, y):
    from paper_2502_07155_amd import bandlimited_nfft
    f = bandlimited_nfft(fhat, x, plan)
    return (f - y).abs().pow(2).sum()


@pytest.mark.parametrize("d,M,L,m,N", [(1, 64, 128, 5, 800), (2, 32, 64, 4, 1500), (3, 16, 32, 3, 700),
                                       (2, 40, 96, 5, 1200)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f32c", "f32d"])
def test_autograd_matches_oracle_gradients(d, M, L, m, N, prec):
    p = W.custom_problem(d, M, L, m, N, seed=500 + d, precision="f32" if prec != "f64" else "f64",
                         with_targets=True)
    plan, fhat, x, y = _setup(p, prec)
    loss = _loss(plan, fhat, x, y)
    loss.backward()
    f = O.forward_shannon(p.fhat, p.x, L, m)
    G = 2 * (f - p.y)
    g_fhat = O.adjoint_shannon(G, p.x, M, L, m)
    g_x = O.grad_x_shannon(p.fhat, G, p.x, L, m)
    tol = 1e-11 if prec == "f64" else 5e-5
    got_fhat = fhat.grad.cpu().numpy().astype(np.complex128)
    got_x = x.grad.cpu().numpy().astype(np.float64)
    assert O.rel_err_inf(got_fhat, g_fhat) <= tol
    assert O.rel_err_inf(got_x, g_x) <= tol


def test_backward_after_intervening_forward_restores_state():
    """A second forward on the same plan before backward must not change the gradients."""
    import torch
    p = W.custom_problem(2, 32, 64, 4, 1000, seed=77, with_targets=True)
    plan, fhat, x, y = _setup(p, "f64")
    loss = _loss(plan, fhat, x, y)
    other = W.custom_problem(2, 32, 64, 4, 300, seed=78)
    plan.set_nodes(torch.from_numpy(other.x).cuda())
    plan.forward(torch.from_numpy(other.fhat).cuda())
    loss.backward()
    f = O.forward_shannon(p.fhat, p.x, 64, 4)
    G = 2 * (f - p.y)
    assert O.rel_err_inf(x.grad.cpu().numpy(), O.grad_x_shannon(p.fhat, G, p.x, 64, 4)) <= 1e-11


def test_differentiation_workload_vs_finite_differences():
    """d=2, M=256, L=512, m=6, N=200000: FP32 forward + hand-written backward, checked
    along random directions against central differences (h = 1e-4) of the FP64 transform.
    grad fhat: the loss is quadratic in fhat, so central differences are exact up to
    rounding.  grad x: Richardson extrapolation (4 D(h/2) - D(h)) / 3 removes the
    O((pi M h)^2) truncation error of plain central differences."""
    import torch
    from paper_2502_07155_amd import Plan
    p = W.make_problem("d2_M256_L512_m6_N200k", precision="f32", with_targets=True)
    plan, fhat, x, y = _setup(p, "f32")
    loss = _loss(plan, fhat, x, y)
    loss.backward()
    gf = fhat.grad.detach().to(torch.complex128)
    gx = x.grad.detach().to(torch.float64)

    plan64 = Plan(p.d, p.M, p.L, p.m, precision="f64")
    fh64 = torch.from_numpy(p.fhat).cuda()
    x64 = torch.from_numpy(p.x).cuda()
    y64 = torch.from_numpy(p.y).cuda()

    def L64(fh, xx):
        plan64.set_nodes(xx)
        return float((plan64.forward(fh) - y64).abs().pow(2).sum())

    gen = torch.Generator(device="cuda").manual_seed(1234)
    h = 1e-4
    for _ in range(2):
        D = torch.complex(torch.randn(fh64.shape, generator=gen, device="cuda", dtype=torch.float64),
                          torch.randn(fh64.shape, generator=gen, device="cuda", dtype=torch.float64))
        fd = (L64(fh64 + h * D, x64) - L64(fh64 - h * D, x64)) / (2 * h)
        an = float((gf.real * D.real + gf.imag * D.imag).sum())
        assert abs(fd - an) <= 1e-4 * abs(an), (fd, an)
    for _ in range(2):
        Dx = torch.randn(x64.shape, generator=gen, device="cuda", dtype=torch.float64).clamp(-5, 5)
        # nodes within 1e-3 of +-1/2 are not moved, so every stencil point stays in [-1/2, 1/2)
        Dx = torch.where(x64.abs() > 0.5 - 1e-3, torch.zeros_like(Dx), Dx)
        c1 = (L64(fh64, x64 + h * Dx) - L64(fh64, x64 - h * Dx)) / (2 * h)
        c2 = (L64(fh64, x64 + h / 2 * Dx) - L64(fh64, x64 - h / 2 * Dx)) / h
        rich = (4 * c2 - c1) / 3
        an = float((gx * Dx).sum())
        assert abs(rich - an) <= 1e-4 * abs(an), (rich, an)
        assert abs(c1 - an) <= 2e-2 * abs(an), (c1, an)
