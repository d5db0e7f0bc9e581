"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types an oracle formula: each compares the oracle with an independent
route (closed forms, exact rational arithmetic, a dense matrix product, a direct
definition with pure-Python loops, invariants such as interpolation, separability and
the adjoint identity, finite differences, and the paper's own qualitative claims).
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import i0, i1, j1

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- elementary pieces

def test_scaled_offset_matches_exact_rationals():
    rng = np.random.default_rng(11)
    x = rng.random(400) - 0.5
    for a in (512, 1000, 2468, 16372, 4093):
        n = np.rint(a * x)
        got = O.scaled_offset(a, x, n)
        for xi, ni, gi in zip(x[:80], n[:80], got[:80]):
            exact = Fraction(a) * Fraction(float(xi)) - Fraction(int(ni))
            assert abs(Fraction(float(gi)) - exact) <= abs(exact) * Fraction(1, 2 ** 52) + Fraction(1, 2 ** 80)


def test_node_offsets_edge_distance_matches_exact_rationals():
    """e = m - |L x - l| for every candidate l, including nodes a few ulps from a grid
    point, where the window's square-root end makes that distance decide the weight."""
    rng = np.random.default_rng(12)
    for L, m in ((32, 5), (1024, 6), (4096, 8)):
        k = rng.integers(-L // 2, L // 2, 40)
        delta = np.concatenate([rng.random(20) - 0.5, 10.0 ** rng.uniform(-16, -12, 20)])
        x = (k + delta) / L
        ell, t, e = O.node_offsets(x, L, m)
        for i in range(x.size):
            for j in range(ell.shape[1]):
                exact = Fraction(m) - abs(Fraction(L) * Fraction(float(x[i])) - Fraction(int(ell[i, j])))
                assert abs(Fraction(float(e[i, j])) - exact) <= abs(exact) * Fraction(1, 2 ** 52) + Fraction(1, 2 ** 90)


def test_window_near_the_end_of_its_support():
    """Just inside |t| = m the sinh window is sinh(beta sqrt(1-(t/m)^2))/sinh(beta) with
    1 - (t/m)^2 = e (2m - e) / m^2, e = m - |t|; passing e exactly keeps that value where
    the rounded t cannot (eq. (3.4))."""
    m, beta = 5, 7.853981633974483
    for e in (6.7e-16, 1e-15, 3e-14, 1e-9):
        t = -(m - e)                                   # rounds in double
        exact = math.sinh(beta * math.sqrt(e * (2 * m - e)) / m) / math.sinh(beta)
        got = float(O.phi_g(np.array([t]), m, beta, "sinh", np.array([e]))[0])
        assert abs(got - exact) <= 1e-15 * exact


def test_sinpi_special_values_and_small_arguments():
    n = np.arange(-20, 21, dtype=np.float64)
    assert np.all(O.sinpi(n) == 0.0)
    assert np.all(O.sinpi(n + 0.5) == np.where(np.mod(n, 2) == 0, 1.0, -1.0))
    t = np.linspace(-0.25, 0.25, 101)
    assert np.max(np.abs(O.sinpi(t) - np.sin(np.pi * t))) < 4e-16
    # reduction: sin(pi (n + r)) = (-1)^n sin(pi r), near integers where the plain form fails
    r = np.array([1e-9, -3e-12, 2.5e-7])
    for k in (3.0, -8.0, 101.0):
        assert np.allclose(O.sinpi(k + r), (-1) ** abs(int(k)) * np.sin(np.pi * ((k + r) - k)),
                           rtol=1e-6, atol=0)


@pytest.mark.parametrize("win", ["sinh", "ckb"])
def test_windows_are_in_class_Phi_mL(win):
    """Section 3: even, supported on [-m/L, m/L], values in [0,1], non-increasing on
    [0, inf), phi(0) = 1."""
    for m, beta in [(4, 6.0), (6, 9.4), (8, 20.0)]:
        t = np.linspace(0, m + 2, 2001)
        ph = O.phi_g(t, m, beta, win)
        assert ph[0] == pytest.approx(1.0, abs=1e-15)
        assert np.all(ph >= 0) and np.all(ph <= 1.0 + 1e-15)
        assert np.all(np.diff(ph) <= 1e-15)
        assert np.all(ph[t >= m] == 0.0)
        assert np.array_equal(O.phi_g(-t, m, beta, win), ph)


def test_regularized_sinc_definition_points():
    """psi(u) = sinc(L pi u) phi(u) (4.2): psi vanishes at nonzero grid points and is 1 at 0."""
    m, beta = 6, O.default_beta(256, 512, 6)
    ell = np.arange(-m - 2, m + 3, dtype=np.float64)
    vals = O.psi_g(ell, m, beta)
    assert vals[ell == 0][0] == 1.0
    assert np.all(vals[ell != 0] == 0.0)


# ---------------------------------------------------------------- window transforms

def _phihat_sinh_closed(v, L, m, beta):
    """Fourier transform of the sinh-type window in closed form (Bessel I1 / J1)."""
    w = 2 * math.pi * m * v / L
    c = math.pi * m * beta / (L * math.sinh(beta))
    if abs(w) < beta:
        r = math.sqrt(beta * beta - w * w)
        return c * i1(r) / r
    if abs(w) > beta:
        r = math.sqrt(w * w - beta * beta)
        return c * j1(r) / r
    return c * 0.5


def _phihat_ckb_closed(v, L, m, beta):
    """Fourier transform of the continuous Kaiser-Bessel window in closed form."""
    w = 2 * math.pi * m * v / L
    pre = (m / L) / (i0(beta) - 1.0)
    sw = 2.0 if w == 0 else 2.0 * math.sin(w) / w
    if abs(w) < beta:
        r = math.sqrt(beta * beta - w * w)
        return pre * (2.0 * math.sinh(r) / r - sw)
    if abs(w) > beta:
        r = math.sqrt(w * w - beta * beta)
        return pre * (2.0 * math.sin(r) / r - sw)
    return pre * (2.0 - sw)


@pytest.mark.parametrize("L,M,m", [(512, 256, 6), (1024, 512, 5), (80, 40, 5), (256, 128, 4)])
def test_phihat_quadrature_vs_closed_form(L, M, m):
    beta = O.default_beta(M, L, m)
    v = np.array([0.0, 0.5, 3.0, M / 4, M / 2 - 1, M / 2, L / 2, 0.8 * L])
    got = O.phihat1(v, L, m, beta, "sinh")
    ref = np.array([_phihat_sinh_closed(vi, L, m, beta) for vi in v])
    assert np.max(np.abs(got - ref)) < 1e-15 * m / L * 200
    beta2 = O.default_beta(M, L, m, "nfft")
    got2 = O.phihat1(v, L, m, beta2, "sinh")
    ref2 = np.array([_phihat_sinh_closed(vi, L, m, beta2) for vi in v])
    assert np.max(np.abs(got2 - ref2)) < 1e-15 * m / L * 200
    got3 = O.phihat1(v, L, m, beta, "ckb")
    ref3 = np.array([_phihat_ckb_closed(vi, L, m, beta) for vi in v])
    assert np.max(np.abs(got3 - ref3)) < 1e-15 * m / L * 200


@pytest.mark.parametrize("L,M,m", [(512, 256, 6), (80, 40, 5)])
def test_psihat_is_box_convolution_of_phihat(L, M, m):
    """psi = sinc(L pi .) phi, and the transform of sinc(L pi u) is (1/L) on [-L/2, L/2],
    so psihat(v) = (1/L) int_{v-L/2}^{v+L/2} phihat(w) dw (convolution theorem)."""
    beta = O.default_beta(M, L, m)
    for v in (0.0, 7.0, M / 2 - 1, -M / 2, 0.75 * L):
        val, _ = quad(lambda w: _phihat_sinh_closed(w, L, m, beta), v - L / 2, v + L / 2,
                      limit=800, epsabs=1e-17, epsrel=1e-13)
        assert O.psihat1(v, L, m, beta)[0] == pytest.approx(val / L, rel=1e-12, abs=2e-14 / L)


def test_psihat_quadrature_converged_and_near_one_over_L():
    """Section 5 observes |I_L| psihat(k) ~ 1 on I_M for these windows."""
    for (M, L, m) in [(256, 512, 6), (512, 1024, 5), (128, 256, 4), (40, 80, 5)]:
        beta = O.default_beta(M, L, m)
        k = O.band(M)
        a = O.psihat1(k, L, m, beta, nq=256)
        b = O.psihat1(k, L, m, beta, nq=512)
        assert np.max(np.abs(a - b)) * L < 1e-13
        assert np.max(np.abs(L * a - 1.0)) < 2e-2
        assert np.all(a > 0)


# ---------------------------------------------------------------- FFT step and wiring

def _dft_definition_1d(hat, L):
    """(4.7) written out with pure-Python loops, phases reduced in integers."""
    out = []
    for ell in range(-L // 2, L // 2):
        s = 0j
        for i, k in enumerate(range(-L // 2, L // 2)):
            ph = ((k * ell) % L) / L
            s += hat[i] * complex(math.cos(2 * math.pi * ph), math.sin(2 * math.pi * ph))
        out.append(s / L)
    return np.array(out)


def test_inverse_fft_step_matches_definition():
    rng = np.random.default_rng(3)
    for L in (8, 12, 16):
        hat = rng.standard_normal(L) + 1j * rng.standard_normal(L)
        assert np.max(np.abs(O.inverse_fft_step(hat) - _dft_definition_1d(hat, L))) < 1e-15
    # d = 2: row/column application of the 1-D definition
    L = 8
    hat = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
    rows = np.array([_dft_definition_1d(r, L) for r in hat])
    both = np.array([_dft_definition_1d(c, L) for c in rows.T]).T
    assert np.max(np.abs(O.inverse_fft_step(hat) - both)) < 1e-15


@pytest.mark.parametrize("d,M,L,m,N", [(1, 8, 16, 3, 40), (1, 10, 14, 2, 30), (2, 6, 12, 2, 25),
                                       (2, 8, 12, 3, 20), (3, 4, 8, 2, 12)])
@pytest.mark.parametrize("method", ["shannon", "nfft"])
def test_fast_equals_dense_matrix_form(d, M, L, m, N, method):
    """(4.11) f = Psi F D_psihat fhat (and B F D fhat for Algorithm 2.1) as dense matrices."""
    p = W.custom_problem(d, M, L, m, N, seed=100 + d + L)
    beta = O.default_beta(M, L, m, method)
    if method == "shannon":
        fast = O.forward_shannon(p.fhat, p.x, L, m, beta)
    else:
        fast = O.forward_nfft(p.fhat, p.x, L, m, beta)
    dense = O.dense_forward(p.fhat, p.x, L, m, beta, method=method)
    assert O.rel_err_inf(fast, dense) < 1e-13


def test_gather_definition_pure_python_tiny():
    """Step 3 of Algorithm 4.2 with the index set J_{L,m}(x) of (4.8) enumerated
    term by term; psi written from (4.2) with math.sin / math.sinh."""
    L, m, M = 12, 3, 6
    beta = O.default_beta(M, L, m)
    rng = np.random.default_rng(5)
    theta = rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))
    x = rng.random((15, 2)) - 0.5

    def psi1(u):
        z = L * math.pi * u
        s = 1.0 if z == 0 else math.sin(z) / z
        q = L * u / m
        if abs(q) > 1:
            return 0.0
        return s * math.sinh(beta * math.sqrt(1 - q * q)) / math.sinh(beta)

    ref = []
    for xj in x:
        tot = 0j
        for l1 in range(math.ceil(L * xj[0] - m), math.floor(L * xj[0] + m) + 1):
            for l2 in range(math.ceil(L * xj[1] - m), math.floor(L * xj[1] + m) + 1):
                if -L // 2 <= l1 < L // 2 and -L // 2 <= l2 < L // 2:
                    tot += theta[l1 + L // 2, l2 + L // 2] * psi1(xj[0] - l1 / L) * psi1(xj[1] - l2 / L)
        ref.append(tot)
    got = O.gather_shannon(theta, x, L, m, beta)
    assert np.max(np.abs(got - np.array(ref))) < 1e-13


def test_interpolation_property():
    """Section 3: R f(k/L) = f(k/L); the short sums at x = l/L return theta_l exactly."""
    M, L, m = 16, 32, 5
    beta = O.default_beta(M, L, m)
    rng = np.random.default_rng(8)
    fh = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    _, _, theta = O.forward_shannon(fh, np.zeros((1, 2)), L, m, beta, return_stages=True)
    ells = np.array(list(itertools.product(range(-L // 2, L // 2), repeat=2)))
    x = ells / L
    f = O.gather_shannon(theta, x, L, m, beta)
    ref = theta[ells[:, 0] + L // 2, ells[:, 1] + L // 2]
    assert np.max(np.abs(f - ref)) < 1e-14 * np.max(np.abs(theta))


def test_separability_tensor_product_input():
    """A tensor-product fhat gives the product of 1-D outputs (pins axis order)."""
    M, L, m = 32, 64, 5
    rng = np.random.default_rng(9)
    a = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    b = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    x = rng.random((60, 3)) - 0.5
    f2 = O.forward_shannon(np.multiply.outer(a, b), x[:, :2], L, m)
    fa = O.forward_shannon(a, x[:, :1], L, m)
    fb = O.forward_shannon(b, x[:, 1:2], L, m)
    assert O.rel_err_inf(f2, fa * fb) < 1e-13
    f3 = O.forward_shannon(np.multiply.outer(np.multiply.outer(a, b), c), x, L, m)
    fc = O.forward_shannon(c, x[:, 2:3], L, m)
    assert O.rel_err_inf(f3, fa * fb * fc) < 1e-13


# ---------------------------------------------------------------- targets

def test_direct_sum_pure_python_tiny():
    M = 6
    rng = np.random.default_rng(12)
    fh = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    x = rng.random((7, 2)) - 0.5
    ref = []
    for xj in x:
        s = 0j
        for i1_, k1 in enumerate(range(-M // 2, M // 2)):
            for i2_, k2 in enumerate(range(-M // 2, M // 2)):
                ph = 2 * math.pi * (k1 * xj[0] + k2 * xj[1])
                s += fh[i1_, i2_] * complex(math.cos(ph), math.sin(ph))
        ref.append(s)
    assert np.max(np.abs(O.direct_sum(fh, x) - np.array(ref))) < 1e-13


def test_direct_sum_of_ones_is_dirichlet_product():
    """sum_{k in I_M} e^{2 pi i k x} = e^{-i pi x} sin(M pi x)/sin(pi x), per dimension."""
    rng = np.random.default_rng(13)
    for d, M in [(1, 256), (2, 64), (3, 16)]:
        x = rng.random((40, d)) - 0.5
        ones = np.ones((M,) * d, dtype=np.complex128)
        assert O.rel_err_inf(O.direct_sum(ones, x), O.dirichlet(x, M)) < 1e-12


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8, 10])
def test_error_vs_direct_sum_decays_like_exp_minus_beta(m):
    """Accuracy target of Algorithm 4.2 (reading of the cited estimates): on nodes of the
    truncated domain, max error / max |f| <= d exp(-beta), beta = pi m (L-M)/L."""
    M, L = 256, 512
    p = W.custom_problem(1, M, L, m, 800, seed=20 + m, nodes="truncated")
    err = O.rel_err_inf(O.forward_shannon(p.fhat, p.x, L, m), O.direct_sum(p.fhat, p.x))
    assert err <= math.exp(-O.default_beta(M, L, m))
    assert err >= 1e-3 * math.exp(-O.default_beta(M, L, m))   # not suspiciously exact


def test_error_decays_with_oversampling_and_in_two_dims():
    m = 6
    errs = []
    for L in (384, 512, 768, 1024):
        p = W.custom_problem(1, 256, L, m, 600, seed=31, nodes="truncated")
        e = O.rel_err_inf(O.forward_shannon(p.fhat, p.x, L, m), O.direct_sum(p.fhat, p.x))
        assert e <= math.exp(-O.default_beta(256, L, m))
        errs.append(e)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    p = W.custom_problem(2, 128, 256, 5, 400, seed=32, nodes="truncated")
    e2 = O.rel_err_inf(O.forward_shannon(p.fhat, p.x, 256, 5), O.direct_sum(p.fhat, p.x))
    assert e2 <= 2 * math.exp(-O.default_beta(128, 256, 5))


def test_ones_reproduce_dirichlet_not_sinc():
    """fhat = 1 on I_M: the method reproduces prod D_M(x_t) to the method's accuracy; the
    continuous-band target prod M sinc(M pi x_t) differs by the periodisation."""
    for d, M, L, m in [(1, 256, 512, 6), (2, 64, 128, 5), (3, 32, 64, 4)]:
        rng = np.random.default_rng(40 + d)
        a = 0.5 - m / L
        x = (rng.random((150, d)) * 2 - 1) * a
        f = O.forward_shannon(np.ones((M,) * d, dtype=np.complex128), x, L, m)
        dm = O.dirichlet(x, M)
        beta = O.default_beta(M, L, m)
        assert O.rel_err_inf(f, dm) <= d * math.exp(-beta)
        sincs = np.prod(M * O.sinc_pi(M * x), axis=1)
        assert O.rel_err_inf(f, sincs) > O.rel_err_inf(f, dm)


def test_boundary_nodes_are_outside_the_method_domain():
    """Section 5 (Figure 5.1a): outside the truncated domain the approximation fails."""
    M, L, m = 256, 512, 6
    rng = np.random.default_rng(50)
    x = np.concatenate([0.5 - rng.random((50, 1)) * (m / L), -0.5 + rng.random((50, 1)) * (m / L) * 0.5])
    fh = W.complex_normal(rng, M)
    e = O.rel_err_inf(O.forward_shannon(fh, x, L, m), O.direct_sum(fh, x))
    assert e > 0.05


def test_nfft_with_standard_beta_tracks_direct_sum():
    p = W.custom_problem(1, 256, 512, 6, 500, seed=3)
    err = O.rel_err_inf(O.forward_nfft(p.fhat, p.x, 512, 6), O.direct_sum(p.fhat, p.x))
    assert err < 1e-9


def test_example_5_1_qualitative_outcome():
    """Example 5.1: equal errors for M <= 80, then only Algorithm 4.2 keeps improving."""
    with open(os.path.join(GOLDEN, "example_5_1.json")) as fh:
        g = json.load(fh)
    m = g["m"]
    res = {}
    for M in g["M_values"]:
        L = (1 + g["lambda"]) * M
        N = M // 2
        x = W.chebyshev_nodes(N, L, m)[:, None]
        fh_ = W.triangle_fhat(M)
        exact = O.example51_f(x[:, 0], M)
        beta = O.default_beta(M, L, m)
        e_bl = np.max(np.abs(O.forward_shannon(fh_, x, L, m, beta) - exact))
        e_nf = np.max(np.abs(O.forward_nfft(fh_, x, L, m, beta) - exact))
        res[M] = (e_bl, e_nf)
    assert sorted(res) == list(range(20, 1001, 20))
    # equal errors for M <= 80
    for M in (20, 40, 60, 80):
        assert res[M][1] / res[M][0] < 1.2
    # beyond that Algorithm 2.1 (same beta) stalls at its M = 100 level ...
    for M in range(100, 1001, 20):
        assert abs(res[M][1] / res[100][1] - 1.0) < 0.01
    # ... while Algorithm 4.2 keeps improving, well below it
    assert res[1000][0] < res[20][0] / 300
    assert res[1000][0] < res[100][0] / 40
    for M in range(120, 1001, 20):
        assert res[M][0] < res[M][1] / 2


# ---------------------------------------------------------------- adjoint and gradients

@pytest.mark.parametrize("d,M,L,m,N", [(1, 16, 32, 4, 50), (2, 8, 16, 3, 40), (3, 4, 8, 2, 15)])
def test_adjoint_inner_product_identity(d, M, L, m, N):
    p = W.custom_problem(d, M, L, m, N, seed=60 + d, with_targets=True)
    Af = O.forward_shannon(p.fhat, p.x, L, m)
    AHg = O.adjoint_shannon(p.y, p.x, M, L, m)
    lhs = np.vdot(p.y, Af)
    rhs = np.vdot(AHg, p.fhat)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    Bf = O.forward_nfft(p.fhat, p.x, L, m)
    BHg = O.adjoint_nfft(p.y, p.x, M, L, m)
    assert abs(np.vdot(p.y, Bf) - np.vdot(BHg, p.fhat)) < 1e-13 * abs(np.vdot(p.y, Bf))


def test_adjoint_equals_dense_conjugate_transpose():
    d, M, L, m, N = 2, 6, 12, 2, 20
    p = W.custom_problem(d, M, L, m, N, seed=70, with_targets=True)
    beta = O.default_beta(M, L, m)
    A = O.dense_Psi(p.x, L, m, beta) @ O.dense_F(M, L, d) @ np.diag(O.dense_D(M, L, d, m, beta))
    ref = (A.conj().T @ p.y).reshape(M, M)
    assert O.rel_err_inf(O.adjoint_shannon(p.y, p.x, M, L, m), ref) < 1e-13


def test_adjoint_entries_equal_dense_conjugate_transpose():
    """adjoint_at (entries of A^H g one frequency at a time) against the dense A^H of (4.11)
    and the dense B^H of (2.4)-(2.6), including nodes whose windows leave I_L."""
    d, M, L, m, N = 2, 6, 12, 2, 20
    p = W.custom_problem(d, M, L, m, N, seed=71, with_targets=True)
    ks = np.array([[-3, -3], [0, 0], [2, -1], [-1, 2], [2, 2]])
    idx = tuple((ks + M // 2).T)
    beta = O.default_beta(M, L, m)
    A = O.dense_Psi(p.x, L, m, beta) @ O.dense_F(M, L, d) @ np.diag(O.dense_D(M, L, d, m, beta))
    ref = (A.conj().T @ p.y).reshape(M, M)[idx]
    assert O.rel_err_inf(O.adjoint_at(p.y, p.x, M, L, m, ks), ref) < 1e-13
    bn = O.default_beta(M, L, m, "nfft")
    B = O.dense_B(p.x, L, m, bn) @ O.dense_F(M, L, d) @ np.diag(O.dense_D(M, L, d, m, bn, method="nfft"))
    refn = (B.conj().T @ p.y).reshape(M, M)[idx]
    assert O.rel_err_inf(O.adjoint_at(p.y, p.x, M, L, m, ks, method="nfft"), refn) < 1e-13


@pytest.mark.parametrize("d,M,L,m,N", [(1, 16, 40, 4, 60), (3, 8, 16, 3, 50)])
def test_adjoint_entries_equal_fft_adjoints(d, M, L, m, N):
    p = W.custom_problem(d, M, L, m, N, seed=72 + d, with_targets=True)
    ks = W.rng_for(73).integers(-M // 2, M // 2, size=(6, d))
    idx = tuple((ks + M // 2).T)
    full = O.adjoint_shannon(p.y, p.x, M, L, m)
    assert O.rel_err_inf(O.adjoint_at(p.y, p.x, M, L, m, ks), full[idx]) < 1e-13
    fulln = O.adjoint_nfft(p.y, p.x, M, L, m)
    assert O.rel_err_inf(O.adjoint_at(p.y, p.x, M, L, m, ks, method="nfft"), fulln[idx]) < 1e-13


def test_grad_x_matches_richardson_finite_differences():
    M, L, m = 16, 32, 4
    p = W.custom_problem(2, M, L, m, 20, seed=5, with_targets=True)
    f = O.forward_shannon(p.fhat, p.x, L, m)
    gx = O.grad_x_shannon(p.fhat, 2 * (f - p.y), p.x, L, m)
    D = np.random.default_rng(1).standard_normal(p.x.shape)

    def loss(xx):
        return np.sum(np.abs(O.forward_shannon(p.fhat, xx, L, m) - p.y) ** 2)

    h = 1e-4
    c1 = (loss(p.x + h * D) - loss(p.x - h * D)) / (2 * h)
    c2 = (loss(p.x + h / 2 * D) - loss(p.x - h / 2 * D)) / h
    rich = (4 * c2 - c1) / 3
    ana = np.sum(gx * D)
    assert abs(rich - ana) < 1e-6 * abs(ana)


def test_grad_fhat_is_adjoint_of_residual():
    """For loss = sum |A fhat - y|^2 the conjugate-Wirtinger gradient is A^H 2(f - y);
    checked against central differences along a random complex direction."""
    M, L, m = 16, 32, 4
    p = W.custom_problem(1, M, L, m, 30, seed=6, with_targets=True)
    f = O.forward_shannon(p.fhat, p.x, L, m)
    g = O.adjoint_shannon(2 * (f - p.y), p.x, M, L, m)
    D = W.complex_normal(np.random.default_rng(2), p.fhat.shape)

    def loss(fh):
        return np.sum(np.abs(O.forward_shannon(fh, p.x, L, m) - p.y) ** 2)

    h = 1e-3
    fd = (loss(p.fhat + h * D) - loss(p.fhat - h * D)) / (2 * h)
    ana = np.sum(g.real * D.real + g.imag * D.imag)
    assert abs(fd - ana) < 1e-8 * abs(ana)


@pytest.mark.parametrize("win", ["sinh", "ckb"])
@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8])
def test_dphi_dpsi_match_difference_quotients(win, m):
    """The window derivatives (sinh eq. (3.4), continuous Kaiser-Bessel Remark 3.1) and
    the regularized-sinc derivative against central differences of phi_g and psi_g, which
    share no code with the derivative formulas; zero at and beyond the end of the support."""
    beta = O.default_beta(256, 512, m)
    t = np.linspace(-m + 0.01, m - 0.01, 197)
    h = 1e-6
    fd_phi = (O.phi_g(t + h, m, beta, win) - O.phi_g(t - h, m, beta, win)) / (2 * h)
    assert np.max(np.abs(O.dphi_g(t, m, beta, win) - fd_phi)) < 1e-7
    fd_psi = (O.psi_g(t + h, m, beta, win) - O.psi_g(t - h, m, beta, win)) / (2 * h)
    assert np.max(np.abs(O.dpsi_g(t, m, beta, win) - fd_psi)) < 1e-7
    edge = np.array([-m, m, m + 1.0, -m - 0.5])
    assert np.all(O.dpsi_g(edge, m, beta, win) == 0.0)
    assert np.all(O.dphi_g(edge, m, beta, win) == 0.0)


def test_dphi_ckb_has_a_finite_limit_at_the_support_end():
    """The continuous Kaiser-Bessel window ends like 1 - (t/m)^2 (Remark 3.1), so its
    derivative tends to the one-sided difference quotient at |t| = m, unlike the sinh
    window's square-root end; the limit is -2 beta^2 / (2 m (I0(beta) - 1)) by the series
    I0(z) = 1 + z^2/4 + ...  (d/dt of beta^2 (1 - (t/m)^2) / 4 at t = m)."""
    from scipy.special import i0
    m = 5
    beta = O.default_beta(256, 512, m)
    lim = -beta ** 2 / (2.0 * m * (i0(beta) - 1.0))
    t = m - 1e-7
    assert abs(float(O.dphi_g(np.array([t]), m, beta, "ckb")[0]) - lim) < 1e-6 * abs(lim)
    h = 1e-5
    one_sided = (O.phi_g(np.array([m - h]), m, beta, "ckb")[0] - 0.0) / (-h)
    assert abs(one_sided - lim) < 1e-4 * abs(lim)


# ---------------------------------------------------------------- Figure 5.1

def test_exponential_approximations_at_integer_frequencies_equal_the_transforms():
    """At an integer v = k in I_M the right-hand side of (5.1) is Algorithm 2.1 applied to
    the unit coefficient vector e_k, and that of (5.2) is Algorithm 4.2 applied to e_k times
    L psihat(k) (the deconvolution (5.2) leaves out): an explicit-exponential path against
    the FFT path."""
    M, L, m = 20, 40, 5
    x = np.linspace(-0.5 + m / L, 0.5 - m / L, 301)[:-1, None]
    b = O.default_beta(M, L, m)
    for k in (-10, -3, 0, 7, 9):
        e = np.zeros(M, dtype=np.complex128)
        e[k + M // 2] = 1.0
        nf = O.forward_nfft(e, x, L, m, b)
        assert np.max(np.abs(O.exp_approx_nfft(float(k), x[:, 0], L, m, b) - nf)) <= 1e-13 * np.max(np.abs(nf))
        sh = O.forward_shannon(e, x, L, m, b) * L * O.psihat1(float(k), L, m, b)[0]
        assert np.max(np.abs(O.exp_approx_shannon(float(k), x[:, 0], L, m, b) - sh)) <= 1e-13 * np.max(np.abs(sh))


def _fig51_errors(x, L, m, vs, beta_nfft):
    M = 20
    b = O.default_beta(M, L, m)
    e_sh, e_nf = [], []
    for v in vs:
        ex = np.exp(2j * np.pi * v * x)
        e_sh.append(np.max(np.abs(ex - O.exp_approx_shannon(v, x, L, m, b))))
        e_nf.append(np.max(np.abs(ex - O.exp_approx_nfft(v, x, L, m, beta_nfft))))
    return np.array(e_sh), np.array(e_nf)


def test_figure_5_1_qualitative_outcome():
    """Figure 5.1's statements (coarse grid: S = 4, 2000 points): on [-1/2, 1/2) the sum
    (5.2) fails everywhere and (5.1) works only at integer v; on the truncated interval both
    work for |v| <= M/2 and fail beyond, (5.2) with the smaller error when both use the same
    beta.  With the standard NFFT beta, (5.1) beats (5.2) instead (reading A1)."""
    g = json.load(open(os.path.join(GOLDEN, "figure_5_1.json")))
    M, L, m = g["M"], g["L"], g["m"]
    vs = O.fig51_frequencies(M, m, 4)
    inband = np.abs(vs) <= M / 2
    integer = np.abs(vs - np.rint(vs)) < 1e-12
    P = 2000
    full = -0.5 + np.arange(P) / P
    a, b = -0.5 + m / L, 0.5 - m / L
    trunc = a + np.arange(P) * (b - a) / P
    same = O.default_beta(M, L, m)
    sh, nf = _fig51_errors(full, L, m, vs, same)
    assert sh.min() > 0.5
    assert nf[inband & integer].max() < 0.02 and nf[inband & ~integer].max() > 1.0
    sh, nf = _fig51_errors(trunc, L, m, vs, same)
    assert sh[inband].max() < 1e-3 and nf[inband].max() < 2e-2
    assert sh[np.abs(vs) >= M / 2 + 1].min() > 5 * sh[inband].max()   # grows beyond the band
    assert sh[np.abs(vs) >= M / 2 + m - 1e-9].min() > 0.1
    assert sh[inband].max() < nf[inband].max() / 5
    _, nf_std = _fig51_errors(trunc, L, m, vs[inband], O.default_beta(M, L, m, "nfft"))
    assert nf_std.max() < sh[inband].max() / 100
