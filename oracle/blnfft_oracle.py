"""FP64 CPU oracle for the NFFT-like procedure for bandlimited functions
(Kircheis & Potts, "Nonequispaced fast Fourier transforms for bandlimited functions").

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's oracle
leg (its CPU baseline and its error checks) may import or run this module.  The GPU library never calls it, shares no code
with it, and must fail loudly rather than fall back to it.

Everything here is plain, slow and written to be checked against the paper by eye:
float64 / complex128 numpy, a library FFT as the one allowed primitive for the iFFT
step, Gauss-Legendre quadrature for the window transforms, and loops over the
(2m+1)^d candidate neighbours of each node exactly as the index sets are defined.

Notation (paper, Sections 1-4): d dimensions, bandwidth M (even), oversampled grid L
(even, L >= M), truncation m with 2m < L, band I_M = [-M/2, M/2)^d as integer vectors,
nodes x_j in [-1/2, 1/2)^d.  Arrays over I_M or I_L are stored centred: array index
i_t holds k_t = i_t - M/2 (or l_t = i_t - L/2).

Readings of points the paper leaves open:
* The d-variate window is the tensor product of the univariate one, so psi and its
  transform factor over dimensions.
* L must be even (I_L is defined like I_M, which needs an even size).
* Nodes outside the truncated domain [-1/2 + m/L, 1/2 - m/L)^d are evaluated with the
  zero-extended sum over l in I_L (samples theta_l with l outside I_L are zero), as the
  first form of the final sum in Section 4 states.
* The sinh-type window's beta defaults to pi*m*(L-M)/L for the bandlimited method; the
  classical NFFT defaults to 2*pi*m*(1 - M/(2L)).  Both are arguments.
* The adjoint is the exact matrix adjoint of the factorisation (4.11).

Functions whose result has no pin other than the others here are marked
"parity unpinned" in their docstring.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

# ---------------------------------------------------------------------------
# Accurate elementary pieces
# ---------------------------------------------------------------------------

_SPLIT = 134217729.0  # 2^27 + 1, Veltkamp splitting constant for float64


def _veltkamp(x: np.ndarray):
    """Split float64 x into hi + lo with hi holding at most 26 significant bits."""
    c = _SPLIT * x
    hi = c - (c - x)
    return hi, x - hi


def scaled_offset(a, x, n):
    """Return a*x - n with a single rounding.

    `a` and `n` are integer-valued (|a| < 2^26).  a*hi and a*lo are exact products
    of the Veltkamp halves, a*hi - n is exact because the two are close, so only the
    final addition rounds.  Used for L*x_j - l (the grid offset of a node) and for the
    phase k*x_j of the direct sum, where a plain product would lose up to ~1e-13."""
    a = np.asarray(a, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    hi, lo = _veltkamp(x)
    return (a * hi - n) + a * lo


def sinpi(t: np.ndarray) -> np.ndarray:
    """sin(pi t) with exact reduction: t = n + r, |r| <= 1/2, sin(pi t) = (-1)^n sin(pi r)."""
    t = np.asarray(t, dtype=np.float64)
    n = np.rint(t)
    r = t - n
    sign = np.where(np.fmod(np.abs(n), 2.0) == 0.0, 1.0, -1.0)
    return sign * np.sin(np.pi * r)


def cospi(t: np.ndarray) -> np.ndarray:
    """cos(pi t) with exact reduction."""
    t = np.asarray(t, dtype=np.float64)
    n = np.rint(t)
    r = t - n
    sign = np.where(np.fmod(np.abs(n), 2.0) == 0.0, 1.0, -1.0)
    return sign * np.cos(np.pi * r)


def sinc_pi(t: np.ndarray) -> np.ndarray:
    """sinc(pi t) = sin(pi t) / (pi t), with sinc(0) = 1 (Section 3)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.ones_like(t)
    nz = t != 0.0
    out[nz] = sinpi(t[nz]) / (np.pi * t[nz])
    return out


def dsinc_pi(t: np.ndarray) -> np.ndarray:
    """d/dt sinc(pi t) = (pi t cos(pi t) - sin(pi t)) / (pi t^2); -pi^2 t/3 near 0."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    small = np.abs(t) < 1e-4
    ts = t[small]
    z = np.pi * ts
    out[small] = np.pi * (-z / 3.0 + z ** 3 / 30.0)
    tb = t[~small]
    out[~small] = (np.pi * tb * cospi(tb) - sinpi(tb)) / (np.pi * tb * tb)
    return out


# ---------------------------------------------------------------------------
# Window functions of Remark 3.1, written in grid units t = L*u
# (phi(u) = phi_g(L*u); the support [-m/L, m/L] becomes |t| <= m).
# ---------------------------------------------------------------------------

def default_beta(M: int, L: int, m: int, method: str = "shannon") -> float:
    """beta for the sinh-type window (3.4); the paper only asks for "certain beta > 0".

    shannon: beta = pi*m*(L-M)/L = pi*m*lambda/(1+lambda), the choice of the regularized
             Shannon literature the paper builds on.
    nfft:    beta = 2*pi*m*(1 - M/(2L)), the usual NFFT choice for oversampling L/M."""
    if method == "shannon":
        return math.pi * m * (L - M) / L
    if method == "nfft":
        return 2.0 * math.pi * m * (1.0 - M / (2.0 * L))
    raise ValueError(method)


def _edge(t, m: int, e):
    """Distance m - |t| to the end of the support: the given e, else formed from t."""
    t = np.asarray(t, dtype=np.float64)
    return (m - np.abs(t)) if e is None else np.asarray(e, dtype=np.float64)


def _root(t, m: int, e) -> np.ndarray:
    """sqrt(1 - (t/m)^2) for |t| <= m, as sqrt(e (m + |t|)) / m with e = m - |t|: near the
    end of the support the value depends on e only, which callers can pass exactly."""
    t = np.asarray(t, dtype=np.float64)
    return np.sqrt(np.maximum(e, 0.0) * (m + np.abs(t))) / m


def phi_g(t, m: int, beta: float, win: str = "sinh", e=None) -> np.ndarray:
    """Window phi in grid units, zero outside |t| <= m.

    sinh: sinh(beta*sqrt(1-(t/m)^2)) / sinh(beta)               eq. (3.4)
    ckb:  (I0(beta*sqrt(1-(t/m)^2)) - 1) / (I0(beta) - 1)       Remark 3.1
    e: optional m - |t| computed without the rounding of t (see node_offsets); the sinh
    window grows like sqrt(m - |t|) at the end of its support, so there that distance
    decides the value."""
    t = np.asarray(t, dtype=np.float64)
    e = _edge(t, m, e)
    inside = e >= 0.0
    s = _root(t, m, e)
    if win == "sinh":
        val = np.sinh(beta * s) / np.sinh(beta)
    elif win == "ckb":
        val = (np.i0(beta * s) - 1.0) / (np.i0(beta) - 1.0)
    else:
        raise ValueError(win)
    return np.where(inside, val, 0.0)


def dphi_g(t, m: int, beta: float, win: str = "sinh", e=None) -> np.ndarray:
    """d/dt of phi_g.  For sinh it behaves like 1/sqrt(m-|t|) at the edge; the value at
    |t| = m itself (and outside) is returned as 0 (it is only ever multiplied by a sinc
    factor that vanishes there).  e as in phi_g."""
    t = np.asarray(t, dtype=np.float64)
    e = _edge(t, m, e)
    inside = e > 0.0
    qq = np.where(inside, t / m, 0.0)
    s = _root(t, m, np.where(inside, e, 0.0))
    s_safe = np.where(inside, s, 1.0)
    dsdt = -(qq / m) / s_safe
    if win == "sinh":
        val = beta * np.cosh(beta * s) / math.sinh(beta) * dsdt
    elif win == "ckb":
        from scipy.special import i1
        val = beta * i1(beta * s) / (np.i0(beta) - 1.0) * dsdt
    else:
        raise ValueError(win)
    return np.where(inside, val, 0.0)


def psi_g(t, m: int, beta: float, win: str = "sinh", e=None) -> np.ndarray:
    """Regularized sinc (4.2) in grid units: psi(u) = sinc(L pi u) phi(u), t = L u."""
    return sinc_pi(t) * phi_g(t, m, beta, win, e)


def dpsi_g(t, m: int, beta: float, win: str = "sinh", e=None) -> np.ndarray:
    """d/dt of psi_g; zero at |t| >= m (psi is C^1 there)."""
    t = np.asarray(t, dtype=np.float64)
    inside = _edge(t, m, e) > 0.0
    val = dsinc_pi(t) * phi_g(t, m, beta, win, e) + sinc_pi(t) * dphi_g(t, m, beta, win, e)
    return np.where(inside, val, 0.0)


# ---------------------------------------------------------------------------
# Continuous Fourier transforms of the windows (convention (3.1)), by quadrature.
# psi is even and real, so psihat(v) = (2/L) * int_0^m psi_g(t) cos(2 pi v t / L) dt.
# The substitution t = m sin(theta) turns sqrt(1 - (t/m)^2) into cos(theta) and
# removes the square-root edge behaviour; Gauss-Legendre on [0, pi/2] then converges
# exponentially.
# ---------------------------------------------------------------------------

_GL_CACHE: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def _gauss_legendre(n: int):
    if n not in _GL_CACHE:
        z, w = np.polynomial.legendre.leggauss(n)
        th = (z + 1.0) * (np.pi / 4.0)
        _GL_CACHE[n] = (th, w * (np.pi / 4.0))
    return _GL_CACHE[n]


def _window_in_theta(theta, beta, win):
    c = np.cos(theta)
    if win == "sinh":
        return np.sinh(beta * c) / math.sinh(beta)
    if win == "ckb":
        return (np.i0(beta * c) - 1.0) / (np.i0(beta) - 1.0)
    raise ValueError(win)


def psihat1(v, L: int, m: int, beta: float, win: str = "sinh", nq: int = 256) -> np.ndarray:
    """Univariate psihat(v) = int psi(u) e^{-2 pi i v u} du (Algorithm 4.2, step 0a)."""
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    th, w = _gauss_legendre(nq)
    t = m * np.sin(th)
    g = sinc_pi(t) * _window_in_theta(th, beta, win) * m * np.cos(th)
    # cos(2 pi v t / L) for every (v, node)
    arg = 2.0 * np.outer(v, t) / L
    return (2.0 / L) * (cospi(arg) @ (w * g))


def phihat1(v, L: int, m: int, beta: float, win: str = "sinh", nq: int = 256) -> np.ndarray:
    """Univariate phihat(v) = int phi(u) e^{-2 pi i v u} du (Algorithm 2.1, step 0a)."""
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    th, w = _gauss_legendre(nq)
    t = m * np.sin(th)
    g = _window_in_theta(th, beta, win) * m * np.cos(th)
    arg = 2.0 * np.outer(v, t) / L
    return (2.0 / L) * (cospi(arg) @ (w * g))


def band(M: int) -> np.ndarray:
    return np.arange(M) - M // 2


def _outer_product(factors):
    out = factors[0]
    for f in factors[1:]:
        out = np.multiply.outer(out, f)
    return out


# ---------------------------------------------------------------------------
# Algorithm 4.2, steps 1-3
# ---------------------------------------------------------------------------

def deconvolve_pad(fhat: np.ndarray, L: int, m: int, beta: float,
                   win: str = "sinh", method: str = "shannon") -> np.ndarray:
    """Step 1: thetahat(k) = fhat(k)/psihat(k) on I_M and 0 on I_L minus I_M.

    Returns the centred L^d array (index k_t + L/2).  method "nfft" divides by phihat
    instead (Algorithm 2.1, step 1)."""
    d = fhat.ndim
    M = fhat.shape[0]
    k = band(M)
    h1 = psihat1(k, L, m, beta, win) if method == "shannon" else phihat1(k, L, m, beta, win)
    hat = _outer_product([h1] * d)
    out = np.zeros((L,) * d, dtype=np.complex128)
    lo = (L - M) // 2
    out[tuple(slice(lo, lo + M) for _ in range(d))] = fhat / hat
    return out


def inverse_fft_step(thetahat: np.ndarray) -> np.ndarray:
    """Step 2, eq. (4.7): theta_l = |I_L|^{-1} sum_{k in I_L} thetahat(k) e^{2 pi i k l / L}.

    numpy's ifftn has exactly this sign and 1/L^d factor; the shifts move between the
    centred storage and the wrapped order the library FFT expects."""
    return np.fft.fftshift(np.fft.ifftn(np.fft.ifftshift(thetahat)))


def node_offsets(x_col: np.ndarray, L: int, m: int):
    """For one coordinate of every node: the 2m+1 candidate indices l = c + o,
    o = -m..m, c = round(L x), their grid offsets t = L x - l, and the distances
    e = m - |L x - l| to the end of the window's support.

    Every l with |L x - l| <= m (the set J_{L,m}(x) of (4.8), per dimension) is among
    the candidates because |L x - c| <= 1/2; candidates with |t| > m get window 0.
    With t0 = L x - c (one rounding) and |t0| <= 1/2, |t| = |o| - sign(o) t0 for o != 0,
    so e = (m - |o|) + sign(o) t0 is rounded once and exact where m - |o| = 0; the
    rounded t itself would lose the distance of a node just inside the support end."""
    c = np.rint(L * x_col)
    t0 = scaled_offset(L, x_col, c)                     # L x - c, one rounding
    o = np.arange(-m, m + 1, dtype=np.float64)
    ell = c[:, None] + o[None, :]
    t = t0[:, None] - o[None, :]
    e = np.where(o[None, :] == 0, m - np.abs(t0)[:, None],
                 (m - np.abs(o))[None, :] + np.sign(o)[None, :] * t0[:, None])
    return ell.astype(np.int64), t, e


def gather_shannon(theta: np.ndarray, x: np.ndarray, L: int, m: int, beta: float,
                   win: str = "sinh", chunk: int = 65536) -> np.ndarray:
    """Step 3: f_j = sum_{l in J_{L,m}(x_j)} theta_l psi(x_j - l/L), with theta_l = 0 for
    l outside I_L (zero-extended sum)."""
    d = theta.ndim
    N = x.shape[0]
    pad = m + 1
    tp = np.pad(theta, pad)                             # zeros outside I_L
    f = np.zeros(N, dtype=np.complex128)
    for s in range(0, N, chunk):
        xs = x[s:s + chunk]
        idx, w = [], []
        for t in range(d):
            ell, off, edge = node_offsets(xs[:, t], L, m)
            idx.append(ell + L // 2 + pad)
            w.append(psi_g(off, m, beta, win, edge))
        acc = np.zeros(xs.shape[0], dtype=np.complex128)
        for combo in itertools.product(range(2 * m + 1), repeat=d):
            wt = w[0][:, combo[0]].copy()
            for t in range(1, d):
                wt *= w[t][:, combo[t]]
            vals = tp[tuple(idx[t][:, combo[t]] for t in range(d))]
            acc += wt * vals
        f[s:s + chunk] = acc
    return f


def forward_shannon(fhat: np.ndarray, x: np.ndarray, L: int, m: int,
                    beta: float | None = None, win: str = "sinh",
                    return_stages: bool = False):
    """Algorithm 4.2 (NFFT-like procedure for bandlimited functions), steps 0a-3."""
    M = fhat.shape[0]
    if beta is None:
        beta = default_beta(M, L, m, "shannon")
    thetahat = deconvolve_pad(fhat, L, m, beta, win, "shannon")
    theta = inverse_fft_step(thetahat)
    f = gather_shannon(theta, x, L, m, beta, win)
    if return_stages:
        return f, thetahat, theta
    return f


# ---------------------------------------------------------------------------
# Algorithm 2.1 (classical NFFT with M_sigma = L), periodic window sums
# ---------------------------------------------------------------------------

def gather_nfft(g: np.ndarray, x: np.ndarray, L: int, m: int, beta: float,
                win: str = "sinh", chunk: int = 65536) -> np.ndarray:
    """Step 3 of Algorithm 2.1: sum over l in I_{L,m}(x_j) (2.5) of g_l times the
    1-periodic window phi~_m(x_j - l/L); indices wrap modulo L."""
    d = g.ndim
    N = x.shape[0]
    f = np.zeros(N, dtype=np.complex128)
    for s in range(0, N, chunk):
        xs = x[s:s + chunk]
        idx, w = [], []
        for t in range(d):
            ell, off, edge = node_offsets(xs[:, t], L, m)
            idx.append(np.mod(ell + L // 2, L))
            w.append(phi_g(off, m, beta, win, edge))
        acc = np.zeros(xs.shape[0], dtype=np.complex128)
        for combo in itertools.product(range(2 * m + 1), repeat=d):
            wt = w[0][:, combo[0]].copy()
            for t in range(1, d):
                wt *= w[t][:, combo[t]]
            acc += wt * g[tuple(idx[t][:, combo[t]] for t in range(d))]
        f[s:s + chunk] = acc
    return f


def forward_nfft(fhat: np.ndarray, x: np.ndarray, L: int, m: int,
                 beta: float | None = None, win: str = "sinh",
                 return_stages: bool = False):
    """Algorithm 2.1 with oversampled size M_sigma = L: divide by phihat, iFFT with
    1/|I_L|, periodic window short sums."""
    M = fhat.shape[0]
    if beta is None:
        beta = default_beta(M, L, m, "nfft")
    ghat = deconvolve_pad(fhat, L, m, beta, win, "nfft")
    g = inverse_fft_step(ghat)
    f = gather_nfft(g, x, L, m, beta, win)
    if return_stages:
        return f, ghat, g
    return f


# ---------------------------------------------------------------------------
# Adjoint and gradients of the factorisation f = Psi F D_psihat fhat  (4.11)
# ---------------------------------------------------------------------------

def spread_shannon(g: np.ndarray, x: np.ndarray, L: int, m: int, beta: float,
                   d: int, win: str = "sinh", chunk: int = 65536) -> np.ndarray:
    """Psi^T g: a_l = sum_j g_j psi(x_j - l/L) for l in I_L (centred L^d array)."""
    N = x.shape[0]
    pad = m + 1
    W = L + 2 * pad
    re = np.zeros(W ** d)
    im = np.zeros(W ** d)
    for s in range(0, N, chunk):
        xs = x[s:s + chunk]
        gs = g[s:s + chunk]
        idx, w = [], []
        for t in range(d):
            ell, off, edge = node_offsets(xs[:, t], L, m)
            idx.append(ell + L // 2 + pad)
            w.append(psi_g(off, m, beta, win, edge))
        for combo in itertools.product(range(2 * m + 1), repeat=d):
            wt = w[0][:, combo[0]].copy()
            flat = idx[0][:, combo[0]].copy()
            for t in range(1, d):
                wt *= w[t][:, combo[t]]
                flat = flat * W + idx[t][:, combo[t]]
            c = gs * wt
            re += np.bincount(flat, weights=c.real, minlength=W ** d)
            im += np.bincount(flat, weights=c.imag, minlength=W ** d)
    full = (re + 1j * im).reshape((W,) * d)
    # keep l in I_L only: columns of Psi exist for l in I_L
    return full[tuple(slice(pad, pad + L) for _ in range(d))]


def adjoint_shannon(g: np.ndarray, x: np.ndarray, M: int, L: int, m: int,
                    beta: float | None = None, win: str = "sinh",
                    return_stages: bool = False):
    """A^H g = D_psihat^H F^H Psi^T g, the exact adjoint of (4.11).  D_psihat is real."""
    d = x.shape[1]
    if beta is None:
        beta = default_beta(M, L, m, "shannon")
    a = spread_shannon(g, x, L, m, beta, d, win)
    # F^H: sum_l a_l e^{-2 pi i k l / L}, unnormalised forward DFT
    A = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(a)))
    lo = (L - M) // 2
    Ak = A[tuple(slice(lo, lo + M) for _ in range(d))]
    h1 = psihat1(band(M), L, m, beta, win)
    Dk = 1.0 / (L ** d * _outer_product([h1] * d))
    out = Dk * Ak
    if return_stages:
        return out, a, A
    return out


def grad_x_shannon(fhat: np.ndarray, G: np.ndarray, x: np.ndarray, L: int, m: int,
                   beta: float | None = None, win: str = "sinh",
                   chunk: int = 65536) -> np.ndarray:
    """gx[j, t] = Re(conj(G_j) * d f_j / d x_jt) with f from Algorithm 4.2.

    d f_j / d x_jt = sum_l theta_l * L * psi_g'(L x_jt - l_t) * prod_{s != t} psi_g(...).
    With G = 2 (f - y) this is the gradient of sum |f_j - y_j|^2 in PyTorch's
    convention for real inputs."""
    M = fhat.shape[0]
    d = x.shape[1]
    if beta is None:
        beta = default_beta(M, L, m, "shannon")
    theta = inverse_fft_step(deconvolve_pad(fhat, L, m, beta, win, "shannon"))
    return grad_x_from_theta(theta, G, x, L, m, beta, win, chunk)


def grad_x_from_theta(theta, G, x, L, m, beta, win, chunk=65536):
    d = theta.ndim
    N = x.shape[0]
    pad = m + 1
    tp = np.pad(theta, pad)
    gx = np.zeros((N, d))
    for s in range(0, N, chunk):
        xs = x[s:s + chunk]
        idx, w, dw = [], [], []
        for t in range(d):
            ell, off, edge = node_offsets(xs[:, t], L, m)
            idx.append(ell + L // 2 + pad)
            w.append(psi_g(off, m, beta, win, edge))
            dw.append(L * dpsi_g(off, m, beta, win, edge))
        der = np.zeros((xs.shape[0], d), dtype=np.complex128)
        for combo in itertools.product(range(2 * m + 1), repeat=d):
            vals = tp[tuple(idx[t][:, combo[t]] for t in range(d))]
            for t in range(d):
                wt = dw[t][:, combo[t]].copy()
                for u in range(d):
                    if u != t:
                        wt *= w[u][:, combo[u]]
                der[:, t] += wt * vals
        gx[s:s + chunk] = np.real(np.conj(G[s:s + chunk])[:, None] * der)
    return gx


def adjoint_nfft(g: np.ndarray, x: np.ndarray, M: int, L: int, m: int,
                 beta: float | None = None, win: str = "sinh") -> np.ndarray:
    """Adjoint of Algorithm 2.1, D^H F^H B^T g, with the periodic window matrix B (2.4).
    parity unpinned beyond the inner-product identity with forward_nfft."""
    d = x.shape[1]
    if beta is None:
        beta = default_beta(M, L, m, "nfft")
    N = x.shape[0]
    acc = np.zeros(L ** d, dtype=np.complex128)
    idx, w = [], []
    for t in range(d):
        ell, off, edge = node_offsets(x[:, t], L, m)
        idx.append(np.mod(ell + L // 2, L))
        w.append(phi_g(off, m, beta, win, edge))
    for combo in itertools.product(range(2 * m + 1), repeat=d):
        wt = w[0][:, combo[0]].copy()
        flat = idx[0][:, combo[0]].copy()
        for t in range(1, d):
            wt *= w[t][:, combo[t]]
            flat = flat * L + idx[t][:, combo[t]]
        c = g * wt
        acc += (np.bincount(flat, weights=c.real, minlength=L ** d)
                + 1j * np.bincount(flat, weights=c.imag, minlength=L ** d))
    a = acc.reshape((L,) * d)
    A = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(a)))
    lo = (L - M) // 2
    Ak = A[tuple(slice(lo, lo + M) for _ in range(d))]
    h1 = phihat1(band(M), L, m, beta, win)
    return Ak / (L ** d * _outer_product([h1] * d))


def adjoint_at(g: np.ndarray, x: np.ndarray, M: int, L: int, m: int, ks,
               method: str = "shannon", beta: float | None = None,
               win: str = "sinh") -> np.ndarray:
    """Entries (A^H g)(k) of the adjoint for the frequencies k in ks (K x d integers in
    [-M/2, M/2)), one at a time from the matrix factorisation ((4.11); for the classical
    NFFT, (2.4)-(2.6)):

        (A^H g)(k) = sum_j g_j prod_t [sum_{l_t} w(L x_jt - l_t) e^{-2 pi i k_t l_t / L}]
                     / (L^d prod_t what(k_t)),

    with w = psi and l_t over I_L only (Psi has no columns outside I_L), or w = phi with
    l_t wrapped mod L (the phase is unchanged by the wrap), and what the window's
    transform.  The inner sum runs over the candidates of node_offsets.  For checking
    sampled entries of adjoints too large for the dense or FFT forms."""
    d = x.shape[1]
    ks = np.atleast_2d(np.asarray(ks, dtype=np.int64))
    if beta is None:
        beta = default_beta(M, L, m, method)
    hat = psihat1 if method == "shannon" else phihat1
    cols = []
    for t in range(d):
        ell, off, edge = node_offsets(x[:, t], L, m)
        if method == "shannon":
            w = psi_g(off, m, beta, win, edge) * ((ell >= -(L // 2)) & (ell < L // 2))
        else:
            w = phi_g(off, m, beta, win, edge)
        cols.append((ell, w))
    lmin = -(L // 2) - m                                # smallest candidate l
    lall = np.arange(lmin, L // 2 + m + 1, dtype=np.int64)
    out = np.empty(len(ks), dtype=np.complex128)
    for i, k in enumerate(ks):
        prod = np.asarray(g, dtype=np.complex128).copy()
        scale = float(L) ** d
        for t in range(d):
            ell, w = cols[t]
            r = np.mod(int(k[t]) * lall, L)             # k l mod L, exact
            phase = cospi(2.0 * r / L) - 1j * sinpi(2.0 * r / L)   # e^{-2 pi i k l / L}
            prod = prod * (w * phase[ell - lmin]).sum(axis=1)
            scale *= float(hat(np.array([float(k[t])]), L, m, beta, win)[0])
        out[i] = prod.sum() / scale
    return out


# ---------------------------------------------------------------------------
# Targets: the direct trigonometric sum (2.1) and closed forms
# ---------------------------------------------------------------------------

def _phase_table(x_col: np.ndarray, M: int) -> np.ndarray:
    """E[j, i] = exp(2 pi i k_i x_j), k_i = i - M/2, phase reduced exactly."""
    k = band(M).astype(np.float64)
    kx = np.multiply.outer(x_col, k)
    n = np.rint(kx)
    r = scaled_offset(k[None, :], x_col[:, None], n)   # k x - n, one rounding
    return cospi(2.0 * r) + 1j * sinpi(2.0 * r)


def direct_sum(fhat: np.ndarray, x: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """f_j = sum_{k in I_M} fhat(k) e^{2 pi i k x_j}, eq. (2.1), cost O(N M^d)."""
    d = fhat.ndim
    M = fhat.shape[0]
    N = x.shape[0]
    out = np.zeros(N, dtype=np.complex128)
    for s in range(0, N, chunk):
        xs = x[s:s + chunk]
        E = [_phase_table(xs[:, t], M) for t in range(d)]
        # contract the last axis first: T[j, i_1..i_{d-1}] = sum_{i_d} E_d[j,i_d] fhat[..., i_d]
        T = E[d - 1] @ fhat.reshape(-1, M).T            # (n, M^{d-1})
        for t in range(d - 2, -1, -1):
            T = T.reshape(xs.shape[0], -1, M)
            T = np.einsum("jai,ji->ja", T, E[t])
        out[s:s + chunk] = T.reshape(-1)
    return out


def dirichlet(x: np.ndarray, M: int) -> np.ndarray:
    """prod_t D_M(x_t), D_M(x) = sum_{k=-M/2}^{M/2-1} e^{2 pi i k x}
    = e^{-i pi x} sin(M pi x) / sin(pi x)  (with D_M(0) = M)."""
    x = np.atleast_2d(x)
    out = np.ones(x.shape[0], dtype=np.complex128)
    for t in range(x.shape[1]):
        xt = x[:, t]
        s = sinpi(xt)
        val = np.where(s != 0.0, sinpi(M * xt) / np.where(s != 0.0, s, 1.0), float(M))
        out *= (cospi(-xt) + 1j * sinpi(-xt)) * val
    return out


# ---------------------------------------------------------------------------
# Section 5, Figure 5.1: approximations of e^{2 pi i v x} at a real frequency v (d = 1)
# ---------------------------------------------------------------------------

def exp_samples(v: float, L: int) -> np.ndarray:
    """e^{2 pi i v l / L} for l in I_L, centred order (index l + L/2)."""
    ell = band(L).astype(np.float64)
    return np.exp(2j * np.pi * v * ell / L)


def exp_approx_nfft(v: float, x: np.ndarray, L: int, m: int, beta: float,
                    win: str = "sinh") -> np.ndarray:
    """Right-hand side of (5.1): (1 / (L phihat(v))) sum_{l in I_L} e^{2 pi i v l/L}
    phi~(x - l/L), the 1-periodic window sum of Algorithm 2.1 at a real v."""
    g = exp_samples(v, L) / (L * phihat1(v, L, m, beta, win)[0])
    return gather_nfft(g, np.asarray(x, dtype=np.float64).reshape(-1, 1), L, m, beta, win)


def exp_approx_shannon(v: float, x: np.ndarray, L: int, m: int, beta: float,
                       win: str = "sinh") -> np.ndarray:
    """Right-hand side of (5.2): sum_{l in I_L} e^{2 pi i v l/L} psi(x - l/L), the
    regularized Shannon sum without the deconvolution (l outside I_L contributes 0)."""
    return gather_shannon(exp_samples(v, L), np.asarray(x, dtype=np.float64).reshape(-1, 1),
                          L, m, beta, win)


def fig51_frequencies(M: int, m: int, S: int) -> np.ndarray:
    """v_s = -M/2 - m + s/S, s = 0..S(M + 2m)  (5.4)."""
    s = np.arange(S * (M + 2 * m) + 1, dtype=np.float64)
    return -M / 2 - m + s / S


def example51_f(x: np.ndarray, M: int) -> np.ndarray:
    """Example 5.1 target f(x) = sinc^2(M pi x / 2)."""
    return sinc_pi(0.5 * M * np.asarray(x, dtype=np.float64)) ** 2


# ---------------------------------------------------------------------------
# Dense matrices (2.2)-(2.4) and (4.9)-(4.10), for brute force on tiny inputs
# ---------------------------------------------------------------------------

def _grid_points(L: int, d: int) -> np.ndarray:
    """All l in I_L, row-major (last coordinate fastest)."""
    g = np.array(list(itertools.product(range(-L // 2, L // 2), repeat=d)), dtype=np.int64)
    return g.reshape(-1, d)


def dense_F(M: int, L: int, d: int) -> np.ndarray:
    """F[l, k] = e^{2 pi i k.l / L}, l in I_L, k in I_M; the phase k.l mod L is reduced
    in integers."""
    ls = _grid_points(L, d)
    ks = _grid_points(M, d)
    ph = np.mod(ls @ ks.T, L).astype(np.float64)
    return cospi(2.0 * ph / L) + 1j * sinpi(2.0 * ph / L)


def dense_Psi(x: np.ndarray, L: int, m: int, beta: float, win: str = "sinh") -> np.ndarray:
    """Psi[j, l] = psi(x_j - l/L) over every l in I_L (4.10)."""
    d = x.shape[1]
    ls = _grid_points(L, d)
    P = np.ones((x.shape[0], ls.shape[0]))
    for t in range(d):
        off = scaled_offset(L, x[:, t][:, None], ls[:, t][None, :].astype(np.float64))
        P *= psi_g(off, m, beta, win)
    return P


def dense_B(x: np.ndarray, L: int, m: int, beta: float, win: str = "sinh") -> np.ndarray:
    """B[j, l] = phi~_m(x_j - l/L) = sum_z phi(x_j - l/L + z), l in I_L (2.4)."""
    d = x.shape[1]
    ls = _grid_points(L, d)
    P = np.ones((x.shape[0], ls.shape[0]))
    for t in range(d):
        tot = np.zeros(P.shape)
        for z in (-1, 0, 1):
            off = scaled_offset(L, x[:, t][:, None],
                                (ls[:, t][None, :] - z * L).astype(np.float64))
            tot += phi_g(off, m, beta, win)
        P *= tot
    return P


def dense_D(M: int, L: int, d: int, m: int, beta: float, win: str = "sinh",
            method: str = "shannon") -> np.ndarray:
    """Diagonal of D_psihat (4.9) or D (2.2): 1/(|I_L| * hat(k)), k in I_M row-major."""
    h1 = psihat1(band(M), L, m, beta, win) if method == "shannon" else \
        phihat1(band(M), L, m, beta, win)
    return (1.0 / (L ** d * _outer_product([h1] * d))).reshape(-1)


def dense_forward(fhat: np.ndarray, x: np.ndarray, L: int, m: int, beta: float,
                  win: str = "sinh", method: str = "shannon") -> np.ndarray:
    """f = Psi F D_psihat fhat (4.11), or B F D fhat for Algorithm 2.1."""
    d = fhat.ndim
    M = fhat.shape[0]
    W = dense_Psi(x, L, m, beta, win) if method == "shannon" else dense_B(x, L, m, beta, win)
    return W @ (dense_F(M, L, d) @ (dense_D(M, L, d, m, beta, win, method) * fhat.reshape(-1)))


# ---------------------------------------------------------------------------
# Error measures (normwise maximum error, as (5.5) on normalised data)
# ---------------------------------------------------------------------------

def rel_err_inf(a: np.ndarray, ref: np.ndarray) -> float:
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(a - ref)) / den) if den > 0 else float(np.max(np.abs(a)))


def rel_err_l2(a: np.ndarray, ref: np.ndarray) -> float:
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / den) if den > 0 else float(np.linalg.norm(a))


def in_truncated_domain(x: np.ndarray, L: int, m: int) -> np.ndarray:
    """Mask of nodes in [-1/2 + m/L, 1/2 - m/L)^d, where Algorithm 4.2 is meant to be
    used (Section 4)."""
    a = 0.5 - m / L
    return np.all((x >= -a) & (x < a), axis=1)
