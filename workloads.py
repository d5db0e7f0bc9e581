"""Seeded synthetic inputs for the bandlimited NFFT workloads.

This module draws random numbers only: nodes x_j, coefficient samples fhat(k) and
target values y_j with the shapes, sizes and distributions of the workloads. It holds
none of the transform's arithmetic, so the CPU oracle, the GPU tests and the benchmark
can all share it without sharing any of the method.

Conventions
-----------
* Nodes are an (N, d) float64 array, row-major, each coordinate in [-1/2, 1/2).
* Coefficients fhat are a complex128 array of shape (M,)*d; array index i_t holds the
  frequency k_t = i_t - M/2, i.e. the band I_M = [-M/2, M/2)^d of Section 1.
* Every generator is driven by numpy's PCG64 with an explicit seed.
* For a run in single precision, inputs are drawn in float64 and rounded once to
  float32 (``round_inputs``); the rounded values then feed every path, the oracle
  included, so that input rounding is not mistaken for transform error.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Workloads, named by what they are.  Sizes: d dimensions, bandwidth M, oversampled
# grid L per dimension, truncation m, N nodes.
WORKLOADS = {
    # d=1 correctness case, uniform nodes, complex normal coefficients.
    "d1_M256_L512_m6_N1k": dict(d=1, M=256, L=512, m=6, N=1000, nodes="uniform",
                                coeff="normal", seed=1),
    # d=2 headline case, uniform nodes, coefficients decaying like 1/(1+|k|^2).
    "d2_M512_L1024_m5_N1M": dict(d=2, M=512, L=1024, m=5, N=1_000_000,
                                 nodes="uniform", coeff="normal_decay", seed=2),
    # d=3, clustered nodes (16-component Gaussian mixture), fhat = 1 on the band.
    "d3_M128_L256_m4_N2M": dict(d=3, M=128, L=256, m=4, N=2_000_000, nodes="gmm16",
                                coeff="ones", seed=3),
    # d=2 differentiation case: uniform nodes, complex normal fhat and targets y.
    "d2_M256_L512_m6_N200k": dict(d=2, M=256, L=512, m=6, N=200_000, nodes="uniform",
                                  coeff="normal", seed=5),
}

BATCHED_SEED = 4
BATCHED_COUNT = 512


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_nodes(rng: np.random.Generator, N: int, d: int) -> np.ndarray:
    """N nodes i.i.d. uniform in [-1/2, 1/2)^d."""
    return rng.random((N, d)) - 0.5


def truncated_uniform_nodes(rng: np.random.Generator, N: int, d: int, L: int,
                            m: int) -> np.ndarray:
    """N nodes uniform in the truncated domain [-1/2 + m/L, 1/2 - m/L)^d."""
    a = 0.5 - m / L
    return (rng.random((N, d)) * 2.0 - 1.0) * a


def gmm_nodes(rng: np.random.Generator, N: int, d: int, components: int = 16,
              sigma: float = 0.02, spread: float = 0.4) -> np.ndarray:
    """Gaussian mixture: `components` centres uniform in [-spread, spread]^d, isotropic
    standard deviation `sigma`, equal weights.  Samples outside [-1/2, 1/2)^d are
    rejected and redrawn."""
    centres = (rng.random((components, d)) * 2.0 - 1.0) * spread
    out = np.empty((0, d))
    need = N
    while need > 0:
        lab = rng.integers(0, components, size=need)
        pts = centres[lab] + sigma * rng.standard_normal((need, d))
        ok = np.all((pts >= -0.5) & (pts < 0.5), axis=1)
        out = np.concatenate([out, pts[ok]], axis=0)
        need = N - out.shape[0]
    return out


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """(n1 + i n2) with n1, n2 i.i.d. standard normal."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def band_frequencies(M: int) -> np.ndarray:
    """Integer frequencies of I_M in array order: k = i - M/2, i = 0..M-1."""
    return np.arange(M) - M // 2


def coefficients(rng: np.random.Generator, M: int, d: int, kind: str) -> np.ndarray:
    shape = (M,) * d
    if kind == "normal":
        return complex_normal(rng, shape)
    if kind == "normal_decay":
        k = band_frequencies(M).astype(np.float64)
        ksq = np.zeros(shape)
        for t in range(d):
            sh = [1] * d
            sh[t] = M
            ksq = ksq + (k ** 2).reshape(sh)
        return complex_normal(rng, shape) / (1.0 + ksq)
    if kind == "ones":
        return np.ones(shape, dtype=np.complex128)
    raise ValueError(kind)


def nodes_for(rng: np.random.Generator, kind: str, N: int, d: int, L: int = 0,
              m: int = 0) -> np.ndarray:
    if kind == "uniform":
        return uniform_nodes(rng, N, d)
    if kind == "gmm16":
        return gmm_nodes(rng, N, d)
    if kind == "truncated":
        return truncated_uniform_nodes(rng, N, d, L, m)
    raise ValueError(kind)


_F32_BELOW_HALF = float(np.nextafter(np.float32(0.5), np.float32(0.0)))


def round_inputs(x: np.ndarray | None = None, fhat: np.ndarray | None = None,
                 dtype=np.float32):
    """Round float64 inputs once to `dtype` and return them as float64 / complex128.

    A coordinate that rounds up to +1/2 is moved to the largest value below 1/2, so
    the rounded nodes stay in [-1/2, 1/2)."""
    xo = fo = None
    if x is not None:
        xr = x.astype(dtype)
        if dtype == np.float32:
            xr = np.where(xr >= np.float32(0.5), np.float32(_F32_BELOW_HALF), xr)
        xo = xr.astype(np.float64)
    if fhat is not None:
        cdt = np.complex64 if dtype == np.float32 else np.complex128
        fo = fhat.astype(cdt).astype(np.complex128)
    return xo, fo


@dataclass
class Problem:
    name: str
    d: int
    M: int
    L: int
    m: int
    x: np.ndarray
    fhat: np.ndarray
    y: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.x.shape[0]


def make_problem(name: str, N: int | None = None, precision: str = "f64",
                 with_targets: bool = False) -> Problem:
    """Build a named workload.  `N` overrides the node count (a smaller case drawn from
    the same distribution, same seed).  precision "f32" rounds the inputs per
    ``round_inputs``."""
    spec = WORKLOADS[name]
    rng = rng_for(spec["seed"])
    n = spec["N"] if N is None else N
    d, M, L, m = spec["d"], spec["M"], spec["L"], spec["m"]
    x = nodes_for(rng, spec["nodes"], n, d, L, m)
    fhat = coefficients(rng, M, d, spec["coeff"])
    y = complex_normal(rng, n) if with_targets else None
    if precision == "f32":
        x, fhat = round_inputs(x, fhat)
        if y is not None:
            y = y.astype(np.complex64).astype(np.complex128)
    return Problem(name, d, M, L, m, x, fhat, y)


def custom_problem(d: int, M: int, L: int, m: int, N: int, seed: int,
                   nodes: str = "uniform", coeff: str = "normal",
                   precision: str = "f64", with_targets: bool = False) -> Problem:
    rng = rng_for(seed)
    x = nodes_for(rng, nodes, N, d, L, m)
    fhat = coefficients(rng, M, d, coeff)
    y = complex_normal(rng, N) if with_targets else None
    if precision == "f32":
        x, fhat = round_inputs(x, fhat)
        if y is not None:
            y = y.astype(np.complex64).astype(np.complex128)
    return Problem(f"custom_d{d}_M{M}_L{L}_m{m}_N{N}", d, M, L, m, x, fhat, y)


@dataclass
class BatchedInstance:
    M: int
    L: int
    m: int
    x: np.ndarray     # (N,) float64
    fhat: np.ndarray  # (M,) complex128


def batched_instances(count: int = BATCHED_COUNT, seed: int = BATCHED_SEED,
                      precision: str = "f32", n_scale: float = 1.0,
                      m_choices=(4, 6, 8), m_range=(32, 4096),
                      n_range=(1e3, 2e5)) -> list[BatchedInstance]:
    """Independent d=1 instances: M = 2*round(exp(U[ln 32, ln 4096])) (so M is even in
    [64, 8192]), L = 2M, m uniform in {4, 6, 8}, N = round(exp(U[ln 1e3, ln 2e5])),
    nodes uniform in [-1/2, 1/2), fhat complex normal.  `n_scale` shrinks every N (for
    small test variants of the same draw)."""
    rng = rng_for(seed)
    out = []
    lo_m, hi_m = math.log(m_range[0]), math.log(m_range[1])
    lo_n, hi_n = math.log(n_range[0]), math.log(n_range[1])
    for _ in range(count):
        half = int(round(math.exp(rng.uniform(lo_m, hi_m))))
        M = 2 * half
        L = 2 * M
        m = int(rng.choice(m_choices))
        N = int(round(math.exp(rng.uniform(lo_n, hi_n))))
        N = max(1, int(round(N * n_scale)))
        x = uniform_nodes(rng, N, 1)[:, 0]
        fhat = complex_normal(rng, M)
        if precision == "f32":
            xr, fr = round_inputs(x[:, None], fhat)
            x, fhat = xr[:, 0], fr
        out.append(BatchedInstance(M, L, m, x, fhat))
    return out


def chebyshev_nodes(N: int, L: int, m: int) -> np.ndarray:
    """Scaled Chebyshev points of Example 5.1, eq. (5.6):
    x_j = cos((j-1) pi / N) * (1/2 - m/L), j = 1..N."""
    j = np.arange(1, N + 1)
    return np.cos((j - 1) * np.pi / N) * (0.5 - m / L)


def triangle_fhat(M: int) -> np.ndarray:
    """Samples at k in I_M of the Fourier transform in Example 5.1:
    fhat(v) = (2/M) (1 - |2v/M|) for |v| <= M/2."""
    k = band_frequencies(M).astype(np.float64)
    return ((2.0 / M) * (1.0 - np.abs(2.0 * k / M))).astype(np.complex128)
