"""Figure 5.1 (Section 5) on the GPU: the approximations (5.1) and (5.2) of e^{2 pi i v x}
at real frequencies v, each the short sums of one plan (bl_interpolate) on the samples
e^{2 pi i v l/L}, for M = 20, L = 40 (not a power of two: no FFT is involved), m = 5.
Both sides sum the same samples (for (5.1) divided by the oracle's L phihat(v)); the
figure's statements are checked on the GPU values (S = 8, P = 20000)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "figure_5_1.json")


def _samples(vs, M, L, m, method, beta):
    """e^{2 pi i v l/L} per frequency (rows), for (5.1) divided by L phihat(v) of the oracle,
    so that the GPU and the oracle sum the same samples."""
    th = np.stack([O.exp_samples(v, L) for v in vs])
    if method == "nfft":
        th = th / (L * O.phihat1(vs, L, m, beta))[:, None]
    return th


def _interpolate(x, theta, M, L, m, method, beta):
    import torch
    from paper_2502_07155_amd import Plan
    plan = Plan(1, M, L, m, precision="f64", method=method, beta=beta)
    plan.set_nodes(torch.from_numpy(x[:, None]).cuda())
    assert plan.stats()["beta"] == pytest.approx(beta, rel=1e-15)
    td = torch.from_numpy(theta).cuda()
    h = np.stack([plan.interpolate(td[i]).cpu().numpy() for i in range(theta.shape[0])])
    plan.close()
    return h


def test_figure_5_1_on_the_gpu():
    g = json.load(open(GOLDEN))
    M, L, m = g["M"], g["L"], g["m"]
    vs = O.fig51_frequencies(M, m, 8)
    inband = np.abs(vs) <= M / 2
    integer = np.abs(vs - np.rint(vs)) < 1e-12
    P = 20000
    a, b = -0.5 + m / L, 0.5 - m / L
    xs = {"full": -0.5 + np.arange(P) / P, "truncated": a + np.arange(P) * (b - a) / P}
    same = O.default_beta(M, L, m)
    err = {}
    for name, x in xs.items():
        ex = np.exp(2j * np.pi * np.outer(vs, x))
        for label, method, beta in (("sh", "shannon", same), ("nf", "nfft", same),
                                     ("nfstd", "nfft", O.default_beta(M, L, m, "nfft"))):
            theta = _samples(vs, M, L, m, method, beta)
            h = _interpolate(x, theta, M, L, m, method, beta)
            sub = np.arange(0, P, 97)
            gather = O.gather_shannon if method == "shannon" else O.gather_nfft
            for i in range(0, vs.size, 23):
                ref = gather(theta[i], x[sub, None], L, m, beta)
                if method == "shannon":
                    assert O.rel_err_inf(h[i, sub], ref) <= 1e-12, (name, label, vs[i])
                else:
                    # Outside the main lobe of phihat the samples 1/(L phihat(v)) reach ~350
                    # while |h| ~ 1: the sum cancels, so the bar is relative to the sum of
                    # absolute terms, sum_l |g_l| phi(x - l/L) (phi >= 0).
                    absum = O.gather_nfft(np.abs(theta[i]).astype(np.complex128), x[sub, None],
                                          L, m, beta).real
                    assert np.max(np.abs(h[i, sub] - ref) / absum) <= 1e-13, (name, label, vs[i])
            err[name, label] = np.max(np.abs(h - ex), axis=1)
    sh, nf = err["full", "sh"], err["full", "nf"]
    assert sh.min() > 0.5                                          # (5.2) needs the truncated interval
    assert nf[inband & integer].max() < 0.02 and nf[inband & ~integer].max() > 1.0
    sh, nf, nfs = err["truncated", "sh"], err["truncated", "nf"], err["truncated", "nfstd"]
    assert sh[inband].max() < 1e-3 and nf[inband].max() < 2e-2
    assert sh[np.abs(vs) >= M / 2 + 1].min() > 5 * sh[inband].max()
    assert sh[inband].max() < nf[inband].max() / 5                # same beta: (5.2) is better
    assert nfs[inband].max() < sh[inband].max() / 100             # standard beta: (5.1) is better


def test_forward_and_adjoint_at_the_figures_L():
    """L = 40 (not a power of two) runs steps 1-2 by the chirp-z passes: forward and adjoint
    of an FP64 plan against the oracle."""
    import torch
    from paper_2502_07155_amd import Plan
    M, L, m = 20, 40, 5
    p = W.custom_problem(1, M, L, m, 300, seed=41, with_targets=True)
    plan = Plan(1, M, L, m, precision="f64")
    plan.set_nodes(torch.from_numpy(p.x).cuda())
    f = plan.forward(torch.from_numpy(p.fhat).cuda()).cpu().numpy()
    assert O.rel_err_inf(f, O.forward_shannon(p.fhat, p.x, L, m)) <= 1e-12
    a = plan.adjoint(torch.from_numpy(p.y).cuda()).cpu().numpy()
    assert O.rel_err_inf(a, O.adjoint_shannon(p.y, p.x, M, L, m)) <= 1e-12
    plan.close()
