"""Batched d = 1 transforms (one graph launch for many independent instances of
Algorithm 4.2) against the FP64 oracle, instance by instance."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5   # normwise relative error of FP32 data, per instance


def _instances(spec, seed):
    """Instances with the given (M, L, m, N); nodes uniform in [-1/2, 1/2), fhat complex
    normal, both rounded to float32."""
    rng = W.rng_for(seed)
    out = []
    for M, L, m, N in spec:
        x = W.uniform_nodes(rng, N, 1)
        fhat = W.complex_normal(rng, M)
        xr, fr = W.round_inputs(x, fhat)
        out.append(W.BatchedInstance(M, L, m, xr[:, 0], fr))
    return out


def _run(insts, precision="f32"):
    import torch
    from paper_2502_07155_amd import BatchPlan
    bp = BatchPlan([i.M for i in insts], [i.L for i in insts], [i.m for i in insts],
                   [i.x.size for i in insts], precision=precision)
    x = torch.from_numpy(np.concatenate([i.x for i in insts]).astype(np.float32)).cuda()
    fhat = torch.from_numpy(np.concatenate([i.fhat for i in insts]).astype(np.complex64)).cuda()
    bp.set_nodes(x)
    f = bp.forward(fhat)
    torch.cuda.synchronize()
    return bp, x, fhat, f


def _check(bp, insts, f, tol=TOL, sample=None, seed=0):
    rng = np.random.default_rng(seed)
    got = f.cpu().numpy().astype(np.complex128)
    for i, inst in enumerate(insts):
        gi = got[bp.node_offsets[i]:bp.node_offsets[i + 1]]
        if inst.x.size == 0:
            assert gi.size == 0
            continue
        idx = np.arange(inst.x.size) if sample is None or inst.x.size <= sample \
            else np.sort(rng.choice(inst.x.size, sample, replace=False))
        ref = O.forward_shannon(inst.fhat, inst.x[idx, None].astype(np.float64), inst.L, inst.m)
        err = O.rel_err_inf(gi[idx], ref)
        assert err <= tol, (i, inst.M, inst.L, inst.m, inst.x.size, err)


# (M, L, m, N): power-of-two and other even L, the smallest M, an empty instance, the
# largest single-piece transform (L + M - 1 <= 4096) and ones split into 4 and 8 pieces
MIXED = [(8, 16, 2, 50), (40, 60, 3, 300), (64, 128, 4, 1000), (100, 250, 5, 0),
         (256, 512, 6, 2000), (128, 160, 8, 700), (2, 6, 2, 10), (4000, 8000, 4, 1500),
         (8192, 16384, 8, 3000), (6000, 12000, 6, 2000), (1000, 1500, 7, 4000)]


@pytest.mark.parametrize("precision", ["f32", "f32c"])
def test_batch_mixed_instances(precision):
    insts = _instances(MIXED, seed=41)
    bp, _, _, f = _run(insts, precision)
    _check(bp, insts, f)


def test_batch_small_pieces(monkeypatch):
    """With the in-LDS transform size lowered to 256 points, instances split into 2, 4 and
    8 pieces (and one that fits) on small sizes."""
    monkeypatch.setenv("BL_BATCH_LDS_FFT", "256")
    insts = _instances([(100, 250, 5, 700), (300, 600, 6, 900), (500, 1000, 4, 1100),
                        (60, 120, 3, 300)], seed=48)
    bp, _, _, f = _run(insts)
    _check(bp, insts, f)


def test_batch_single_instance_matches_plan():
    """A batch of one instance against the single-transform plan on the same inputs."""
    import torch
    from paper_2502_07155_amd import Plan
    insts = _instances([(512, 1024, 6, 5000)], seed=42)
    bp, x, fhat, f = _run(insts)
    plan = Plan(1, 512, 1024, 6, precision="f32")
    plan.set_nodes(x.reshape(-1, 1).contiguous())
    g = plan.forward(fhat)
    torch.cuda.synchronize()
    assert O.rel_err_inf(f.cpu().numpy(), g.cpu().numpy()) <= 2e-6


def test_batch_replays_rebinding_and_determinism():
    """Graph replays with eager work in between give identical results; new nodes and new
    coefficients after the capture are picked up."""
    import torch
    insts = _instances([(64, 128, 4, 900), (300, 600, 6, 1200), (2048, 4096, 8, 800)], seed=43)
    bp, x, fhat, f0 = _run(insts)
    f0 = f0.clone()
    out = torch.empty_like(f0)
    for rep in range(5):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda") * 2
        bp.forward(fhat, out)
        junk.sum().item()
        torch.cuda.synchronize()
        assert torch.equal(out, f0), rep
    _check(bp, insts, f0)
    insts2 = _instances([(64, 128, 4, 900), (300, 600, 6, 1200), (2048, 4096, 8, 800)], seed=44)
    x2 = torch.from_numpy(np.concatenate([i.x for i in insts2]).astype(np.float32)).cuda()
    fhat2 = torch.from_numpy(np.concatenate([i.fhat for i in insts2]).astype(np.complex64)).cuda()
    bp.set_nodes(x2)
    fhat.copy_(fhat2)
    f2 = bp.forward(fhat, out)
    torch.cuda.synchronize()
    _check(bp, insts2, f2)


def test_batch_node_errors():
    import torch
    from paper_2502_07155_amd import BLNFFTError
    insts = _instances([(64, 128, 4, 100), (32, 64, 3, 100)], seed=45)
    bp, x, fhat, f = _run(insts)
    for bad in (0.5, float("nan"), -0.75):
        xb = x.clone()
        xb[150] = bad
        with pytest.raises(BLNFFTError) as e:
            bp.set_nodes(xb)
        assert e.value.status == 2   # BL_EDOMAIN
        with pytest.raises(BLNFFTError) as e:
            bp.forward(fhat)
        assert e.value.status == 5   # BL_ESTATE
    bp.set_nodes(x)
    g = bp.forward(fhat)
    torch.cuda.synchronize()
    assert torch.equal(g, f)


def test_batch_edge_nodes():
    """Nodes on grid points, at -1/2, just below 1/2, and many nodes in one cell."""
    L = 256
    M = 128
    xs = np.concatenate([np.arange(-L // 2, L // 2) / L, [-0.5, np.nextafter(np.float32(0.5), 0)],
                         np.full(3000, 0.123, dtype=np.float64)]).astype(np.float32).astype(np.float64)
    rng = W.rng_for(46)
    fhat = W.complex_normal(rng, M).astype(np.complex64).astype(np.complex128)
    insts = [W.BatchedInstance(M, L, 5, xs, fhat), W.BatchedInstance(M, L, 8, xs[::-1].copy(), fhat)]
    bp, _, _, f = _run(insts)
    _check(bp, insts, f)


def test_batched_workload_full_size_sampled():
    """The 512-instance workload (M = 2 round(exp(U[ln 32, ln 4096])), L = 2M, m in
    {4, 6, 8}, N log-uniform in [1e3, 2e5]) at full size, in the launch configuration the
    benchmark times, checked on 64 sampled nodes per instance."""
    insts = W.batched_instances()
    bp, _, _, f = _run(insts)
    _check(bp, insts, f, sample=64, seed=47)
