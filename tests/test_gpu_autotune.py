"""The autotuner: FFT lines per workgroup timed at plan creation, the short sums' tile edge
and chunk capacity timed at the first large node binding, both cached in a JSON file keyed
by device, shape, precision and node-density class.  Whatever it picks, the transforms stay
within the parity tolerance of the oracle."""
import json

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _forward(plan, p):
    import torch
    plan.set_nodes(torch.from_numpy(p.x).to(torch.float32).cuda())
    return plan.forward(torch.from_numpy(p.fhat).to(torch.complex64).cuda()).cpu().numpy().astype(np.complex128)


def test_tuned_choices_are_measured_then_cached(tmp_path, monkeypatch):
    from paper_2502_07155_amd import Plan
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("BL_TUNE_CACHE", str(cache))
    monkeypatch.delenv("BL_AUTOTUNE", raising=False)
    monkeypatch.delenv("BL_TILE", raising=False)
    monkeypatch.delenv("BL_FFT_LINES", raising=False)
    d, M, L, m, N = 2, 128, 256, 5, 120_000
    p = W.custom_problem(d, M, L, m, N, seed=3100, precision="f32")
    first = Plan(d, M, L, m, precision="f32c")
    assert first.stats()["tuned"]["fft"] == 1
    f1 = _forward(first, p)
    s1 = first.stats()
    assert s1["tuned"]["tiles"] == 1
    assert all(b > 0 for b in s1["fft_lines"][0][:d]) and all(b > 0 for b in s1["fft_lines"][1][:d])
    entries = json.loads(cache.read_text())
    assert any(k.startswith("fft|") for k in entries) and any(k.startswith("tiles|") for k in entries)
    second = Plan(d, M, L, m, precision="f32c")
    assert second.stats()["tuned"]["fft"] == 2
    f2 = _forward(second, p)
    s2 = second.stats()
    assert s2["tuned"]["tiles"] == 2
    assert s2["tile"] == s1["tile"] and s2["chunk_cap"] == s1["chunk_cap"]
    assert s2["fft_lines"] == s1["fft_lines"]
    idx = np.sort(W.rng_for(3).choice(N, 3000, replace=False))
    ref = O.forward_shannon(p.fhat, p.x[idx], L, m)
    for f in (f1, f2):
        assert O.rel_err_inf(f[idx], ref) <= 1e-6
    # a rebinding of as many nodes keeps the plan's choice
    _forward(second, p)
    assert second.stats()["tile"] == s1["tile"]
    first.close()
    second.close()


def test_overrides_and_off_switch(tmp_path, monkeypatch):
    from paper_2502_07155_amd import Plan
    monkeypatch.setenv("BL_TUNE_CACHE", str(tmp_path / "t.json"))
    d, M, L, m, N = 2, 64, 128, 4, 70_000
    p = W.custom_problem(d, M, L, m, N, seed=3101, precision="f32")
    monkeypatch.setenv("BL_TILE", "12")
    plan = Plan(d, M, L, m, precision="f32")
    _forward(plan, p)
    assert plan.stats()["tuned"]["tiles"] == 0 and plan.stats()["tile"][0] == 12
    plan.close()
    monkeypatch.delenv("BL_TILE")
    monkeypatch.setenv("BL_AUTOTUNE", "0")
    plan = Plan(d, M, L, m, precision="f32")
    f = _forward(plan, p)
    st = plan.stats()
    assert st["tuned"] == {"fft": 0, "tiles": 0} and st["fft_lines"] == ((0, 0, 0), (0, 0, 0))
    ref = O.forward_shannon(p.fhat, p.x[:2000], L, m)
    assert O.rel_err_inf(f[:2000], ref) <= 1e-5
    plan.close()


@pytest.mark.parametrize("spec", [(1, 1000, 2000, 5, 80_000), (3, 40, 64, 3, 100_000)])
def test_tuned_plans_keep_parity(spec, tmp_path, monkeypatch):
    """Tuned d = 1 (chirp-z, L = 2000) and d = 3 plans: forward and adjoint against the oracle."""
    import torch
    from paper_2502_07155_amd import Plan
    monkeypatch.setenv("BL_TUNE_CACHE", str(tmp_path / "t.json"))
    d, M, L, m, N = spec
    p = W.custom_problem(d, M, L, m, N, seed=3102 + d, precision="f64", with_targets=True)
    plan = Plan(d, M, L, m, precision="f64")
    plan.set_nodes(torch.from_numpy(p.x).cuda())
    assert plan.stats()["tuned"] == {"fft": 1, "tiles": 1}
    f = plan.forward(torch.from_numpy(p.fhat).cuda()).cpu().numpy()
    idx = np.sort(W.rng_for(4).choice(N, 2000, replace=False))
    assert O.rel_err_inf(f[idx], O.forward_shannon(p.fhat, p.x[idx], L, m)) <= 1e-12
    a = plan.adjoint(torch.from_numpy(p.y).cuda()).cpu().numpy()
    h = M // 2
    ks = W.rng_for(5).integers(-h, h, size=(6, d))
    assert O.rel_err_inf(a[tuple((ks + h).T)], O.adjoint_at(p.y, p.x, M, L, m, ks)) <= 1e-12
    plan.close()
