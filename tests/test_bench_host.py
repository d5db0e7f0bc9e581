"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the algorithmic flop and byte
counts behind `roofline`, the counter scaling of `traffic`, and the rule that a traffic
figure taken on other gather sources is not reported."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_flops_per_node():
    # headline short sum: (2m)^d = 100 terms of 2 FMAs, plus d * 2m = 20 weights
    assert bench.mac_flops_per_node(2, 5) == 400
    assert bench.gather_flops_per_node(2, 5) == 400 + 20 * bench.WEIGHT_EVAL_FLOPS
    assert bench.gather_flops_per_node(3, 4) == 4 * 512 + 24 * bench.WEIGHT_EVAL_FLOPS
    assert bench.mac_flops_per_node(1, 6) == 48


def test_algorithmic_bytes_headline():
    ab = bench.algorithmic_bytes(2, 512, 1024, 1_000_000, 8, 4)
    # pass over the last axis: M rows of M in, M rows of L out; then L columns of M in,
    # L columns of L out (complex64)
    assert ab["fft"] == (512 * 512 + 512 * 1024 + 512 * 1024 + 1024 * 1024) * 8
    # grid once, nodes (d floats), f, permutation
    assert ab["gather"] == 1024 * 1024 * 8 + 1_000_000 * (2 * 4 + 8 + 4)
    assert ab["total"] == ab["fft"] + ab["gather"]


def _counter_csv(directory, rows):
    os.makedirs(directory, exist_ok=True)
    with open(os.path.join(directory, "run_counter_collection.csv"), "w") as fh:
        fh.write("Kernel_Name,Counter_Value\n")
        for name, v in rows:
            fh.write(f"\"{name}\",{v}\n")


def test_traffic_scaling(tmp_path):
    gib_kib = float(1 << 20)
    _counter_csv(tmp_path / "f", [("k_gather<float, 2>", 100.0), ("k_gather<float, 2>", 300.0),
                                 ("k_fft_pass<...>", 1e9)])
    _counter_csv(tmp_path / "w", [("k_gather<float, 2>", 500.0)])
    _counter_csv(tmp_path / "cf", [("copy", gib_kib / 2)] * 5)   # FETCH_SIZE reads half the bytes
    _counter_csv(tmp_path / "cw", [("copy", gib_kib)] * 5)
    text = bench.summarize_traffic(str(tmp_path / "f"), str(tmp_path / "w"),
                                   str(tmp_path / "cf"), str(tmp_path / "cw"))
    vals = dict(line.split(":", 1) for line in text.splitlines())
    # (200 KiB / 0.5 + 500 KiB / 1.0) per dispatch
    assert float(vals["traffic_bytes_per_launch"]) == pytest.approx((400 + 500) * 1024)
    assert vals["source_sha256"].strip() == bench.source_digest(bench.GATHER_SOURCES)


def test_traffic_is_dropped_for_other_sources(monkeypatch):
    path = os.path.join(ROOT, bench.TRAFFIC_FILE)
    if not os.path.exists(path):
        pytest.skip("no committed traffic summary")
    monkeypatch.setattr(bench, "source_digest", lambda paths: "0" * 64)
    assert bench.measured_traffic() is None
