"""CPU checks of the benchmark's contract that need no GPU: more than one
GPU is refused with a message and a non-zero exit, before anything touches
a device; the algorithmic operation counts it prices the kernels with are
the documented ones; the stored traffic summary is used only while the
kernel sources are the ones it was taken on."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_operation_counts():
    import bench
    assert bench.FLOP_PER_STEP == 830.0 and bench.FLOP_PER_PAIR == 35.0 and bench.FLOP_PER_UPDATE == 500.0
    assert bench.algorithmic_flops([10, 20, 30]) == 10 * 830.0 + 20 * 35.0 + 30 * 500.0
    # 256 CUs x 2.4 GHz x 128 FLOP per clock
    assert bench.ALU_PEAK_TFLOPS == pytest.approx(78.6432)


def test_stored_traffic_follows_the_sources(tmp_path, monkeypatch):
    import bench
    rec = {"source_sha256": bench.source_sha256(), "hbm_bytes_per_launch": 123.0}
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "t.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash covers the sources under ROOT: a tree without them hashes
    # differently from the repository's, so the record no longer applies
    assert bench.stored_traffic("t.json") is None
    rec["source_sha256"] = bench.source_sha256()
    (d / "t.json").write_text(json.dumps(rec))
    assert bench.stored_traffic("t.json") == 123.0
    assert bench.stored_traffic("missing.json") is None


def test_hbm_roofline_and_dedup_bytes():
    """The secondary rooflines: bytes over time against 8 TB/s, and the
    duplicate-removal byte count from its stated per-track, per-entry and
    per-hit terms."""
    import torch

    import bench
    r = bench.hbm_roofline(8e9, 1000.0, "x")
    assert r["bound"] == "hbm" and abs(r["achieved"] - 8.0) < 1e-9 and abs(r["frac"] - 1e-3) < 1e-12
    S, K, H = 4, 2, 5
    hits = torch.full((S * K, H), -3, dtype=torch.int32)
    hits[0, :3] = torch.tensor([0, 1, 9])      # 9 is not a hit of a 5-hit batch
    hits[2 * K, :2] = torch.tensor([2, 3])
    hits[1, :] = 4                              # slot 1 is not read
    out = dict(S=S, K=K, hits=hits, n_cands=torch.tensor([1, 0, 1, 1], dtype=torch.int32))
    entries = 2 + 2
    assert bench.dedup_bytes(out, 5) == S * (12 * H + 52) + 20 * entries + 4 * 5


def test_roofline_against_the_fp32_peak():
    import bench
    # 256 CUs x 2.4 GHz x 256 FLOP per clock (packed FP32, the published peak)
    assert bench.FP32_PEAK_TFLOPS == pytest.approx(157.2864)
    st = [1e6, 2e6, 5e5]
    r = bench.alu_roofline(st, 1.0, "k", None)
    flops = 1e6 * 830 + 2e6 * 35 + 5e5 * 500
    assert r["bound"] == "alu" and r["peak"] == bench.FP32_PEAK_TFLOPS
    assert r["achieved"] == pytest.approx(flops / 1e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.2864)
    assert r["frac_of_issue_peak"] == pytest.approx(2 * r["frac"])
    assert r["fp64_flop_share"] == pytest.approx((1e6 * 55 + 2e6 * 10 + 5e5 * 500) / flops)


def test_parity_sample_spans_the_batch():
    import bench
    import kfsynth
    ev = kfsynth.generate("batch256", n_events=40)
    idx = bench.parity_sample(ev)
    assert idx.size >= 2000 and np.unique(idx).size == idx.size
    assert np.unique(ev.trk_event[idx]).size >= 16
    one = kfsynth.generate("build5k", tracks_per_event=3000)
    assert bench.parity_sample(one).size >= 2000
