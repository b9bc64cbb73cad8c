"""Host logic of the benchmark (no GPU): the byte model, the network's flop
count, the refusal of more than one GPU, and the rule that counter-measured
traffic is reported only for the kernel sources it was measured on."""
import os
import subprocess
import sys

import bench
from paper_2010_14823_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_headline_domain():
    cfg = synth.CONFIGS["c3"]
    mask = synth.cloud_mask(cfg)
    ncloudy = int(mask.sum())
    assert ncloudy == round(0.5 * cfg.ncol)
    # 14 reads + 12 writes of 8 B per point of a cloudy column, 8 + 12 per
    # point of a clear one, 8 surface values per column
    want = cfg.nlev * (ncloudy * (14 + 12) * 8 + (cfg.ncol - ncloudy) * (8 + 12) * 8) + cfg.ncol * 8 * 8
    assert bench.algorithmic_bytes(cfg, mask) == want == 23219666944
    # warm: no ice-phase inputs (8 and 5 fields read), still 12 tendencies
    warm = cfg.nlev * (ncloudy * (8 + 12) * 8 + (cfg.ncol - ncloudy) * (5 + 12) * 8) + cfg.ncol * 64
    assert bench.algorithmic_bytes(cfg, mask, warm=True) == warm


def test_network_flop_per_point():
    # 12 -> 128 -> 128 -> 128 -> 12, one multiply and one add per weight
    assert bench.NET_FLOP_PER_POINT == 2 * (12 * 128 + 2 * 128 * 128 + 128 * 12) == 71680


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single" in r.stderr
    assert r.stdout == ""


def test_traffic_is_reported_only_for_the_measured_sources(monkeypatch, tmp_path):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "sweep_kernel_w_fp64_hbm_counters.md").write_text(
        "# counters\n\n- source_sha256: " + "ab" * 32 + "\n- hbm_bytes_per_launch: 2.551890e+10\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sweep_source_digest", lambda: "ab" * 32)
    assert bench.recorded_traffic("w", "fp64") == 2.55189e10
    monkeypatch.setattr(bench, "sweep_source_digest", lambda: "cd" * 32)
    assert bench.recorded_traffic("w", "fp64") is None
    assert bench.recorded_traffic("no_such_workload", "fp64") is None
