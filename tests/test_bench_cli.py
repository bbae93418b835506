"""Host-side checks of the benchmark driver (no GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


def test_unknown_time_to_design_leg_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--ttd-steps", "1", "--ttd-modes", "fp16"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode != 0 and "--ttd-modes" in p.stderr


def test_recorded_traffic_is_current():
    """Every committed counter record was taken on the kernel sources as they
    stand (a stale record makes the bench report its traffic as null)."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        recs = json.load(fh)
    assert recs
    for key, rec in recs.items():
        name = key.split(" @ ")[0]
        family = "heat" if name.startswith("heat") else ("el3d" if name.startswith("el3d") else "el2d")
        assert rec["source_digest"] == bench.source_digest(family), key


def test_bytes_per_cell():
    """Algorithmic bytes per cell and sweep: state and velocity read and written
    once plus one material value (FP32)."""
    assert bench.bytes_per_cell("heat_batch64") == 4 * (2 + 2) + 4
    assert bench.bytes_per_cell("multimaterial3d_256x128x18") == 4 * (6 + 6) + 4
    assert bench.bytes_per_cell("cantilever3d_128x64x64") == 52
    assert bench.bytes_per_cell("cantilever2d_1024x512") == 4 * (4 + 4) + 4
    assert bench.RHS_BYTES_PER_CELL["el2d"] == 8 and bench.RHS_BYTES_PER_CELL["el3d"] == 12


def test_oracle_extrapolation_uses_the_fp64_sweeps():
    cpu = {"sweep_seconds": 0.01, "sensitivity_and_phase_seconds": 0.5, "cores": 1, "sample": "s"}
    ttd = {"config": {"design_steps": 4}, "fp64_plain": {"sweeps": 1000}}
    ex = bench.oracle_extrapolation(cpu, ttd)
    assert ex["seconds"] == 0.01 * 1000 + 0.5 * 4 and ex["cores"] == 1
    assert bench.oracle_extrapolation(None, ttd) is None


def test_recorded_traffic_needs_matching_sources(tmp_path, monkeypatch):
    digest = bench.source_digest("el2d")
    rec = {"k @ w": {"source_digest": digest, "fetch_kib": 10.0, "fetch_factor": 2.0, "write_kib": 4.0,
                     "write_factor": 1.0}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    real_root = bench.ROOT
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # sources are read from the real tree
    monkeypatch.setattr(bench, "source_digest", lambda fam: digest)
    assert bench.recorded_traffic("el2d", "k", "w") == (10.0 * 2.0 + 4.0) * 1024
    monkeypatch.setattr(bench, "source_digest", lambda fam: "changed")
    assert bench.recorded_traffic("el2d", "k", "w") is None
    assert bench.recorded_traffic("el2d", "other", "w") is None
    assert real_root
