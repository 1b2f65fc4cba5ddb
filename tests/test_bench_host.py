"""Host logic of bench.py (no GPU): the single-GPU guard, the algorithmic bytes per cell
update that the roofline entry divides by, and the rule that counter traffic is reported
only while the sweep sources still hash to the value the counters were taken on."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_bytes_per_fluid_cell_update():
    import bench
    from synth import workload
    wl3 = workload("c3_foam_384")
    # each population read once and written once, plus the type byte
    assert bench.bytes_per_fluid_cell(wl3, "fp32") == 2 * 19 * 4 + 2 * 7 * 4 + 1 == 209
    assert bench.bytes_per_fluid_cell(wl3, "f16s") == 2 * 19 * 2 + 2 * 7 * 4 + 1 == 133
    assert bench.bytes_per_fluid_cell(wl3, "f16s_g16") == 2 * 19 * 2 + 2 * 7 * 2 + 1 == 105
    wl2 = dict(wl3, dim=2)
    assert bench.bytes_per_fluid_cell(wl2, "fp64") == 2 * 9 * 8 + 2 * 5 * 8 + 1


def test_traffic_is_reported_only_for_the_hashed_sources(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "kernel.h"
    src.write_bytes(b"// sweep source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "traffic.md"
    prof.write_text(f"    source_sha256: {sha}\n    traffic_bytes_per_launch k<3,4,8,256>: 4617801172\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(prof))
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", (str(src),))
    assert bench.measured_traffic("k<3,4,8,256>") == 4617801172
    assert bench.measured_traffic("k<3,1,4,256>") is None
    src.write_bytes(b"// sweep source, edited\n")
    assert bench.measured_traffic("k<3,4,8,256>") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("k<3,4,8,256>") is None
