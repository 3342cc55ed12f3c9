"""CPU checks of the benchmark's command-line contract (no GPU needed)."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
    assert "--gpus" in r.stderr or "gpus" in r.stderr


def test_traffic_record_is_ignored_for_other_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    for p in bench.TRAFFIC_SOURCES:
        f = tmp_path / p
        f.parent.mkdir(parents=True, exist_ok=True)
        f.write_text("kernel source A")
    rec = {"sources_digest": bench.sources_digest(),
           "kernels": {"lu": {"hbm_bytes_per_launch": 123.0}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.recorded_traffic("lu") == 123.0
    (tmp_path / bench.TRAFFIC_SOURCES[0]).write_text("kernel source B")
    assert bench.recorded_traffic("lu") is None
