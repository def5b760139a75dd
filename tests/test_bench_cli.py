"""The benchmark's command-line contract that holds without a GPU: it measures one GPU only
and refuses a multi-GPU request with a message; its stored-counter lookups go stale with the
kernel sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_stored_counter_figures_follow_the_source_hash(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash("step_bgk.hip")
    assert bench.kernel_source_hash("step_elbm.hip") != h
    (tmp_path / "profiles").mkdir()
    rec = {"source_hash": h, "hbm_bytes_per_launch": 123}
    (tmp_path / "profiles" / "traffic_x.json").write_text(json.dumps(rec))
    rec_stale = dict(rec, source_hash="0" * 16)
    (tmp_path / "profiles" / "traffic_y.json").write_text(json.dumps(rec_stale))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda tu="step_bgk.hip": h)
    assert bench.stored_traffic("x", 1) == 123
    assert bench.stored_traffic("y", 1) is None
    assert bench.stored_traffic("missing", 1) is None
