"""Host-side checks of the measurement plumbing: the traffic mode of
profile_summary.py (counter scaling by the calibration copies, per-step
sums, the source hash) and bench.measured_traffic (a figure is used only
while the kernel sources still hash to the recorded value)."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, dispatch_id int, "
                "counter_name text, value real, duration real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?)",
                    [(k, i, counter, v, d) for i, (k, v, d) in enumerate(rows)])
    con.commit()
    con.close()


def _traffic(tmp_path, *extra):
    copy = 1 << 30
    # the copies read as half their bytes (FETCH) and as their bytes (WRITE)
    _db(tmp_path / "f.db", "FETCH_SIZE",
        [("__amd_rocclr_copyBuffer", copy / 2048, 5e5)] * 2 +
        [("kern_a", 1000.0, 50e3), ("kern_a", 3000.0, 50e3), ("kern_a", 1.0, 1e3),
         ("kern_b", 10.0, 30e3)])
    _db(tmp_path / "w.db", "WRITE_SIZE",
        [("__amd_rocclr_copyBuffer", copy / 1024, 5e5)] * 2 +
        [("kern_a", 500.0, 50e3), ("kern_a", 500.0, 50e3), ("kern_a", 0.0, 1e3),
         ("kern_b", 20.0, 30e3)])
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    out = subprocess.run(
        [sys.executable, os.path.join(ROOT, "profile_summary.py"), str(tmp_path / "f.db"),
         "--write-db", str(tmp_path / "w.db"), "--match", "kern_a|kern_b", "--min-us", "20",
         "--source", str(src), "--config", "CFG", *extra],
        capture_output=True, text=True, check=True).stdout
    line = [x for x in out.splitlines() if x.startswith("TRAFFIC ")][0]
    return json.loads(line[len("TRAFFIC "):])


def test_traffic_long_dispatch_means(tmp_path):
    rec = _traffic(tmp_path)
    # kern_a: mean of the two long dispatches; kern_b: one; KiB x 1024 x factor
    assert rec["fetch_factor"] == pytest.approx(2.0)
    assert rec["write_factor"] == pytest.approx(1.0)
    assert rec["read_bytes"] == round((2000.0 + 10.0) * 1024 * 2)
    assert rec["write_bytes"] == round((500.0 + 20.0) * 1024)
    assert rec["bytes_per_step"] == rec["read_bytes"] + rec["write_bytes"]
    assert len(rec["source_sha256"]) == 64


def test_traffic_per_step_totals(tmp_path):
    rec = _traffic(tmp_path, "--per-step", "2")
    # every dispatch counts (the short one too), divided by the step count
    assert rec["read_bytes"] == round((4001.0 + 10.0) / 2 * 1024 * 2)
    assert rec["write_bytes"] == round((1000.0 + 20.0) / 2 * 1024)
    assert rec["per_step"] == 2


def test_measured_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    import hashlib

    import bench
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "a.hip"
    src.write_text("one\n")
    src2 = tmp_path / "b.h"
    src2.write_text("two\n")
    sha = hashlib.sha256(b"one\ntwo\n").hexdigest()
    rec = {"config": "CFG", "bytes_per_step": 1234, "sources": ["a.hip", "b.h"],
           "source_sha256": sha}
    (tmp_path / "profiles" / "p.md").write_text("text\nTRAFFIC " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("CFG") == (1234, os.path.join("profiles", "p.md"))
    assert bench.measured_traffic("OTHER") == (None, None)
    src2.write_text("changed\n")
    assert bench.measured_traffic("CFG") == (None, None)
