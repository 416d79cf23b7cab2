"""Host-side logic of bench.py: the roofline's traffic and its VALU-issue
figures come from the committed counter files only when those were taken on
the current scatter source (checked by hash); and the benchmark refuses more
than one GPU."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _counters(tmp_path, src_text, sha=None, valu=1.5e9, per64=89.4, bytes_per_launch=5_000_000_000):
    src = tmp_path / "wt_scatter.hip"
    src.write_text(src_text)
    c = {"source_sha256": sha if sha is not None else hashlib.sha256(src.read_bytes()).hexdigest(),
         "bytes_per_launch": bytes_per_launch,
         "valu_per_step": valu, "valu_per_64_symbols": per64, "lds_per_64_symbols": 13.0,
         "sq": {"per_dispatch_median": {"SQ_INSTS_VALU": valu}, "valu_per_64_symbols": per64,
                "lds_per_64_symbols": 13.0}}
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(c))
    return str(src), str(path)


def test_counters_used_when_source_matches(tmp_path, monkeypatch):
    src, path = _counters(tmp_path, "kernel source A")
    monkeypatch.setattr(bench, "SCATTER_SRC", src)
    assert bench.scatter_traffic(1, path) == 5_000_000_000
    # 1.5e9 VALU instructions in 2.5 ms against 1024 SIMDs x 2.4 GHz / 4
    frac = 1.5e9 / (2.5e-3 * 1024 * 2.4e9 / 4)
    for alu in (bench.alu_issue("w", 2.5, path), bench.single_alu_issue(2.5, path)):
        assert alu["frac"] == round(frac, 4)
        assert alu["peak"] == 614.4 and alu["valu_per_64_symbols"] == 89.4


def test_counters_ignored_when_source_changed(tmp_path, monkeypatch):
    src, path = _counters(tmp_path, "kernel source A", sha="0" * 64)
    monkeypatch.setattr(bench, "SCATTER_SRC", src)
    assert bench.scatter_traffic(1, path) is None
    assert bench.alu_issue("w", 2.5, path) is None and bench.single_alu_issue(2.5, path) is None


def test_counters_missing(tmp_path, monkeypatch):
    src, _ = _counters(tmp_path, "kernel source A")
    monkeypatch.setattr(bench, "SCATTER_SRC", src)
    missing = str(tmp_path / "none.json")
    assert bench.scatter_traffic(1, missing) is None
    assert bench.alu_issue("w", 2.5, missing) is None and bench.single_alu_issue(2.5, missing) is None
    # the roofline then names no limiter it has not measured
    assert bench.bound_fields("no such workload", 2.5)["bound"] == "hbm"


def test_committed_counters_are_well_formed():
    for path in (bench.COUNTERS, bench.PAIR_COUNTERS):
        c = json.load(open(path))
        assert len(c["source_sha256"]) == 64
        # each figure is rounded down on its own
        assert abs(c["bytes_per_launch"] - c["fetch_bytes_per_launch"] - c["write_bytes_per_launch"]) <= 1
        assert c["sq"]["per_dispatch_median"]["SQ_INSTS_VALU"] > 0


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
