"""Host-side logic of bench.py: the roofline's traffic and limiter come from the
committed counter files only when those were taken on the current scatter
source (checked by hash); and the benchmark refuses more than one GPU."""
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
         "sq": {"per_dispatch_median": {"SQ_INSTS_VALU": valu}, "valu_per_64_symbols": per64}}
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(c))
    return str(src), str(path)


def test_counters_used_when_source_matches(tmp_path, monkeypatch):
    src, path = _counters(tmp_path, "kernel source A")
    monkeypatch.setattr(bench, "SCATTER_SRC", src)
    assert bench.scatter_traffic(1, path) == 5_000_000_000
    # 1.5e9 VALU instructions in 2.5 ms against 1024 SIMDs x 2.4 GHz / 4
    lim = bench.valu_limiter(path, "7 levels", 2.5)
    frac = 1.5e9 / (2.5e-3 * 1024 * 2.4e9 / 4)
    assert f"about {round(100 * frac)}%" in lim
    assert "about 89 VALU instructions per 64 symbols for 7 levels" in lim


def test_counters_ignored_when_source_changed(tmp_path, monkeypatch):
    src, path = _counters(tmp_path, "kernel source A", sha="0" * 64)
    monkeypatch.setattr(bench, "SCATTER_SRC", src)
    assert bench.scatter_traffic(1, path) is None
    assert "not taken" in bench.valu_limiter(path, "7 levels", 2.5)


def test_counters_missing(tmp_path, monkeypatch):
    src, _ = _counters(tmp_path, "kernel source A")
    monkeypatch.setattr(bench, "SCATTER_SRC", src)
    missing = str(tmp_path / "none.json")
    assert bench.scatter_traffic(1, missing) is None
    assert "not taken" in bench.valu_limiter(missing, "7 levels", 2.5)


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
