"""Host logic of bench.py (CPU only): the kernel-source hash ignores comments,
the PMC summaries are found for the configurations they were taken for and
only those, the 1-D resolution spreads are read from the oracle's study, and
more than one GPU is refused."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_kernel_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    srcs = []
    for rel in bench.STEP_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), dst)
        srcs.append(dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_hash()
    assert h0 == bench.kernel_hash()
    hdr = next(p for p in srcs if p.name == "kc_stream.h")
    text = hdr.read_text()
    assert "#pragma once\n" in text
    hdr.write_text("// a new comment line\n/* and a block\n   comment */\n" +
                   text.replace("#pragma once\n", "#pragma once // trailing\n", 1) + "\n\n")
    assert bench.kernel_hash() == h0
    assert "R(0.5)" in text
    hdr.write_text(text.replace("R(0.5)", "R(0.25)", 1))
    assert bench.kernel_hash() != h0


def test_pmc_summaries_match_their_configurations_only():
    found = 0
    for cand in bench.CANDIDATES_4096:
        t = bench.measured_traffic(*cand)
        c = bench.measured_counters(*cand)
        if t is None:
            continue
        found += 1
        assert 335544320 <= t <= 2 * 335544320
        assert 33 <= c["valu_issued_per_update"] <= 60 and 0 < c["valu_busy"] <= 1
    assert found == len(bench.CANDIDATES_4096)
    assert bench.measured_traffic(4, 36, 4, 1) is None
    assert bench.measured_counters(3, 35, 4, 1) is None


def test_resolution_spreads_of_the_1d_study():
    sp = bench.resolution_spread(400)
    assert len(sp) == 30
    assert all(0 <= v <= 0.02 for v in sp.values())
    assert bench.resolution_spread(12345) == {}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
    assert r.stdout == ""
