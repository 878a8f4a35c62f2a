"""Host logic of bench.py (CPU): the algorithmic byte model, the kernel-code
hash that ties a counter summary to the sources it was taken on, the HBM
traffic from calibrated counters, and the per-root cost summary."""
import os
import shutil

import numpy as np
import pytest

import bench

# search statistics of one launch on the 20M-edge, 36-motif workload (the
# instrumented kernel's counts, equal to the oracle's window logs)
CFG2_STATS = {"win_list": 514_840_325, "win_all": 0, "ent_list": 4_434_811_793, "ent_all": 0,
              "push": 141_617_592, "credit": 369_698_594, "roots": 20_000_000}


def test_algorithmic_bytes_of_the_headline_workload():
    # 16 B per root edge, 16 B per window, 8 B per entry (u32 id + u32 time)
    b = bench.algorithmic_bytes(CFG2_STATS, 4, 20_000_000)
    assert b == 44_035_939_544
    # 64-bit times: 4 more bytes per entry
    assert bench.algorithmic_bytes(CFG2_STATS, 8, 20_000_000) - b == 4 * 4_434_811_793
    # whole-list entries carry both endpoints
    st = dict(CFG2_STATS, win_all=1, ent_all=10)
    assert bench.algorithmic_bytes(st, 4, 20_000_000) - b == 16 + 10 * 12


def test_kernel_hash_ignores_comments_and_layout(tmp_path, monkeypatch):
    h0 = bench.kernel_source_hash()
    csrc = tmp_path / "paper_2507_14813_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(bench.ROOT, "paper_2507_14813_amd", "csrc", f), csrc / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    p = csrc / "search.h"
    src = p.read_text()
    p.write_text("// a new comment\n/* and a block\n   comment */\n" + src.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash() == h0
    p.write_text(src + "\nstatic_assert(true, \"x\");\n")
    assert bench.kernel_source_hash() != h0


def test_counter_record_is_tied_to_workload_and_code(monkeypatch):
    rec = bench.counter_record(20_000_000)
    if rec is not None:
        # a record is only used while it matches the sources it was taken on
        assert rec["kernel_source_sha256"] == bench.kernel_source_hash()
        traffic = bench.measured_traffic(rec)
        assert 0 < traffic < bench.algorithmic_bytes(CFG2_STATS, 4, 20_000_000)
        assert 0.0 < rec["tcc_hit"] / (rec["tcc_hit"] + rec["tcc_miss"]) < 1.0
    assert bench.counter_record(20_000_001) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.counter_record(20_000_000) is None
    assert bench.measured_traffic(None) is None


def test_measured_traffic_scales_each_counter():
    rec = {"fetch_kib": 100.0, "write_kib": 10.0, "fetch_factor": 2.0, "write_factor": 1.0}
    assert bench.measured_traffic(rec) == 1024.0 * 210.0


def test_cost_distribution():
    c = np.array([0, 1, 5, 11, 0, 101], dtype=np.uint64)   # 1 + entries, 0 = not searched
    d = bench.cost_distribution(c)
    assert d["roots"] == 4 and d["max"] == 100.0 and d["p50"] == 7.0
    assert d["mean"] == pytest.approx((0 + 4 + 10 + 100) / 4)
    assert bench.cost_distribution(np.zeros(5, np.uint64)) is None
