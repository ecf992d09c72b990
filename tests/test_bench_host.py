"""Host logic of bench.py (no GPU): the roofline's byte counts and the rule that ties
the committed rocprofv3 summaries to the kernel sources they were taken on."""
import os
import shutil

import pytest

import bench


def test_stage_bytes_per_cell():
    """Algorithmic bytes of one stage launch, averaged over the three stages of a step:
    stage 1 reads U^n and writes U^(1) (2 x 15 values), stages 2 and 3 read U^(s-1)
    and U^n and write U^(s) (3 x 15 values): 160 B per cell in FP32, 320 in FP64, and
    eight array passes of 60 / 120 B per step (480 / 960 B per cell-update)."""
    assert bench.stage_bytes_per_cell(4) == 160.0
    assert bench.stage_bytes_per_cell(8) == 320.0
    assert 3 * bench.stage_bytes_per_cell(4) == 480.0
    assert 3 * bench.stage_bytes_per_cell(8) == 960.0


def test_committed_counters_match_the_current_kernels():
    """The committed summaries carry the hash of the kernel sources they were taken on;
    they are current, so bench.py reads their per-launch figures for the built tile."""
    assert bench.measured_traffic([32, 8]) is not None
    assert bench.measured_valu([32, 8]) is not None
    assert 0.3 * 167772160 < bench.measured_traffic([32, 8]) < 1.5 * 167772160
    assert bench.measured_traffic([16, 16]) is None     # taken on another tile shape


def test_hash_ignores_comments_and_follows_code(tmp_path):
    """A comment edit keeps the hash (the kernel is the same); a code edit changes it."""
    root = tmp_path
    for p in bench.KERNEL_SOURCES:
        os.makedirs(os.path.dirname(root / p), exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, p), root / p)
    h0 = bench.kernel_source_hash(str(root))
    assert h0 == bench.kernel_source_hash()
    k = root / bench.KERNEL_SOURCES[0]
    txt = k.read_text()
    k.write_text(txt + "\n// a comment\n/* and another */\n")
    assert bench.kernel_source_hash(str(root)) == h0
    k.write_text(txt.replace("R(0.5)", "R(0.25)", 1))
    assert bench.kernel_source_hash(str(root)) != h0


def test_counter_file_with_another_hash_is_ignored(tmp_path, monkeypatch):
    src = open(bench.COUNTER_FILE).read()
    bad = tmp_path / "counters.txt"
    bad.write_text(src.replace("kernel_source_sha256_16:", "kernel_source_sha256_16: 0000 stale"))
    assert bench._counter_value(str(bad), "hbm_bytes_per_launch", [32, 8]) is None
    good = tmp_path / "good.txt"
    good.write_text(src)
    assert bench._counter_value(str(good), "hbm_bytes_per_launch", [32, 8]) == pytest.approx(
        bench.measured_traffic([32, 8]))
