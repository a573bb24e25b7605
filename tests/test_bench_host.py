"""Host-side checks of the benchmark driver (no GPU): the one-GPU guard and
the kernel-code hash that keys the stored traffic measurements."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_code_text_drops_comments_and_blank_lines_only():
    src = "int a; // note\n\n   // whole-line comment\n  b = a * 2;   \nc();"
    assert bench.code_text(src) == "int a;\n  b = a * 2;\nc();"
    # a comment edit leaves the hash input unchanged, a code edit does not
    assert bench.code_text("x = 1; // old") == bench.code_text("x = 1; // new words")
    assert bench.code_text("x = 1;") != bench.code_text("x = 2;")


def test_kernel_hash_is_stable_and_stored_entries_are_well_formed():
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    for key, entry in bench.MEASURED_TRAFFIC.items():
        wl, prec, storage = key.split("/")
        assert wl in ("c1", "c2", "c4") and prec in ("fp32", "fp64", "fp32x")
        assert storage in ("OM", "OM+AR", "f") and (storage == "f" or prec == "fp32")
        assert len(entry["source"]) == 16 and entry["bytes_per_launch"] > 0
        assert entry["tile_rows"] >= 1
        # FETCH_SIZE counts the kernels' 128 B reads as 64 B: scaled by 2
        assert entry["bytes_per_launch"] == 1024 * (2 * entry["fetch_kib"] + entry["write_kib"])


def test_algorithmic_bytes_per_update():
    # 16 values read and written once per Euler step; RK3 moves 128 values
    assert bench.bytes_per_csu("fp32", 0) == 128 and bench.bytes_per_csu("fp64", 0) == 256
    assert bench.bytes_per_csu("fp32x", 0) == 192 and bench.bytes_per_csu("fp32", 1) == 512
    # A-block residuals: four 2-byte values more, each way
    assert bench.bytes_per_csu("fp32", 0, "OM+AR") == 144
    assert bench.STORAGE_NAMES == {0: "OM", 1: "f", 2: "OM+AR"}


def test_stored_traffic_needs_the_same_code_and_tile_rows(monkeypatch):
    entry = {"source": bench.kernel_source_hash(), "tile_rows": 512, "fetch_kib": 1.0,
             "write_kib": 2.0, "bytes_per_launch": 4096.0}
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "c4/fp32/OM", entry)
    assert bench.stored_traffic("c4", "fp32", "OM", 512) == 4096.0
    assert bench.stored_traffic("c4", "fp32", "OM", 256) is None        # other tile rows
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "c4/fp32/OM", dict(entry, source="0" * 16))
    assert bench.stored_traffic("c4", "fp32", "OM", 512) is None        # other kernel code
    assert bench.stored_traffic("c1", "fp32", "OM", 2) is None          # never measured


def test_default_tile_rows_apply_to_the_timed_workload_only():
    assert bench.DEFAULT_TILE_ROWS == {"c4": 512}
