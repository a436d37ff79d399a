"""Host logic that turns rocprofv3 counter CSVs into the committed profile
records, and the bench's use of those records (no GPU involved)."""
import csv
import json
import os

import pytest

import bench
from paper_1210_3165_amd import profiling
from paper_1210_3165_amd.build import kernel_source_sha

KERNEL = "void bz::bz_page_kernel<256, 1, 0, false>(bz::PageArgs)"
OTHER = "void bz::bz_page_kernel<256, 1, 1, false>(bz::PageArgs)"


def write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], r)))


def test_traffic_scales_by_the_copy_kernel(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    copy = profiling.COPY_KERNEL
    # the copy moves 16 MiB each way; its counters read 8192 KiB fetched and
    # 16384 KiB written, so fetch counts are scaled by 2 and writes by 1
    write_csv(f, [(copy, 1, "FETCH_SIZE", 8192.0), (copy, 1, "FETCH_SIZE", 8192.0),
                  (KERNEL, 262144, "FETCH_SIZE", 9000.0), (KERNEL, 131072, "FETCH_SIZE", 10000.0),
                  (OTHER, 262144, "FETCH_SIZE", 1.0)])
    write_csv(w, [(copy, 1, "WRITE_SIZE", 16384.0), (KERNEL, 262144, "WRITE_SIZE", 16384.0),
                  (KERNEL, 131072, "WRITE_SIZE", 16384.0)])
    rec = profiling.traffic(str(f), str(w), "<256, 1, 0, false>", 16 * 2**20, "w", ["cmd"],
                            ("bz_tile.hpp",))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["bytes_per_launch"] == int((9500.0 * 2 + 16384.0) * 1024)
    assert rec["per_grid_fetch_kib_raw"] == {"131072": 10000.0, "262144": 9000.0}
    assert rec["source_sha"] == kernel_source_sha(("bz_tile.hpp",))
    assert rec["kernels"] == [KERNEL]


def test_traffic_needs_copy_and_kernel_rows(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(f, [(KERNEL, 1, "FETCH_SIZE", 1.0)])
    write_csv(w, [(KERNEL, 1, "WRITE_SIZE", 1.0)])
    with pytest.raises(SystemExit):
        profiling.traffic(str(f), str(w), "bz_page", 16 * 2**20, "w", [], ("bz_tile.hpp",))


def test_valu_lane_ops_per_pixel(tmp_path):
    p = tmp_path / "sq.csv"
    px = 4096 * 4096
    write_csv(p, [(KERNEL, 262144, "SQ_INSTS_VALU", 10_000_000.0), (KERNEL, 131072, "SQ_INSTS_VALU", 12_000_000.0),
                  (KERNEL, 262144, "SQ_WAVES", 4096.0), (KERNEL, 131072, "SQ_WAVES", 2048.0),
                  (OTHER, 262144, "SQ_INSTS_VALU", 1.0)])
    rec = profiling.valu(str(p), "<256, 1, 0, false>", px, "w", ["cmd"], ("bz_tile.hpp",))
    assert rec["kernel"] == "<256, 1, 0, false>" and rec["kernels"] == [KERNEL]
    assert rec["per_dispatch"] == {"SQ_WAVES": 3072.0, "SQ_INSTS_VALU": 11_000_000.0}
    assert rec["valu_lane_ops_per_px"] == round(11_000_000 * 64 / px, 3)
    with pytest.raises(SystemExit):
        profiling.valu(str(p), "no such kernel", px, "w", [], ("bz_tile.hpp",))


def test_bench_uses_records_of_the_current_source_only(tmp_path, monkeypatch):
    rec = {"source_sha": kernel_source_sha(), "valu_lane_ops_per_px": 40.0, "bytes_per_launch": 123}
    path = tmp_path / "r.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "VALU_FILE", str(path))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    px, ms = 4096 * 4096, 0.04
    v = bench.measured_valu(px, ms)
    assert v["lane_ops_per_px"] == 40.0
    assert v["peak_T_lane_ops_s"] == pytest.approx(39.3216)
    assert v["frac"] == pytest.approx(40.0 * px / 40e-6 / 39.3216e12)
    assert bench.measured_traffic() == 123
    path.write_text(json.dumps(dict(rec, source_sha="0" * 64)))
    assert bench.measured_valu(px, ms) is None and bench.measured_traffic() is None


def test_bench_refuses_more_than_one_gpu():
    """The bench measures one GPU; asked for more it exits with a message and
    without touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for extra, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *extra], capture_output=True,
                           text=True, timeout=120, env={**os.environ, **env})
        assert r.returncode == 2 and "one GPU only" in r.stderr, (extra, env, r.stderr)


def test_percentile_matches_numpy():
    import numpy as np
    rng = np.random.default_rng(3)
    for n in (1, 2, 5, 40):
        v = list(rng.uniform(1, 100, n))
        for q in (10, 50, 90):
            assert abs(profiling._pct(v, q) - float(np.percentile(v, q))) < 1e-9


def _fake_amd_smi(tmp_path, text):
    tool = tmp_path / "amd-smi"
    (tmp_path / "out.txt").write_text(text)
    tool.write_text(f"#!/bin/sh\ncat {tmp_path / 'out.txt'}\n")
    tool.chmod(0o755)
    return str(tmp_path)


def test_sclk_sampler_reads_every_xcd_under_load(tmp_path, monkeypatch):
    """The bench's clock sampler parses the GFX clock of each XCD from the
    tool's text, keeps the steps running while it reads, and summarises the
    readings; the memory clock and limits are not taken for GFX clocks."""
    text = ("GPU: 0\n    CLOCK:\n"
            + "".join(f"        GFX_{i}:\n            CLK: {2390 + i} MHz\n            MIN_CLK: 500 MHz\n"
                      f"            MAX_CLK: 2400 MHz\n" for i in range(8))
            + "        MEM_0:\n            CLK: 2000 MHz\n")
    monkeypatch.setenv("PATH", _fake_amd_smi(tmp_path, text) + os.pathsep + os.environ["PATH"])
    steps = []
    res = bench.sample_sclk(lambda: steps.append(1), min_samples=2, seconds=0.1, limit_s=5.0,
                            sync=lambda: None)
    assert res is not None and res["xcds"] == 8 and res["readings"] >= 2
    assert (res["min"], res["max"]) == (2390, 2397) and 2390 <= res["median"] <= 2397
    assert len(steps) > 0


def test_sclk_sampler_without_clock_readings(tmp_path, monkeypatch):
    monkeypatch.setenv("PATH", _fake_amd_smi(tmp_path, "no GPU found\n") + os.pathsep + os.environ["PATH"])
    assert bench.sample_sclk(lambda: None, seconds=0.05, limit_s=1.0, sync=lambda: None) is None
    monkeypatch.setenv("PATH", str(tmp_path / "empty"))
    assert bench.sample_sclk(lambda: None, seconds=0.05, limit_s=1.0, sync=lambda: None) is None


def test_overlap_summary_counts_launches_in_flight(tmp_path):
    """Runs split where the kernel or grid changes; a serial run has one
    launch in flight, an overlapping one reports its mean depth and the share
    of its span with two or more in flight."""
    cols = ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"]
    rows = [("void k<1>(A)", 100, 0, 10_000), ("void k<1>(A)", 100, 10_000, 20_000),   # serial
            ("void k<1>(A)", 50, 30_000, 40_000), ("void k<1>(A)", 50, 35_000, 45_000),  # overlap
            ("void other(B)", 100, 50_000, 60_000)]
    with open(tmp_path / "t_kernel_trace.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        w.writerows(rows)
    table = profiling.overlap_summary(str(tmp_path), "t", "k<1>").strip().split("\n")
    assert len(table) == 4
    serial = [c.strip() for c in table[2].split("|")[1:-1]]
    over = [c.strip() for c in table[3].split("|")[1:-1]]
    assert serial[2:] == ["100", "2", "10.0", "20.0", "10.0", "1.00", "0.00"]
    assert over[2:] == ["50", "2", "10.0", "15.0", "7.5", "1.33", "0.33"]
    assert len(profiling.overlap_summary(str(tmp_path), "t", "k<1>", min_launches=3).strip().split("\n")) == 2
