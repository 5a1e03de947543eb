"""Host-side tooling (no GPU): the profile summaries and the bench's one-GPU contract."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _trace_db(path):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, duration integer)")
    con.executemany("insert into kernels values (?, ?)",
                    [("anb::k_tile<float, 0, true>(anb::Dev, ...)", 20000), ("anb::k_tile<float, 0, true>(anb::Dev, ...)", 22000),
                     ("anb::k_prepare(anb::Dev, ...)", 4000)])
    con.commit()


def _pmc_db(path, tile_kib, copy_kib):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, dispatch_id integer, counter_name text, value real)")
    rows = []
    for i, v in enumerate(tile_kib):
        rows += [("k_tile<float, 0, true>", i, "FETCH_SIZE", v / 2), ("k_tile<float, 0, true>", i, "FETCH_SIZE", v / 2)]
    rows.append(("__amd_rocclr_copyBuffer", 99, "FETCH_SIZE", copy_kib))
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()


def test_kernel_trace_summary(tmp_path):
    from paper_2608_12691_amd import profiling as P
    db = str(tmp_path / "t.db")
    _trace_db(db)
    out = str(tmp_path / "t.txt")
    P.kernels_summary(db, out, "cmd")
    lines = open(out).read().splitlines()
    assert lines[1] == "command: cmd"
    tile = [l for l in lines if l.startswith("k_tile")][0].split()
    calls, total, avg, med, mx = int(tile[-6]), float(tile[-5]), float(tile[-4]), float(tile[-3]), float(tile[-2])
    assert (calls, total, avg, med, mx) == (2, 42.0, 21.0, 21.0, 22.0)


def test_traffic_scaling_by_calibration_copy(tmp_path):
    """Counter KiB are scaled by what the counter reads for a copy of known size (per dispatch sums)."""
    from paper_2608_12691_amd import profiling as P
    f = str(tmp_path / "f.db")
    w = str(tmp_path / "w.db")
    _pmc_db(f, [100.0, 300.0], 512.0)
    con = sqlite3.connect(w)
    con.execute("create table counters_collection (kernel_name text, dispatch_id integer, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)",
                    [("k_tile<float, 0, true>", 0, "WRITE_SIZE", 50.0), ("__amd_rocclr_copyBuffer", 9, "WRITE_SIZE", 1024.0)])
    con.commit()
    out = str(tmp_path / "traffic.json")
    P.traffic(f, w, out, "cmd", "k_tile<float, 0, true>", 1 << 20)
    rec = json.load(open(out))
    # a 1 MiB copy read as 512 KiB: 2 bytes per counter KiB; tile mean 200 KiB -> 409600 bytes
    assert rec["FETCH_SIZE"]["bytes_per_counter_kib"] == pytest.approx(2.0)
    assert rec["FETCH_SIZE"]["bytes_per_launch"] == pytest.approx(200 * 1024 * 2.0)
    assert rec["WRITE_SIZE"]["bytes_per_launch"] == pytest.approx(50 * 1024 * 1.0)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(200 * 2048 + 50 * 1024)
    assert rec["kernel_source_hash"] == P.kernel_source_hash()


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
