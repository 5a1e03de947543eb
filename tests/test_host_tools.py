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


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_frame_plan_covers_every_leg():
    """The walk holds the warm-up, the timed calls and the CPU sample at the
    driver's arguments (--steps 20 --warmup 5) and at the defaults."""
    b = _bench_module()
    assert b.plan_frames(5, 20, 200) == 205
    assert b.plan_frames(50, 1000, 200) == 1050
    assert b.plan_frames(5, 20, 0) == 25
    with pytest.raises(ValueError):
        b.plan_frames(5, 0, 10)


def test_bench_times_a_sample_of_the_tile_launches():
    """At the driver's 20 steps two launches are bracketed (every 10th);
    at 1,000 steps every 16th; never more than every call."""
    b = _bench_module()
    assert b.timing_every(20) == 10
    assert b.timing_every(1000) == 64
    assert b.timing_every(1) == 1 and b.timing_every(3) == 1
    assert all(1 <= b.timing_every(k) <= 64 for k in range(1, 2000))
    assert all(k // b.timing_every(k) >= 2 for k in range(4, 2000))  # at least two timed launches


def test_bench_cpu_baseline_on_a_short_walk():
    """The oracle legs stay inside the frames they are given (a 25-frame walk,
    W = 5: at most 20 calls) and report both thread counts."""
    from paper_2608_12691_amd import systems
    b = _bench_module()
    w = systems.make_config(2)
    s = w.systems[0]
    W, K = 5, 20
    traj = systems.perturbation_walk(s, W + K, 0.01, seed=7)
    lams = systems.lambda_draws(W + K, seed=8)
    rec = b.cpu_baseline(w, traj, lams, W, 200, budget_s=0.2, budget_1core_s=0.2)
    assert rec["kind"] == "oracle" and rec["unit"] == "pair-evals/s" and rec["value"] > 0
    assert rec["cores"] == b.host_threads() and rec["single_core"]["cores"] == 1
    assert rec["single_core"]["value"] > 0
    # a sample that starts past the last frame is an error, not an index fault
    with pytest.raises(ValueError):
        b._oracle_leg(w, traj, lams, W + K, 10, 1.0, 1)
    # GPU results at the sample's first call are compared with the oracle's
    import oracle as O
    ref = O.evaluate(traj[W], s.types, s.is_solute, s.exclusions, s.box, w.ff.sigma, w.ff.epsilon, w.ff.charge,
                     O.Params.of(w), lams[W])
    exact = dict(forces=ref["forces"].copy(), dudl=ref["terms"][9], terms=ref["terms"].copy())
    off = dict(forces=ref["forces"] * (1 + 1e-6), dudl=ref["terms"][9] + 1e-3 * ref["abs_terms"][9],
               terms=ref["terms"] + 2e-7 * ref["abs_terms"])
    rec = b.cpu_baseline(w, traj, lams, W, 2, budget_s=0.2, budget_1core_s=0.2,
                         gpu_first={"fp32": off, "fp64": exact})
    e = rec["error_vs_oracle"]
    assert e["call"] == W
    assert e["fp64"] == {"force_rms_rel": 0.0, "dudl_rel": 0.0, "energy_rel": 0.0}
    assert abs(e["fp32"]["force_rms_rel"] - 1e-6) < 1e-9
    assert abs(e["fp32"]["energy_rel"] - 2e-7) < 1e-9
    d = abs(ref["terms"][9])
    S = ref["abs_terms"][9]
    want = 1e-3 * S / d if d >= 1e-2 * S else 1e-3
    assert abs(e["fp32"]["dudl_rel"] - want) < 1e-9 * max(1.0, want)


def test_bench_optional_leg_failure_is_recorded():
    b = _bench_module()
    line = {}
    b.optional(line, "leg", lambda: 1 / 0)
    assert "ZeroDivisionError" in line["leg"]["error"]
    b.optional(line, "ok", lambda: 3)
    assert line["ok"] == 3
