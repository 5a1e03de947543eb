"""Summaries of rocprofv3 output for the committed profile records.

    python -m paper_2608_12691_amd.profiling kernels DB OUT.txt "COMMAND"
        per-kernel launch counts and durations (from --kernel-trace --stats)
    python -m paper_2608_12691_amd.profiling traffic FETCH_DB WRITE_DB OUT.json "COMMAND" \
        --kernel 'k_tile<float, 0, true>' --copy-bytes N
        HBM bytes per launch of a kernel from two --pmc runs (FETCH_SIZE, then
        WRITE_SIZE), each scaled by what the counter reads for the
        calibration copy of N bytes that the profiled command performs
        (bench.py --copy-calibration); the record carries the hash of the
        kernel sources it was taken on.
    python -m paper_2608_12691_amd.profiling counters DB OUT.txt "COMMAND" --kernel K [--launch-us T]
        mean per-launch counter values of one kernel (from --pmc runs)
"""
import hashlib
import json
import os
import sqlite3
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("tile_kernels.hip", "anb_internal.h", "erfc_coeffs.h", "lane_ops.h", "pair_math.h")


def kernel_source_hash():
    """Hash of the tile kernel's sources: a traffic record applies only to the code it was taken on."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_12691_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _durations(db):
    con = sqlite3.connect(db)
    out = {}
    for name, dur in con.execute("select name, duration from kernels"):
        out.setdefault(name, []).append(dur / 1e3)
    return out


def kernels_summary(db, out_path, command):
    d = _durations(db)
    rows = sorted(d.items(), key=lambda kv: -sum(kv[1]))
    total = sum(sum(v) for v in d.values())
    lines = ["rocprofv3 kernel trace (durations in microseconds)", "command: %s" % command, "",
             "%-64s %7s %10s %9s %9s %9s %6s" % ("kernel", "calls", "total_us", "avg_us", "med_us", "max_us", "pct")]
    for name, v in rows:
        v = np.asarray(v)
        short = name.replace("anb::", "").replace("(anb::Dev", "(Dev")
        short = short if len(short) <= 64 else short[:61] + "..."
        lines.append("%-64s %7d %10.1f %9.3f %9.3f %9.2f %6.2f" % (short, len(v), v.sum(), v.mean(), np.median(v),
                                                                   v.max(), 100 * v.sum() / total))
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(db, counter, pattern):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name = ? "
                       "group by dispatch_id", (counter,)).fetchall()
    return [(k, v) for k, _, v in rows if pattern(k)]


def traffic(fetch_db, write_db, out_path, command, kernel, copy_bytes):
    def is_kernel(k):
        return kernel in k

    def is_copy(k):
        return "copyBuffer" in k or "elementwise" in k

    rec = dict(command=command, kernel=kernel, kernel_source_hash=kernel_source_hash(), copy_bytes=copy_bytes)
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        tile = [v for _, v in _counter(db, counter, is_kernel)]
        copies = [v for _, v in _counter(db, counter, is_copy)]
        cal = max(copies)                       # the calibration copy is the largest copy
        factor = copy_bytes / (cal * 1024.0)    # bytes per counter KiB
        rec[counter] = dict(kib_per_launch_mean=float(np.mean(tile)), kib_per_launch_median=float(np.median(tile)),
                            launches=len(tile), calibration_kib=float(cal), bytes_per_counter_kib=factor,
                            bytes_per_launch=float(np.mean(tile) * 1024.0 * factor))
    rec["hbm_bytes_per_launch"] = rec["FETCH_SIZE"]["bytes_per_launch"] + rec["WRITE_SIZE"]["bytes_per_launch"]
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def counters_summary(db, out_path, command, kernel, launch_us=None):
    """Mean per-launch value of every counter collected for a kernel (sums over the device).
    With the kernel's launch time (from a trace without counters), the FP32
    (and FP64) VALU instruction counts become counter-derived FLOP/s (64 lanes
    per wave instruction, FMA = 2 FLOP; an upper bound: inactive lanes are
    counted)."""
    con = sqlite3.connect(db)
    rows = con.execute("select counter_name, avg(v), count(*) from (select dispatch_id, counter_name, sum(value) v "
                       "from counters_collection where kernel_name like ? group by dispatch_id, counter_name) "
                       "group by counter_name", ("%" + kernel + "%",)).fetchall()
    c = {name: v for name, v, _ in rows}
    lines = ["rocprofv3 counters of %s (mean per launch, device totals)" % kernel, "command: %s" % command, ""]
    lines += ["%-28s %16.6g  (%d launches)" % r for r in rows]
    for prec in ("F32", "F64"):
        keys = ["SQ_INSTS_VALU_%s_%s" % (op, prec) for op in ("FMA", "MUL", "ADD")]
        if launch_us and all(k in c for k in keys):
            flop = 64 * (2 * c[keys[0]] + c[keys[1]] + c[keys[2]] + c.get("SQ_INSTS_VALU_TRANS_" + prec, 0.0))
            name = "FP32" if prec == "F32" else "FP64"
            lines += ["", "%s FLOP per launch (counter-derived, lanes x ops): %.4g" % (name, flop),
                      "launch time (kernel trace): %.3f us" % launch_us,
                      "counter-derived %s rate: %.3f TFLOP/s" % (name, flop / (launch_us * 1e-6) / 1e12)]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main(argv):
    if argv[0] == "kernels":
        kernels_summary(argv[1], argv[2], argv[3])
    elif argv[0] == "counters":
        us = float(argv[argv.index("--launch-us") + 1]) if "--launch-us" in argv else None
        counters_summary(argv[1], argv[2], argv[3], argv[argv.index("--kernel") + 1], us)
    elif argv[0] == "traffic":
        kernel = argv[argv.index("--kernel") + 1]
        nbytes = int(argv[argv.index("--copy-bytes") + 1])
        traffic(argv[1], argv[2], argv[3], argv[4], kernel, nbytes)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
