"""Summaries of rocprofv3 output for the benchmark's records.

``python -m paper_2308_01654_amd.profsum traffic FETCH_DIR WRITE_DIR OUT.json``
    FETCH_SIZE / WRITE_SIZE runs of ``bench.py --probe N`` (one counter per
    run): bytes per dispatch of the iteration and combine kernels, scaled by
    what the same counters read for the calibration copy of known size.
``python -m paper_2308_01654_amd.profsum counters DIR [DIR ...] OUT.json``
    SQ counter runs of ``bench.py --probe N``: per-dispatch values of the
    iteration kernel (the last dispatch), per-wave figures and the executed
    FP32 instruction mix.
``python -m paper_2308_01654_amd.profsum stats DIR``
    Kernel-trace statistics (``--kernel-trace --stats``) as a Markdown table.
``python -m paper_2308_01654_amd.profsum trace DIR OUT.json``
    The same statistics of the iteration and combine kernels as a record
    (calls, average, minimum and maximum duration in ns).

Every JSON record carries the hash of the kernel source it was taken on;
bench.py reports a record only while that hash matches the source.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "mppi_kernels.hip")
COPY_BYTES = 256 << 20   # bench.py --probe: mppi_bench_copy(256 MiB) reads and writes this


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no counter_collection.csv under %s" % d)
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows):
    """{dispatch id: (kernel name, {counter: value summed over dimensions})}"""
    out = {}
    for r in rows:
        did = int(r["Dispatch_Id"])
        name, vals = out.setdefault(did, (r["Kernel_Name"], collections.defaultdict(float)))
        vals[r["Counter_Name"]] += float(r["Counter_Value"])
    return out


def _last(disp, key):
    ids = [i for i, (n, _) in disp.items() if key in n]
    if not ids:
        raise KeyError(key)
    i = max(ids)
    return disp[i][0], dict(disp[i][1])


def traffic(fetch_dir, write_dir, out):
    df, dw = _per_dispatch(_rows(fetch_dir)), _per_dispatch(_rows(write_dir))
    _, cf = _last(df, "k_copy")
    _, cw = _last(dw, "k_copy")
    fetch_scale = COPY_BYTES / (cf["FETCH_SIZE"] * 1024.0)
    write_scale = COPY_BYTES / (cw["WRITE_SIZE"] * 1024.0)
    kn, kf = _last(df, "k_batch")
    _, kw = _last(dw, "k_batch")
    cn, cbf = _last(df, "k_combine")
    _, cbw = _last(dw, "k_combine")
    rec = dict(kernel=kn, kernel_source_sha256_16=kernel_source_hash(),
               fetch_scale=fetch_scale, write_scale=write_scale,
               fetch_bytes_per_launch=kf["FETCH_SIZE"] * 1024.0 * fetch_scale,
               write_bytes_per_launch=kw["WRITE_SIZE"] * 1024.0 * write_scale,
               combine_kernel=cn,
               combine_fetch_bytes_per_launch=cbf["FETCH_SIZE"] * 1024.0 * fetch_scale,
               combine_write_bytes_per_launch=cbw["WRITE_SIZE"] * 1024.0 * write_scale)
    rec["hbm_bytes_per_launch"] = int(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])
    rec["counters_kib_per_dispatch"] = {"k_copy": [cf["FETCH_SIZE"], cw["WRITE_SIZE"]],
                                       "k_batch": [kf["FETCH_SIZE"], kw["WRITE_SIZE"]],
                                       "k_combine": [cbf["FETCH_SIZE"], cbw["WRITE_SIZE"]]}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def counters(dirs, out):
    vals, kn = {}, None
    for d in dirs:
        kn, v = _last(_per_dispatch(_rows(d)), "k_batch")
        vals.update(v)
    rec = dict(kernel=kn, kernel_source_sha256_16=kernel_source_hash(), per_dispatch=vals)
    w = vals.get("SQ_WAVES")
    if w:
        rec["per_wave"] = {k: v / w for k, v in vals.items() if k != "SQ_WAVES"}
    if "SQ_INSTS_VALU_FLOPS_FP32" in vals:
        # wave-level instruction counts: an FMA is two flops, every lane of
        # the wave counted (64 per instruction)
        rec["executed_fp32_flop_per_dispatch"] = 64.0 * vals["SQ_INSTS_VALU_FLOPS_FP32"]
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def stats(d):
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    with open(files[0]) as f:
        rows = list(csv.DictReader(f))
    print("| kernel | calls | total ns | average ns | % | min ns | max ns |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print("| %s | %s | %s | %.1f | %.2f | %s | %s |" % (
            r["Name"], r["Calls"], r["TotalDurationNs"], float(r["AverageNs"]),
            float(r["Percentage"]), r["MinNs"], r["MaxNs"]))


def _stat_rows(d):
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no kernel_stats.csv under %s" % d)
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def trace(d, out):
    rec = dict(kernel_source_sha256_16=kernel_source_hash())
    for key, name in (("k_batch", "iteration"), ("k_combine", "combine")):
        # the row of the kernel that ran most often (the benchmark's launches)
        rows = [r for r in _stat_rows(d) if key in r["Name"]]
        if not rows:
            raise KeyError(key)
        r = max(rows, key=lambda x: int(x["Calls"]))
        rec[name] = dict(kernel=r["Name"], calls=int(r["Calls"]),
                         average_ns=float(r["AverageNs"]), min_ns=float(r["MinNs"]),
                         max_ns=float(r["MaxNs"]))
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4])
    elif cmd == "counters":
        counters(sys.argv[2:-1], sys.argv[-1])
    elif cmd == "stats":
        stats(sys.argv[2])
    elif cmd == "trace":
        trace(sys.argv[2], sys.argv[3])
    else:
        raise SystemExit(__doc__)
