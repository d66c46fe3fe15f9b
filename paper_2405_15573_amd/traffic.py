"""HBM traffic per kernel launch from two rocprofv3 counter runs.

rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE each write a counter_collection.csv with
one row per dispatch and counter (values in KiB).  Each counter is scaled by what it
reads for a plain device copy of known size (a 1 GiB copy run in the same program), so
that the result is in bytes of the same scale as the algorithmic byte counts.

    python -m paper_2405_15573_amd.traffic FETCH.csv WRITE.csv --n 262144 -o out.json [--match REGEX]
        [--trace KERNEL_TRACE.csv]

--match keeps the kernels whose short name matches the regular expression.  --trace reads
the kernel trace of the FETCH_SIZE run (rocprofv3 --kernel-trace in the same command) and
adds, per kernel, the bytes and the time summed over all its dispatches and their ratio,
for kernels whose dispatches differ in size.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30        # bytes read and written by each calibration copy
CALIBRATION_COPIES = 3      # bench.py --copy-calibration runs this many before anything else


def kernel_source_sha256() -> str:
    h = hashlib.sha256()
    with open(os.path.join(HERE, "csrc", "uhm.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def _short(name: str) -> str:
    """'void (anonymous namespace)::k_backward<1>(double2 const*, ...)' -> 'k_backward<1>'."""
    base = name.replace("(anonymous namespace)::", "").replace("uhm_detail::", "")
    if base.startswith("void "):
        base = base[5:]
    return base.split("(")[0].strip()


def _rows(path: str, counter: str):
    with open(path) as f:
        rows = [r for r in csv.DictReader(f) if r.get("Counter_Name") == counter]
    return sorted(rows, key=lambda r: int(r.get("Dispatch_Id", 0)))


def per_kernel(path: str, counter: str) -> dict:
    vals = defaultdict(list)
    for row in _rows(path, counter):
        vals[_short(row["Kernel_Name"])].append(float(row["Counter_Value"]))
    return vals


def calibration_kib(path: str, counter: str) -> float:
    """Counter reading (KiB) of the calibration copies: the first CALIBRATION_COPIES device
    copies of more than 64 MiB in dispatch order, which the program runs before anything
    else."""
    big = [float(r["Counter_Value"]) for r in _rows(path, counter)
           if "copy" in r["Kernel_Name"].lower() and float(r["Counter_Value"]) > 65536.0]
    if len(big) < CALIBRATION_COPIES:
        raise RuntimeError("calibration copies not found")
    return sum(big[:CALIBRATION_COPIES]) / CALIBRATION_COPIES


def summarize(fetch_csv: str, write_csv: str, match: str = "") -> dict:
    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    sf = COPY_BYTES / (calibration_kib(fetch_csv, "FETCH_SIZE") * 1024.0)
    sw = COPY_BYTES / (calibration_kib(write_csv, "WRITE_SIZE") * 1024.0)
    out = {}
    for k in set(fetch) | set(write):
        if not k.startswith("k_") or (match and not re.search(match, k)):
            continue
        f = sum(fetch.get(k, [0.0])) / max(1, len(fetch.get(k, [])))
        w = sum(write.get(k, [0.0])) / max(1, len(write.get(k, [])))
        out[k] = {"fetch_bytes": f * 1024.0 * sf, "write_bytes": w * 1024.0 * sw,
                  "bytes": f * 1024.0 * sf + w * 1024.0 * sw, "dispatches": len(fetch.get(k, []))}
    return {"copy_fetch_scale": sf, "copy_write_scale": sw, "kernels": out}


def durations(trace_csv: str) -> dict:
    """Kernel durations (s) from a rocprofv3 kernel-trace CSV, by short name."""
    out = defaultdict(list)
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            out[_short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    return out


def totals(fetch_csv: str, write_csv: str, trace_csv: str, match: str = "") -> dict:
    """Per kernel: bytes (copy-calibrated FETCH_SIZE + WRITE_SIZE) and time summed over its
    dispatches, and their ratio in TB/s."""
    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    dur = durations(trace_csv)
    sf = COPY_BYTES / (calibration_kib(fetch_csv, "FETCH_SIZE") * 1024.0)
    sw = COPY_BYTES / (calibration_kib(write_csv, "WRITE_SIZE") * 1024.0)
    out = {}
    for k in set(fetch) | set(write):
        if not k.startswith("k_") or (match and not re.search(match, k)):
            continue
        b = sum(fetch.get(k, [])) * 1024.0 * sf + sum(write.get(k, [])) * 1024.0 * sw
        t = sum(dur.get(k, []))
        out[k] = {"total_bytes": b, "total_seconds": t, "dispatches": len(dur.get(k, [])),
                  "tb_per_s": b / t / 1e12 if t > 0 else None}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("-o", "--out", required=True)
    ap.add_argument("--match", default="", help="keep kernels whose short name matches this regex")
    ap.add_argument("--trace", default="", help="kernel trace of the FETCH_SIZE run: adds summed bytes, time, TB/s")
    a = ap.parse_args()
    s = summarize(a.fetch_csv, a.write_csv, a.match)
    if a.trace:
        s["totals"] = totals(a.fetch_csv, a.write_csv, a.trace, a.match)
        print(json.dumps(s["totals"]))
    s["n"] = a.n
    s["source_sha256"] = kernel_source_sha256()
    s["bytes_per_launch"] = {k: v["bytes"] for k, v in s["kernels"].items()}
    with open(a.out, "w") as f:
        json.dump(s, f, indent=1)
    print(json.dumps(s["bytes_per_launch"]))


if __name__ == "__main__":
    main()
