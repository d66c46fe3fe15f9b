"""Matrix-core utilisation per kernel from one rocprofv3 counter run.

    rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_MFMA_MOPS_BF16 \\
        SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_LDS_BANK_CONFLICT \\
        SQ_LDS_IDX_ACTIVE GRBM_GUI_ACTIVE --output-format csv -d DIR -o run -- <program>
    python -m paper_2405_15573_amd.mfma_util DIR/run_counter_collection.csv [--match REGEX]

The CSV has one row per dispatch and counter.  Per kernel, summed over its dispatches:

* busy: SQ_VALU_MFMA_BUSY_CYCLES over the SIMD-cycles of the dispatches.  GRBM_GUI_ACTIVE
  arrives summed over the chip's 8 XCDs, so the GPU's busy cycles are GRBM_GUI_ACTIVE / 8,
  and the SIMD-cycles are that times 256 CUs x 4 SIMDs;
* rate: 512 flops per SQ_INSTS_VALU_MFMA_MOPS_* unit, over the dispatches' time
  (End_Timestamp - Start_Timestamp), against the dense peak of the dominant type
  (bf16 2500, fp32 157.3, fp64 78.6 TFLOP/s);
* LDS: SQ_LDS_BANK_CONFLICT over SQ_LDS_IDX_ACTIVE.
"""
from __future__ import annotations

import argparse
import csv
import re
from collections import defaultdict

from .traffic import _short

XCDS, CUS, SIMDS = 8, 256, 4
MOPS_FLOPS = 512
PEAK_TFLOPS = {"BF16": 2500.0, "F32": 157.3, "F64": 78.6}
COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F32",
            "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "GRBM_GUI_ACTIVE")


def summarize(path: str, match: str = "") -> dict:
    disp = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            k = _short(r["Kernel_Name"])
            if not k.startswith("k_") or (match and not re.search(match, k)):
                continue
            d = disp.setdefault(int(r["Dispatch_Id"]), {"kernel": k, "t": 1e-9 * (int(r["End_Timestamp"]) -
                                                                                int(r["Start_Timestamp"]))})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    acc = defaultdict(lambda: defaultdict(float))
    for d in disp.values():
        a = acc[d["kernel"]]
        a["dispatches"] += 1
        a["t"] += d["t"]
        for c in COUNTERS:
            a[c] += d.get(c, 0.0)
    out = {}
    for k, a in acc.items():
        simd_cycles = a["GRBM_GUI_ACTIVE"] / XCDS * CUS * SIMDS
        typ = max(PEAK_TFLOPS, key=lambda t: a["SQ_INSTS_VALU_MFMA_MOPS_" + t])
        flops = MOPS_FLOPS * a["SQ_INSTS_VALU_MFMA_MOPS_" + typ]
        tflops = flops / a["t"] / 1e12 if a["t"] > 0 else 0.0
        out[k] = {
            "dispatches": int(a["dispatches"]),
            "mean_us": 1e6 * a["t"] / a["dispatches"],
            "mfma_busy": a["SQ_VALU_MFMA_BUSY_CYCLES"] / simd_cycles if simd_cycles > 0 else 0.0,
            "type": typ if flops > 0 else None,
            "tflops": tflops,
            "frac_of_peak": tflops / PEAK_TFLOPS[typ] if flops > 0 else 0.0,
            "lds_conflict": (a["SQ_LDS_BANK_CONFLICT"] / a["SQ_LDS_IDX_ACTIVE"]
                             if a["SQ_LDS_IDX_ACTIVE"] > 0 else 0.0),
        }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("csv")
    ap.add_argument("--match", default="", help="keep kernels whose short name matches this regex")
    a = ap.parse_args()
    s = summarize(a.csv, a.match)
    print("| kernel | dispatches | mean (us) | MFMA busy | MFMA rate | of dense peak | LDS bank conflicts |")
    print("|---|---|---|---|---|---|---|")
    for k, v in sorted(s.items(), key=lambda kv: -kv[1]["mean_us"] * kv[1]["dispatches"]):
        rate = f"{v['tflops']:.1f} TFLOP/s {v['type']}" if v["type"] else "-"
        print(f"| {k} | {v['dispatches']} | {v['mean_us']:.1f} | {100 * v['mfma_busy']:.1f}% | {rate} | "
              f"{100 * v['frac_of_peak']:.1f}% | {100 * v['lds_conflict']:.1f}% |")


if __name__ == "__main__":
    main()
