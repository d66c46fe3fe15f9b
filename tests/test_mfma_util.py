"""Host logic of the matrix-core utilisation summary (synthetic counter rows, no GPU)."""
import csv

import pytest

from paper_2405_15573_amd import mfma_util


def _write(path, dispatches):
    """dispatches: list of (kernel name, duration ns, {counter: value})."""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 1000
        for i, (name, dur, cnt) in enumerate(dispatches):
            for c, v in cnt.items():
                w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v,
                            "Start_Timestamp": t, "End_Timestamp": t + dur})
            t += dur + 10


def test_busy_rate_and_conflicts(tmp_path):
    # 1 ms at 2 GHz on every XCD: GRBM reads 8 x 2e6; half the SIMD-cycles busy; 50 TFLOP/s fp32
    cycles = 2.0e6
    simd_cycles = cycles * 256 * 4
    cnt = {"GRBM_GUI_ACTIVE": 8 * cycles, "SQ_VALU_MFMA_BUSY_CYCLES": 0.5 * simd_cycles,
           "SQ_INSTS_VALU_MFMA_MOPS_F32": 50e12 * 1e-3 / 512, "SQ_INSTS_VALU_MFMA_MOPS_BF16": 0.0,
           "SQ_INSTS_VALU_MFMA_MOPS_F64": 0.0, "SQ_LDS_BANK_CONFLICT": 25.0, "SQ_LDS_IDX_ACTIVE": 100.0}
    p = tmp_path / "c.csv"
    _write(p, [("void (anonymous namespace)::k_lp_coupling<1, 4>(int)", 1_000_000, cnt)] * 2 +
           [("void at::native::other_kernel(int)", 5, {"GRBM_GUI_ACTIVE": 1.0})])
    s = mfma_util.summarize(str(p))
    assert list(s) == ["k_lp_coupling<1, 4>"]
    k = s["k_lp_coupling<1, 4>"]
    assert k["dispatches"] == 2 and k["type"] == "F32"
    assert k["mfma_busy"] == pytest.approx(0.5)
    assert k["tflops"] == pytest.approx(50.0)
    assert k["frac_of_peak"] == pytest.approx(50.0 / 157.3)
    assert k["lds_conflict"] == pytest.approx(0.25)
    assert mfma_util.summarize(str(p), match="^k_lp_forward") == {}
