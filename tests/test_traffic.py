"""Host logic of the HBM-traffic summary: kernel-name parsing and copy calibration."""
import csv

from paper_2405_15573_amd import traffic


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_short_names():
    assert traffic._short("void (anonymous namespace)::k_backward<1>(HIP_vector_type<double, 2u> const*, int)") \
        == "k_backward<1>"
    assert traffic._short("void uhm_detail::(anonymous namespace)::k_coupling(double const*)") == "k_coupling"
    assert traffic._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_summary_scales_by_the_copy(tmp_path):
    gib_kib = float(1 << 20)
    cal = traffic.CALIBRATION_COPIES
    # the counters read each 1 GiB calibration copy as 0.5 GiB fetched and 2 GiB written
    # (scales 2 and 1/2); later, larger copies of the same program must not be taken for it
    fetch = [("__amd_rocclr_copyBuffer", gib_kib / 2)] * cal + [
        ("__amd_rocclr_copyBuffer", 8.0), ("void (anonymous namespace)::k_coupling(int)", 1000.0),
        ("void (anonymous namespace)::k_coupling(int)", 3000.0), ("__amd_rocclr_copyBuffer", 4 * gib_kib)]
    write = [("__amd_rocclr_copyBuffer", 2 * gib_kib)] * cal + [
        ("__amd_rocclr_copyBuffer", 8.0), ("void (anonymous namespace)::k_coupling(int)", 400.0),
        ("void (anonymous namespace)::k_coupling(int)", 400.0), ("__amd_rocclr_copyBuffer", 16 * gib_kib)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    s = traffic.summarize(str(fp), str(wp))
    assert abs(s["copy_fetch_scale"] - 2.0) < 1e-12 and abs(s["copy_write_scale"] - 0.5) < 1e-12
    k = s["kernels"]["k_coupling"]
    assert k["dispatches"] == 2
    assert abs(k["fetch_bytes"] - 2000.0 * 1024 * 2) < 1e-6
    assert abs(k["write_bytes"] - 400.0 * 1024 / 2) < 1e-6
    assert "__amd_rocclr_copyBuffer" not in s["kernels"]


def test_missing_calibration_is_an_error(tmp_path):
    import pytest
    fp = tmp_path / "f.csv"
    _write(fp, "FETCH_SIZE", [("void (anonymous namespace)::k_coupling(int)", 1000.0)])
    with pytest.raises(RuntimeError):
        traffic.summarize(str(fp), str(fp))


def test_match_keeps_only_the_named_kernels(tmp_path):
    gib_kib = float(1 << 20)
    cal = traffic.CALIBRATION_COPIES
    rows = [("__amd_rocclr_copyBuffer", gib_kib)] * cal + [
        ("void (anonymous namespace)::k_coupling(int)", 10.0), ("void (anonymous namespace)::k_aca<8>(int)", 99.0),
        ("void (anonymous namespace)::k_coupling_sym(int)", 20.0)]
    fp = tmp_path / "f.csv"
    _write(fp, "FETCH_SIZE", rows)
    wp = tmp_path / "w.csv"
    _write(wp, "WRITE_SIZE", rows)
    s = traffic.summarize(str(fp), str(wp), match=r"^k_coupling")
    assert sorted(s["kernels"]) == ["k_coupling", "k_coupling_sym"]


def test_totals_sum_bytes_and_time_over_dispatches(tmp_path):
    """Dispatches of different sizes: the rate is summed bytes over summed time, not the
    mean of per-dispatch rates."""
    gib_kib = float(1 << 20)
    cal = traffic.CALIBRATION_COPIES
    k = "void uhm_detail::(anonymous namespace)::k_qr_step<8>(QrStep, int)"
    fetch = [("__amd_rocclr_copyBuffer", gib_kib)] * cal + [(k, 1000.0), (k, 3000.0)]
    write = [("__amd_rocclr_copyBuffer", gib_kib)] * cal + [(k, 500.0), (k, 500.0)]
    fp, wp, tp = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.csv"
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    with open(tp, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerow({"Dispatch_Id": 10, "Kernel_Name": k, "Start_Timestamp": 1000, "End_Timestamp": 3000})
        w.writerow({"Dispatch_Id": 11, "Kernel_Name": k, "Start_Timestamp": 5000, "End_Timestamp": 11000})
    t = traffic.totals(str(fp), str(wp), str(tp))["k_qr_step<8>"]
    assert t["dispatches"] == 2
    assert abs(t["total_bytes"] - 5000.0 * 1024) < 1e-6
    assert abs(t["total_seconds"] - 8000e-9) < 1e-18
    assert abs(t["tb_per_s"] - 5000.0 * 1024 / 8000e-9 / 1e12) < 1e-12
