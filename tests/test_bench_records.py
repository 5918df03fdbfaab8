"""Host logic of bench.py's measurement records: the per-workload source
hashes that invalidate a record when its kernel changes, the MFMA
utilization and shader-clock arithmetic from a rocprofv3 counter file, the
split of the bfloat16 product's dispatches into its two products, and the
traffic scaling by the plain-copy calibration."""
import csv
import json

import pytest

import bench

FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
          "End_Timestamp"]


def _write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, counter, value, t0, t1) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value, "Start_Timestamp": t0, "End_Timestamp": t1})


def test_source_hash_depends_on_the_workload_kernel():
    # the bfloat16 workloads time the bfloat16 product, the others the float one
    assert bench.kernel_source_hash("gemm_nn", "bf16_20000x15000") != bench.kernel_source_hash("gemm_nn", "dense8000")
    assert bench.kernel_source_hash("gemm_nn", "dense8000") == bench.kernel_source_hash("gemm_nn", "paper_dense8000")
    assert bench.kernel_source_hash("spmm", "csr100k") != bench.kernel_source_hash("gemm_nn", "dense8000")


def test_record_mfma_float_products(tmp_path):
    nn = "void rqlp::gemm_kernel<float, 7, false, true, true, 2>(float const*)"
    tn = "void rqlp::gemm_kernel<float, 7, true, true, true, 2>(float const*)"
    rows = []
    # two dispatches each: busy cycles summed over 1024 SIMDs, active cycles
    # summed over 8 XCDs, 250 us per dispatch
    for name, busy, active in ((nn, 4.0e8, 8 * 5.0e5), (tn, 3.0e8, 8 * 5.0e5)):
        for d in range(2):
            t0 = 1_000_000 * (d + 1)
            rows.append((name, "SQ_VALU_MFMA_BUSY_CYCLES", busy, t0, t0 + 250_000))
            rows.append((name, "GRBM_GUI_ACTIVE", active, t0, t0 + 250_000))
            rows.append((name, "SQ_INSTS_VALU_MFMA_MOPS_F32", 1.0e6, t0, t0 + 250_000))
    rows.append(("void rqlp::chol_kernel<8, 14>(double*)", "GRBM_GUI_ACTIVE", 1.0, 0, 1))
    src = tmp_path / "mf.csv"
    _write_csv(src, rows)
    out = tmp_path / "mfma.json"
    bench.record_mfma("dense8000", str(src), path=str(out))
    rec = json.loads(out.read_text())["dense8000"]
    assert set(rec) == {"gemm_nn", "gemm_tn"}
    assert rec["gemm_nn"]["mfma_util"] == pytest.approx(4.0e8 / (5.0e5 * 1024))
    assert rec["gemm_tn"]["mfma_util"] == pytest.approx(3.0e8 / (5.0e5 * 1024))
    # 5e5 active cycles per XCD in 250 us: 2 GHz
    assert rec["gemm_nn"]["clock_ghz"] == pytest.approx(2.0)
    assert rec["gemm_nn"]["mfma_flops"] == pytest.approx(512.0e6)
    assert rec["gemm_nn"]["dispatches"] == 2
    assert rec["gemm_nn"]["source_hash"] == bench.kernel_source_hash("gemm_nn", "dense8000")
    util, clock = bench.load_mfma_record("dense8000", "gemm_tn", path=str(out))
    assert util == pytest.approx(3.0e8 / (5.0e5 * 1024)) and clock == pytest.approx(2.0)
    # a record taken on other sources is not used
    rec["gemm_tn"]["source_hash"] = "0" * 16
    out.write_text(json.dumps({"dense8000": rec}))
    assert bench.load_mfma_record("dense8000", "gemm_tn", path=str(out)) == (None, None)


def test_record_mfma_bf16_dispatches_alternate(tmp_path):
    name = "void rqlp::gemm_bf16_kernel<9>(unsigned short const*)"
    rows = []
    # dispatches alternate A X, A^T X: even ones busier than odd ones
    for d in range(4):
        busy = 6.0e8 if d % 2 == 0 else 2.0e8
        t0 = 1_000_000 * (d + 1)
        rows.append((name, "SQ_VALU_MFMA_BUSY_CYCLES", busy, t0, t0 + 400_000))
        rows.append((name, "GRBM_GUI_ACTIVE", 8 * 8.0e5, t0, t0 + 400_000))
        rows.append((name, "SQ_INSTS_VALU_MFMA_MOPS_BF16", 2.0e6, t0, t0 + 400_000))
    src = tmp_path / "bm.csv"
    _write_csv(src, rows)
    out = tmp_path / "mfma.json"
    bench.record_mfma("bf16_20000x15000", str(src), path=str(out))
    rec = json.loads(out.read_text())["bf16_20000x15000"]
    assert rec["gemm_nn"]["mfma_util"] == pytest.approx(6.0e8 / (8.0e5 * 1024))
    assert rec["gemm_tn"]["mfma_util"] == pytest.approx(2.0e8 / (8.0e5 * 1024))
    assert rec["gemm_nn"]["dispatches"] == 2 and rec["gemm_tn"]["dispatches"] == 2
    assert rec["gemm_nn"]["clock_ghz"] == pytest.approx(2.0)
    assert rec["gemm_nn"]["mfma_mops_counter"] == "SQ_INSTS_VALU_MFMA_MOPS_BF16"
    assert rec["gemm_nn"]["source_hash"] == bench.kernel_source_hash("gemm_nn", "bf16_20000x15000")


def test_record_traffic_scales_by_the_copy(tmp_path):
    nn = "void rqlp::gemm_kernel<float, 7, false, true, true, 2>(float const*)"
    copy = "__amd_rocclr_copyBuffer"
    cal_bytes = float(1 << 30)
    fetch, write, calf, calw = (tmp_path / n for n in ("f.csv", "w.csv", "cf.csv", "cw.csv"))
    # the copy of 1 GiB reads FETCH_SIZE = 0.5 GiB and WRITE_SIZE = 1 GiB (KiB units)
    _write_csv(calf, [(copy, "FETCH_SIZE", (1 << 20) / 2, 0, 1)])
    _write_csv(calw, [(copy, "WRITE_SIZE", float(1 << 20), 0, 1)])
    _write_csv(fetch, [(nn, "FETCH_SIZE", 1000.0, 0, 1), (nn, "FETCH_SIZE", 3000.0, 2, 3)])
    _write_csv(write, [(nn, "WRITE_SIZE", 500.0, 0, 1), (nn, "WRITE_SIZE", 500.0, 2, 3)])
    out = tmp_path / "traffic.json"
    bench.record_traffic("dense8000", str(fetch), str(write), str(calf), str(calw), cal_bytes, path=str(out))
    rec = json.loads(out.read_text())["dense8000"]["gemm_nn"]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert rec["write_bytes"] == pytest.approx(500.0 * 1024)
    assert bench.load_traffic("dense8000", "gemm_nn", path=str(out)) == pytest.approx(2000.0 * 2048 + 500.0 * 1024)


def test_record_alias_shares_the_product_records(tmp_path):
    # the q = 0 form of the 8000^2 workload runs the same products
    out = tmp_path / "mfma.json"
    h = bench.kernel_source_hash("gemm_nn", "dense8000")
    out.write_text(json.dumps({"dense8000": {"gemm_nn": {"mfma_util": 0.5, "clock_ghz": 2.0, "source_hash": h}}}))
    assert bench.load_mfma_record("dense8000_q0", "gemm_nn", path=str(out)) == (0.5, 2.0)
    assert bench.load_mfma_record("csr100k", "gemm_nn", path=str(out)) == (None, None)


def test_committed_records_match_current_sources():
    """The committed records were taken on the kernels as they are now, so
    that the bench line carries them (a kernel change without a new PMC run
    makes this fail)."""
    for workload, kernels in (("dense8000", ("gemm_nn", "gemm_tn")), ("bf16_20000x15000", ("gemm_nn", "gemm_tn"))):
        for k in kernels:
            util, clock = bench.load_mfma_record(workload, k)
            assert util is not None and 0.0 < util < 1.0 and 1.5 < clock < 2.5, (workload, k)
            assert bench.load_traffic(workload, k) is not None, (workload, k)
    assert bench.load_traffic("csr100k", "spmm") is not None
