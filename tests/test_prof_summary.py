"""The profile summariser behind the committed traffic records and pass times,
on small hand-written rocprofv3-style CSV files: marker segmentation, the
dropped warm dispatch, counter calibration against the marker copy, and the
shortened kernel names."""
import csv
import json
import os

import pytest

from paper_2406_18356_amd import prof_summary as ps

COPY = "__amd_rocclr_copyBuffer"
COPY_GRID = 131072


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _trace(tmp_path):
    # an untimed setup dispatch, then two marked passes: copy, warm dispatch, timed dispatches
    rows, t = [], 0

    def add(name, dur, grid):
        nonlocal t
        rows.append({"Kernel_Name": name, "Grid_Size": grid, "Start_Timestamp": t, "End_Timestamp": t + dur})
        t += dur + 10

    add("void msr::setup<float>(int)", 500, 64)
    add(COPY, 100, COPY_GRID)
    add("void msr::row_kernel<float, 64, EpiResid<float> >(msr::RowArgs<float>, int)", 9000, 512)  # warm
    for d in (1000, 2000, 3000):
        add("void msr::row_kernel<float, 64, EpiResid<float> >(msr::RowArgs<float>, int)", d, 512)
    add(COPY, 100, COPY_GRID)
    add("void msr::col_kernel<float, 64, ModePsf<float> >(msr::ColArgs<float>, int)", 7000, 256)  # warm
    for d in (4000, 6000):
        add("void msr::col_kernel<float, 64, ModePsf<float> >(msr::ColArgs<float>, int)", d, 256)
    _write(tmp_path / "p_kernel_trace.csv", ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"], rows)


def test_passes_take_the_timed_dispatches_of_each_segment(tmp_path):
    _trace(tmp_path)
    out = tmp_path / "passes.txt"
    ps.passes(str(tmp_path), "p", str(out), "cmd", [("resid", "EpiResid", "-2"), ("psf", "ModePsf", "-1")])
    lines = out.read_text().splitlines()
    resid = next(ln for ln in lines if ln.startswith("resid")).split()
    psf = next(ln for ln in lines if ln.startswith("psf")).split()
    assert resid[1:5] == ["3", "2.00", "1.00", "3.00"]  # the 9 us warm dispatch is dropped
    assert psf[1:5] == ["2", "5.00", "4.00", "6.00"]


def _counters(tmp_path, prefix, counter, copy_kib, kernel_kib):
    rows, d = [], 0

    def add(name, grid, v):
        nonlocal d
        d += 1
        rows.append({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                     "Counter_Value": v})

    add(COPY, COPY_GRID, copy_kib)
    add("row_kernel<EpiResid>", 512, 99999.0)  # warm
    for v in kernel_kib:
        add("row_kernel<EpiResid>", 512, v)
    _write(tmp_path / f"{prefix}_counter_collection.csv",
           ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], rows)


def test_traffic_is_scaled_by_what_the_counters_read_for_the_copy(tmp_path):
    copy_bytes = 64.0 * 1024 * 1024
    # the fetch counter reads half the copy's bytes (scale 2), the write counter all of them (scale 1)
    _counters(tmp_path, "f", "FETCH_SIZE", copy_bytes / 1024 / 2, [1000.0, 3000.0])
    _counters(tmp_path, "w", "WRITE_SIZE", copy_bytes / 1024, [500.0, 500.0])
    out = tmp_path / "t.json"
    rec = ps.traffic(str(tmp_path), "f", "w", str(out), "EpiResid", 12345.0, copy_bytes, "cmd", -1)
    assert rec["fetch_scale"] == pytest.approx(2.0)
    assert rec["write_scale"] == pytest.approx(1.0)
    assert rec["dispatches"] == 2
    assert rec["fetch_bytes"] == pytest.approx(2000.0 * 2.0 * 1024)
    assert rec["write_bytes"] == pytest.approx(500.0 * 1024)
    assert rec["traffic_bytes"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["source_sha256"] == ps.kernel_source_hash()
    assert json.loads(out.read_text())["algorithmic_bytes"] == 12345.0


def test_short_names():
    assert ps._short("_ZN12_GLOBAL__N_114conv3x3_kernelIDF16bLb0EEEvNS_6ConvInIT_EENS_7ConvOutE") == \
        "conv3x3_kernel<bf16, false>"
    assert ps._short("_ZN12_GLOBAL__N_114conv3x3_kernelIfLb1EEEvNS_6ConvInIT_EENS_7ConvOutE") == \
        "conv3x3_kernel<float, true>"
    assert ps._short("(anonymous namespace)::pool_kernel(bool _Accum const*, int)") == "pool_kernel"
    assert ps._short("void msr::row_kernel<float, 8, msr::EpiLoad<float> >(msr::RowArgs<float>, int)") == \
        "row_kernel<float, 8, msr::EpiLoad<float> >"


def test_a_run_without_marker_copies_is_refused(tmp_path):
    _write(tmp_path / "p_kernel_trace.csv", ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"],
           [{"Kernel_Name": "k", "Grid_Size": 1, "Start_Timestamp": 0, "End_Timestamp": 1}])
    with pytest.raises(SystemExit):
        ps.passes(str(tmp_path), "p", str(tmp_path / "o.txt"), "cmd", [("k", "k", "0")])
    assert not os.path.exists(tmp_path / "o.txt")


def test_mfma_use_per_group(tmp_path):
    """Busy cycles over SIMD cycles (GRBM_GUI_ACTIVE summed over the 8 XCDs)
    and counted flops (512 per MOP) over GPU-active time; the first dispatch
    of each group is dropped as the warm launch."""
    rows, d = [], 0
    # per dispatch: GRBM = 8 x 2.4e6 cycles (1 ms), 1.6e6 MFMA instructions of 32 busy cycles
    for name in ["conv3x3_kernelIDF16bLb0E"] * 3 + ["conv3x3_wgrad_kernelIDF16b"] * 2:
        for cname, v in (("GRBM_GUI_ACTIVE", 8 * 2.4e6), ("SQ_INSTS_VALU_MFMA_BF16", 1.6e6),
                         ("SQ_INSTS_VALU_MFMA_MOPS_BF16", 64 * 1.6e6), ("SQ_VALU_MFMA_BUSY_CYCLES", 32 * 1.6e6)):
            rows.append({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": 256, "Counter_Name": cname,
                         "Counter_Value": v})
        d += 1
    _write(tmp_path / "m_counter_collection.csv",
           ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], rows)
    out = tmp_path / "mfma.txt"
    ps.mfma(str(tmp_path), "m", str(out), "cmd", [("fwd", "conv3x3_kernelIDF16b"), ("wgrad", "wgrad_kernel")])
    fwd = next(ln for ln in out.read_text().splitlines() if ln.startswith("fwd")).split()
    assert fwd[1] == "2"                                   # two timed dispatches
    assert float(fwd[3]) == pytest.approx(2 * 1.6e6 * 32768 / 1e12, abs=5e-4)  # TFLOP, printed to 3 places
    assert float(fwd[4]) == pytest.approx(2.0, rel=1e-3)   # active ms
    busy = 2 * 32 * 1.6e6 / (1024 * 2 * 2.4e6)
    assert float(fwd[5]) == pytest.approx(busy, abs=1e-3)
    assert float(fwd[7]) == pytest.approx(2 * 1.6e6 * 32768 / 2e-3 / 1e12 / 2500, abs=1e-3)
