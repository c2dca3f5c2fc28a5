"""The rocprofv3 summary tool on small synthetic counter files (CPU only):
the VALU-mix table turns per-dispatch instruction counts into
64 x (add + mul + 2 fma + trans) FLOPs over the dispatch's own duration, and
the LDS table gives bank-conflict cycles per LDS issue cycle."""
import csv

from paper_1307_2265_amd import profsummary as S

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
        "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
        "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
        "Counter_Value", "Start_Timestamp", "End_Timestamp"]
KERNEL = "void ppm::sweep_kernel<ppm::PrecF64, false, false, false, false>(ppm::PatchDev const*)"


def _write(path, counters):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(COLS)
        for disp in (1, 2):   # two dispatches of 1 ms each
            for name, value in counters.items():
                w.writerow([disp, disp, "Agent 1", 1, 1, 1, 262144, 7, KERNEL, 256, 0, 0, 256, 0,
                            32, name, value, 1_000_000 * disp, 1_000_000 * disp + 1_000_000])


def test_valu_mix_and_lds_tables(tmp_path):
    flops, lds = tmp_path / "flops.csv", tmp_path / "lds.csv"
    # per dispatch: 1e6 adds, 2e6 muls, 3e6 fmas, 1e6 trans in FP64, nothing in FP32
    _write(flops, {"SQ_INSTS_VALU_ADD_F64": 1e6, "SQ_INSTS_VALU_MUL_F64": 2e6,
                   "SQ_INSTS_VALU_FMA_F64": 3e6, "SQ_INSTS_VALU_TRANS_F64": 1e6,
                   "SQ_INSTS_VALU_ADD_F32": 0, "SQ_INSTS_VALU_MUL_F32": 0,
                   "SQ_INSTS_VALU_FMA_F32": 0, "SQ_INSTS_VALU_TRANS_F32": 0})
    _write(lds, {"SQ_INSTS_LDS": 4e6, "SQ_ACTIVE_INST_LDS": 8e6, "SQ_LDS_BANK_CONFLICT": 2e6,
                 "SQ_WAVES": 4096})
    out = tmp_path / "x.md"
    S.valu(str(flops), str(lds), "cmd-flops", "cmd-lds", str(out))
    text = out.read_text()
    # 64 x (1 + 2 + 6 + 1) e6 = 640 MFLOP per 1 ms dispatch = 0.64 TFLOP/s
    row = [ln for ln in text.splitlines() if ln.startswith("| `sweep_kernel") and "TFLOP" not in ln]
    assert "| 2 | 1.000 | 1.0 / 2.0 / 3.0 / 1.0 | 0.64 (0.008) |" in row[0], row[0]
    assert "| 2 | 4.00 | 8.00 | 2.000 | 0.250 |" in row[1], row[1]
    assert "cmd-flops" in text and "cmd-lds" in text


def test_traffic_is_calibrated_by_the_largest_copies(tmp_path):
    # a 2 GiB device-to-device copy for which FETCH_SIZE reads half the bytes
    # and WRITE_SIZE all of them; a sweep dispatch reading 4 and writing 3 GB
    cols = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    gib2 = float(1 << 31)

    def write(path, counter, copy_v, sweep_v):
        with open(path, "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(cols)
            for d in (1, 2, 3):
                w.writerow([d, 4096, "__amd_rocclr_copyBuffer", counter, copy_v])
            w.writerow([4, 4096, "__amd_rocclr_copyBuffer", counter, copy_v / 8])  # smaller copy
            w.writerow([5, 262144, KERNEL, counter, sweep_v])
    fetch, wr = tmp_path / "f.csv", tmp_path / "w.csv"
    write(fetch, "FETCH_SIZE", gib2 / 2 / 1024, 2e9 / 1024)
    write(wr, "WRITE_SIZE", gib2 / 1024, 3e9 / 1024)
    out, js = tmp_path / "t.md", tmp_path / "t.json"
    S.traffic(str(fetch), str(wr), 512, 3, "cf", "cw", str(out), str(js))
    import json
    k = json.load(open(js))["kernels"]["sweep_kernel<PrecF64, false, false, false, false>"]
    assert abs(k["fetch_bytes"] - 4e9) < 1e3 and abs(k["write_bytes"] - 3e9) < 1e3
