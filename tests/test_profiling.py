"""Host logic of the rocprofv3 summaries (synthetic CSV files, no GPU)."""

import csv
import os

from paper_1805_04791_amd import profiling as pf

TRACE_COLS = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
              "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
              "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z",
              "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
PMC_COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
ZK = "void vie::k_zpass<float, 16, 16, 3, 0>(vie::cx<float>*, vie::cx<float> const*, vie::ZArgs, vie::cx<float> const*)"
CK = "void at::native::vectorized_elementwise_kernel<4, at::native::MulFunctor<float> >(int, float*)"


def write_csv(path, cols, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow({c: r.get(c, 0) for c in cols})


def test_short_name_strips_namespace_and_arguments():
    assert pf.short_name(ZK) == "k_zpass<float, 16, 16, 3, 0>"
    assert pf.short_name("void vie::(anonymous namespace)::k_dots(vie::cx<double> const*, long)") == "k_dots"


def test_stats_groups_dispatches_by_launch_shape(tmp_path):
    d = tmp_path / "kt"
    os.makedirs(d)
    write_csv(d / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                                           "MaxNs", "StdDev"], [{"Name": ZK, "Calls": 6, "TotalDurationNs": 7000,
                                                                 "AverageNs": 1166.7, "Percentage": 100}])
    rows = []
    for i, (dur, wg) in enumerate([(1000, 256)] * 5 + [(2000, 64)]):
        rows.append({"Kernel_Name": ZK, "Start_Timestamp": 10 * i, "End_Timestamp": 10 * i + dur,
                     "Workgroup_Size_X": wg, "Workgroup_Size_Y": 1, "Workgroup_Size_Z": 1,
                     "Grid_Size_X": 4096, "Grid_Size_Y": 1, "Grid_Size_Z": 1})
    write_csv(d / "run_kernel_trace.csv", TRACE_COLS, rows)
    text = pf.stats_summary(str(d), "python3 bench.py")
    assert "| `k_zpass<float, 16, 16, 3, 0>` | 4096 | 256 | 5 | 1.0 | 1.0 |" in text
    assert "| 4096 | 64 |" not in text            # fewer than 4 dispatches
    assert "python3 bench.py" in text


def test_traffic_scales_counters_by_the_copy_kernel(tmp_path):
    f, w = tmp_path / "f", tmp_path / "w"
    os.makedirs(f)
    os.makedirs(w)
    copy = float(2 ** 30)
    # the copy kernel reports half its bytes on FETCH and all on WRITE
    frows = [{"Kernel_Name": CK, "Grid_Size": 1 << 20, "Workgroup_Size": 128, "Counter_Name": "FETCH_SIZE",
              "Counter_Value": copy / 2 / 1024}] * 3
    frows += [{"Kernel_Name": ZK, "Grid_Size": 8 << 20, "Workgroup_Size": 256, "Counter_Name": "FETCH_SIZE",
               "Counter_Value": 1000.0}] * 4
    wrows = [{"Kernel_Name": CK, "Grid_Size": 1 << 20, "Workgroup_Size": 128, "Counter_Name": "WRITE_SIZE",
              "Counter_Value": copy / 1024}] * 3
    wrows += [{"Kernel_Name": ZK, "Grid_Size": 8 << 20, "Workgroup_Size": 256, "Counter_Name": "WRITE_SIZE",
               "Counter_Value": 500.0}] * 4
    write_csv(f / "run_counter_collection.csv", PMC_COLS, frows)
    write_csv(w / "run_counter_collection.csv", PMC_COLS, wrows)
    text = pf.traffic_summary(str(f), str(w), r"k_zpass<float", "cmd", "MulFunctor", copy, algorithmic=3072000)
    out = tmp_path / "t.md"
    out.write_text(text)
    traffic, kernel, digest = pf.read_traffic(str(out))
    assert traffic == 2 * 1000 * 1024 + 500 * 1024
    assert kernel == "k_zpass<float, 16, 16, 3, 0>"
    assert digest == pf.source_digest()
    assert pf.read_traffic(str(tmp_path / "missing.md")) is None
