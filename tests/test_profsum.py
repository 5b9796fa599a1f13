"""The rocprofv3 summary tool on small synthetic counter files (CPU only)."""
import csv
import json

from paper_2410_21888_amd import profsum

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size", "Kernel_Id",
        "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
        "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
INTS = "void rimp2::gemm_f64_kernel<128, 128, 16, false, 0, true, false>(rimp2::GemmParams)"
GAMMA = "void rimp2::gemm_f64_kernel<128, 128, 16, true, 1, true, false>(rimp2::GemmParams)"


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for i, (name, value) in enumerate(rows):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 256, 1, name, 256, 0, 0, 64, 0, 32, counter, value, 0, 1])


def test_roles_of_kernel_symbols():
    assert profsum.role_of(INTS) == "ints_gemm"
    assert profsum.role_of(GAMMA) == "gamma_gemm"
    assert profsum.role_of(GAMMA.replace("true, 1", "false, 1")) == "gamma_metric"
    # the instantiation with the two-chunks-ahead loader carries one more argument
    assert profsum.role_of(INTS.replace("true, false>", "true, false, true>")) == "ints_gemm"
    assert profsum.role_of("void rimp2::gemm_f64_grouped<64, 64, 16, false, 3, true, true>(rimp2::GemmGroup)") == "pij_gemm"
    assert profsum.role_of("rimp2::amplitude_kernel(double*, ...)") == "amplitude"
    assert profsum.role_of("__amd_rocclr_copyBuffer") == "(runtime copy)"
    assert profsum.role_of("void rimp2::gemm_oz8_kernel<7, 1>(rimp2::OzParams)") == "oz8 S=7"
    assert profsum.role_of("void rimp2::gemm_oz8_grouped<5, 2>(rimp2::OzGroup, long, long)") == "oz8 S=5 (grouped)"
    assert profsum.role_of("void (anonymous namespace)::digit_split_grouped<5, 0>(DigitOp const*)") == "digit_split"


def test_traffic_scales_by_the_calibration_copy(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    # the 1 GiB copy: FETCH_SIZE counts half of the bytes it moved, WRITE_SIZE all of them
    write_counters(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 524288.0), (INTS, 1000.0), (INTS, 3000.0),
                                     (GAMMA, 10.0)])
    write_counters(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1048576.0), (INTS, 100.0), (INTS, 300.0),
                                     (GAMMA, 1.0)])
    roles, cal = profsum.traffic(str(f), str(w))
    assert abs(cal["fetch_scale"] - 2.0) < 1e-12 and abs(cal["write_scale"] - 1.0) < 1e-12
    assert roles["ints_gemm"]["launches"] == 2
    assert abs(roles["ints_gemm"]["bytes_per_launch"] - (2000.0 * 2 + 200.0) * 1024) < 1e-6
    assert abs(roles["gamma_gemm"]["bytes_per_launch"] - (10.0 * 2 + 1.0) * 1024) < 1e-6
    out = tmp_path / "t.json"
    assert profsum.main(["traffic", str(f), str(w), "--workload", "w", "--json", str(out)]) == 0
    with open(out) as fh:
        d = json.load(fh)
    assert d["w"]["ints_gemm"]["source_hash"] == profsum.kernel_source_hash()


def test_traffic_splits_two_runs_into_two_workloads(tmp_path):
    """One process runs the same kernels twice (two paths): --first keeps the
    first launches under the role's name, and --later-workload files the rest
    under a second workload."""
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    write_counters(f, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 524288.0), (GAMMA, 10.0), (GAMMA, 10.0),
                                     (GAMMA, 40.0), (INTS, 5.0)])
    write_counters(w, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 1048576.0), (GAMMA, 1.0), (GAMMA, 1.0),
                                     (GAMMA, 4.0), (INTS, 1.0)])
    out = tmp_path / "t.json"
    assert profsum.main(["traffic", str(f), str(w), "--workload", "a", "--first", "gamma_gemm=2",
                         "--first", "ints_gemm=0", "--later-workload", "b", "--json", str(out)]) == 0
    with open(out) as fh:
        d = json.load(fh)
    assert set(d["a"]) == {"gamma_gemm"} and set(d["b"]) == {"gamma_gemm", "ints_gemm"}
    assert d["a"]["gamma_gemm"]["launches"] == 2 and d["b"]["gamma_gemm"]["launches"] == 1
    assert abs(d["a"]["gamma_gemm"]["bytes_per_launch"] - (10.0 * 2 + 1.0) * 1024) < 1e-6
    assert abs(d["b"]["gamma_gemm"]["bytes_per_launch"] - (40.0 * 2 + 4.0) * 1024) < 1e-6


def test_mfma_occupancy_and_clock(tmp_path):
    c = tmp_path / "m_counter_collection.csv"
    a = tmp_path / "m_agent_info.csv"
    with open(a, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Node_Id", "Simd_Count", "Num_Xcc"])
        w.writerow([0, 0, 0])          # the CPU agent
        w.writerow([1, 1024, 8])
    with open(c, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        # 1 ms at 2.4 GHz on 8 XCCs, matrix units busy 90% of 1024 SIMDs' cycles
        for i, (cn, v) in enumerate((("GRBM_GUI_ACTIVE", 8 * 2.4e6), ("SQ_VALU_MFMA_BUSY_CYCLES", 0.9 * 2.4e6 * 1024))):
            w.writerow([7, 7, "Agent 1", 1, 1, 1, 256, 1, INTS, 256, 0, 0, 64, 0, 32, cn, v, 1000000, 2000000])
    r = profsum.mfma(str(c))
    e = r["ints_gemm"]
    assert e["launches"] == 1
    assert abs(e["avg_ms"] - 1.0) < 1e-12
    assert abs(e["clock_ghz"] - 2.4) < 1e-9
    assert abs(e["mfma_busy"] - 0.9) < 1e-12
    # with first={role: 0} the launch is filed as "(later)"
    r2 = profsum.mfma(str(c), first={"ints_gemm": 0})
    assert set(r2) == {"ints_gemm (later)"} and abs(r2["ints_gemm (later)"]["mfma_busy"] - 0.9) < 1e-12


def test_source_hash_ignores_comments_and_spacing():
    a = {fn: "int f(int x) {\n  return x + 1;  // one\n}\nconst char* s = \"// kept\";\n" for fn in profsum.FRAGMENT_SOURCES}
    b = {fn: "/* header */\nint f(int x) {\n\n    return x + 1;\n}\nconst char* s = \"// kept\";\n" for fn in profsum.FRAGMENT_SOURCES}
    c = dict(a)
    c[profsum.FRAGMENT_SOURCES[0]] = a[profsum.FRAGMENT_SOURCES[0]].replace("x + 1", "x + 2")
    d = dict(a)
    d[profsum.FRAGMENT_SOURCES[0]] = a[profsum.FRAGMENT_SOURCES[0]].replace('"// kept"', '"// kepT"')
    h = profsum.sources_hash
    assert h(a.get) == h(b.get)
    assert h(a.get) != h(c.get)          # code changes the hash
    assert h(a.get) != h(d.get)          # so does a string literal that looks like a comment
