"""Host-side logic with no GPU: the 48-instance workload recipe and the
arithmetic that turns rocprofv3 counter files into HBM bytes and MFMA
figures."""
import csv
import json
import os

import numpy as np


def test_batch_instances_follow_the_recipe():
    import bench
    insts = bench.batch_instances()
    assert len(insts) == 48
    for i, w in enumerate(insts):
        assert 10 <= w["n"] <= 24 and w["N"] == w["n"] and w["two_s"] == w["n"] % 2
        assert w["D"] in (64, 128, 256, 512)
        assert w["seed"] == 1000 + i and w["k"] == w["n"] // 2 - 1
        g = w["g"]
        # density-fitting integrals: 8-fold symmetric, (pp|pp) > 0
        assert np.allclose(g, g.transpose(1, 0, 2, 3)) and np.allclose(g, g.transpose(2, 3, 0, 1))
        assert (np.einsum("pppp->p", g) > 0).all()
        assert np.allclose(w["h"], w["h"].T)
    # seeded: the same list every time
    again = bench.batch_instances()
    assert all(a["n"] == b["n"] and a["D"] == b["D"] and np.array_equal(a["h"], b["h"]) for a, b in zip(insts, again))


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_scales_counters_by_the_copy_and_sums_the_last_launches(tmp_path):
    import rocprof_summary as rs
    # a 2 MiB copy that the fetch counter reports as half (in KiB), and
    # three GEMM launches of which the last two form the H*psi
    copy_kib = 2 * 1024.0
    fetch = [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Value": copy_kib / 2},
             {"Dispatch_Id": 2, "Kernel_Name": "void gemm_bf16_padded<2, 64, 64>(...)", "Counter_Value": 999.0},
             {"Dispatch_Id": 3, "Kernel_Name": "void gemm_bf16_padded<2, 64, 64>(...)", "Counter_Value": 100.0},
             {"Dispatch_Id": 4, "Kernel_Name": "void gemm_bf16_wave<1>(...)", "Counter_Value": 50.0}]
    write = [{"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Value": copy_kib},
             {"Dispatch_Id": 2, "Kernel_Name": "void gemm_bf16_padded<2, 64, 64>(...)", "Counter_Value": 7.0},
             {"Dispatch_Id": 3, "Kernel_Name": "void gemm_bf16_padded<2, 64, 64>(...)", "Counter_Value": 10.0},
             {"Dispatch_Id": 4, "Kernel_Name": "void gemm_bf16_wave<1>(...)", "Counter_Value": 20.0}]
    _write_counters(tmp_path / "f", fetch)
    _write_counters(tmp_path / "w", write)
    out = tmp_path / "t.json"
    assert rs.main(["traffic", str(tmp_path / "f"), str(tmp_path / "w"), "2", "2", str(out)]) == 0
    t = json.loads(out.read_text())
    assert abs(t["fetch"]["scale"] - 2.0) < 1e-12 and abs(t["write"]["scale"] - 1.0) < 1e-12
    assert abs(t["fetch"]["hbm_bytes_last_hpsi"] - 2.0 * 150.0 * 1024) < 1e-6
    assert abs(t["write"]["hbm_bytes_last_hpsi"] - 30.0 * 1024) < 1e-6
    assert abs(t["hbm_bytes_per_hpsi"] - (300.0 + 30.0) * 1024) < 1e-6
    assert t["source_sha256"] == rs.source_sha256() and t["launches"] == 2


def test_bench_reports_traffic_only_for_the_kernel_source_it_was_taken_on():
    # roofline.traffic comes from the committed counter file while its hash
    # matches the executor source, and is null otherwise
    import bench
    from rocprof_summary import source_sha256
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    total, detail = bench.measured_traffic("cas82_d4096")
    if t["source_sha256"] == source_sha256():
        assert total == t["hbm_bytes_per_hpsi"] and detail["launches"] == t["launches"]
    else:
        assert total is None and detail is None
    assert bench.measured_traffic("cas32_d1024") == (None, None)


def test_mfma_counters_give_executed_flops_and_busy_fraction(tmp_path):
    # several counters per dispatch; the last two BF16 GEMM dispatches form
    # the H*psi.  One BF16 MFMA MOP is 512 flops; GRBM_GUI_ACTIVE is summed
    # over the 8 XCDs and the busy cycles over the 1024 SIMDs.
    import rocprof_summary as rs
    rows = []
    for di, name, mops, busy, grbm in ((1, "void gemm_bf16_pipe<2, 64, 64, 3>(...)", 5.0, 7.0, 8.0),
                                       (2, "void gemm_bf16_pipe<2, 64, 64, 3>(...)", 100.0, 1024.0, 64.0),
                                       (3, "void gemm_bf16_padded<1, 64, 64, false, false>(...)", 300.0, 3072.0, 64.0),
                                       (4, "void reduce_kernel<1>(...)", 1e6, 1e6, 1e6)):
        for cname, v in (("SQ_INSTS_VALU_MFMA_MOPS_BF16", mops), ("SQ_VALU_MFMA_BUSY_CYCLES", busy),
                         ("GRBM_GUI_ACTIVE", grbm)):
            rows.append({"Dispatch_Id": di, "Kernel_Name": name, "Counter_Name": cname, "Counter_Value": v})
    os.makedirs(tmp_path / "m", exist_ok=True)
    with open(tmp_path / "m" / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)
    out = tmp_path / "m.json"
    assert rs.main(["counters", str(tmp_path / "m"), "2", str(out), "102400"]) == 0
    m = json.loads(out.read_text())
    assert m["launches"] == 2 and m["counters"]["SQ_INSTS_VALU_MFMA_MOPS_BF16"] == 400.0
    assert m["mfma_flops_executed"] == 400.0 * 512 and abs(m["executed_over_algorithmic"] - 2.0) < 1e-12
    # 4096 busy SIMD cycles over 128 / 8 = 16 active cycles x 1024 SIMDs
    assert abs(m["mfma_busy_fraction"] - 4096.0 / (16.0 * 1024.0)) < 1e-12
    assert m["source_sha256"] == rs.source_sha256()


def test_bench_reports_mfma_counters_only_for_the_kernel_source_they_were_taken_on():
    import bench
    from rocprof_summary import source_sha256
    with open(bench.MFMA_FILE) as f:
        m = json.load(f)
    got = bench.measured_mfma("cas82_d4096")
    if m["source_sha256"] == source_sha256():
        assert got["busy_fraction"] == m["mfma_busy_fraction"] and got["launches"] == m["launches"]
    else:
        assert got is None
    assert bench.measured_mfma("cas32_d1024") is None


def test_e4m3_reference_quantizer_matches_the_format():
    """The numpy E4M3 quantizer the FP8 GPU tests compare against: 127 finite
    non-negative values, largest 448, smallest subnormal 2^-9, and round to
    nearest with ties to the even code (facts of the OCP 8-bit float format)."""
    from tests.test_gpu_kernel import _e4m3_values, _quantize_e4m3
    v = _e4m3_values()
    assert len(v) == 127 and v[0] == 0.0 and v[1] == 2.0 ** -9 and v[-1] == 448.0
    assert v[8] == 2.0 ** -6  # first normal: exponent field 1, mantissa 0
    x = np.array([1.0625, 1.1875, -1.0625, 2.0 ** -10, 3 * 2.0 ** -10, 500.0, -1e9, 0.3])
    # 1.0625 lies halfway between 1 (code 0x38, even) and 1.125 (0x39): 1;
    # 1.1875 between 1.125 (0x39) and 1.25 (0x3a, even): 1.25; half the
    # smallest subnormal ties to 0 (even); 1.5 * 2^-9 ties to 2^-8 (code 2);
    # beyond 448 saturates; 0.3 rounds to 0.3125 (nearest: 0.28125 / 0.3125)
    want = np.array([1.0, 1.25, -1.0, 0.0, 2.0 ** -8, 448.0, -448.0, 0.3125])
    assert np.array_equal(_quantize_e4m3(x), want)
