"""Host-side pieces of bench.py: the algorithmic flop counts behind the
reported rates (against the counts the scope table gives for the measured
workloads) and the conversion of two counter runs into per-launch HBM bytes
(synthetic counter files: a 1 GiB calibration copy and the K-build kernels)."""
import csv
import json
import os

import bench


def test_algorithmic_flop_counts():
    # F_alg = 6 Ng^2 Npair + 8 Ng Npair^2 + (18 n + 10) Ng Npair
    assert bench.f_alg(128, 16, 150000) == 1196722886400000          # 1.197e15 at N=128, Ng=150 000
    assert abs(bench.f_alg(8, 2, 2000) - 8.9e8) / 8.9e8 < 0.01
    assert abs(bench.f_alg(64, 8, 50000) - 3.30e13) / 3.30e13 < 0.01
    # K build of one chunk: 6 rows Ng Npair
    assert bench.f_kbuild(128, 7500, 150000) == 6 * 7500 * 150000 * 8256
    # adjoint: 12 Ng^2 Npair + 14 Ng Npair^2 (about 5.9e14 at N=96, Ng=100 000)
    assert abs(bench.f_backward(96, 100000) - 5.9e14) / 5.9e14 < 0.01
    # open shell: the two-body terms once per spin channel
    P = 128 * 129 // 2
    assert bench.f_alg(128, 16, 150000, 2) - bench.f_alg(128, 16, 150000) == 8 * 150000 * P * P + 298 * 150000 * P
    assert bench.f_backward(96, 100000, 2) - bench.f_backward(96, 100000) == 14 * 100000 * 4656 ** 2


def _counter_csv(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for did, name, value in rows:
            # two device instances per dispatch, summed by the reader
            w.writerow([did, name, counter, value / 2])
            w.writerow([did, name, counter, value / 2])


def test_traffic_from_counter_runs(tmp_path):
    kib = 1024.0
    # the copy moves 2^30 bytes: FETCH_SIZE reads half of that (factor 2), WRITE_SIZE all of it
    fetch = [(1, "__amd_rocclr_copyBuffer", 2 ** 29 / kib),
             (2, "void xtc::k_build_K_lp<0, 3, 3>(double const*, ...)", 10e9 / kib),
             (3, "xtc::k_reduce_K(float const*, int)", 3e9 / kib),
             (4, "xtc::k_unrelated(int)", 7e9 / kib)]
    write = [(1, "__amd_rocclr_copyBuffer", 2 ** 30 / kib),
             (2, "void xtc::k_build_K_lp<0, 3, 3>(double const*, ...)", 1e9 / kib),
             (3, "xtc::k_reduce_K(float const*, int)", 0.5e9 / kib)]
    _counter_csv(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _counter_csv(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = str(tmp_path / "traffic.json")
    bench.traffic_from(str(tmp_path / "f"), str(tmp_path / "w"), "W", "bf16x3", 7500, path=out)
    rec = json.load(open(out))["W/bf16x3/7500"]
    assert abs(rec["fetch_factor"] - 2.0) < 1e-12 and abs(rec["write_factor"] - 1.0) < 1e-12
    per = rec["per_kernel_bytes"]
    assert set(per) == {"k_build_K_lp", "k_reduce_K"}                # unrelated kernels are not counted
    assert abs(per["k_build_K_lp"]["fetch"] - 20e9) < 1 and abs(per["k_reduce_K"]["write"] - 0.5e9) < 1
    assert abs(rec["bytes_per_launch"] - (20e9 + 6e9 + 1e9 + 0.5e9)) < 4
    assert rec["sources"] == bench.kernel_sources_hash()


def test_host_info_and_cpu_baseline_fields():
    info = bench.host_info()
    assert info["cores"] >= 1 and isinstance(info["cpu_model"], (str, type(None)))
    cb = bench.cpu_baseline("N128-occ16-Ng150k", 600)
    assert cb["kind"] == "oracle" and cb["cores"] == info["cores"] and cb["value"] > 0
    assert "24 of 128" in cb["sample"] and cb["full_workload_seconds_extrapolated"] > cb["seconds"]
    assert 0.5 < cb["k_build_share_of_sample_flops"] < 1.0


def test_kernel_rooflines_from_per_step_totals():
    """Per-kernel rates use the kernel's algorithmic flops per step over its
    summed device time, whatever the number of launches."""
    P = 128 * 129 // 2
    t_lp = 2.4                      # seconds of k_build_K_lp in one step, over 40 launches
    times = {"k_build_K_lp": (40, t_lp), "k_build_K_occ": (20, 0.35), "k_gemm_tn_lds": (40, 0.23),
             "k_reduce_K": (40, 0.06)}
    r = bench.kernel_rooflines(times, 128, 16, 150000, "bf16x3")
    assert abs(r["k_build_K_lp"]["tflops"] - 6 * 150000 ** 2 * P / t_lp / 1e12) < 1e-9
    assert abs(r["k_build_K_lp"]["frac"] - r["k_build_K_lp"]["tflops"] / 2500.0) < 1e-12
    assert abs(r["k_build_K_occ"]["tflops"] - 6 * 150000 ** 2 * 136 / 0.35 / 1e12) < 1e-9
    assert r["k_build_K_occ"]["peak_tflops"] == 78.6 and "frac" not in r["k_reduce_K"]
    assert abs(sum(e["share_of_step"] for e in r.values()) - 1.0) < 1e-12
    assert abs(r["k_build_K_lp"]["avg_ms"] - t_lp / 40 * 1e3) < 1e-9


def test_integer_occupied_block_roofline():
    """The integer occupied block is rated by its executed int8 work (21 digit
    products per useful one over its 16-pair tiles) against the int8 peak,
    with its useful FP64-class rate beside it."""
    assert bench.occ_i8_columns(16) == 144          # 136 pairs: nine tiles
    assert bench.occ_i8_columns(8) == 48            # 36 pairs: three tiles
    assert bench.occ_i8_columns(17) == 160          # 153 pairs: two groups of five tiles
    t = 0.27                                        # seconds per step
    r = bench.kernel_rooflines({"k_build_K_occ_i8": (20, t)}, 128, 16, 150000, "bf16x3")["k_build_K_occ_i8"]
    executed = 6 * 150000 ** 2 * 144 * 21
    assert abs(r["tflops"] - executed / t / 1e12) < 1e-9 and r["peak_tflops"] == 5000.0
    assert abs(r["useful_tflops"] - 6 * 150000 ** 2 * 136 / t / 1e12) < 1e-9
