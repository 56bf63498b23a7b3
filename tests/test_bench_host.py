"""Host-side logic of bench.py, no GPU: kernel names as the profiler prints
them, the counter files the roofline reads, workload names and the
refusals (more than one GPU; packed lists for the batched preset)."""
import argparse
import subprocess
import sys

import bench


def test_kernel_names_match_the_profiler():
    assert bench.kernel_key("bfs", 5, 8) == "k_balanced<unsigned long, 0>"
    assert bench.kernel_key("sssp", 3, 4) == "k_wave<unsigned int, 1, true>"
    assert bench.kernel_key("cc", 0, 4) == "k_group<unsigned int, 2, 1>"
    assert bench.kernel_key("sssp", 4, 8) == "k_block<unsigned long, 1>"
    assert bench.kernel_key("sssp", 5, 8, packed=True) == "k_balanced_packed<1>"
    assert bench.kernel_key("bfs", 2, 4, packed=True) == "k_balanced_packed<0>"  # packed: V5 only


def test_profiler_names_shorten_to_kernel_keys():
    """The counter file is keyed by kernel_key's names: the summarizer drops
    the return type, the namespace and the argument list."""
    assert bench._short_name("void emogi::k_balanced<unsigned long, 1>(emogi::ScanArgs, emogi::OpArgs)") == \
        bench.kernel_key("sssp", 5, 8)
    assert bench._short_name("void emogi::k_bu_probe<unsigned int>(emogi::BuArgs)") == \
        bench.kernel_key("bfs", 6, 4)
    assert bench._short_name("emogi::k_bits_count(unsigned int const*, unsigned long)") == "k_bits_count"
    assert bench._short_name("void emogi::k_balanced_packed<0>(emogi::ScanArgs, emogi::OpArgs)") == \
        bench.kernel_key("bfs", 5, 8, packed=True)
    assert bench._short_name("void emogi::k_bu_probe_packed<8>(emogi::BuArgs)") == \
        bench.kernel_key("bfs", 6, 8, packed=True)


def test_counter_files_and_workload_names():
    a = argparse.Namespace(config="kron27", col_bytes=8, pack=False, workload="kron", scale=27)
    assert bench.counters_path(a).endswith("profiles/counters_kron27_u64.json")
    assert "u64 col + u32 weights" in bench.workload_name(a)
    a.pack = True
    assert bench.counters_path(a).endswith("profiles/counters_kron27_u64_packed.json")
    assert "packed lists" in bench.workload_name(a)


def test_refusals():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
    r = subprocess.run([sys.executable, bench.__file__, "--pack", "--config", "batched26"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "--pack" in r.stderr


def test_link_rate_check_flags_rates_above_the_copy_peak():
    """A link rate above the measured copy peak counts bytes that the timed
    kernels did not move (the sampled-CC bytes once divided by the time of
    its later passes only gave 3206 GB/s on a 57 GB/s link)."""
    line = {"host_link": {"scan_GBps": 41.2, "pinned_memcpy_peak_GBps": 57.3},
            "per_algorithm": {"bfs": {"link_GBps": 50.1, "sector_link_GBps": 53.0},
                              "cc": {"link_GBps": 3206.36}},
            "pagerank": {"link_GBps": 51.3},
            "arms": {"packed": {"bfs_link_GB": 10.9}}}
    bad = bench.link_rate_violations(line, 57.28)
    assert bad == [("per_algorithm.cc.link_GBps", 3206.36)]
    line["per_algorithm"]["cc"]["link_GBps"] = 59.0  # within 5 % of the peak
    assert bench.link_rate_violations(line, 57.28) == []


def test_host_link_summary_littles_law():
    """The knee the calibration sweep should show: the sweep's best rate
    times the round trip, in R-byte requests (Sec. 3.3)."""
    prof = {"memcpy_GBps": 57.28, "request_unit": 256, "seq_read_GBps": {4: 57.6, 8: 57.6, 16: 56.1},
            "latency_us": 1.184, "waves_GBps": {16: 3.0, 256: 40.0, 512: 55.0, 1024: 56.0}, "knee_waves": 512,
            "offset_GBps": {0: 50.0, 16: 30.0, 256: 50.0}, "noncoherent": {"memcpy_GBps": 56.0}}
    h = bench.host_link_summary(prof)
    assert h["littles_law_waves"] == 259  # ceil(56e9 * 1.184e-6 / 256)
    assert h["knee_waves"] == 512 and h["waves_in_flight_GBps"]["1024"] == 56.0


def test_profile_summary_scales_counters_by_the_copy_kernel(tmp_path):
    """--summarize on synthetic rocprofv3 CSVs: per-dispatch averages, the copy
    kernel's scale factors (1 GiB read once), kernel names as bench keys them."""
    import csv
    for sub in ("t", "f", "i"):
        (tmp_path / sub / "host").mkdir(parents=True)

    def write(path, header, rows):
        with open(path, "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(header)
            w.writerows(rows)

    sssp = "void emogi::k_balanced<unsigned long, 1>(emogi::ScanArgs, emogi::OpArgs)"
    copy = "void emogi::k_seq_read<4>(unsigned char const*, unsigned long, unsigned long long*)"
    write(tmp_path / "t/host/trace_kernel_stats.csv",
          ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
          [[sssp, 2, 8e6, 4e6, 80, 1, 1, 0], [copy, 1, 2e6, 2e6, 20, 1, 1, 0]])
    cc = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    write(tmp_path / "f/host/fetch_counter_collection.csv", cc,
          [[1, copy, "FETCH_SIZE", 524288], [2, sssp, "FETCH_SIZE", 1000], [3, sssp, "FETCH_SIZE", 3000]])
    write(tmp_path / "i/host/io_counter_collection.csv", cc,
          [[1, copy, "TCC_EA0_RDREQ_IO_32B_sum", (1 << 30) // 32], [1, copy, "WRITE_SIZE", 0],
           [1, copy, "TCC_EA0_RDREQ_DRAM_32B_sum", 0],
           [2, sssp, "TCC_EA0_RDREQ_IO_32B_sum", 100], [3, sssp, "TCC_EA0_RDREQ_IO_32B_sum", 300],
           [2, sssp, "WRITE_SIZE", 10], [3, sssp, "WRITE_SIZE", 30],
           [2, sssp, "TCC_EA0_RDREQ_DRAM_32B_sum", 5], [3, sssp, "TCC_EA0_RDREQ_DRAM_32B_sum", 7]])
    a = argparse.Namespace(summarize=[str(tmp_path / d) for d in ("t", "f", "i")], summary_name="s",
                           config="kron27", pack=False, col_bytes=8, workload="kron", scale=27,
                           algos=("bfs", "sssp", "cc"))
    bench.summarize_profiles(a, out_dir=str(tmp_path))
    import json
    doc = json.load(open(tmp_path / "counters_kron27_u64.json"))
    assert doc["fetch_factor"] == 2.0 and doc["io_factor"] == 1.0
    assert doc["kernel_sources_sha1"] == bench.kernel_sources_sha1()
    k = doc["kernels"][bench.kernel_key("sssp", 5, 8)]
    assert k["dispatches"] == 2
    assert k["link_bytes_per_dispatch"] == 200 * 32
    assert k["fetch_bytes_per_dispatch_scaled"] == 2000 * 1024 * 2.0
    assert k["write_bytes_per_dispatch"] == 20 * 1024
    assert k["hbm_read_bytes_per_dispatch"] == 6 * 32
    md = (tmp_path / "s.md").read_text()
    assert "rocprofv3 --pmc FETCH_SIZE" in md and "k_balanced<unsigned long, 1>" in md
