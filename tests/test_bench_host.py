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
