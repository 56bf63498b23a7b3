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
