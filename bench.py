#!/usr/bin/env python3
"""Benchmark of the zero-copy traversal hot path on one MI355X.

Workload (default): R-MAT/Kronecker scale 27, edgefactor 16,
(a, b, c) = (0.57, 0.19, 0.19), symmetrised, simple; uint64 neighbour ids
(~34 GB) and uint32 weights in [1, 255] (~17 GB) in pinned host memory read
in place by the GPU; 8 random sources with degree > 0 (seed 2).

One step = BFS + SSSP from the step's source and CC over the whole graph
(every row of the hot path: placement is done once beforehand, as the paper
maps everything at set-up).  Value = GTEPS of the whole timed region:
(reached edges of BFS + reached edges of SSSP + all edges for CC) / seconds.
Reached edges = sum of out-degrees of the vertices a traversal reaches.

The JSON line also carries the host-link rate of the neighbour-scan kernels
against the measured pinned memcpy peak, the HBM and managed placements run
once after the timed region, the roofline of the dominant kernel and the
oracle's CPU rate on a bounded sample.

Other workloads (``--config``):
  kron16     R-MAT scale 16, uint32 ids, BFS only from the lowest-id vertex
             with degree > 0 (the small single-source case);
  uniform27  uniform random graph, 2^27 vertices, 2^27 * 32 samples
             (~8.6 billion directed edges), uint32 ids + uint32 weights;
  batched26  R-MAT scale 26, uint32 ids + weights: one step = 64 BFS sources
             (degrees log-spaced 1..max, seed 4) in one batched call plus 64
             SSSP sources (seed 5) in another, against 64 plain runs of each.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PCIE5_X16_GBPS = 64.0  # published per-direction rate of the MI355X host link (PCIe 5.0 x16)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PRESETS = {
    "kron27": dict(workload="kron", scale=27, col_bytes=8, sources=8, steps=8,
                   algos=("bfs", "sssp", "cc")),
    "kron16": dict(workload="kron", scale=16, col_bytes=4, sources=1, steps=50,
                   algos=("bfs",)),
    "uniform27": dict(workload="uniform", scale=27, col_bytes=4, sources=8, steps=8,
                      algos=("bfs", "sssp", "cc")),
    "batched26": dict(workload="kron", scale=26, col_bytes=4, sources=64, steps=2,
                      algos=("bfs", "sssp")),
}


def workload_name(args):
    kind = "Kronecker/R-MAT" if args.workload == "kron" else "uniform random"
    size = f"scale {args.scale}, edgefactor 16" if args.workload == "kron" else \
        f"2^{args.scale} vertices, 2^{args.scale} x 32 samples"
    if args.pack:
        return (f"{kind} {size}, packed lists (from u{8 * args.col_bytes} ids + u32 weights; ids and weights "
                f"bit-packed per list) in pinned host zero-copy memory")
    return f"{kind} {size}, u{8 * args.col_bytes} col + u32 weights in pinned host zero-copy memory"


def build_graph(args, E, graphgen):
    import numpy as np
    t = time.time()
    if args.workload == "kron":
        h = graphgen.rmat(args.scale, 16, 0.57, 0.19, 0.19, seed=1)
    else:
        h = graphgen.uniform(args.scale, (1 << args.scale) * 32, seed=1)
    V, M = h.num_vertices, h.num_edges
    log(f"[bench] generated {h.name}: V={V} E={M} in {time.time() - t:.1f}s")
    t = time.time()
    rp = np.empty(V + 1, dtype=np.uint64)
    col = E.PinnedArray(M, np.uint64 if args.col_bytes == 8 else np.uint32, noncoherent=args.noncoherent)
    w = E.PinnedArray(M, np.uint32, noncoherent=args.noncoherent)
    h.export_into(rp.ctypes.data, col.ptr, args.col_bytes, w.ptr, 3)
    h.free()
    log(f"[bench] exported into pinned memory in {time.time() - t:.1f}s")
    return rp, col, w


def run_step(G, src, out, algos=("bfs", "sssp", "cc"), keep=None):
    """The step's traversals (BFS, SSSP from src; CC); per-algorithm stats.
    With `keep` (a dict), each algorithm's output is also copied into it."""
    res = {}
    for a in algos:
        if a == "cc":
            G.cc(out)
        else:
            getattr(G, a)(src, out)
        res[a] = G.stats()
        if keep is not None:
            keep[a] = out.clone()
    return res


def outputs_equal(ref, got):
    """Per algorithm: whether an arm's output equals the plain zero-copy run's
    (levels, distances and labels are unique, so every arm must match)."""
    import torch
    return {a: bool(torch.equal(ref[a], got[a])) for a in got if a in ref}


def kernel_key(algo, variant, col_bytes, packed=False):
    """The scan kernel's template name as the profiler prints it (variant 6:
    a bottom-up BFS level, whose probe kernel carries nearly all its time)."""
    t = "unsigned long" if col_bytes == 8 else "unsigned int"
    a = {"bfs": 0, "sssp": 1, "cc": 2}[algo]
    if variant == 6:  # packed: the probe decodes 8 ids per vertex
        return "k_bu_probe_packed<8>" if packed else f"k_bu_probe<{t}>"
    if packed:
        return f"k_balanced_packed<{a}>"
    names = [f"k_group<{t}, {a}, 1>", f"k_group<{t}, {a}, 16>", f"k_wave<{t}, {a}, false>",
             f"k_wave<{t}, {a}, true>", f"k_block<{t}, {a}>", f"k_balanced<{t}, {a}>"]
    return names[variant]


KERNEL_SOURCES = ["paper_2006_06890_amd/csrc/traverse.hip", "paper_2006_06890_amd/csrc/wave.h",
                  "paper_2006_06890_amd/csrc/internal.h", "paper_2006_06890_amd/csrc/tier.h",
                  "paper_2006_06890_amd/csrc/packed.h"]


def counters_path(args):
    tag = "_packed" if args.pack else ""
    return os.path.join(ROOT, "profiles", f"counters_{args.config}_u{8 * args.col_bytes}{tag}.json")


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def counter_traffic(args, kernel):
    """Per-dispatch bytes from the committed rocprofv3 counter runs, or None
    when the kernel sources changed since they were taken."""
    path = counters_path(args)
    if not os.path.exists(path):
        return None
    c = json.load(open(path))
    if c.get("kernel_sources_sha1") != kernel_sources_sha1() or kernel not in c["kernels"]:
        return None
    return c["kernels"][kernel]


def host_cpu():
    """CPU model and the logical CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}


def link_rate_violations(result, peak, slack=1.05):
    """Every host-link rate in the line (keys ending in link_GBps or
    scan_GBps) that exceeds the measured copy peak by more than `slack`:
    such a rate counts bytes the timed kernels did not move."""
    bad = []

    def walk(x, path):
        if isinstance(x, dict):
            for k, v in x.items():
                p = f"{path}.{k}" if path else k
                if isinstance(v, (int, float)) and (k.endswith("link_GBps") or k == "scan_GBps"):
                    if v > slack * peak:
                        bad.append((p, v))
                else:
                    walk(v, p)

    walk(result, "")
    return bad


PROFILE_ARGS = "--steps 1 --warmup 0 --no-arms --no-cpu-baseline --no-batch --no-learned --pagerank-iters 0"
COPY_KERNEL = "k_seq_read<4>"  # the calibration's wave-merged read of 1 GiB of pinned host memory


def _short_name(name):
    """'void emogi::k_balanced<unsigned long, 1>(emogi::ScanArgs, ...)' -> 'k_balanced<unsigned long, 1>'."""
    n = name.strip()
    for p in ("void ", "emogi::"):
        if n.startswith(p):
            n = n[len(p):]
    n = n.replace("emogi::", "")
    depth, out = 0, []
    for ch in n:  # drop the argument list (the first '(' outside template brackets)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out).strip()


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        sys.exit(f"no *{suffix} under {d}")
    return rows


def _trace_table(stats, top=18):
    lines = ["| kernel | calls | total ms | avg ms | % |", "|---|---|---|---|---|"]
    stats = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))
    for r in stats[:top]:
        lines.append(f"| `{r['Name'][:100]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    return lines


def _summarize_trace_only(args, stats, out_dir):
    """A kernel-trace summary without counters (--summarize TRACE_DIR - -)."""
    flags = f"--config {args.config}" + (" --pack" if args.pack else "")
    extra = " --no-autotune" if args.config == "batched26" else ""
    cmd = f"python3 $R/bench.py {flags} --steps 1 --warmup 0 --no-cpu-baseline{extra}"
    td = os.path.basename(os.path.normpath(args.summarize[0]))
    lines = [f"# Kernel trace: {workload_name(args)}", "",
             "Commands (run from /tmp with TMPDIR=/tmp; R = repository root):", "", "```",
             f"rocprofv3 --kernel-trace --stats -d $R/gpurun_out/{td} -o trace --output-format csv -- {cmd}",
             f"python3 $R/bench.py {flags} --summarize $R/gpurun_out/{td} - - --summary-name {args.summary_name}",
             "```", "", "## rocprofv3 --kernel-trace --stats (top kernels)", ""] + _trace_table(stats)
    md = os.path.join(out_dir, args.summary_name + ".md")
    with open(md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {md}")


def summarize_profiles(args, out_dir=None):
    """Writes profiles/<name>.md and the counters JSON bench.py reads, from
    three rocprofv3 runs of `bench.py <args> PROFILE_ARGS`: --kernel-trace
    --stats, --pmc FETCH_SIZE, --pmc WRITE_SIZE TCC_EA0_RDREQ_IO_32B_sum
    TCC_EA0_RDREQ_DRAM_32B_sum.  Counters are scaled by what they read for the
    copy kernel (1 GiB of pinned host memory read once per dispatch)."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    trace_d, fetch_d, io_d = args.summarize
    stats = _csv_rows(trace_d, "kernel_stats.csv")
    if fetch_d == "-" and io_d == "-":
        return _summarize_trace_only(args, stats, out_dir)
    per = {}
    for d in (fetch_d, io_d):
        for r in _csv_rows(d, "counter_collection.csv"):
            k = _short_name(r["Kernel_Name"])
            e = per.setdefault(k, {"dispatch_ids": set()})
            e["dispatch_ids"].add(r["Dispatch_Id"])
            c = r["Counter_Name"]
            e[c] = e.get(c, 0.0) + float(r["Counter_Value"])
            e.setdefault("_n_" + c, set()).add(r["Dispatch_Id"])
    copy = per.get(COPY_KERNEL)
    if copy is None:
        sys.exit(f"the counter runs hold no {COPY_KERNEL} dispatch to scale by")
    n_copy = len(copy["_n_FETCH_SIZE"])
    copy_bytes = float(1 << 30)
    fetch_factor = copy_bytes / (copy["FETCH_SIZE"] * 1024 / n_copy)
    io_factor = copy_bytes / (copy["TCC_EA0_RDREQ_IO_32B_sum"] * 32 / len(copy["_n_TCC_EA0_RDREQ_IO_32B_sum"]))
    kernels = {}
    for k, e in per.items():
        nf = len(e.get("_n_FETCH_SIZE", ())) or 1
        ni = len(e.get("_n_TCC_EA0_RDREQ_IO_32B_sum", ())) or 1
        kernels[k] = {
            "dispatches": ni,
            "link_bytes_per_dispatch": e.get("TCC_EA0_RDREQ_IO_32B_sum", 0.0) * 32 * io_factor / ni,
            "fetch_bytes_per_dispatch_scaled": e.get("FETCH_SIZE", 0.0) * 1024 * fetch_factor / nf,
            "write_bytes_per_dispatch": e.get("WRITE_SIZE", 0.0) * 1024 / ni,
            "hbm_read_bytes_per_dispatch": e.get("TCC_EA0_RDREQ_DRAM_32B_sum", 0.0) * 32 / ni,
        }
    workload = workload_name(args) + "; one bench step (" + "+".join(a.upper() for a in args.algos) + ")"
    doc = {"workload": workload, "kernel_sources_sha1": kernel_sources_sha1(),
           "fetch_factor": fetch_factor, "io_factor": io_factor,
           "copy_kernel": f"{COPY_KERNEL}, 1 GiB of pinned host memory per dispatch", "kernels": kernels}
    cpath = os.path.join(out_dir, os.path.basename(counters_path(args)))
    with open(cpath, "w") as f:
        json.dump(doc, f, indent=1)
    flags = f"--config {args.config}" + (" --pack" if args.pack else "")
    cmd = f"python3 $R/bench.py {flags} {PROFILE_ARGS}"
    td, fd, iod = (os.path.basename(os.path.normpath(x)) for x in (trace_d, fetch_d, io_d))
    lines = [f"# Kernel trace + counters: {workload}", "",
             f"Kernel sources sha1 {doc['kernel_sources_sha1']} (the files bench.py hashes).",
             "Commands (run from /tmp with TMPDIR=/tmp; R = repository root):", "", "```",
             f"rocprofv3 --kernel-trace --stats -d $R/gpurun_out/{td} -o trace --output-format csv -- {cmd}",
             f"rocprofv3 --pmc FETCH_SIZE -d $R/gpurun_out/{fd} -o fetch --output-format csv -- {cmd}",
             f"rocprofv3 --pmc WRITE_SIZE TCC_EA0_RDREQ_IO_32B_sum TCC_EA0_RDREQ_DRAM_32B_sum -d $R/gpurun_out/{iod} "
             f"-o io --output-format csv -- {cmd}",
             f"python3 $R/bench.py {flags} --summarize $R/gpurun_out/{td} $R/gpurun_out/{fd} $R/gpurun_out/{iod} "
             f"--summary-name {args.summary_name}", "```", "",
             "## rocprofv3 --kernel-trace --stats (top kernels)", ""] + _trace_table(stats)
    lines += ["", "## Counters (rocprofv3 --pmc; per dispatch, averaged over each kernel's dispatches)", "",
              f"Scale factors from `{COPY_KERNEL}` ({n_copy} dispatches x 1 GiB of pinned host memory read once): "
              f"FETCH_SIZE x {fetch_factor:.3f}, TCC_EA0_RDREQ_IO_32B x 32 B x {io_factor:.3f}.  WRITE_SIZE (the "
              f"copy kernel writes nothing) and TCC_EA0_RDREQ_DRAM_32B x 32 B (GPU-memory read requests past L2) "
              f"are taken at face value.", "",
              "| kernel | dispatches | link GB (IO_32B x 32) | link MB / dispatch | FETCH x factor MB / dispatch "
              "| WRITE MB / dispatch | GPU-memory read MB / dispatch |", "|---|---|---|---|---|---|---|"]
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["link_bytes_per_dispatch"] * kv[1]["dispatches"]):
        lines.append(f"| `{k}` | {v['dispatches']} | {v['link_bytes_per_dispatch'] * v['dispatches'] / 1e9:.2f} | "
                     f"{v['link_bytes_per_dispatch'] / 1e6:.2f} | {v['fetch_bytes_per_dispatch_scaled'] / 1e6:.2f} | "
                     f"{v['write_bytes_per_dispatch'] / 1e6:.2f} | {v['hbm_read_bytes_per_dispatch'] / 1e6:.2f} |")
    md = os.path.join(out_dir, args.summary_name + ".md")
    with open(md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {md} and {cpath}")


def cpu_baseline(args, rp, col_array, src):
    """The oracle, as it stands, on a bounded sample of the benchmark's own
    workload: queue BFS from the step's first source over the very arrays the
    GPU reads (the pinned buffers, read by the CPU), repeated to >= 5 s on
    small graphs.  SSSP and CC are not sampled: single-threaded Dijkstra and
    union-find over billions of edges take minutes."""
    import oracle
    secs, reps, lv = 0.0, 0, None
    while reps == 0 or secs < 5.0:
        t = time.perf_counter()
        lv = oracle.bfs(rp, col_array, src)
        secs += time.perf_counter() - t
        reps += 1
    reached = oracle.reached_edges(rp, lv)
    M = int(rp[-1])
    return {
        "value": reps * reached / secs / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
        "threads_used": 1, "host_cpu": host_cpu(),
        "sample": (f"single-threaded oracle queue BFS from source {src} on the benchmark's own graph "
                   f"({workload_name(args)}; {M} directed edges, {reached} reached), read from the same "
                   f"pinned arrays; {reps} run(s), {secs:.1f}s of CPU"
                   + (".  SSSP and CC not sampled (Dijkstra and union-find over this graph take minutes "
                      "on one core)" if len(args.algos) > 1 else "")),
        "compare_with": "per_algorithm.bfs.gteps" if args.config != "batched26" else "batched.bfs.plain_gteps",
    }


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: per config)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", choices=sorted(PRESETS), default="kron27",
                    help="workload preset (default: R-MAT scale 27, uint64 ids)")
    ap.add_argument("--scale", type=int, default=None)
    ap.add_argument("--col-bytes", type=int, choices=[4, 8], default=None)
    ap.add_argument("--sources", type=int, default=None)
    ap.add_argument("--scheduler", default="heuristic")
    ap.add_argument("--request-unit", type=int, default=256)
    ap.add_argument("--no-arms", action="store_true", help="skip the HBM/managed comparison runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-source batched runs")
    ap.add_argument("--noncoherent", action="store_true", help="pin the edge arrays non-coherent")
    ap.add_argument("--pack", action="store_true",
                    help="measure the packed lists (EMOGI_F_PACK) instead of the plain arrays; "
                         "no batched runs, tier or packed arms")
    ap.add_argument("--no-learned", action="store_true", help="skip the scheduler comparison")
    ap.add_argument("--no-autotune", action="store_true", help="batched26: keep the default batch parameters")
    ap.add_argument("--pagerank-iters", type=int, default=3,
                    help="PageRank iterations run once after the timed region (0: skip)")
    ap.add_argument("--tier-fracs", default="0.1,0.25",
                    help="HBM tier budgets (fractions of the edge-list bytes) run as extra arms; '' for none")
    ap.add_argument("--calib-bytes", type=int, default=1 << 30)
    ap.add_argument("--calibrate-only", action="store_true",
                    help="run the link calibration (plain zero-copy read kernels) and exit")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "IO_DIR"),
                    help="write the profile summary and counters file from three rocprofv3 runs (no GPU)")
    ap.add_argument("--summary-name", default=None, help="with --summarize: profiles/<name>.md")
    args = ap.parse_args()
    if args.pack:
        if args.config == "batched26":
            sys.exit("--pack: batched traversal reads plain lists")
        args.no_batch = True
        args.tier_fracs = ""
    preset = PRESETS[args.config]
    args.workload = preset["workload"]
    args.algos = preset["algos"]
    for k in ("scale", "col_bytes", "sources", "steps"):
        if getattr(args, k) is None:
            setattr(args, k, preset[k])
    return args


def base_result(args, value, elapsed, V, M, profile):
    return {
        "metric": "GTEPS and achieved host-link GB/s (% of measured pinned peak), zero-copy vs managed",
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * elapsed / max(1, args.steps), 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded graph generator; no dataset)",
        "config": {
            "workload": workload_name(args) + "; " + "+".join(a.upper() for a in args.algos) + " per step",
            "preset": args.config, "vertices": V, "directed_edges": M, "col_bytes": args.col_bytes,
            "placement": "host_zero_copy", "request_unit": args.request_unit, "packed": bool(args.pack),
        },
        "host_link": host_link_summary(profile),
    }


def host_link_summary(profile):
    """The calibration (Sec. 3.3's toy study): peaks, R, latency, the
    waves-in-flight sweep with the knee Little's law predicts, start
    offsets, and coherent vs non-coherent pinning."""
    import math
    R = profile["request_unit"]
    waves = profile.get("waves_GBps", {})
    best = max(waves.values()) if waves else 0.0
    # outstanding R-byte requests needed to carry the sweep's best rate over one round trip
    model = math.ceil(best * 1e9 * profile["latency_us"] * 1e-6 / R) if best else None
    nc = profile.get("noncoherent", {})
    return {
        "pinned_memcpy_peak_GBps": round(profile["memcpy_GBps"], 2),
        "request_unit_measured": R,
        "kernel_seq_read_GBps": round(max(profile["seq_read_GBps"].values()), 2),
        "latency_us": round(profile["latency_us"], 3),
        "waves_in_flight_GBps": {str(k): round(v, 2) for k, v in waves.items()},
        "knee_waves": profile.get("knee_waves"),
        "littles_law_waves": model,
        "offset_GBps": {str(k): round(v, 2) for k, v in profile.get("offset_GBps", {}).items()},
        "noncoherent": {k: round(v, 2) for k, v in nc.items()},
    }


def roofline(args, kernels, peak, profile=None):
    """The dominant kernel: algorithmic link bytes per launch ((e + 4) per
    scanned edge for SSSP, e for BFS and CC: the per-unit figures of the
    measurement plan) over its average HIP-event launch time, against the
    link's published rate."""
    dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["ms"])
    achieved = dom["bytes"] / (dom["ms"] * 1e6)
    r = {
        "bound": "host_link",
        "kernel": dom_name,
        "achieved": round(achieved, 2),
        "peak": PCIE5_X16_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / PCIE5_X16_GBPS, 4),
        "frac_of_measured_memcpy": round(achieved / peak, 4),
        "traffic": None,
        "launches": dom["launches"],
        "avg_launch_ms": round(dom["ms"] / max(1, dom["launches"]), 4),
        "algorithmic_bytes_per_launch": round(dom["bytes"] / max(1, dom["launches"])),
        "sector_model_bytes_per_launch": round(dom.get("sector_bytes", 0) / max(1, dom["launches"])),
    }
    ct = counter_traffic(args, dom_name)
    if ct is not None:
        # host-link bytes per launch from TCC_EA0_RDREQ_IO_32B x 32 B (copy-kernel factor applied);
        # FETCH_SIZE (scaled) + WRITE_SIZE per launch beside it for the HBM side
        r["traffic"] = round(ct["link_bytes_per_dispatch"])
        # the counters come from runs from the first source: compare with that source's models
        s0 = dom.get("src0", {})
        if s0.get("launches"):
            alg0 = s0["bytes"] / s0["launches"]
            sec0 = s0["sector_bytes"] / s0["launches"]
            r["first_source"] = {"algorithmic_bytes_per_launch": round(alg0),
                                 "sector_model_bytes_per_launch": round(sec0),
                                 "counted_over_algorithmic": round(r["traffic"] / max(1.0, alg0), 4),
                                 "counted_over_sector_model": round(r["traffic"] / max(1.0, sec0), 4)}
        r["traffic_fetch_write"] = round(ct["fetch_bytes_per_dispatch_scaled"] + ct["write_bytes_per_dispatch"])
        r["traffic_source"] = os.path.relpath(counters_path(args), ROOT)
        if profile and profile.get("hbm_read_GBps"):
            # the vertex state's side: GPU-memory bytes per launch (read requests to
            # DRAM, TCC_EA0_RDREQ_DRAM_32B x 32, + WRITE_SIZE) over the launch time
            hbm_b = round(ct.get("hbm_read_bytes_per_dispatch", 0) + ct["write_bytes_per_dispatch"])
            hbm_gbps = hbm_b / (r["avg_launch_ms"] * 1e6)
            r["hbm"] = {"bytes_per_launch": hbm_b, "achieved_GBps": round(hbm_gbps, 1),
                        "measured_read_peak_GBps": round(profile["hbm_read_GBps"], 1),
                        "measured_copy_peak_GBps": round(profile["hbm_copy_GBps"], 1),
                        "frac_of_read_peak": round(hbm_gbps / profile["hbm_read_GBps"], 4)}
    return r


def bfs_directions(G, src, out, ref_levels=None):
    """BFS from src with the per-level direction rule and all top-down (with
    ref_levels: both outputs must equal them, recorded in "levels_equal")."""
    import torch
    r = {}
    for mode in ("auto", "top_down"):
        G.set_direction(mode)
        G.bfs(src, out)
        if ref_levels is not None:
            r.setdefault("levels_equal", {})[mode] = bool(torch.equal(out, ref_levels))
        st = G.stats()
        r[f"{mode}_ms"] = round(st["total_ms"], 2)
        if mode == "auto":
            r["bottom_up_levels"] = st["bottom_up_levels"]
            r["level_direction"] = st["level_direction"]
            r["level_ms"] = [round(x, 2) for x in st["level_ms"]]
        else:
            r["top_down_level_ms"] = [round(x, 2) for x in st["level_ms"]]
    G.set_direction("auto")
    r["speedup"] = round(r["top_down_ms"] / r["auto_ms"], 3)
    return r


def bench_plain(args, E, G, rp, col, w, sources, out, profile, torch, graphgen):
    import numpy as np
    V, M = rp.shape[0] - 1, int(rp[-1])
    peak = profile["memcpy_GBps"]
    for i in range(args.warmup):
        run_step(G, sources[i % len(sources)], out, args.algos)
        log(f"[bench] warmup step {i} done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for i in range(args.steps):
        steps.append((sources[i % len(sources)], run_step(G, sources[i % len(sources)], out, args.algos)))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, (s, r) in enumerate(steps):
        log(f"[bench] step {i} src={s}: " + ", ".join(f"{a} {r[a]['total_ms']:.1f} ms" for a in r))

    # --- throughput ---
    teps_edges = 0
    per = {a: {"ms": 0.0, "edges": 0, "scan_ms": 0.0, "bytes": 0, "sector_bytes": 0} for a in args.algos}
    kernels = {}
    for s, r in steps:
        reached = r["bfs"]["reached_edges"]  # out-degrees of the vertices BFS reached
        for a in args.algos:
            st = r[a]
            e = M if a == "cc" else reached
            teps_edges += e
            per[a]["ms"] += st["total_ms"]
            per[a]["edges"] += e
            per[a]["scan_ms"] += st["expand_ms"]
            per[a]["bytes"] += st["useful_link_bytes"]
            # the same lists at the link's 32-byte sector granularity (packed: encoded bytes)
            per[a]["sector_bytes"] += (st["useful_link_bytes"] if args.pack
                                       else st["id_sector_bytes"] + st["weight_sector_bytes"])
            # algorithmic link bytes per scanned list element: the id, and for
            # SSSP its weight ((e + 4) per edge, whether or not the scan needed
            # the weight); packed lists: their encoded bytes.  The sector model
            # (each list, and each weight read, rounded out to 32-byte sectors)
            # is spread over the levels by their edges, beside it.
            if args.pack:
                eb = st["useful_link_bytes"] / max(1, st["edges_scanned"])
            else:
                eb = args.col_bytes + (4 if a == "sssp" else 0)
            sb = (st["id_sector_bytes"] + st["weight_sector_bytes"]) / max(1, st["edges_scanned"])
            first = s == sources[0]  # the profiled runs traverse from the first source
            for v, ms, ed in zip(st["level_variant"], st["level_ms"], st["level_edges"]):
                k = kernel_key(a, v, args.col_bytes, args.pack)
                kk = kernels.setdefault(k, {"ms": 0.0, "bytes": 0, "launches": 0, "sector_bytes": 0,
                                            "src0": {"bytes": 0, "sector_bytes": 0, "launches": 0}})
                kk["ms"] += ms
                kk["bytes"] += ed * eb
                kk["sector_bytes"] += ed * sb
                kk["launches"] += 1
                if first:
                    kk["src0"]["bytes"] += ed * eb
                    kk["src0"]["sector_bytes"] += ed * sb
                    kk["src0"]["launches"] += 1
    value = teps_edges / elapsed / 1e9
    link_bytes = sum(p["bytes"] for p in per.values())
    scan_ms = sum(p["scan_ms"] for p in per.values())
    link_gbps = link_bytes / (scan_ms * 1e6) if scan_ms else 0.0

    result = base_result(args, value, elapsed, V, M, profile)
    result["config"].update(
        sources=sources, scheduler=args.scheduler,
        bfs_direction="per level (top-down or bottom-up, alpha 14, beta 24)",
        create_time_passes=("host encode of the packed lists (untimed, as the paper maps at set-up)" if args.pack
                            else "none: the lists are mapped as given, no weight bounds (EMOGI_F_WEIGHT_BOUND off)"))
    result["per_algorithm"] = {
        a: {"gteps": round(p["edges"] / (p["ms"] * 1e6), 4) if p["ms"] else None,
            "link_GBps": round(p["bytes"] / (p["scan_ms"] * 1e6), 2) if p["scan_ms"] else None,
            "sector_link_GBps": round(p["sector_bytes"] / (p["scan_ms"] * 1e6), 2) if p["scan_ms"] else None,
            "ms_per_run": round(p["ms"] / len(steps), 3)}
        for a, p in per.items()
    }
    if "bfs" in per:
        result["per_algorithm"]["bfs"]["bottom_up_levels_per_run"] = round(
            sum(r["bfs"]["bottom_up_levels"] for _, r in steps) / len(steps), 2)
    result["host_link"].update(scan_GBps=round(link_gbps, 2), pct_of_pinned_peak=round(100 * link_gbps / peak, 1))
    result["roofline"] = roofline(args, kernels, peak, profile)

    # outputs of the plain zero-copy method for the first source, untimed: every
    # arm below (other placements, tier, packed, batched) must reproduce them
    ref = {}
    if not (args.no_arms and args.no_batch):
        run_step(G, sources[0], out, args.algos, keep=ref)
    checks = {}

    # --- the two systems patterns, each against the plain method on this GPU ---
    if not args.no_batch and "sssp" in args.algos:
        # 64 sources of log-spaced degrees in one batched call each; the plain
        # method on these same sources is timed by the batched26 preset
        srcs64 = graphgen.degree_spread_sources(rp, 64, seed=4)
        out64 = torch.empty(len(srcs64) * V, dtype=torch.int32, device="cuda")
        deg_t = torch.from_numpy(np.diff(rp).astype(np.int64)).to("cuda")
        bat = {"sources": len(srcs64), "source_degrees": "log-spaced 1..max (seed 4)"}
        j = int(np.argmax(np.diff(rp)[srcs64]))  # the batch's highest-degree source
        plain_j = {}
        run_step(G, srcs64[j], out, ("bfs", "sssp"), keep=plain_j)
        for a in ("bfs", "sssp"):
            getattr(G, a + "_batch")(srcs64, out64)
            st = G.stats()
            o = out64.view(len(srcs64), V)
            reached = sum(int(((o[i] != -1).to(torch.int64) * deg_t).sum()) for i in range(len(srcs64)))
            bat[f"{a}_ms"] = round(st["total_ms"], 1)
            bat[f"{a}_gteps"] = round(reached / (st["total_ms"] * 1e6), 3)
            checks.setdefault("batched", {})[a] = bool(torch.equal(o[j], plain_j[a]))
        del plain_j
        bat["params"] = G.get_batch_params()
        result["batched"] = bat
        del out64, deg_t
        log(f"[bench] batched: {result['batched']}")
    weights = os.path.join(ROOT, "paper_2006_06890_amd", "scheduler_weights.json")
    if not args.no_learned:
        sched = {}
        modes = [("fixed_v3", 3), ("heuristic", "heuristic")]
        if os.path.exists(weights):
            G.load_scheduler(weights)
            modes.append(("learned", "learned"))
        for name, mode in modes:
            if isinstance(mode, int):
                G.set_variant(mode)
            else:
                G.set_scheduler(mode)
            r = run_step(G, sources[0], out, args.algos)
            sched[name] = {a: round(r[a]["total_ms"], 2) for a in r}
            sched[name]["step_ms"] = round(sum(r[a]["total_ms"] for a in r), 2)
            if name == "learned":
                sched[name]["levels_by_network"] = {a: f"{r[a]['levels_by_network']} of {len(r[a]['level_variant'])}"
                                                    for a in r}
        result["schedulers"] = sched
        log(f"[bench] schedulers (one step, source {sources[0]}): {sched}")

    if "bfs" in args.algos and not args.no_arms:
        G.set_scheduler("heuristic")
        result["direction"] = {"zero_copy": bfs_directions(G, sources[0], out, ref.get("bfs"))}
        log(f"[bench] direction (zero-copy): {result['direction']['zero_copy']}")

    if args.pagerank_iters > 0 and "cc" in args.algos:
        # PageRank (the paper's fourth workload): every iteration streams all lists
        pr = torch.empty(V, dtype=torch.int64, device="cuda")
        G.pagerank(args.pagerank_iters, out=pr)
        st = G.stats()
        it_ms = st["expand_ms"] / max(1, st["iterations"])
        result["pagerank"] = {
            "iterations": st["iterations"], "fixed_point_bits": 40, "damping": 0.85,
            "ms_per_iteration": round(st["total_ms"] / max(1, st["iterations"]), 2),
            "scan_ms_per_iteration": round(it_ms, 2),
            "gteps": round(M / (st["total_ms"] / max(1, st["iterations"]) * 1e6), 3),
            "link_GBps": round(st["useful_link_bytes"] / max(1, st["iterations"]) / (it_ms * 1e6), 2),
        }
        del pr
        log(f"[bench] pagerank: {result['pagerank']}")

    arms = {}
    fracs = [float(x) for x in args.tier_fracs.split(",") if x.strip()]
    if fracs and not args.no_arms:
        # HBM tier arms: the same zero-copy graph with the hub lists copied to GPU memory
        G.set_scheduler(args.scheduler if not args.scheduler.isdigit() else "heuristic")
        eb = args.col_bytes + 4
        for f in fracs:
            nv, nb = G.set_hbm_tier(int(f * M * eb))
            got = {}
            r = run_step(G, sources[0], out, args.algos, keep=got)
            checks[f"hbm_tier_{f:g}"] = outputs_equal(ref, got)
            del got
            reached = r["bfs"]["reached_edges"]
            ms = sum(r[a]["total_ms"] for a in r)
            if "direction" in result:
                result["direction"][f"hbm_tier_{f:g}"] = bfs_directions(G, sources[0], out, ref.get("bfs"))
            arms[f"hbm_tier_{f:g}"] = {
                "tier_vertices": nv, "tier_GB": round(nb / 1e9, 2),
                "tier_edge_share": round(nb / (M * eb), 4),
                "gteps": round(sum(M if a == "cc" else reached for a in r) / (ms * 1e6), 4),
                **{f"{a}_ms": round(r[a]["total_ms"], 2) for a in r},
                **{f"{a}_tier_edge_frac": round(r[a]["tier_edges"] / max(1, r[a]["edges_scanned"]), 3) for a in r},
            }
            log(f"[bench] arm hbm_tier_{f:g}: {arms[f'hbm_tier_{f:g}']}")
        G.set_hbm_tier(0)
    G.close()
    if not args.no_arms and "sssp" in args.algos and not args.pack:
        # the optional create-time weight bounds (EMOGI_F_WEIGHT_BOUND): their
        # pass over col + weights against what they save per SSSP
        t0 = time.perf_counter()
        Wb = E.Graph(rp, col, w, placement="host_zero_copy", symmetric=True, borrow=True, weight_bound=True)
        create_s = time.perf_counter() - t0
        Wb.set_scheduler("heuristic")
        Wb.sssp(sources[0], out)
        with_ms = Wb.stats()["total_ms"]
        checks["sssp_weight_bound"] = outputs_equal(ref, {"sssp": out})
        setup_ms = Wb.setup_ms()
        Wb.close()
        plain_ms = steps[0][1]["sssp"]["total_ms"]
        saving = plain_ms - with_ms
        arms["sssp_weight_bound"] = {
            "create_s": round(create_s, 2), "in_min_pass_ms": round(setup_ms, 1),
            "in_min_pass_link_GB": round(M * (args.col_bytes + 4) / 1e9, 2),
            "sssp_ms_with_bound": round(with_ms, 1), "sssp_ms_without": round(plain_ms, 1),
            "saving_ms_per_sssp": round(saving, 1),
            "break_even_sssp_runs": round(setup_ms / saving, 1) if saving > 0 else None,
        }
        log(f"[bench] arm sssp_weight_bound: {arms['sssp_weight_bound']}")
    if not args.no_arms:
        for placement in ("hbm", "managed"):
            try:
                H = E.Graph(rp, col.array, w.array, placement=placement, symmetric=True)
            except E.EmogiError as e:
                arms[placement] = {"status": str(e)}
                continue
            H.set_scheduler("heuristic")
            got = {}
            r = run_step(H, sources[0], out, args.algos, keep=got)
            checks[placement] = outputs_equal(ref, got)
            del got
            reached = r["bfs"]["reached_edges"]
            ms = sum(r[a]["total_ms"] for a in r)
            arms[placement] = {
                "gteps": round(sum(M if a == "cc" else reached for a in r) / (ms * 1e6), 4),
                **{f"{a}_ms": round(r[a]["total_ms"], 2) for a in r},
            }
            if "direction" in result:
                result["direction"][placement] = bfs_directions(H, sources[0], out, ref.get("bfs"))
            H.close()
            log(f"[bench] arm {placement}: {arms[placement]}")
    if not args.no_arms and not args.pack:
        # packed lists (the compression Sec. 6 proposes): the same graph with
        # ids and weights bit-packed per list, every source of the step
        t0 = time.perf_counter()
        try:
            P = E.Graph(rp, col, w, symmetric=True, borrow=True, pack=True)
        except E.EmogiError as e:  # e.g. no room to pin the packed copy beside the plain arrays
            arms["packed"] = {"status": str(e)}
            log(f"[bench] arm packed: {arms['packed']}")
            result["arms"] = arms
            result["output_checks"] = checks
            result["link_rate_violations"] = link_rate_violations(result, peak)
            return result
        create_s = time.perf_counter() - t0
        P.set_scheduler("heuristic")
        ids_b, w_b = P.packed_bytes()
        ms_a, edges, tot_ms, link, bu = {}, 0, 0.0, {}, 0
        for s in sources:
            got = {} if s == sources[0] else None
            r = run_step(P, s, out, args.algos, keep=got)
            if got is not None:
                checks["packed"] = outputs_equal(ref, got)
                del got
            reached = r["bfs"]["reached_edges"]
            bu += r["bfs"]["bottom_up_levels"]
            for a in r:
                ms_a[a] = ms_a.get(a, 0.0) + r[a]["total_ms"]
                link[a] = link.get(a, 0) + r[a]["useful_link_bytes"]
                edges += M if a == "cc" else reached
                tot_ms += r[a]["total_ms"]
        arms["packed"] = {
            "ids_GB": round(ids_b / 1e9, 2), "weights_GB": round(w_b / 1e9, 2),
            "id_bytes_per_edge": round(ids_b / M, 3), "weight_bytes_per_edge": round(w_b / M, 3),
            "create_s": round(create_s, 1),
            "gteps": round(edges / (tot_ms * 1e6), 4),
            **{f"{a}_ms": round(ms_a[a] / len(sources), 2) for a in ms_a},
            **{f"{a}_link_GB": round(link[a] / len(sources) / 1e9, 2) for a in link},
            "bfs_bottom_up_levels_per_run": round(bu / len(sources), 2),
        }
        P.close()
        log(f"[bench] arm packed: {arms['packed']}")
    if arms:
        result["arms"] = arms
    # every arm's outputs against the plain zero-copy run of the same source
    for k, v in result.get("direction", {}).items():
        if "levels_equal" in v:
            checks[f"bfs_direction_{k}"] = v.pop("levels_equal")
    result["output_checks"] = checks
    bad = [f"{k}.{a}" for k, v in checks.items() for a, ok in v.items() if not ok]
    if bad:
        log(f"[bench] OUTPUT MISMATCH against the plain zero-copy run: {bad}")
    result["link_rate_violations"] = link_rate_violations(result, peak)
    return result


def bench_batched(args, E, G, rp, sources, profile, torch):
    """One step = every BFS source in one batched call + every SSSP source in
    another; reported against one plain run per source."""
    import numpy as np
    V, M = rp.shape[0] - 1, int(rp[-1])
    bfs_srcs, sssp_srcs = sources
    out = torch.empty(max(len(bfs_srcs), len(sssp_srcs)) * V, dtype=torch.int32, device="cuda")
    params = {}
    for a, srcs in (("bfs", bfs_srcs), ("sssp", sssp_srcs)):
        if args.no_autotune:
            params[a] = G.get_batch_params()
        else:
            best, trials = G.autotune_batch(a, srcs, out)
            params[a] = best
            log(f"[bench] autotuned {a}: {best} over {len(trials)} trials")

    def step():
        st = {}
        for a, srcs in (("bfs", bfs_srcs), ("sssp", sssp_srcs)):
            G.set_batch_params(**params[a])
            getattr(G, a + "_batch")(srcs, out[:len(srcs) * V])
            st[a] = G.stats()
        return st

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup step {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # reached edges per source (the TEPS numerator), from the last outputs
    deg = torch.from_numpy(np.diff(rp).astype(np.int64)).to("cuda")
    reached = {}
    for a, srcs in (("bfs", bfs_srcs), ("sssp", sssp_srcs)):
        getattr(G, a + "_batch")(srcs, out[:len(srcs) * V])
        o = out[:len(srcs) * V].view(len(srcs), V)
        reached[a] = [int(((o[i] != -1).to(torch.int64) * deg).sum()) for i in range(len(srcs))]
    teps_edges = args.steps * (sum(reached["bfs"]) + sum(reached["sssp"]))
    value = teps_edges / elapsed / 1e9

    # the plain method, one run per source
    plain = {}
    G.set_scheduler("heuristic")
    one = out[:V]
    for a, srcs in (("bfs", bfs_srcs), ("sssp", sssp_srcs)):
        ms = 0.0
        for s in srcs:
            getattr(G, a)(s, one)
            ms += G.stats()["total_ms"]
        plain[a] = ms
        log(f"[bench] plain {a}: {len(srcs)} runs in {ms:.0f} ms")
    G.close()

    result = base_result(args, value, elapsed, V, M, profile)
    result["config"].update(bfs_sources=len(bfs_srcs), sssp_sources=len(sssp_srcs),
                            source_degrees="log-spaced 1..max (BFS seed 4, SSSP seed 5)",
                            batch_params=params)
    result["batched"] = {}
    for a in ("bfs", "sssp"):
        ms = sum(r[a]["total_ms"] for r in runs) / len(runs)
        result["batched"][a] = {
            "sources": len(reached[a]), "ms_per_call": round(ms, 1),
            "gteps": round(sum(reached[a]) / (ms * 1e6), 3),
            "plain_ms_all_sources": round(plain[a], 1),
            "plain_gteps": round(sum(reached[a]) / (plain[a] * 1e6), 3),
            "speedup_vs_plain": round(plain[a] / ms, 2),
            "link_bytes_per_call": runs[-1][a]["useful_link_bytes"],
        }
    log(f"[bench] batched: {result['batched']}")
    return result


def main():
    args = parse_args()
    if args.summarize:
        if not args.summary_name:
            sys.exit("--summarize needs --summary-name")
        summarize_profiles(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(sharding over several GPUs is described in the design notes, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import graphgen
    import paper_2006_06890_amd as E

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    E.lib()
    # Link calibration (hot-path row a0): memcpy peak, kernel read rates, R, latency.
    profile = E.calibrate_link(args.calib_bytes)
    log(f"[bench] link: memcpy {profile['memcpy_GBps']:.2f} GB/s, seq read {profile['seq_read_GBps']}, "
        f"R {profile['request_unit']} B, latency {profile['latency_us']:.2f} us")
    if args.calibrate_only:
        print(json.dumps({"link_profile": profile}), flush=True)
        return
    os.environ.setdefault("GG_VERBOSE", "1")  # generator prints its phases (progress)

    rp, col, w = build_graph(args, E, graphgen)
    V = rp.shape[0] - 1
    deg = np.diff(rp)
    G = E.Graph(rp, col, w, placement="host_zero_copy", symmetric=True, borrow=True, pack=args.pack)
    G.set_request_unit(args.request_unit)
    if args.scheduler.isdigit():
        G.set_variant(int(args.scheduler))
    else:
        G.set_scheduler(args.scheduler)

    if args.config == "batched26":
        srcs = (graphgen.degree_spread_sources(rp, args.sources, seed=4),
                graphgen.degree_spread_sources(rp, args.sources, seed=5))
        result = bench_batched(args, E, G, rp, srcs, profile, torch)
    else:
        if args.config == "kron16":
            sources = [int(np.flatnonzero(deg > 0)[0])]  # lowest id with degree > 0
        else:
            sources = graphgen.random_sources(graphgen.CSR(rp, col.array), args.sources, seed=2)
        out = torch.empty(V, dtype=torch.int32, device="cuda")
        result = bench_plain(args, E, G, rp, col, w, sources, out, profile, torch, graphgen)

    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the CPU sample")
        if args.config == "batched26":
            first = graphgen.random_sources(graphgen.CSR(rp, col.array), 1, seed=2)[0]
        else:
            first = sources[0]
        result["cpu_baseline"] = cpu_baseline(args, rp, col.array, first)
    col.free()
    w.free()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
