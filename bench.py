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


def run_step(G, src, out, torch):
    """BFS + SSSP from src, CC; returns per-algorithm stats."""
    res = {}
    G.bfs(src, out)
    res["bfs"] = G.stats()
    G.sssp(src, out)
    res["sssp"] = G.stats()
    G.cc(out)
    res["cc"] = G.stats()
    return res


def kernel_key(algo, variant, col_bytes):
    """The scan kernel's template name as the profiler prints it."""
    t = "unsigned long" if col_bytes == 8 else "unsigned int"
    a = {"bfs": 0, "sssp": 1, "cc": 2}[algo]
    names = [f"k_group<{t}, {a}, 1>", f"k_group<{t}, {a}, 16>", f"k_wave<{t}, {a}, false>",
             f"k_wave<{t}, {a}, true>", f"k_block<{t}, {a}>", f"k_balanced<{t}, {a}>"]
    return names[variant]


KERNEL_SOURCES = ["paper_2006_06890_amd/csrc/traverse.hip", "paper_2006_06890_amd/csrc/wave.h",
                  "paper_2006_06890_amd/csrc/internal.h"]
COUNTERS = os.path.join(ROOT, "profiles", "counters_kron27_u64.json")


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def counter_traffic(kernel):
    """Per-dispatch bytes from the committed rocprofv3 counter runs, or None
    when the kernel sources changed since they were taken."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("kernel_sources_sha1") != kernel_sources_sha1() or kernel not in c["kernels"]:
        return None
    return c["kernels"][kernel]


def cpu_baseline(args):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np
    import graphgen
    import oracle
    scale = args.cpu_scale
    g = graphgen.rmat(scale, 16, 0.57, 0.19, 0.19, seed=1).to_csr(args.col_bytes, weights=True)
    src = graphgen.random_sources(g, 1, seed=2)[0]
    t = time.perf_counter()
    lv = oracle.bfs(g.row_ptr, g.col, src)
    t_bfs = time.perf_counter() - t
    t = time.perf_counter()
    oracle.dijkstra(g.row_ptr, g.col, g.weights, src)
    t_sssp = time.perf_counter() - t
    t = time.perf_counter()
    oracle.cc(g.row_ptr, g.col)
    t_cc = time.perf_counter() - t
    reached = oracle.reached_edges(g.row_ptr, lv)
    edges = 2 * reached + g.num_edges
    secs = t_bfs + t_sssp + t_cc
    return {
        "value": edges / secs / 1e9, "unit": "GTEPS", "cores": 1, "kind": "oracle",
        "sample": (f"single-threaded oracle (queue BFS + binary-heap Dijkstra + union-find CC) on "
                   f"R-MAT scale {scale} from the same generator and seeds, one source; "
                   f"{secs:.1f}s of CPU (bfs {t_bfs:.1f}s, sssp {t_sssp:.1f}s, cc {t_cc:.1f}s)"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["kron", "uniform"], default="kron")
    ap.add_argument("--scale", type=int, default=27)
    ap.add_argument("--col-bytes", type=int, choices=[4, 8], default=8)
    ap.add_argument("--sources", type=int, default=8)
    ap.add_argument("--scheduler", default="heuristic")
    ap.add_argument("--request-unit", type=int, default=256)
    ap.add_argument("--no-arms", action="store_true", help="skip the HBM/managed comparison runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-source batched runs")
    ap.add_argument("--noncoherent", action="store_true", help="pin the edge arrays non-coherent")
    ap.add_argument("--no-learned", action="store_true", help="skip the scheduler comparison")
    ap.add_argument("--cpu-scale", type=int, default=24)
    ap.add_argument("--calib-bytes", type=int, default=1 << 30)
    ap.add_argument("--calibrate-only", action="store_true",
                    help="run the link calibration (plain zero-copy read kernels) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
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
    peak = profile["memcpy_GBps"]
    log(f"[bench] link: memcpy {peak:.2f} GB/s, seq read {profile['seq_read_GBps']}, "
        f"R {profile['request_unit']} B, latency {profile['latency_us']:.2f} us")
    if args.calibrate_only:
        print(json.dumps({"link_profile": profile}), flush=True)
        return
    os.environ.setdefault("GG_VERBOSE", "1")  # generator prints its phases (progress)

    rp, col, w = build_graph(args, E, graphgen)
    V = rp.shape[0] - 1
    M = int(rp[-1])
    csr = graphgen.CSR(rp, col.array)
    sources = graphgen.random_sources(csr, args.sources, seed=2)
    out = torch.empty(V, dtype=torch.int32, device="cuda")

    G = E.Graph(rp, col, w, placement="host_zero_copy", symmetric=True, borrow=True)
    G.set_request_unit(args.request_unit)
    if args.scheduler.isdigit():
        G.set_variant(int(args.scheduler))
    else:
        G.set_scheduler(args.scheduler)

    for i in range(args.warmup):
        run_step(G, sources[i % len(sources)], out, torch)
        log(f"[bench] warmup step {i} done")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for i in range(args.steps):
        steps.append((sources[i % len(sources)], run_step(G, sources[i % len(sources)], out, torch)))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for i, (s, r) in enumerate(steps):
        log(f"[bench] step {i} src={s}: bfs {r['bfs']['total_ms']:.1f} ms, sssp {r['sssp']['total_ms']:.1f} ms, "
            f"cc {r['cc']['total_ms']:.1f} ms")

    # --- throughput ---
    teps_edges = 0
    per = {a: {"ms": 0.0, "edges": 0, "scan_ms": 0.0, "bytes": 0} for a in ("bfs", "sssp", "cc")}
    kernels = {}
    for s, r in steps:
        reached = r["bfs"]["edges_scanned"]  # BFS expands every reached vertex once
        for a in ("bfs", "sssp", "cc"):
            st = r[a]
            e = M if a == "cc" else reached
            teps_edges += e
            per[a]["ms"] += st["total_ms"]
            per[a]["edges"] += e
            per[a]["scan_ms"] += st["expand_ms"]
            per[a]["bytes"] += st["useful_link_bytes"]
            eb = args.col_bytes + (4 if a == "sssp" else 0)
            for v, ms, ed in zip(st["level_variant"], st["level_ms"], st["level_edges"]):
                k = kernel_key(a, v, args.col_bytes)
                kk = kernels.setdefault(k, {"ms": 0.0, "bytes": 0, "launches": 0})
                kk["ms"] += ms
                kk["bytes"] += ed * eb
                kk["launches"] += 1
    value = teps_edges / elapsed / 1e9
    link_bytes = sum(p["bytes"] for p in per.values())
    scan_ms = sum(p["scan_ms"] for p in per.values())
    link_gbps = link_bytes / (scan_ms * 1e6) if scan_ms else 0.0
    dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["ms"])
    achieved = dom["bytes"] / (dom["ms"] * 1e6)

    result = {
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
        "data": "synthetic (seeded R-MAT generator; no dataset)",
        "config": {
            "workload": (f"{'Kronecker/R-MAT' if args.workload == 'kron' else 'uniform'} scale {args.scale}, "
                         f"edgefactor 16, u{8 * args.col_bytes} col + u32 weights in pinned host "
                         f"zero-copy memory; BFS+SSSP+CC per step"),
            "vertices": V, "directed_edges": M, "col_bytes": args.col_bytes,
            "placement": "host_zero_copy", "sources": sources, "scheduler": args.scheduler,
            "request_unit": args.request_unit,
        },
        "per_algorithm": {
            a: {"gteps": round(p["edges"] / (p["ms"] * 1e6), 4) if p["ms"] else None,
                "link_GBps": round(p["bytes"] / (p["scan_ms"] * 1e6), 2) if p["scan_ms"] else None,
                "ms_per_run": round(p["ms"] / len(steps), 2)}
            for a, p in per.items()
        },
        "host_link": {
            "scan_GBps": round(link_gbps, 2),
            "pinned_memcpy_peak_GBps": round(peak, 2),
            "pct_of_pinned_peak": round(100 * link_gbps / peak, 1),
            "request_unit_measured": profile["request_unit"],
            "kernel_seq_read_GBps": round(max(profile["seq_read_GBps"].values()), 2),
            "latency_us": round(profile["latency_us"], 3),
        },
        "roofline": {
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
        },
    }
    ct = counter_traffic(dom_name)
    if ct is not None:
        # host-link bytes per launch from TCC_EA0_RDREQ_IO_32B x 32 B (copy-kernel factor applied);
        # FETCH_SIZE (scaled) + WRITE_SIZE per launch beside it for the HBM side
        result["roofline"]["traffic"] = round(ct["link_bytes_per_dispatch"])
        result["roofline"]["traffic_fetch_write"] = round(ct["fetch_bytes_per_dispatch_scaled"]
                                                          + ct["write_bytes_per_dispatch"])
        result["roofline"]["traffic_source"] = "profiles/counters_kron27_u64.json"

    # --- the two systems patterns, each against the plain method on this GPU ---
    plain_bfs_ms = per["bfs"]["ms"] / len(steps)
    plain_sssp_ms = per["sssp"]["ms"] / len(steps)
    if not args.no_batch:
        srcs64 = graphgen.degree_spread_sources(rp, 64, seed=4)
        out64 = torch.empty(len(srcs64) * V, dtype=torch.int32, device="cuda")
        G.bfs_batch(srcs64, out64)
        sb = G.stats()
        G.sssp_batch(srcs64, out64)
        ss = G.stats()
        del out64
        result["batched"] = {
            "sources": len(srcs64), "source_degrees": "log-spaced 1..max (seed 4)",
            "bfs_ms": round(sb["total_ms"], 1), "sssp_ms": round(ss["total_ms"], 1),
            "plain_bfs_ms_x_sources": round(plain_bfs_ms * len(srcs64), 1),
            "plain_sssp_ms_x_sources": round(plain_sssp_ms * len(srcs64), 1),
            "bfs_speedup_vs_plain": round(plain_bfs_ms * len(srcs64) / sb["total_ms"], 2),
            "sssp_speedup_vs_plain": round(plain_sssp_ms * len(srcs64) / ss["total_ms"], 2),
            "params": G.get_batch_params(),
        }
        log(f"[bench] batched: {result['batched']}")
    weights = os.path.join(ROOT, "paper_2006_06890_amd", "scheduler_weights.json")
    if not args.no_learned:
        sched = {}
        modes = [("fixed_v3", 3), ("heuristic", "heuristic")]
        if os.path.exists(weights):
            G.set_scheduler_weights(json.load(open(weights))["params"])
            modes.append(("learned", "learned"))
        for name, mode in modes:
            if isinstance(mode, int):
                G.set_variant(mode)
            else:
                G.set_scheduler(mode)
            r = run_step(G, sources[0], out, torch)
            sched[name] = {a: round(r[a]["total_ms"], 1) for a in r}
            sched[name]["step_ms"] = round(sum(r[a]["total_ms"] for a in r), 1)
        result["schedulers"] = sched
        log(f"[bench] schedulers (one step, source {sources[0]}): {sched}")

    G.close()
    if not args.no_arms:
        arms = {}
        for placement in ("hbm", "managed"):
            try:
                H = E.Graph(rp, col.array, w.array, placement=placement, symmetric=True)
            except E.EmogiError as e:
                arms[placement] = {"status": str(e)}
                continue
            H.set_scheduler("heuristic")
            r = run_step(H, sources[0], out, torch)
            reached = r["bfs"]["edges_scanned"]
            ms = sum(r[a]["total_ms"] for a in r)
            arms[placement] = {
                "gteps": round((2 * reached + M) / (ms * 1e6), 4),
                "bfs_gteps": round(reached / (r["bfs"]["total_ms"] * 1e6), 4),
                "sssp_ms": round(r["sssp"]["total_ms"], 2),
                "cc_ms": round(r["cc"]["total_ms"], 2),
            }
            H.close()
            log(f"[bench] arm {placement}: {arms[placement]}")
        result["arms"] = arms

    col.free()
    w.free()
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the CPU sample")
        result["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
