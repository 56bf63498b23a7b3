"""Trains the per-level variant scheduler and evaluates it on held-out graphs.

1. Harvest: on training graphs shaped like the benchmark configurations
   (R-MAT scale 16 with 4-byte ids; R-MAT with 8-byte ids; uniform random with
   4-byte ids; scales up to 24 with graph seeds 1, 2, 3, and R-MAT 27 / uniform
   2^27 at seed 2), run BFS, SSSP and CC in probe mode: every
   level is run with all six access variants on the same state, and the 16
   frontier features plus the six kernel times are kept.  The label of a level
   is its fastest variant.
2. Train: the 16-64-64-6 network is trained on the GPU by the library's own
   HIP kernels (emogi_mlp_train: forward, softmax cross-entropy, backward,
   Adam), from a seeded He-uniform initialisation.  The range of every
   feature over the training levels is kept with the weights: outside it the
   library uses the heuristic (the network is not extrapolated).
3. Evaluate: on held-out locality-ordered power-law graphs (10^8 vertices,
   mean degree 36, exponent 2.1, runs of 1024; seeds 101-103),
   time each traversal (every BFS level top-down, so that the modes differ
   only in the access variant) with the fixed aligned-wave variant (the
   paper's choice), the built-in heuristic, the learned scheduler, and report
   the per-level best (sum over levels of the fastest variant's probe time).

Writes ``scheduler_weights.json`` next to this file:
``{"params": [5638 floats], "feature_lo": [16], "feature_hi": [16], "train": {...},
"eval": {...}}``.

Usage: python -m paper_2006_06890_amd.train_scheduler [--quick]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "scheduler_weights.json")


def log(*a):
    print("[train]", *a, flush=True)


PINNED_SCALE = 25  # graphs from this scale on are written straight into pinned memory


def eligible(X):
    """The straggler guard of the library's pick (k_mlp_pick) from the
    features: a thread per vertex (V0) only if every frontier list is below
    16 ids, a 16-lane group (V1) below 64, a wave (V2, V3) below 4096; the
    workgroup (V4) and the edge-balanced scan (V5) always.  X[:, 4 + b] > 0:
    some frontier vertex has a degree in bin b (<=1, [2,4), [4,8), [8,16),
    [16,64), [64,256), [256,4096), >=4096)."""
    X = np.asarray(X)
    has = [(X[:, 4 + b:12] > 0).any(axis=1) for b in range(8)]
    return np.stack([~has[4], ~has[5], ~has[7], ~has[7],
                     np.ones(X.shape[0], bool), np.ones(X.shape[0], bool)], axis=1)


class _PinnedGraph:
    """A generated graph exported into pinned host memory, used in place
    (borrowed) by the library: the benchmark-sized training graphs would
    otherwise need a second, copied edge array."""

    def __init__(self, E, h, col_bytes):
        V, M = h.num_vertices, h.num_edges
        self.row_ptr = np.empty(V + 1, dtype=np.uint64)
        self.col = E.PinnedArray(M, np.uint64 if col_bytes == 8 else np.uint32)
        self.weights = E.PinnedArray(M, np.uint32)
        h.export_into(self.row_ptr.ctypes.data, self.col.ptr, col_bytes, self.weights.ptr, 3)
        self.num_vertices = V

    def degrees(self):
        return np.diff(self.row_ptr)


def _graph(E, graphgen, spec):
    kind, size, col_bytes, seed = spec
    if kind == "rmat":
        h = graphgen.rmat(size, 16, seed=seed)
    elif kind == "uniform":
        h = graphgen.uniform(size, (1 << size) * 32, seed=seed)
    else:
        h = graphgen.power_law(size, seed=seed)
    if kind != "powerlaw" and size >= PINNED_SCALE:
        g = _PinnedGraph(E, h, col_bytes)
    else:
        g = h.to_csr(col_bytes, weights=True)
    h.free()
    return g


def _open(E, g):
    borrow = isinstance(g, _PinnedGraph)
    return E.Graph(g.row_ptr, g.col, g.weights, placement="host_zero_copy", symmetric=True, borrow=borrow)


def _sources(g, k, seed):
    deg = g.degrees()
    rng = np.random.Generator(np.random.PCG64(seed))
    nz = np.flatnonzero(deg > 0)
    return [int(x) for x in rng.choice(nz, size=min(k, nz.shape[0]), replace=False)]


def _runs(G, g, out, algo, srcs):
    if algo == "cc":
        G.cc(out)
        yield G.stats()
    else:
        for s in srcs:
            getattr(G, algo)(s, out)
            yield G.stats()


def harvest(E, graphgen, specs, torch):
    X, T = [], []
    for spec in specs:
        t0 = time.time()
        g = _graph(E, graphgen, spec)
        out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
        with _open(E, g) as G:
            G.set_scheduler("probe", record=True)
            for algo, k in (("bfs", 3), ("sssp", 2), ("cc", 1)):
                for st in _runs(G, g, out, algo, _sources(g, k, spec[3] + 17)):
                    for f, p in zip(st["level_features"], st["level_probe_ms"]):
                        X.append(f)
                        T.append(p)
                    log(f"  {spec} {algo}: {len(st['level_probe_ms'])} levels ({time.time() - t0:.1f}s)")
        log(f"harvested {spec}: {len(X)} levels so far ({time.time() - t0:.1f}s)")
        del g, out  # before the next graph is generated (the largest are 50-70 GB)
    return np.array(X, dtype=np.float32), np.array(T, dtype=np.float32)


def he_uniform(seed):
    from_shapes = [(64, 16), (64,), (64, 64), (64,), (6, 64), (6,)]
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in from_shapes:
        if len(s) == 2:
            lim = np.sqrt(6.0 / s[1])
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def evaluate(E, graphgen, specs, params, torch, lo=None, hi=None):
    rows = []
    for spec in specs:
        g = _graph(E, graphgen, spec)
        out = torch.empty(g.num_vertices, dtype=torch.int32, device="cuda")
        srcs = _sources(g, 2, spec[3] + 5)
        with _open(E, g) as G:
            G.set_scheduler_weights(params, lo, hi)
            G.set_direction("top_down")  # the modes differ only in the access variant
            for algo in ("bfs", "sssp", "cc"):
                res = {}
                for mode in ("fixed_v3", "heuristic", "learned", "probe"):
                    if mode == "fixed_v3":
                        G.set_variant(3)
                    else:
                        G.set_scheduler(mode, record=(mode == "learned"))
                    scan = 0.0
                    total = 0.0
                    best = 0.0
                    picks = []
                    for st in _runs(G, g, out, algo, srcs):
                        scan += st["expand_ms"]
                        total += st["total_ms"]
                        if mode == "probe":
                            best += float(np.sum(np.min(np.array(st["level_probe_ms"]).reshape(-1, 6), axis=1)))
                        if mode == "learned":
                            picks += st["level_variant"]
                    # scan-kernel time (what the choice affects); end-to-end beside it
                    res[mode] = best if mode == "probe" else scan
                    if mode != "probe":
                        res[mode + "_total"] = total
                    if mode == "learned":
                        res["learned_picks"] = np.bincount(picks, minlength=6).tolist()
                row = {"graph": list(spec), "algo": algo, "ms": {k: round(v, 3) for k, v in res.items()
                                                                if k != "learned_picks"},
                       "learned_picks": res["learned_picks"]}
                rows.append(row)
                log(f"eval {spec} {algo}: {row['ms']} picks {row['learned_picks']}")
        del g, out
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="small graphs (a smoke run)")
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--eval-vertices", type=int, default=100_000_000)
    ap.add_argument("--out", default=WEIGHTS, help="where to write the weights JSON")
    ap.add_argument("--harvest-out", metavar="NPZ", help="also save the harvested levels (features, times)")
    ap.add_argument("--harvest-set", choices=("all", "small", "large"), default="all",
                    help="harvest every training graph, those below scale 25, or those from 25 on")
    ap.add_argument("--harvest-only", action="store_true", help="stop after saving the harvest (--harvest-out)")
    ap.add_argument("--harvest-in", metavar="NPZ", nargs="+",
                    help="skip harvesting: train on levels saved by --harvest-out (several files are joined)")
    ap.add_argument("--eval-only", metavar="WEIGHTS_JSON",
                    help="skip harvesting and training: evaluate these weights and write them, "
                         "with the new evaluation rows, to --out")
    args = ap.parse_args()

    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import graphgen
    import paper_2006_06890_amd as E

    if args.quick:
        train_specs = [("rmat", 14, 4, 1), ("rmat", 14, 8, 2), ("uniform", 14, 4, 3)]
        eval_specs = [("powerlaw", 1 << 16, 4, 101)]
    else:
        train_specs = []
        for seed in (1, 2, 3):
            train_specs += [("rmat", 16, 4, seed), ("rmat", 21, 8, seed), ("rmat", 22, 4, seed),
                            ("rmat", 24, 8, seed), ("uniform", 20, 4, seed), ("uniform", 22, 4, seed),
                            ("uniform", 24, 4, seed)]
        # the benchmark's shapes at full size (R-MAT 27 with 8-byte ids, uniform
        # 2^27 with 4-byte ids), on a graph seed the benchmark does not use
        train_specs += [("rmat", 27, 8, 2), ("uniform", 27, 4, 2)]
        eval_specs = [("powerlaw", args.eval_vertices, 4, s) for s in (101, 102, 103)]

    if args.eval_only:
        doc = json.load(open(args.eval_only))
        params = np.asarray(doc["params"], dtype=np.float32)
        doc["eval"] = evaluate(E, graphgen, eval_specs, params, torch, doc.get("feature_lo"), doc.get("feature_hi"))
        json.dump(doc, open(args.out, "w"))
        log(f"wrote {args.out}")
        return

    if args.harvest_in:
        parts = [np.load(f) for f in args.harvest_in]
        X = np.concatenate([d["X"] for d in parts])
        T = np.concatenate([d["T"] for d in parts])
        train_specs = [json.loads(str(x)) for d in parts for x in d["specs"]]
    else:
        if args.harvest_set != "all":
            large = args.harvest_set == "large"
            train_specs = [sp for sp in train_specs if (sp[1] >= PINNED_SCALE) == large]
        X, T = harvest(E, graphgen, train_specs, torch)
        if args.harvest_out:
            np.savez(args.harvest_out, X=X, T=T, specs=np.array([json.dumps(list(x)) for x in train_specs]))
            log(f"saved {X.shape[0]} levels to {args.harvest_out}")
        if args.harvest_only:
            return
    # The label is the fastest variant the library's straggler guard lets the
    # network pick for that frontier (a worker narrower than the frontier's
    # longest list is not eligible; see k_mlp_pick): at inference the argmax
    # is taken over the same variants.
    ok = eligible(X)
    Te = np.where(ok, T, np.inf)
    y = np.argmin(Te, axis=1).astype(np.int32)
    log(f"{X.shape[0]} levels; label histogram {np.bincount(y, minlength=6).tolist()}")
    # Cost-sensitive sampling: a level is repeated in proportion to what a wrong
    # pick among its eligible variants can cost there (slowest - fastest, in
    # units of 0.05 ms, at most 40 copies), so cheap levels with noisy labels
    # weigh little.
    spread = np.where(ok, T, -np.inf).max(axis=1) - Te.min(axis=1)
    copies = 1 + np.minimum(40, np.floor(spread / 0.05)).astype(np.int64)
    Xw, yw = np.repeat(X, copies, axis=0), np.repeat(y, copies)
    # replicate small datasets so every epoch has several full minibatches
    reps = max(1, 2048 // Xw.shape[0])
    Xr, yr = np.tile(Xw, (reps, 1)), np.tile(yw, reps)
    p0 = he_uniform(7)
    params, hist = E.emogi.mlp_train(Xr, yr, p0, epochs=args.epochs, batch=min(256, Xr.shape[0]),
                                     lr=1e-3, seed=11)
    log(f"loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    # the network is only trusted inside the feature range it was trained on
    lo, hi = X.min(axis=0).astype(np.float32), X.max(axis=0).astype(np.float32)
    rows = evaluate(E, graphgen, eval_specs, params, torch, lo, hi)
    json.dump({
        "params": [float(x) for x in params],
        "feature_lo": [float(x) for x in lo],
        "feature_hi": [float(x) for x in hi],
        "train": {"specs": train_specs, "levels": int(X.shape[0]),
                  "label_hist": np.bincount(y, minlength=6).tolist(),
                  "labels": "fastest eligible variant (straggler guard)",
                  "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
                  "epochs": args.epochs},
        "eval": rows,
    }, open(args.out, "w"))
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
