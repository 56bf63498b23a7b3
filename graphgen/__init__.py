"""Seeded synthetic CSR inputs shared by the tests, the bench and the oracle checks.

This package only makes inputs: it holds none of the traversal arithmetic,
never imports the oracle or the HIP library, and both sides take its output
as plain arrays.  The heavy generators (R-MAT/Kronecker, uniform, Chung-Lu)
live in ``csrgen.c`` (OpenMP); small hand-shaped graphs are built in numpy.
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrgen.c")
_LIB_PATH = os.path.join(_HERE, "libcsrgen.so")
_lib = None


def build(force=False):
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-std=gnu11", "-Wall", "-Werror", "-shared",
             "-fPIC", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p, u64, i32, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        sig = {
            "gg_rmat": (p, [i32, u64, dbl, dbl, dbl, u64, i32]),
            "gg_uniform": (p, [i32, u64, u64]),
            "gg_chung_lu": (p, [u64, u64, dbl, dbl, u64, i32]),
            "gg_from_edges": (p, [u64, u64, p, p]),
            "gg_num_vertices": (u64, [p]),
            "gg_num_edges": (u64, [p]),
            "gg_export": (i32, [p, p, p, i32, p, u64]),
            "gg_relabel": (i32, [p, p]),
            "gg_locality_order": (i32, [p, u64, u64, p]),
            "gg_free": (None, [p]),
            "gg_stream_key": (u64, [u64, u64]),
            "gg_draw": (u64, [u64, u64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


@dataclass
class CSR:
    """A CSR graph: row_ptr uint64[V+1], col uint32|uint64[E], weights uint32[E] or None."""
    row_ptr: np.ndarray
    col: np.ndarray
    weights: Optional[np.ndarray] = None
    symmetric: bool = False
    name: str = ""

    @property
    def num_vertices(self):
        return self.row_ptr.shape[0] - 1

    @property
    def num_edges(self):
        return int(self.row_ptr[-1])

    def degrees(self):
        return np.diff(self.row_ptr)


class Handle:
    """A generated graph still inside the C builder (list storage is uint32)."""

    def __init__(self, ptr, name):
        if not ptr:
            raise MemoryError("graph generation failed (host memory)")
        self._p = ptr
        self.name = name

    @property
    def num_vertices(self):
        return int(_load().gg_num_vertices(self._p))

    @property
    def num_edges(self):
        return int(_load().gg_num_edges(self._p))

    def export_into(self, row_ptr_addr, col_addr, col_bytes, weights_addr=None, weight_seed=3):
        """Writes the CSR into caller memory (addresses as ints, e.g. pinned buffers)."""
        rc = _load().gg_export(self._p, row_ptr_addr, col_addr, col_bytes,
                               weights_addr, weight_seed)
        if rc:
            raise ValueError("bad col_bytes")

    def to_csr(self, col_bytes=4, weights=False, weight_seed=3):
        V, E = self.num_vertices, self.num_edges
        rp = np.empty(V + 1, dtype=np.uint64)
        col = np.empty(E, dtype=np.uint32 if col_bytes == 4 else np.uint64)
        w = np.empty(E, dtype=np.uint32) if weights else None
        self.export_into(rp.ctypes.data, col.ctypes.data, col_bytes,
                         None if w is None else w.ctypes.data, weight_seed)
        return CSR(rp, col, w, symmetric=True, name=self.name)

    def locality_order(self, run=1024, seed=1):
        """Relabels in first-visit order from the top-degree vertex, runs of ``run`` ids shuffled."""
        new_id = np.empty(self.num_vertices, dtype=np.uint64)
        if _load().gg_locality_order(self._p, run, seed, new_id.ctypes.data):
            raise MemoryError("locality order failed")
        self.relabel(new_id)
        return new_id

    def relabel(self, new_id):
        new_id = np.ascontiguousarray(new_id, dtype=np.uint64)
        if _load().gg_relabel(self._p, new_id.ctypes.data):
            raise MemoryError("relabel failed")

    def free(self):
        if self._p:
            _load().gg_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rmat(scale, edgefactor=16, a=0.57, b=0.19, c=0.19, seed=1, permute=True):
    """R-MAT / Kronecker graph, symmetrised, simple, ascending lists."""
    return Handle(_load().gg_rmat(scale, edgefactor, a, b, c, seed, int(permute)),
                  f"rmat{scale}_ef{edgefactor}_s{seed}")


def uniform(scale, samples, seed=1):
    """2^scale vertices, ``samples`` uniform endpoint pairs, symmetrised, simple."""
    return Handle(_load().gg_uniform(scale, samples, seed), f"uniform{scale}_m{samples}_s{seed}")


def chung_lu(num_vertices, samples, gamma=2.1, i0=None, seed=1, permute=True):
    """Chung-Lu power-law graph: expected degree of i ~ (i + i0)^(-1/(gamma-1))."""
    if i0 is None:
        i0 = max(1.0, num_vertices ** 0.1)
    return Handle(_load().gg_chung_lu(num_vertices, samples, gamma, i0, seed, int(permute)),
                  f"chunglu{num_vertices}_g{gamma}_s{seed}")


def power_law(num_vertices, mean_degree=36, gamma=2.1, seed=1, run=1024):
    """Chung-Lu power law with ~mean_degree directed edges per vertex after
    symmetrising and deduplication, locality-ordered in runs of ``run``."""
    samples = int(num_vertices * mean_degree / 2 * 1.18)  # ~15% of hub pairs repeat
    h = chung_lu(num_vertices, samples, gamma=gamma, seed=seed, permute=False)  # relabelled below
    h.locality_order(run=run, seed=seed)
    h.name = f"powerlaw{num_vertices}_d{mean_degree}_g{gamma}_s{seed}"
    return h


def stream_key(seed, stream):
    return int(_load().gg_stream_key(seed, stream))


def draw(key, n):
    return int(_load().gg_draw(key, n))


# ---------------------------------------------------------------------------
# small hand-shaped graphs (numpy)
# ---------------------------------------------------------------------------

def from_edges(n, edges, symmetric=True, col_dtype=np.uint32, simple=True,
               weights=None):
    """CSR from an edge list.  With ``symmetric`` every (u,v) also adds (v,u).
    With ``simple`` self-loops and duplicate pairs are dropped.  ``weights``
    (per input edge) is carried to both directions; for duplicates the first
    kept entry after sorting wins."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = None if weights is None else np.asarray(weights, dtype=np.uint64).reshape(-1)
    if symmetric:
        e = np.concatenate([e, e[:, ::-1]], axis=0)
        if w is not None:
            w = np.concatenate([w, w])
    if simple and e.shape[0]:
        keep = e[:, 0] != e[:, 1]
        e = e[keep]
        if w is not None:
            w = w[keep]
    if e.shape[0]:
        order = np.lexsort((e[:, 1], e[:, 0]))
        e = e[order]
        if w is not None:
            w = w[order]
        if simple:
            first = np.ones(e.shape[0], dtype=bool)
            first[1:] = np.any(e[1:] != e[:-1], axis=1)
            e = e[first]
            if w is not None:
                w = w[first]
    counts = np.bincount(e[:, 0], minlength=n) if e.shape[0] else np.zeros(n, dtype=np.int64)
    rp = np.zeros(n + 1, dtype=np.uint64)
    rp[1:] = np.cumsum(counts)
    col = e[:, 1].astype(col_dtype) if e.shape[0] else np.zeros(0, dtype=col_dtype)
    wt = None if w is None else w.astype(np.uint32)
    return CSR(rp, col, wt, symmetric=symmetric)


def pair_weights(csr, seed=3):
    """Symmetric per-pair weights in [1, 255], same rule as the C builder."""
    key = stream_key(seed, 3)
    V = csr.num_vertices
    src = np.repeat(np.arange(V, dtype=np.uint64), np.diff(csr.row_ptr).astype(np.int64))
    dst = csr.col.astype(np.uint64)
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    packed = (lo << np.uint64(32)) | hi
    return _mix64_np(np.uint64(key) ^ packed).__mod__(np.uint64(255)).astype(np.uint32) + np.uint32(1)


def _mix64_np(z):
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def path(n, **kw):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], **kw)


def cycle(n, **kw):
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], **kw)


def star(n, **kw):
    return from_edges(n, [(0, i) for i in range(1, n)], **kw)


def complete(n, **kw):
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], **kw)


def grid(k, **kw):
    edges = []
    for r in range(k):
        for c in range(k):
            v = r * k + c
            if c + 1 < k:
                edges.append((v, v + 1))
            if r + 1 < k:
                edges.append((v, v + k))
    return from_edges(k * k, edges, **kw)


def binary_tree(n, **kw):
    return from_edges(n, [((i - 1) // 2, i) for i in range(1, n)], **kw)


def edgeless(n, **kw):
    return from_edges(n, np.zeros((0, 2), dtype=np.int64), **kw)


def disjoint_cliques(sizes, **kw):
    edges, base = [], 0
    for s in sizes:
        edges += [(base + i, base + j) for i in range(s) for j in range(i + 1, s)]
        base += s
    return from_edges(base, edges, **kw)


def random_sources(csr, count, seed):
    """``count`` distinct vertices with out-degree > 0, uniform, seeded."""
    deg = np.diff(csr.row_ptr)
    cand = np.flatnonzero(deg > 0)
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, cand.shape[0])
    return [int(x) for x in rng.choice(cand, size=count, replace=False)]


def degree_spread_sources(row_ptr, count, seed):
    """``count`` vertices whose degrees are closest to log-spaced targets in
    [1, max degree]; ties broken by a seeded shuffle; duplicates skipped."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.uint64)).astype(np.int64)
    order = np.random.Generator(np.random.PCG64(seed)).permutation(deg.shape[0])
    d = deg[order]
    pos = np.flatnonzero(d > 0)
    if pos.shape[0] == 0:
        return []
    dmax = int(d.max())
    targets = np.unique(np.round(np.geomspace(1, dmax, count)).astype(np.int64))
    by = np.argsort(d[pos], kind="stable")
    sd = d[pos][by]
    picked, seen = [], set()
    for t in targets:
        i = int(np.searchsorted(sd, t))
        for j in (i, i - 1, i + 1, i - 2, i + 2):
            if 0 <= j < sd.shape[0]:
                v = int(order[pos[by[j]]])
                if v not in seen:
                    seen.add(v)
                    picked.append(v)
                    break
    k = 0
    while len(picked) < min(count, pos.shape[0]) and k < pos.shape[0]:
        v = int(order[pos[k]])
        if v not in seen:
            seen.add(v)
            picked.append(v)
        k += 1
    return picked[:count]
