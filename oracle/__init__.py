"""Oracle for the zero-copy graph traversal: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2006_06890_amd``) and never imports it.

Contents
--------
* ``bfs``, ``dijkstra``, ``cc``: the plain definitions of BFS levels, integer
  shortest-path distances and min-id component labels (EMOGI Sec. 2.1,
  Algorithm 1; Sec. 5.1 lists BFS, SSSP and CC as the evaluated workloads),
  written in ``oracle.c`` (queue BFS, binary-heap Dijkstra, union-find).
* ``floyd_warshall``, ``cc_closure``: independent all-pairs / closure
  computations for tiny graphs.
* ``certify_distances``, ``certify_cc``: linear-time certificates used where a
  full run is too slow.
* ``pagerank``: the power iteration of PageRank (EMOGI's fourth workload,
  Sec. 5.1) in fixed point, so every sum is exact.
* ``request_bytes``: host-link bytes of a request-granular scan (Sec. 3.3,
  Sec. 4.3.2), ``reached_edges``: the TEPS numerator.
* ``mlp``: fp64 reference of the per-level scheduler network.
* ``linkmodel``: the closed-form link arithmetic of Sec. 3.3.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
INF = 0xFFFFFFFF

_lib = None


def build(force=False):
    """Compile oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-Wall", "-Werror", "-shared", "-fPIC",
             _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
        sig = {
            "oracle_validate_csr": (i32, [u64, p, p, i32, i32, i32]),
            "oracle_bfs": (i32, [u64, p, p, i32, u64, p]),
            "oracle_dijkstra": (i32, [u64, p, p, i32, p, u64, p]),
            "oracle_cc": (i32, [u64, p, p, i32, p]),
            "oracle_floyd_warshall": (i32, [u64, p, p, i32, p, p]),
            "oracle_cc_closure": (i32, [u64, p, p, i32, p]),
            "oracle_certify_distances": (i32, [u64, p, p, i32, p, u64, p]),
            "oracle_certify_cc": (i32, [u64, p, p, i32, p]),
            "oracle_request_bytes": (u64, [u64, p, i32, u64, p]),
            "oracle_reached_edges": (u64, [u64, p, p]),
            "oracle_pagerank": (i32, [u64, p, p, i32, ctypes.c_uint32, u64, ctypes.c_uint32, p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return None if a is None else a.ctypes.data


def _csr(row_ptr, col):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    col = np.asarray(col)
    if col.dtype not in (np.uint32, np.uint64):
        raise OracleError("col must be uint32 or uint64")
    col = np.ascontiguousarray(col)
    V = row_ptr.shape[0] - 1
    if V < 0 or int(row_ptr[-1]) != col.shape[0]:
        raise OracleError("row_ptr[V] must equal len(col)")
    return V, row_ptr, col, col.dtype.itemsize


def _w(weights, E):
    if weights is None:
        return None
    w = np.ascontiguousarray(weights, dtype=np.uint32)
    if w.shape[0] != E:
        raise OracleError("weights must have one entry per edge")
    return w


def validate_csr(row_ptr, col, simple=False, symmetric=False):
    """0 when the CSR is well formed; otherwise the failed check number."""
    V, rp, c, cb = _csr(row_ptr, col)
    return _load().oracle_validate_csr(V, _ptr(rp), _ptr(c), cb, int(simple), int(symmetric))


def bfs(row_ptr, col, src):
    V, rp, c, cb = _csr(row_ptr, col)
    out = np.empty(V, dtype=np.uint32)
    rc = _load().oracle_bfs(V, _ptr(rp), _ptr(c), cb, src, _ptr(out))
    if rc:
        raise OracleError(f"oracle_bfs failed ({rc})")
    return out


def dijkstra(row_ptr, col, weights, src):
    """Returns uint32 distances; raises OracleError(-6) on 32-bit overflow."""
    V, rp, c, cb = _csr(row_ptr, col)
    w = _w(weights, c.shape[0])
    out = np.empty(V, dtype=np.uint32)
    rc = _load().oracle_dijkstra(V, _ptr(rp), _ptr(c), cb, _ptr(w), src, _ptr(out))
    if rc == -6:
        raise OracleError("distance overflow (-6)")
    if rc:
        raise OracleError(f"oracle_dijkstra failed ({rc})")
    return out


def cc(row_ptr, col):
    V, rp, c, cb = _csr(row_ptr, col)
    out = np.empty(V, dtype=np.uint32)
    rc = _load().oracle_cc(V, _ptr(rp), _ptr(c), cb, _ptr(out))
    if rc:
        raise OracleError(f"oracle_cc failed ({rc})")
    return out


def pagerank(row_ptr, col, frac_bits, damping_fixed, iters):
    """Fixed-point PageRank after ``iters`` iterations (oracle_pagerank):
    uint64 scores with ``frac_bits`` fractional bits, damping factor
    ``damping_fixed`` / 2^frac_bits."""
    V, rp, c, cb = _csr(row_ptr, col)
    out = np.empty(V, dtype=np.uint64)
    rc = _load().oracle_pagerank(V, _ptr(rp), _ptr(c), cb, frac_bits, damping_fixed, iters, _ptr(out))
    if rc:
        raise OracleError(f"oracle_pagerank failed ({rc})")
    return out


def floyd_warshall(row_ptr, col, weights=None):
    """All-pairs distances (uint64, UINT64_MAX unreachable); tiny graphs only."""
    V, rp, c, cb = _csr(row_ptr, col)
    if V > 512:
        raise OracleError("floyd_warshall is for tiny graphs")
    w = _w(weights, c.shape[0])
    D = np.empty((V, V), dtype=np.uint64)
    _load().oracle_floyd_warshall(V, _ptr(rp), _ptr(c), cb, _ptr(w), _ptr(D))
    return D


def cc_closure(row_ptr, col):
    V, rp, c, cb = _csr(row_ptr, col)
    if V > 2048:
        raise OracleError("cc_closure is for tiny graphs")
    out = np.empty(V, dtype=np.uint32)
    _load().oracle_cc_closure(V, _ptr(rp), _ptr(c), cb, _ptr(out))
    return out


def certify_distances(row_ptr, col, src, dist, weights=None):
    """0 iff ``dist`` is exactly the distance vector from ``src`` (w >= 1)."""
    V, rp, c, cb = _csr(row_ptr, col)
    w = _w(weights, c.shape[0])
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    return _load().oracle_certify_distances(V, _ptr(rp), _ptr(c), cb, _ptr(w), src, _ptr(d))


def certify_cc(row_ptr, col, labels):
    V, rp, c, cb = _csr(row_ptr, col)
    lab = np.ascontiguousarray(labels, dtype=np.uint32)
    return _load().oracle_certify_cc(V, _ptr(rp), _ptr(c), cb, _ptr(lab))


def request_bytes(row_ptr, elem_bytes, R, mask=None):
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    return int(_load().oracle_request_bytes(rp.shape[0] - 1, _ptr(rp), elem_bytes, R, _ptr(m)))


def reached_edges(row_ptr, dist):
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    return int(_load().oracle_reached_edges(rp.shape[0] - 1, _ptr(rp), _ptr(d)))
