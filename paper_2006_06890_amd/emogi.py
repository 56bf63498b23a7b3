"""Python binding of the zero-copy traversal library (``include/emogi.h``).

Argument marshalling only: every step of a traversal runs in the HIP kernels
of ``libemogi.so``.  PyTorch supplies device memory (output tensors) and
streams.  The binding fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libemogi.so")

PLACEMENTS = {"hbm": 0, "host_zero_copy": 1, "managed": 2}
F_SYMMETRIC, F_VALIDATE, F_BORROW, F_PIN_NONCOHERENT = 0x1, 0x2, 0x4, 0x8
SCHED_HEURISTIC, SCHED_LEARNED = 16, 17
VARIANTS = ["V0_thread", "V1_group16", "V2_wave", "V3_wave_aligned", "V4_block", "V5_balanced"]
N_SCHED_PARAMS = 5638
INF = 0xFFFFFFFF
MAX_LEVEL_STATS = 512

STATUS = {
    0: "ok", -1: "invalid argument", -2: "out of host memory", -3: "out of device memory",
    -4: "HIP runtime error", -5: "graph is not symmetric", -6: "distance overflow",
    -7: "iteration cap reached", -8: "unsupported",
}


class EmogiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_uint32),
        ("variant_hist", ctypes.c_uint32 * 6),
        ("vertices_expanded", ctypes.c_uint64),
        ("edges_scanned", ctypes.c_uint64),
        ("useful_link_bytes", ctypes.c_uint64),
        ("request_bytes", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
        ("expand_ms", ctypes.c_double),
        ("expand_launches", ctypes.c_uint32),
        ("request_unit", ctypes.c_uint32),
        ("level_count", ctypes.c_uint32),
        ("level_variant", ctypes.c_uint8 * MAX_LEVEL_STATS),
        ("level_frontier", ctypes.c_uint32 * MAX_LEVEL_STATS),
        ("level_ms", ctypes.c_float * MAX_LEVEL_STATS),
        ("level_edges", ctypes.c_uint64 * MAX_LEVEL_STATS),
    ]

    def as_dict(self):
        n = self.level_count
        return {
            "iterations": self.iterations,
            "variant_hist": list(self.variant_hist),
            "vertices_expanded": self.vertices_expanded,
            "edges_scanned": self.edges_scanned,
            "useful_link_bytes": self.useful_link_bytes,
            "request_bytes": self.request_bytes,
            "total_ms": self.total_ms,
            "expand_ms": self.expand_ms,
            "expand_launches": self.expand_launches,
            "request_unit": self.request_unit,
            "level_variant": list(self.level_variant[:n]),
            "level_frontier": list(self.level_frontier[:n]),
            "level_ms": list(self.level_ms[:n]),
            "level_edges": list(self.level_edges[:n]),
        }


_lib = None


def lib():
    """Loads libemogi.so; raises if it has not been built (no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2006_06890_amd.build`"
            )
        L = ctypes.CDLL(LIB_PATH)
        p, u64, u32, i32, sz = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                ctypes.c_int, ctypes.c_size_t)
        sig = {
            "emogi_host_alloc": (i32, [sz, u32, ctypes.POINTER(ctypes.c_void_p)]),
            "emogi_host_free": (i32, [p]),
            "emogi_graph_create": (i32, [p, u64, p, u32, p, i32, u32, ctypes.POINTER(ctypes.c_void_p)]),
            "emogi_graph_destroy": (i32, [p]),
            "emogi_set_request_unit": (i32, [p, u32]),
            "emogi_set_scheduler": (i32, [p, i32]),
            "emogi_set_scheduler_weights": (i32, [p, p, sz]),
            "emogi_bfs": (i32, [p, u64, p, p]),
            "emogi_sssp": (i32, [p, u64, p, p]),
            "emogi_cc": (i32, [p, p, p]),
            "emogi_last_stats": (i32, [p, ctypes.POINTER(Stats)]),
            "emogi_num_vertices": (u64, [p]),
            "emogi_num_edges": (u64, [p]),
            "emogi_strerror": (ctypes.c_char_p, [i32]),
            "emogi_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != 0:
        msg = lib().emogi_last_error().decode(errors="replace")
        raise EmogiError(code, msg)


class PinnedArray:
    """Pinned, GPU-mapped host memory from emogi_host_alloc, viewed as numpy."""

    def __init__(self, count, dtype, noncoherent=False):
        self.dtype = np.dtype(dtype)
        self.count = int(count)
        nbytes = max(1, self.count * self.dtype.itemsize)
        ptr = ctypes.c_void_p()
        check(lib().emogi_host_alloc(nbytes, F_PIN_NONCOHERENT if noncoherent else 0,
                                     ctypes.byref(ptr)))
        self.ptr = ptr.value
        buf = (ctypes.c_char * nbytes).from_address(self.ptr)
        self.array = np.frombuffer(buf, dtype=self.dtype, count=self.count)

    def free(self):
        if self.ptr:
            self.array = None
            check(lib().emogi_host_free(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _addr(a):
    if a is None:
        return None
    if isinstance(a, PinnedArray):
        return a.ptr
    return a.ctypes.data


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Graph:
    """A CSR graph placed for traversal (``emogi_graph_create``).

    row_ptr: uint64[V+1]; col: uint32|uint64[E] (numpy or PinnedArray);
    weights: uint32[E] or None.  With ``borrow`` the edge arrays must be
    PinnedArray objects and are used in place (host zero-copy only).
    """

    def __init__(self, row_ptr, col, weights=None, placement="host_zero_copy",
                 symmetric=False, validate=False, borrow=False, noncoherent=False):
        rp = np.ascontiguousarray(row_ptr, dtype=np.uint64)
        col_arr = col.array if isinstance(col, PinnedArray) else np.ascontiguousarray(col)
        if col_arr.dtype not in (np.uint32, np.uint64):
            raise TypeError("col must be uint32 or uint64")
        if weights is not None and not isinstance(weights, PinnedArray):
            weights = np.ascontiguousarray(weights, dtype=np.uint32)
        if not isinstance(col, PinnedArray):
            col = col_arr
        self._keep = (rp, col, weights)
        flags = ((F_SYMMETRIC if symmetric else 0) | (F_VALIDATE if validate else 0)
                 | (F_BORROW if borrow else 0) | (F_PIN_NONCOHERENT if noncoherent else 0))
        h = ctypes.c_void_p()
        V = rp.shape[0] - 1
        check(lib().emogi_graph_create(rp.ctypes.data, V, _addr(col), col_arr.dtype.itemsize,
                                       _addr(weights), PLACEMENTS[placement], flags,
                                       ctypes.byref(h)))
        self._h = h.value
        self.num_vertices = V
        self.num_edges = int(rp[-1])
        self.col_bytes = col_arr.dtype.itemsize
        self.placement = placement
        if not borrow:
            self._keep = None  # copied by the library

    # -- configuration -------------------------------------------------------
    def set_variant(self, v):
        check(lib().emogi_set_scheduler(self._h, int(v)))

    def set_scheduler(self, mode):
        modes = {"heuristic": SCHED_HEURISTIC, "learned": SCHED_LEARNED}
        check(lib().emogi_set_scheduler(self._h, modes[mode] if isinstance(mode, str) else int(mode)))

    def set_scheduler_weights(self, params):
        if params is None:
            check(lib().emogi_set_scheduler_weights(self._h, None, 0))
            return
        p = np.ascontiguousarray(params, dtype=np.float32)
        check(lib().emogi_set_scheduler_weights(self._h, p.ctypes.data, p.shape[0]))

    def set_request_unit(self, nbytes):
        check(lib().emogi_set_request_unit(self._h, int(nbytes)))

    # -- traversals ----------------------------------------------------------
    def _out(self, out):
        import torch
        if out is None:
            out = torch.empty(max(1, self.num_vertices), dtype=torch.int32, device="cuda")
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous():
            raise TypeError("output must be a contiguous int32 CUDA/HIP tensor")
        if out.numel() < self.num_vertices:
            raise ValueError("output tensor too small")
        return out

    def bfs(self, src, out=None, stream=None):
        out = self._out(out)
        check(lib().emogi_bfs(self._h, int(src), out.data_ptr(), _stream_handle(stream)))
        return out

    def sssp(self, src, out=None, stream=None):
        out = self._out(out)
        check(lib().emogi_sssp(self._h, int(src), out.data_ptr(), _stream_handle(stream)))
        return out

    def cc(self, out=None, stream=None):
        out = self._out(out)
        check(lib().emogi_cc(self._h, out.data_ptr(), _stream_handle(stream)))
        return out

    def stats(self):
        s = Stats()
        check(lib().emogi_last_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            check(lib().emogi_graph_destroy(self._h))
            self._h = None
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def to_u32(t):
    """int32 device tensor -> uint32 numpy array on the host."""
    return t.detach().cpu().numpy().view(np.uint32)
