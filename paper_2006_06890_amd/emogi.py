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
F_SYMMETRIC, F_VALIDATE, F_BORROW, F_PIN_NONCOHERENT, F_PACK, F_WEIGHT_BOUND = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
SCHED_HEURISTIC, SCHED_LEARNED, SCHED_PROBE, SCHED_RECORD = 16, 17, 18, 0x100
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
        ("tier_edges", ctypes.c_uint64),
        ("weights_read", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
        ("expand_ms", ctypes.c_double),
        ("expand_launches", ctypes.c_uint32),
        ("request_unit", ctypes.c_uint32),
        ("level_count", ctypes.c_uint32),
        ("level_variant", ctypes.c_uint8 * MAX_LEVEL_STATS),
        ("level_frontier", ctypes.c_uint32 * MAX_LEVEL_STATS),
        ("level_ms", ctypes.c_float * MAX_LEVEL_STATS),
        ("level_edges", ctypes.c_uint64 * MAX_LEVEL_STATS),
        ("level_features", (ctypes.c_float * 16) * MAX_LEVEL_STATS),
        ("level_probe_ms", (ctypes.c_float * 6) * MAX_LEVEL_STATS),
        ("prep_ms", ctypes.c_double),
        ("reached_edges", ctypes.c_uint64),
        ("id_sector_bytes", ctypes.c_uint64),
        ("weight_sector_bytes", ctypes.c_uint64),
        ("levels_by_network", ctypes.c_uint32),
        ("bottom_up_levels", ctypes.c_uint32),
        ("level_direction", ctypes.c_uint8 * MAX_LEVEL_STATS),
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
            "tier_edges": self.tier_edges,
            "weights_read": self.weights_read,
            "total_ms": self.total_ms,
            "expand_ms": self.expand_ms,
            "expand_launches": self.expand_launches,
            "request_unit": self.request_unit,
            "level_variant": list(self.level_variant[:n]),
            "level_frontier": list(self.level_frontier[:n]),
            "level_ms": list(self.level_ms[:n]),
            "level_edges": list(self.level_edges[:n]),
            "level_features": [list(self.level_features[i]) for i in range(n)],
            "level_probe_ms": [list(self.level_probe_ms[i]) for i in range(n)],
            "prep_ms": self.prep_ms,
            "reached_edges": self.reached_edges,
            "id_sector_bytes": self.id_sector_bytes,
            "weight_sector_bytes": self.weight_sector_bytes,
            "levels_by_network": self.levels_by_network,
            "bottom_up_levels": self.bottom_up_levels,
            "level_direction": list(self.level_direction[:n]),
        }


CALIB_BLOCKS = 8
CALIB_WAVES = 10
CALIB_OFFSETS = 17


class LinkProfile(ctypes.Structure):
    _fields_ = [
        ("memcpy_GBps", ctypes.c_double),
        ("seq_read_GBps", ctypes.c_double * 3),
        ("block_bytes", ctypes.c_uint32 * CALIB_BLOCKS),
        ("rand_aligned_GBps", ctypes.c_double * CALIB_BLOCKS),
        ("rand_shift32_GBps", ctypes.c_double * CALIB_BLOCKS),
        ("request_unit", ctypes.c_uint32),
        ("latency_us", ctypes.c_double),
        ("buffer_bytes", ctypes.c_uint64),
        ("waves", ctypes.c_uint32 * CALIB_WAVES),
        ("waves_GBps", ctypes.c_double * CALIB_WAVES),
        ("knee_waves", ctypes.c_uint32),
        ("offset_bytes", ctypes.c_uint32 * CALIB_OFFSETS),
        ("offset_GBps", ctypes.c_double * CALIB_OFFSETS),
        ("nc_memcpy_GBps", ctypes.c_double),
        ("nc_seq_read_GBps", ctypes.c_double),
        ("nc_rand_GBps", ctypes.c_double),
        ("coh_rand_GBps", ctypes.c_double),
        ("hbm_read_GBps", ctypes.c_double),
        ("hbm_copy_GBps", ctypes.c_double),
    ]

    def as_dict(self):
        return {
            "memcpy_GBps": self.memcpy_GBps,
            "seq_read_GBps": dict(zip((4, 8, 16), list(self.seq_read_GBps))),
            "rand_aligned_GBps": dict(zip(list(self.block_bytes), list(self.rand_aligned_GBps))),
            "rand_shift32_GBps": dict(zip(list(self.block_bytes), list(self.rand_shift32_GBps))),
            "request_unit": self.request_unit,
            "latency_us": self.latency_us,
            "buffer_bytes": self.buffer_bytes,
            "waves_GBps": dict(zip(list(self.waves), list(self.waves_GBps))),
            "knee_waves": self.knee_waves,
            "offset_GBps": dict(zip(list(self.offset_bytes), list(self.offset_GBps))),
            "noncoherent": {"memcpy_GBps": self.nc_memcpy_GBps, "seq_read_GBps": self.nc_seq_read_GBps,
                            "rand_GBps": self.nc_rand_GBps, "coherent_rand_GBps": self.coh_rand_GBps},
            "hbm_read_GBps": self.hbm_read_GBps,
            "hbm_copy_GBps": self.hbm_copy_GBps,
        }


class BatchParams(ctypes.Structure):
    _fields_ = [
        ("hub_degree", ctypes.c_uint32),
        ("steps_per_graph", ctypes.c_uint32),
        ("blocks_per_cu", ctypes.c_uint32),
        ("use_graph", ctypes.c_uint32),
        ("sssp_delta", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchTrial(ctypes.Structure):
    _fields_ = [("params", BatchParams), ("ms", ctypes.c_float)]


class TrainConfig(ctypes.Structure):
    _fields_ = [
        ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float), ("batch", ctypes.c_uint32), ("epochs", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]


def mlp_forward(params, X, stream=None):
    """Logits [B,6] of the scheduler network; params/X are float32 device tensors."""
    import torch
    B = X.shape[0]
    Z = torch.empty((B, 6), dtype=torch.float32, device=X.device)
    check(lib().emogi_mlp_forward(params.data_ptr(), X.data_ptr(), B, Z.data_ptr(),
                                  _stream_handle(stream)))
    return Z


def mlp_loss_grad(params, X, y, stream=None):
    """(mean cross-entropy loss, gradient[5638]) from the HIP kernels."""
    import torch
    grad = torch.empty(N_SCHED_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    check(lib().emogi_mlp_loss_grad(params.data_ptr(), X.data_ptr(), y.data_ptr(), X.shape[0],
                                    grad.data_ptr(), loss.data_ptr(), _stream_handle(stream)))
    return loss, grad


def mlp_adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    check(lib().emogi_mlp_adam_step(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                    int(t), lr, beta1, beta2, eps, _stream_handle(stream)))


def mlp_train(X, y, params, epochs=50, batch=256, lr=1e-3, seed=0):
    """Trains on the GPU from host arrays; returns (params float32[5638], loss per epoch)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.int32)
    p = np.ascontiguousarray(params, dtype=np.float32).copy()
    hist = np.zeros(epochs, dtype=np.float32)
    cfg = TrainConfig(lr, 0.9, 0.999, 1e-8, batch, epochs, seed)
    check(lib().emogi_mlp_train(X.ctypes.data, y.ctypes.data, X.shape[0], ctypes.byref(cfg),
                                p.ctypes.data, hist.ctypes.data))
    return p, hist


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
            "emogi_packed_bytes": (i32, [p, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)]),
            "emogi_set_request_unit": (i32, [p, u32]),
            "emogi_set_scheduler": (i32, [p, i32]),
            "emogi_set_sssp_delta": (i32, [p, u32]),
            "emogi_set_cc_algorithm": (i32, [p, i32]),
            "emogi_set_hbm_tier": (i32, [p, u64, p, p]),
            "emogi_set_level_batch": (i32, [p, u32]),
            "emogi_set_frontier_order": (i32, [p, i32]),
            "emogi_set_direction": (i32, [p, i32, u32, u32]),
            "emogi_graph_setup_ms": (i32, [p, ctypes.POINTER(ctypes.c_double)]),
            "emogi_set_scheduler_weights": (i32, [p, p, sz]),
            "emogi_set_scheduler_range": (i32, [p, p, p]),
            "emogi_bfs": (i32, [p, u64, p, p]),
            "emogi_sssp": (i32, [p, u64, p, p]),
            "emogi_cc": (i32, [p, p, p]),
            "emogi_bfs_noalloc": (i32, [p, u64, p, p]),
            "emogi_pagerank": (i32, [p, u32, u32, u64, p, p]),
            "emogi_last_stats": (i32, [p, ctypes.POINTER(Stats)]),
            "emogi_num_vertices": (u64, [p]),
            "emogi_num_edges": (u64, [p]),
            "emogi_calibrate_link": (i32, [sz, ctypes.POINTER(LinkProfile)]),
            "emogi_mlp_forward": (i32, [p, p, u32, p, p]),
            "emogi_mlp_loss_grad": (i32, [p, p, p, u32, p, p, p]),
            "emogi_mlp_adam_step": (i32, [p, p, p, p, u32, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, p]),
            "emogi_mlp_train": (i32, [p, p, u32, ctypes.POINTER(TrainConfig), p, p]),
            "emogi_bfs_batch": (i32, [p, p, u32, p, p]),
            "emogi_sssp_batch": (i32, [p, p, u32, p, p]),
            "emogi_set_batch_params": (i32, [p, ctypes.POINTER(BatchParams)]),
            "emogi_get_batch_params": (i32, [p, ctypes.POINTER(BatchParams)]),
            "emogi_autotune_batch": (i32, [p, i32, p, u32, p, p, ctypes.POINTER(BatchParams),
                                           ctypes.POINTER(BatchTrial), u32]),
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


def calibrate_link(nbytes=1 << 30):
    """Runs emogi_calibrate_link and returns the profile as a dict."""
    p = LinkProfile()
    check(lib().emogi_calibrate_link(int(nbytes), ctypes.byref(p)))
    return p.as_dict()


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
    PinnedArray objects and are used in place (host zero-copy only).  With
    ``pack`` the lists (ascending) are stored compressed and col is read only
    here (``EMOGI_F_PACK``).  ``weight_bound`` computes the SSSP weight-read
    bounds at creation (``EMOGI_F_WEIGHT_BOUND``; a pass over the weights).
    """

    def __init__(self, row_ptr, col, weights=None, placement="host_zero_copy",
                 symmetric=False, validate=False, borrow=False, noncoherent=False, pack=False,
                 weight_bound=False):
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
                 | (F_BORROW if borrow else 0) | (F_PIN_NONCOHERENT if noncoherent else 0)
                 | (F_PACK if pack else 0) | (F_WEIGHT_BOUND if weight_bound else 0))
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

    def packed_bytes(self):
        """(id bytes, weight bytes) of the packed lists (zeros unless created with ``pack``)."""
        b, wb = ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().emogi_packed_bytes(self._h, ctypes.byref(b), ctypes.byref(wb)))
        return b.value, wb.value

    # -- configuration -------------------------------------------------------
    def set_variant(self, v):
        check(lib().emogi_set_scheduler(self._h, int(v)))

    def set_scheduler(self, mode, record=False):
        """mode: 'heuristic' | 'learned' | 'probe' | variant index; record keeps per-level features."""
        modes = {"heuristic": SCHED_HEURISTIC, "learned": SCHED_LEARNED, "probe": SCHED_PROBE}
        m = modes[mode] if isinstance(mode, str) else int(mode)
        check(lib().emogi_set_scheduler(self._h, m | (SCHED_RECORD if record else 0)))

    def set_scheduler_weights(self, params, feature_lo=None, feature_hi=None):
        """Loads the network; with feature_lo/feature_hi (16 each) levels whose
        features fall outside that training range use the heuristic."""
        if params is None:
            check(lib().emogi_set_scheduler_weights(self._h, None, 0))
            check(lib().emogi_set_scheduler_range(self._h, None, None))
            return
        p = np.ascontiguousarray(params, dtype=np.float32)
        check(lib().emogi_set_scheduler_weights(self._h, p.ctypes.data, p.shape[0]))
        if feature_lo is None:
            check(lib().emogi_set_scheduler_range(self._h, None, None))
        else:
            lo = np.ascontiguousarray(feature_lo, dtype=np.float32)
            hi = np.ascontiguousarray(feature_hi, dtype=np.float32)
            if lo.shape != (16,) or hi.shape != (16,):
                raise ValueError("feature bounds must have 16 entries each")
            check(lib().emogi_set_scheduler_range(self._h, lo.ctypes.data, hi.ctypes.data))

    def load_scheduler(self, path):
        """Network and training feature range from a train_scheduler JSON file."""
        import json
        doc = json.load(open(path))
        self.set_scheduler_weights(doc["params"], doc.get("feature_lo"), doc.get("feature_hi"))

    def set_frontier_order(self, ordered):
        """True: list each next frontier in ascending vertex id (bitmap compaction)."""
        check(lib().emogi_set_frontier_order(self._h, int(bool(ordered))))

    def set_direction(self, mode, alpha=0, beta=0):
        """BFS level direction: 'top_down', 'auto' (default) or 'bottom_up';
        alpha/beta of the switching rule (0 keeps the current values)."""
        m = {"top_down": 0, "auto": 1, "bottom_up": 2}[mode]
        check(lib().emogi_set_direction(self._h, m, int(alpha), int(beta)))

    def setup_ms(self):
        """Milliseconds of the create-time pass that found each vertex's
        smallest incoming weight (0 when it did not run)."""
        x = ctypes.c_double(0)
        check(lib().emogi_graph_setup_ms(self._h, ctypes.byref(x)))
        return x.value

    def set_cc_algorithm(self, name):
        """'label_propagation' or 'sampled_union_find' (default)."""
        check(lib().emogi_set_cc_algorithm(
            self._h, {"label_propagation": 0, "sampled_union_find": 1}[name]))

    def set_level_batch(self, levels):
        """BFS levels enqueued per host wait (0: automatic, 1: per-level waits)."""
        check(lib().emogi_set_level_batch(self._h, int(levels)))

    def set_hbm_tier(self, budget_bytes):
        """Copies the highest-degree vertices' lists that fit in budget_bytes
        into GPU memory (0 removes the tier); returns (vertices, bytes) held."""
        nv, nb = ctypes.c_uint64(0), ctypes.c_uint64(0)
        check(lib().emogi_set_hbm_tier(self._h, int(budget_bytes), ctypes.byref(nv), ctypes.byref(nb)))
        return int(nv.value), int(nb.value)

    def set_sssp_delta(self, delta):
        """SSSP near-far band width (0 = plain label correcting)."""
        check(lib().emogi_set_sssp_delta(self._h, int(delta)))

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

    def bfs_noalloc(self, src, out, stream=None):
        """emogi_bfs_noalloc: BFS into `out` (required: nothing is allocated)."""
        out = self._out(out)
        check(lib().emogi_bfs_noalloc(self._h, int(src), out.data_ptr(), _stream_handle(stream)))
        return out

    def sssp(self, src, out=None, stream=None):
        out = self._out(out)
        check(lib().emogi_sssp(self._h, int(src), out.data_ptr(), _stream_handle(stream)))
        return out

    def cc(self, out=None, stream=None):
        out = self._out(out)
        check(lib().emogi_cc(self._h, out.data_ptr(), _stream_handle(stream)))
        return out

    # -- batched multi-source (<= 64 sources share every list read) ----------
    def _batch_out(self, n, out):
        import torch
        if out is None:
            out = torch.empty(n * max(1, self.num_vertices), dtype=torch.int32, device="cuda")
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous():
            raise TypeError("output must be a contiguous int32 CUDA/HIP tensor")
        if out.numel() < n * self.num_vertices:
            raise ValueError("output tensor too small")
        return out

    def _srcs(self, srcs):
        s = np.ascontiguousarray(srcs, dtype=np.uint64)
        if not 1 <= s.shape[0] <= 64:
            raise ValueError("1..64 sources")
        return s

    def pagerank(self, iters, frac_bits=40, damping_fixed=None, out=None, stream=None):
        """Fixed-point PageRank (emogi_pagerank); returns an int64 CUDA tensor
        holding the uint64 scores (view it as uint64 on the host).
        damping_fixed defaults to floor(0.85 * 2^frac_bits)."""
        import torch
        if damping_fixed is None:
            damping_fixed = (85 << frac_bits) // 100
        if out is None:
            out = torch.empty(max(1, self.num_vertices), dtype=torch.int64, device="cuda")
        if out.dtype != torch.int64 or not out.is_cuda or not out.is_contiguous():
            raise TypeError("output must be a contiguous int64 CUDA/HIP tensor")
        if out.numel() < self.num_vertices:
            raise ValueError("output tensor too small")
        check(lib().emogi_pagerank(self._h, int(iters), int(frac_bits), int(damping_fixed), out.data_ptr(),
                                   _stream_handle(stream)))
        return out

    def bfs_batch(self, srcs, out=None, stream=None):
        """Levels from each source, source-major [n * V] int32 tensor."""
        s = self._srcs(srcs)
        out = self._batch_out(s.shape[0], out)
        check(lib().emogi_bfs_batch(self._h, s.ctypes.data, s.shape[0], out.data_ptr(),
                                    _stream_handle(stream)))
        return out

    def sssp_batch(self, srcs, out=None, stream=None):
        s = self._srcs(srcs)
        out = self._batch_out(s.shape[0], out)
        check(lib().emogi_sssp_batch(self._h, s.ctypes.data, s.shape[0], out.data_ptr(),
                                     _stream_handle(stream)))
        return out

    def set_batch_params(self, hub_degree=1024, steps_per_graph=4, blocks_per_cu=8, use_graph=True,
                         sssp_delta=0):
        p = BatchParams(hub_degree, steps_per_graph, blocks_per_cu, int(use_graph), sssp_delta)
        check(lib().emogi_set_batch_params(self._h, ctypes.byref(p)))

    def get_batch_params(self):
        p = BatchParams()
        check(lib().emogi_get_batch_params(self._h, ctypes.byref(p)))
        return p.as_dict()

    def autotune_batch(self, algo, srcs, out=None, stream=None):
        """Tries the candidate parameter sets; keeps and returns the fastest plus the table."""
        s = self._srcs(srcs)
        out = self._batch_out(s.shape[0], out)
        best = BatchParams()
        table = (BatchTrial * 64)()
        check(lib().emogi_autotune_batch(self._h, {"bfs": 0, "sssp": 1}[algo], s.ctypes.data,
                                         s.shape[0], out.data_ptr(), _stream_handle(stream),
                                         ctypes.byref(best), table, 64))
        trials = [dict(t.params.as_dict(), ms=t.ms) for t in table if t.params.blocks_per_cu]
        return best.as_dict(), trials

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


def to_u64(t):
    """int64 device tensor -> uint64 numpy array on the host."""
    return t.detach().cpu().numpy().view(np.uint64)
