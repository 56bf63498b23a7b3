// Graph handle: validation and placement of the CSR (EMOGI Sec. 4.2: the
// vertex list and per-vertex buffers go to GPU memory, the edge list to host
// memory, all mapped once at set-up; Sec. 3.1: pinned + mapped host memory is
// what lets GPU threads read it in place).
#include "internal.h"

#include <chrono>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>
#include <atomic>
#include <new>

namespace emogi {

static thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

// Runs fn(begin, end) over [0, n) on up to hardware_concurrency threads.
template <class F>
static void parallel_for(uint64_t n, F fn) {
    unsigned t = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < (1u << 16) || t == 1) {
        fn(uint64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    uint64_t step = (n + t - 1) / t;
    for (unsigned i = 0; i < t; ++i) {
        uint64_t b = i * step, e = std::min(n, b + step);
        if (b >= e) break;
        th.emplace_back([=] { fn(b, e); });
    }
    for (auto &x : th) x.join();
}

static void parallel_copy(void *dst, const void *src, size_t bytes) {
    const size_t grain = size_t(1) << 22;
    uint64_t blocks = (bytes + grain - 1) / grain;
    parallel_for(blocks, [&](uint64_t b, uint64_t e) {
        for (uint64_t i = b; i < e; ++i) {
            size_t off = i * grain, len = std::min(grain, bytes - off);
            memcpy(static_cast<char *>(dst) + off, static_cast<const char *>(src) + off, len);
        }
    });
}

static inline uint64_t col_at(const void *col, uint32_t cb, uint64_t i) {
    return cb == 4 ? static_cast<const uint32_t *>(col)[i] : static_cast<const uint64_t *>(col)[i];
}

// 0 when well formed, else an EMOGI_E_* code with the reason recorded.
static emogi_status_t validate(const uint64_t *rp, uint64_t V, const void *col, uint32_t cb,
                               bool symmetric) {
    if (rp[0] != 0) {
        set_error("row_ptr[0] must be 0");
        return EMOGI_E_INVALID;
    }
    for (uint64_t u = 0; u < V; ++u)
        if (rp[u + 1] < rp[u]) {
            set_error("row_ptr decreases at vertex %llu", (unsigned long long)u);
            return EMOGI_E_INVALID;
        }
    std::atomic<int> bad{0};
    parallel_for(V, [&](uint64_t b, uint64_t e) {
        for (uint64_t u = b; u < e && !bad.load(std::memory_order_relaxed); ++u)
            for (uint64_t i = rp[u]; i < rp[u + 1]; ++i)
                if (col_at(col, cb, i) >= V) {
                    bad = 1;
                    break;
                }
    });
    if (bad) {
        set_error("a neighbour id is >= num_vertices");
        return EMOGI_E_INVALID;
    }
    if (!symmetric) return EMOGI_OK;
    // u->v must have v->u: sort a copy of each list, then binary-search.
    uint64_t E = rp[V];
    std::vector<uint64_t> sorted(E);
    parallel_for(V, [&](uint64_t b, uint64_t e) {
        for (uint64_t u = b; u < e; ++u) {
            for (uint64_t i = rp[u]; i < rp[u + 1]; ++i) sorted[i] = col_at(col, cb, i);
            std::sort(sorted.begin() + rp[u], sorted.begin() + rp[u + 1]);
        }
    });
    parallel_for(V, [&](uint64_t b, uint64_t e) {
        for (uint64_t u = b; u < e && !bad.load(std::memory_order_relaxed); ++u)
            for (uint64_t i = rp[u]; i < rp[u + 1]; ++i) {
                uint64_t v = sorted[i];
                if (!std::binary_search(sorted.begin() + rp[v], sorted.begin() + rp[v + 1], u)) {
                    bad = 1;
                    break;
                }
            }
    });
    if (bad) {
        set_error("graph is not symmetric");
        return EMOGI_E_NOT_SYMMETRIC;
    }
    return EMOGI_OK;
}

static void release(emogi_graph_s *g) {
    if (!g) return;
    auto free_edges = [](void *p, emogi_graph_s::Kind k) {
        if (!p) return;
        if (k == emogi_graph_s::DEVICE || k == emogi_graph_s::MANAGED) (void)hipFree(p);
        if (k == emogi_graph_s::PINNED) (void)hipHostFree(p);
    };
    free_edges(g->col, g->col_kind);
    free_edges(g->weights, g->w_kind);
    if (g->row_ptr) (void)hipFree(g->row_ptr);
    if (g->in_min) (void)hipFree(g->in_min);
    if (g->packed.on_device && g->packed.stream) (void)hipFree(g->packed.stream);
    if (g->packed.pinned) (void)hipHostFree(g->packed.pinned);
    if (g->packed.wwidth) (void)hipFree(g->packed.wwidth);
    if (g->packed.off) (void)hipFree(g->packed.off);
    if (g->packed.width) (void)hipFree(g->packed.width);
    Pool &p = g->pool;
    for (auto q : p.queue)
        if (q) (void)hipFree(q);
    if (p.bitmap) (void)hipFree(p.bitmap);
    if (p.stamp) (void)hipFree(p.stamp);
    if (p.chunk_scan) (void)hipFree(p.chunk_scan);
    if (p.block_sums) (void)hipFree(p.block_sums);
    if (p.counters) (void)hipFree(p.counters);
    if (p.host_counters) (void)hipHostFree(p.host_counters);
    if (p.pr_acc) (void)hipFree(p.pr_acc);
    if (p.pr_contrib) (void)hipFree(p.pr_contrib);
    if (p.level_ctr) (void)hipFree(p.level_ctr);
    if (p.level_host) (void)hipHostFree(p.level_host);
    if (p.features) (void)hipFree(p.features);
    if (p.degree_hist) (void)hipFree(p.degree_hist);
    for (void *x : {(void *)p.snap_state, (void *)p.snap_stamp, (void *)p.snap_bitmap, (void *)p.snap_nextbits,
                    (void *)p.cc_probe, (void *)p.nextbits, (void *)p.farbits, (void *)p.snap_farbits})
        if (x) (void)hipFree(x);
    if (g->mlp_params) (void)hipFree(g->mlp_params);
    if (g->mlp_range) (void)hipFree(g->mlp_range);
    tier_release(g);
    BatchPool &b = g->batch;
    for (int i = 0; i < 2; ++i) {
        if (b.mask[i]) (void)hipFree(b.mask[i]);
        if (b.hub[i]) (void)hipFree(b.hub[i]);
    }
    for (void *x : {(void *)b.vis, (void *)b.ovf, (void *)b.wait, (void *)b.dist, (void *)b.ctr, (void *)b.srcs})
        if (x) (void)hipFree(x);
    if (b.host_ctr) (void)hipHostFree(b.host_ctr);
    if (b.stream) (void)hipStreamDestroy(b.stream);
    for (hipEvent_t e : {g->ev_begin, g->ev_end, g->ev_k0, g->ev_k1, g->ev_s0})
        if (e) (void)hipEventDestroy(e);
    delete g;
}

// Smallest weight of an edge into each vertex: one coalesced pass over the
// edge list (wherever it is placed) with atomicMin into m; ids at or above V
// are ignored.  The plain read first skips atomics that cannot lower m[v].
template <class ColT>
__global__ __launch_bounds__(256) void k_in_min(const ColT *col, const uint32_t *w, uint64_t E, uint64_t V,
                                                uint32_t *m) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < E; i += stride) {
        const uint64_t v = uint64_t(col[i]);
        const uint32_t x = w[i];
        if (v < V && x < m[v]) atomicMin(&m[v], x);
    }
}

__global__ __launch_bounds__(256) void k_in_min_init(uint32_t *m, uint64_t V) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V; i += stride) m[i] = 0xFFFFFFFFu;
}

__global__ __launch_bounds__(256) void k_in_min_pack(const uint32_t *m, uint64_t V, uint8_t *out) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V; i += stride)
        out[i] = uint8_t(min(m[i], 255u));
}

// Per-vertex smallest incoming weight (uint8, saturated) for SSSP's
// weight-read skipping; computed from the edges, so it holds for directed
// graphs and asymmetric weights alike.
static emogi_status_t compute_in_min(emogi_graph_s *g) {
    const uint64_t V = g->V, E = g->E;
    uint32_t *m = nullptr;
    if (hipMalloc(&m, V * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of %llu bytes for the incoming weight bounds failed",
                  (unsigned long long)(V * sizeof(uint32_t)));
        return EMOGI_E_OOM_DEVICE;
    }
    if (hipMalloc(&g->in_min, V) != hipSuccess) {
        (void)hipGetLastError();
        g->in_min = nullptr;
        (void)hipFree(m);
        set_error("hipMalloc of the incoming weight bounds failed");
        return EMOGI_E_OOM_DEVICE;
    }
    const unsigned grid = 256u * 8u;
    (void)hipDeviceSynchronize();
    const auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(k_in_min_init, dim3(grid), dim3(256), 0, nullptr, m, V);
    if (g->col_bytes == 8)
        hipLaunchKernelGGL(k_in_min<uint64_t>, dim3(grid), dim3(256), 0, nullptr,
                           static_cast<const uint64_t *>(g->col), g->weights, E, V, m);
    else
        hipLaunchKernelGGL(k_in_min<uint32_t>, dim3(grid), dim3(256), 0, nullptr,
                           static_cast<const uint32_t *>(g->col), g->weights, E, V, m);
    hipLaunchKernelGGL(k_in_min_pack, dim3(grid), dim3(256), 0, nullptr, m, V, g->in_min);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipDeviceSynchronize();
    g->in_min_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    (void)hipFree(m);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        set_error("incoming weight bound kernels failed");
        return EMOGI_E_HIP;
    }
    return EMOGI_OK;
}

// Allocates one packed stream where the placement puts the lists: pinned
// host memory written in place, or a host buffer that is copied to HBM later.
static emogi_status_t alloc_stream(emogi_graph_s *g, size_t bytes, void **pinned, uint32_t **host,
                                   std::vector<uint32_t> &staging) {
    if (g->placement == EMOGI_PLACE_HOST_ZERO_COPY) {
        unsigned fl = hipHostMallocMapped;
        if (g->flags & EMOGI_F_PIN_NONCOHERENT) fl |= hipHostMallocNonCoherent;
        if (hipHostMalloc(pinned, bytes, fl) != hipSuccess) {
            (void)hipGetLastError();
            *pinned = nullptr;
            set_error("hipHostMalloc of %zu pinned bytes for the packed lists failed", bytes);
            return EMOGI_E_OOM_HOST;
        }
        *host = static_cast<uint32_t *>(*pinned);
    } else {
        staging.resize(bytes / 4);
        *host = staging.data();
    }
    return EMOGI_OK;
}

// The GPU's view of a stream built by alloc_stream (copied to HBM if placed there).
static emogi_status_t publish_stream(emogi_graph_s *g, size_t bytes, void *pinned, const uint32_t *host,
                                     uint32_t **dev) {
    void *d = nullptr;
    if (g->placement == EMOGI_PLACE_HOST_ZERO_COPY) {
        EMOGI_HIP_TRY(hipHostGetDevicePointer(&d, pinned, 0), EMOGI_E_HIP);
    } else {
        if (hipMalloc(&d, bytes) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of %zu bytes for the packed lists failed", bytes);
            return EMOGI_E_OOM_DEVICE;
        }
        *dev = static_cast<uint32_t *>(d);
        EMOGI_HIP_TRY(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice), EMOGI_E_HIP);
    }
    *dev = static_cast<uint32_t *>(d);
    return EMOGI_OK;
}

// Appends `w`-bit fields to a word stream.
struct BitWriter {
    uint32_t *o;
    uint64_t acc = 0;
    uint32_t nbits = 0;
    void put(uint64_t x, uint32_t w) {  // x < 2^w, w <= 32; nbits < 32 before
        acc |= x << nbits;
        nbits += w;
        if (nbits >= 32) {
            *o++ = uint32_t(acc);
            acc >>= 32;
            nbits -= 32;
        }
    }
    void flush() {
        if (nbits) *o++ = uint32_t(acc);
        acc = 0;
        nbits = 0;
    }
};

// Words of one packed block of `cnt` ids (gap width w, weight width ww).
static inline uint64_t block_words(uint64_t cnt, uint32_t w, uint32_t ww) {
    return 1 + ((cnt - 1) * w + 31) / 32 + (cnt * ww + 31) / 32;
}

// EMOGI_F_PACK: encodes the lists (and weights) on the host threads in two
// passes over col: widths and word counts, then the blocks, straight into
// the stream's final host memory (pinned) or a host buffer copied to HBM.
static emogi_status_t pack_lists(emogi_graph_s *g, const uint64_t *row_ptr, const void *col,
                                 const uint32_t *weights) {
    const uint64_t V = g->V;
    const uint32_t cb = g->col_bytes;
    if (g->placement == EMOGI_PLACE_MANAGED) {
        set_error("packed lists are placed in pinned host memory or HBM, not managed memory");
        return EMOGI_E_UNSUPPORTED;
    }
    std::vector<uint8_t> width(V), wwidth(weights ? V : 0);
    std::vector<uint64_t> off(V + 1, 0), wcount(V, 0);
    std::atomic<uint64_t> bad{~uint64_t(0)};
    parallel_for(V, [&](uint64_t u0, uint64_t u1) {
        for (uint64_t u = u0; u < u1; ++u) {
            const uint64_t b = row_ptr[u], e = row_ptr[u + 1];
            uint64_t maxgap = 0, prev = 0;
            uint32_t maxw = 0;
            for (uint64_t i = b; i < e; ++i) {
                const uint64_t x = col_at(col, cb, i);
                if (x > 0xFFFFFFFFull || (i > b && x < prev)) {
                    uint64_t cur = bad.load();
                    while (u < cur && !bad.compare_exchange_weak(cur, u)) {
                    }
                }
                if ((i - b) % 64 != 0 && x >= prev) maxgap = std::max(maxgap, x - prev);
                prev = x;
                if (weights) maxw = std::max(maxw, weights[i]);
            }
            const uint32_t w = maxgap ? 64u - uint32_t(__builtin_clzll(maxgap)) : 0u;
            const uint32_t ww = maxw ? 32u - uint32_t(__builtin_clz(maxw)) : 0u;
            width[u] = uint8_t(w);
            if (weights) wwidth[u] = uint8_t(ww);
            const uint64_t d = e - b;
            if (d) {
                const uint64_t nb = (d + 63) / 64, last = d - (nb - 1) * 64;
                off[u + 1] = (nb - 1) * block_words(64, w, ww) + block_words(last, w, ww);
                wcount[u] = (nb - 1) * 2 * uint64_t(ww) + (last * ww + 31) / 32;
            }
        }
    });
    if (bad.load() != ~uint64_t(0)) {
        set_error("EMOGI_F_PACK needs ascending lists of ids below 2^32 (vertex %llu)",
                  (unsigned long long)bad.load());
        return EMOGI_E_INVALID;
    }
    uint64_t wwords = 0;
    for (uint64_t u = 0; u < V; ++u) {
        off[u + 1] += off[u];
        wwords += wcount[u];
    }
    Packed &pk = g->packed;
    const uint64_t words = off[V];
    const size_t bytes = std::max<size_t>(8, words * 4);
    uint32_t *host = nullptr;
    std::vector<uint32_t> staging;
    emogi_status_t st = alloc_stream(g, bytes, &pk.pinned, &host, staging);
    if (st != EMOGI_OK) return st;
    parallel_for(V, [&](uint64_t u0, uint64_t u1) {
        for (uint64_t u = u0; u < u1; ++u) {
            const uint64_t b = row_ptr[u], e = row_ptr[u + 1];
            const uint32_t w = width[u], ww = weights ? wwidth[u] : 0u;
            BitWriter bw{host + off[u]};
            for (uint64_t k0 = b; k0 < e; k0 += 64) {
                const uint64_t k1 = std::min(e, k0 + 64);
                uint64_t prev = col_at(col, cb, k0);
                *bw.o++ = uint32_t(prev);
                for (uint64_t i = k0 + 1; i < k1; ++i) {
                    const uint64_t x = col_at(col, cb, i);
                    bw.put(x - prev, w);
                    prev = x;
                }
                bw.flush();
                if (ww) {
                    for (uint64_t i = k0; i < k1; ++i) bw.put(weights[i], ww);
                    bw.flush();
                }
            }
        }
    });
    pk.words = words;
    pk.wwords = wwords;
    if ((st = publish_stream(g, bytes, pk.pinned, host, &pk.stream)) != EMOGI_OK) return st;
    if (g->placement != EMOGI_PLACE_HOST_ZERO_COPY) pk.on_device = true;
    auto upload = [&](void **dst, const void *src, size_t n) -> emogi_status_t {
        if (hipMalloc(dst, std::max<size_t>(n, 8)) != hipSuccess) {
            (void)hipGetLastError();
            *dst = nullptr;
            set_error("hipMalloc of the packed list offsets failed");
            return EMOGI_E_OOM_DEVICE;
        }
        if (n) EMOGI_HIP_TRY(hipMemcpy(*dst, src, n, hipMemcpyHostToDevice), EMOGI_E_HIP);
        return EMOGI_OK;
    };
    if ((st = upload(reinterpret_cast<void **>(&pk.off), off.data(), (V + 1) * 8)) != EMOGI_OK) return st;
    if ((st = upload(reinterpret_cast<void **>(&pk.width), width.data(), V)) != EMOGI_OK) return st;
    if (weights && (st = upload(reinterpret_cast<void **>(&pk.wwidth), wwidth.data(), V)) != EMOGI_OK) return st;
    return EMOGI_OK;
}

// Places one edge-sized array (col or weights) per the placement.
static emogi_status_t place(emogi_graph_s *g, const void *src, size_t bytes, void **dst,
                            emogi_graph_s::Kind *kind) {
    if (bytes == 0) bytes = 8;  // keep a valid pointer for empty graphs
    switch (g->placement) {
    case EMOGI_PLACE_HBM: {
        void *d = nullptr;
        if (hipMalloc(&d, bytes) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of %zu bytes for the edge list failed", bytes);
            return EMOGI_E_OOM_DEVICE;
        }
        *dst = d;
        *kind = emogi_graph_s::DEVICE;
        if (src) EMOGI_HIP_TRY(hipMemcpy(d, src, bytes, hipMemcpyHostToDevice), EMOGI_E_HIP);
        return EMOGI_OK;
    }
    case EMOGI_PLACE_HOST_ZERO_COPY: {
        if (g->flags & EMOGI_F_BORROW) {
            hipPointerAttribute_t attr;
            if (!src || hipPointerGetAttributes(&attr, src) != hipSuccess ||
                attr.type != hipMemoryTypeHost) {
                (void)hipGetLastError();
                set_error("EMOGI_F_BORROW needs memory from emogi_host_alloc");
                return EMOGI_E_INVALID;
            }
            void *d = nullptr;
            EMOGI_HIP_TRY(hipHostGetDevicePointer(&d, const_cast<void *>(src), 0), EMOGI_E_HIP);
            *dst = d;
            *kind = emogi_graph_s::BORROWED;
            return EMOGI_OK;
        }
        unsigned fl = hipHostMallocMapped;
        if (g->flags & EMOGI_F_PIN_NONCOHERENT) fl |= hipHostMallocNonCoherent;
        void *h = nullptr;
        if (hipHostMalloc(&h, bytes, fl) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipHostMalloc of %zu pinned bytes failed", bytes);
            return EMOGI_E_OOM_HOST;
        }
        *kind = emogi_graph_s::PINNED;
        void *d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(h);
            *kind = emogi_graph_s::NONE;
            set_error("hipHostGetDevicePointer failed");
            return EMOGI_E_HIP;
        }
        *dst = d;
        if (src) parallel_copy(h, src, bytes);
        return EMOGI_OK;
    }
    case EMOGI_PLACE_MANAGED: {
        int dev = g->device, managed = 0;
        (void)hipDeviceGetAttribute(&managed, hipDeviceAttributeManagedMemory, dev);
        if (!managed) {
            set_error("managed memory is not supported on this device (no XNACK/HMM)");
            return EMOGI_E_UNSUPPORTED;
        }
        void *m = nullptr;
        if (hipMallocManaged(&m, bytes, hipMemAttachGlobal) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMallocManaged of %zu bytes failed", bytes);
            return EMOGI_E_OOM_HOST;
        }
        *dst = m;
        *kind = emogi_graph_s::MANAGED;
        if (src) parallel_copy(m, src, bytes);
        // Sec. 5.1 (a): the UVM baseline marks the edge list read-mostly.
        (void)hipMemAdvise(m, bytes, hipMemAdviseSetReadMostly, dev);
        (void)hipGetLastError();
        return EMOGI_OK;
    }
    }
    set_error("unknown placement %d", (int)g->placement);
    return EMOGI_E_INVALID;
}

}  // namespace emogi

using namespace emogi;

extern "C" {

emogi_status_t emogi_host_alloc(size_t bytes, uint32_t flags, void **out) {
    if (!out || bytes == 0) {
        set_error("emogi_host_alloc: null out or zero size");
        return EMOGI_E_INVALID;
    }
    unsigned fl = hipHostMallocMapped;
    if (flags & EMOGI_F_PIN_NONCOHERENT) fl |= hipHostMallocNonCoherent;
    void *h = nullptr;
    if (hipHostMalloc(&h, bytes, fl) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipHostMalloc of %zu bytes failed", bytes);
        return EMOGI_E_OOM_HOST;
    }
    *out = h;
    return EMOGI_OK;
}

emogi_status_t emogi_host_free(void *p) {
    if (!p) return EMOGI_OK;
    EMOGI_HIP_TRY(hipHostFree(p), EMOGI_E_HIP);
    return EMOGI_OK;
}

emogi_status_t emogi_graph_create(const uint64_t *row_ptr, uint64_t V, const void *col,
                                  uint32_t col_bytes, const uint32_t *weights,
                                  emogi_placement_t placement, uint32_t flags,
                                  emogi_graph_t *out) {
    if (!out || !row_ptr) {
        set_error("emogi_graph_create: null row_ptr or out");
        return EMOGI_E_INVALID;
    }
    if (col_bytes != 4 && col_bytes != 8) {
        set_error("col_bytes must be 4 or 8");
        return EMOGI_E_INVALID;
    }
    if (V >= 0xFFFFFFFFull) {
        set_error("num_vertices must be below 2^32-1 (outputs are uint32)");
        return EMOGI_E_UNSUPPORTED;
    }
    if ((int)placement < 0 || (int)placement > 2) {
        set_error("unknown placement %d", (int)placement);
        return EMOGI_E_INVALID;
    }
    uint64_t E = row_ptr[V];
    if (E > 0 && !col) {
        set_error("col is null but the graph has edges");
        return EMOGI_E_INVALID;
    }
    if ((flags & EMOGI_F_BORROW) && placement != EMOGI_PLACE_HOST_ZERO_COPY) {
        set_error("EMOGI_F_BORROW is only valid with host zero-copy placement");
        return EMOGI_E_INVALID;
    }
    if (flags & EMOGI_F_VALIDATE) {
        emogi_status_t st = validate(row_ptr, V, col, col_bytes, (flags & EMOGI_F_SYMMETRIC) != 0);
        if (st != EMOGI_OK) return st;
    }
    int dev = 0;
    EMOGI_HIP_TRY(hipGetDevice(&dev), EMOGI_E_HIP);

    auto *g = new (std::nothrow) emogi_graph_s();
    if (!g) {
        set_error("out of host memory");
        return EMOGI_E_OOM_HOST;
    }
    g->V = V;
    g->E = E;
    g->col_bytes = col_bytes;
    g->flags = flags;
    g->placement = placement;
    g->device = dev;
    uint64_t maxd = 0, nz = 0;
    for (uint64_t u = 0; u < V; ++u) {
        const uint64_t d = row_ptr[u + 1] - row_ptr[u];
        maxd = std::max(maxd, d);
        nz += d > 0;
    }
    g->max_degree = maxd;
    g->nonisolated = nz;
    // The smallest weight bounds what an edge can add to a distance: SSSP
    // skips the weight read of an edge whose target is already that close.
    g->min_weight = 0;
    if (weights && E > 0 && (flags & EMOGI_F_WEIGHT_BOUND)) {
        const unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
        std::vector<uint32_t> part(nt, 0xFFFFFFFFu);
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&, t] {
                uint32_t m = 0xFFFFFFFFu;
                for (uint64_t i = E * t / nt, end = E * (t + 1) / nt; i < end; ++i) m = std::min(m, weights[i]);
                part[t] = m;
            });
        for (auto &x : th) x.join();
        g->min_weight = *std::min_element(part.begin(), part.end());
    }

    emogi_status_t st = EMOGI_OK;
    if (hipMalloc(&g->row_ptr, (V + 1) * sizeof(uint64_t)) != hipSuccess) {
        (void)hipGetLastError();
        g->row_ptr = nullptr;
        release(g);
        set_error("hipMalloc of row_ptr failed");
        return EMOGI_E_OOM_DEVICE;
    }
    if (hipMemcpy(g->row_ptr, row_ptr, (V + 1) * sizeof(uint64_t), hipMemcpyHostToDevice) !=
        hipSuccess) {
        (void)hipGetLastError();
        release(g);
        set_error("copy of row_ptr failed");
        return EMOGI_E_HIP;
    }
    if (flags & EMOGI_F_PACK)
        // g->col and g->weights stay null: the scans decode the packed streams
        st = pack_lists(g, row_ptr, col, weights);
    else
        st = place(g, col, E * col_bytes, &g->col, &g->col_kind);
    if (st == EMOGI_OK && weights && !(flags & EMOGI_F_PACK)) {
        void *w = nullptr;
        st = place(g, weights, E * sizeof(uint32_t), &w, &g->w_kind);
        g->weights = static_cast<uint32_t *>(w);
        // the per-target bound pays only where a weight read crosses the
        // host link; from HBM the extra gather costs more than it saves
        if (st == EMOGI_OK && E > 0 && placement == EMOGI_PLACE_HOST_ZERO_COPY && (flags & EMOGI_F_WEIGHT_BOUND))
            st = compute_in_min(g);
    }
    if (st == EMOGI_OK) {
        for (hipEvent_t *e : {&g->ev_begin, &g->ev_end, &g->ev_k0, &g->ev_k1, &g->ev_s0})
            if (hipEventCreate(e) != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipEventCreate failed");
                st = EMOGI_E_HIP;
                break;
            }
    }
    if (st != EMOGI_OK) {
        release(g);
        return st;
    }
    *out = g;
    return EMOGI_OK;
}

emogi_status_t emogi_packed_bytes(emogi_graph_t g, uint64_t *id_bytes, uint64_t *weight_bytes) {
    if (!g || !id_bytes) {
        set_error("null argument");
        return EMOGI_E_INVALID;
    }
    *id_bytes = (g->packed.words - g->packed.wwords) * 4;
    if (weight_bytes) *weight_bytes = g->packed.wwords * 4;
    return EMOGI_OK;
}

emogi_status_t emogi_graph_destroy(emogi_graph_t g) {
    if (!g) return EMOGI_E_INVALID;
    (void)hipDeviceSynchronize();
    release(g);
    return EMOGI_OK;
}

emogi_status_t emogi_set_frontier_order(emogi_graph_t g, int ordered) {
    if (!g) {
        set_error("null graph");
        return EMOGI_E_INVALID;
    }
    g->ordered_frontier = ordered != 0;
    return EMOGI_OK;
}

emogi_status_t emogi_set_cc_algorithm(emogi_graph_t g, int algorithm) {
    if (!g || (algorithm != EMOGI_CC_LABEL_PROPAGATION && algorithm != EMOGI_CC_SAMPLED_UNION_FIND)) {
        set_error("unknown CC algorithm %d", algorithm);
        return EMOGI_E_INVALID;
    }
    g->cc_sampled = algorithm == EMOGI_CC_SAMPLED_UNION_FIND;
    return EMOGI_OK;
}

emogi_status_t emogi_set_level_batch(emogi_graph_t g, uint32_t levels) {
    if (!g || levels > 64) {
        set_error("level batch must be 0 (automatic) .. 64");
        return EMOGI_E_INVALID;
    }
    g->level_batch = levels;
    return EMOGI_OK;
}

emogi_status_t emogi_set_sssp_delta(emogi_graph_t g, uint32_t delta) {
    if (!g) {
        set_error("null graph");
        return EMOGI_E_INVALID;
    }
    g->sssp_delta = delta;
    return EMOGI_OK;
}

emogi_status_t emogi_set_request_unit(emogi_graph_t g, uint32_t bytes) {
    if (!g || bytes < 32 || bytes > 4096 || (bytes & (bytes - 1))) {
        set_error("request unit must be a power of two in [32, 4096]");
        return EMOGI_E_INVALID;
    }
    g->request_unit = bytes;
    return EMOGI_OK;
}

emogi_status_t emogi_set_scheduler(emogi_graph_t g, int mode) {
    const int base = mode & ~int(EMOGI_SCHED_RECORD);
    if (!g || !((base >= 0 && base < EMOGI_NUM_VARIANTS) || base == EMOGI_SCHED_HEURISTIC ||
                base == EMOGI_SCHED_LEARNED || base == EMOGI_SCHED_PROBE)) {
        set_error("unknown scheduler mode %d", mode);
        return EMOGI_E_INVALID;
    }
    g->sched_mode = base;
    g->record_features = (mode & EMOGI_SCHED_RECORD) != 0;
    return EMOGI_OK;
}

emogi_status_t emogi_set_direction(emogi_graph_t g, int mode, uint32_t alpha, uint32_t beta) {
    if (!g || (mode != EMOGI_DIR_TOP_DOWN && mode != EMOGI_DIR_AUTO && mode != EMOGI_DIR_BOTTOM_UP)) {
        set_error("unknown direction mode %d", mode);
        return EMOGI_E_INVALID;
    }
    g->direction = mode;
    if (alpha) g->dir_alpha = alpha;
    if (beta) g->dir_beta = beta;
    return EMOGI_OK;
}

emogi_status_t emogi_graph_setup_ms(emogi_graph_t g, double *in_min_ms) {
    if (!g || !in_min_ms) {
        set_error("null argument");
        return EMOGI_E_INVALID;
    }
    *in_min_ms = g->in_min_ms;
    return EMOGI_OK;
}

emogi_status_t emogi_last_stats(emogi_graph_t g, emogi_stats_t *out) {
    if (!g || !out) {
        set_error("null argument");
        return EMOGI_E_INVALID;
    }
    *out = g->stats;
    return EMOGI_OK;
}

uint64_t emogi_num_vertices(emogi_graph_t g) { return g ? g->V : 0; }
uint64_t emogi_num_edges(emogi_graph_t g) { return g ? g->E : 0; }

const char *emogi_strerror(emogi_status_t e) {
    switch (e) {
    case EMOGI_OK: return "ok";
    case EMOGI_E_INVALID: return "invalid argument";
    case EMOGI_E_OOM_HOST: return "out of host memory";
    case EMOGI_E_OOM_DEVICE: return "out of device memory";
    case EMOGI_E_HIP: return "HIP runtime error";
    case EMOGI_E_NOT_SYMMETRIC: return "graph is not symmetric";
    case EMOGI_E_OVERFLOW: return "distance overflow";
    case EMOGI_E_NOCONVERGE: return "iteration cap reached";
    case EMOGI_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *emogi_last_error(void) { return g_last_error; }

}  // extern "C"
