// Level-synchronous BFS / SSSP / CC over a CSR whose edge list may sit in
// pinned host memory and is read in place by the GPU.
//
// The traversal follows Algorithm 1 of EMOGI (Sec. 2.1): a set of active
// vertices is expanded one level (round) per kernel launch (Sec. 4.2), each
// neighbour runs an application step, and the neighbours that meet the
// application's condition form the next active set.  What the paper changes
// is how a neighbour list is read from zero-copy memory: by a whole wave
// with consecutive lanes on consecutive elements (Sec. 4.3.1, merged) and
// with the start rounded down to the request unit so every wave-wide load
// covers whole request blocks (Sec. 4.3.2, aligned).  Six result-identical
// access variants are provided (see emogi_variant_t).
//
// MI355X specifics:
//  * wave64: one vector load of 64 lanes x 4 B covers 256 B, the request unit
//    at which random host-link reads reach the copy rate;
//  * frontier pushes are compacted per wave with ballot + mbcnt into a
//    per-wave LDS segment; a block writes its segments to the global queue
//    with one atomic at the end (or a wave flushes when its segment fills);
//  * vertex state (levels, distances, labels, visited bitmap, stamps) stays
//    in HBM; only the edge list (and weights) cross the host link.
#include "internal.h"
#include "wave.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace emogi {

enum Algo { A_BFS = 0, A_SSSP = 1, A_CC = 2 };

constexpr int kUnroll = 4;        // loads in flight per lane in the wave variants
constexpr int kChunksPerWave = 8; // V5: consecutive aligned chunks per wave visit
constexpr int kMaxGrid = 256 * 8; // 8 blocks of 4 waves on each of the 256 CUs

// End of a scan block: flush the staged frontier and fold the statistics.
__device__ __forceinline__ void finish_block(Stage &st, uint32_t *next, unsigned long long *ctr,
                                             int lane, int wid, uint64_t edges, uint64_t reqb,
                                             uint64_t verts) {
    finish_queue(st, next, &ctr[C_NEXT], lane, wid);
    edges = wave_sum64(edges);
    reqb = wave_sum64(reqb);
    verts = wave_sum64(verts);
    if (lane == 0) {
        if (edges) atomicAdd(&ctr[C_EDGES], (unsigned long long)edges);
        if (reqb) atomicAdd(&ctr[C_REQBYTES], (unsigned long long)reqb);
        if (verts) atomicAdd(&ctr[C_VERTS], (unsigned long long)verts);
    }
}

// ---------------------------------------------------------------------------
// Application step per neighbour (Algorithm 1's workload + condition).
// ---------------------------------------------------------------------------
struct OpArgs {
    uint32_t *state;    // levels / dist / labels (the caller's output array)
    uint32_t *bitmap;   // BFS visited bits; SSSP overflow marks
    uint32_t *stamp;    // SSSP/CC: last round in which v was pushed
    uint32_t tag;       // BFS: level of the next frontier; SSSP/CC: round number
    uint32_t V;         // neighbour ids at or above V are ignored (malformed input)
    unsigned long long *ctr;
};

template <int A>
__device__ __forceinline__ uint32_t source_value(const OpArgs &a, uint32_t u) {
    if (A == A_BFS) return 0u;
    return a.state[u];
}

// Returns true when v joins the next frontier.
template <int A>
__device__ __forceinline__ bool visit(const OpArgs &a, uint32_t uval, uint32_t v, uint32_t w) {
    if (v >= a.V) return false;
    if (A == A_BFS) {
        // BFS: an unvisited neighbour is visited at the next level.
        uint32_t word = v >> 5, bit = 1u << (v & 31u);
        if (a.bitmap[word] & bit) return false;
        uint32_t old = atomicOr(&a.bitmap[word], bit);
        if (old & bit) return false;
        a.state[v] = a.tag;
        return true;
    } else if (A == A_SSSP) {
        // SSSP: relax the edge; an improved vertex is re-activated once per round.
        uint64_t nd = uint64_t(uval) + w;
        if (nd > 0xFFFFFFFEull) {
            atomicOr(&a.bitmap[v >> 5], 1u << (v & 31u));
            atomicOr(&a.ctr[C_OVERFLOW], 1ull);
            return false;
        }
        if (a.state[v] <= uint32_t(nd)) return false;
        uint32_t old = atomicMin(&a.state[v], uint32_t(nd));
        if (old <= uint32_t(nd)) return false;
        return atomicExch(&a.stamp[v], a.tag) != a.tag;
    } else {
        // CC: push the smaller label; a lowered vertex is re-activated once per round.
        if (a.state[v] <= uval) return false;
        uint32_t old = atomicMin(&a.state[v], uval);
        if (old <= uval) return false;
        return atomicExch(&a.stamp[v], a.tag) != a.tag;
    }
}

struct ScanArgs {
    const uint32_t *queue;  // null: the frontier is every vertex 0..n-1
    uint32_t n;
    const uint64_t *row_ptr;
    const void *col;
    const uint32_t *w;
    uint32_t *next;
    uint64_t align_mask;    // elements per request unit - 1
    uint32_t req_unit;      // bytes
    uint32_t col_bytes;
    const uint64_t *chunk_scan;  // V5 only
};

__device__ __forceinline__ uint64_t request_bytes(uint64_t s, uint64_t e, uint32_t cb, uint32_t R) {
    uint64_t first = (s * cb) / R, last = (e * cb + R - 1) / R;
    return (last - first) * R;
}

__device__ __forceinline__ uint32_t frontier_at(const ScanArgs &s, uint32_t q) {
    return s.queue ? s.queue[q] : q;
}

// ---------------------------------------------------------------------------
// V2/V3: one wave per frontier vertex.  V3 rounds the start down to the
// request unit and masks the lanes below the true start (Sec. 4.3.2).
// ---------------------------------------------------------------------------
template <class ColT, int A, bool ALIGN>
__global__ __launch_bounds__(kBlock) void k_wave(ScanArgs s, OpArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(s.col);
    uint64_t edges = 0, reqb = 0, verts = 0;
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t q = uint64_t(blockIdx.x) * kWavesPerBlock + wid; q < s.n; q += nw) {
        const uint32_t u = uniform32(frontier_at(s, uint32_t(q)));
        const uint64_t b = uniform64(s.row_ptr[u]), e = uniform64(s.row_ptr[u + 1]);
        if (b == e) continue;
        const uint32_t uval = uniform32(source_value<A>(a, u));
        if (lane == 0) {
            edges += e - b;
            reqb += request_bytes(b, e, s.col_bytes, s.req_unit);
            verts += 1;
        }
        const uint64_t start = ALIGN ? (b & ~s.align_mask) : b;
        for (uint64_t j0 = start; j0 < e; j0 += uint64_t(kWave) * kUnroll) {
            uint32_t v[kUnroll], w[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const uint64_t j = j0 + uint64_t(k) * kWave + lane;
                ok[k] = (j >= b) && (j < e);
                v[k] = 0;
                w[k] = 0;
                if (ok[k]) {
                    v[k] = load_col(col, j);
                    if (A == A_SSSP) w[k] = s.w[j];
                }
            }
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const bool p = ok[k] && visit<A>(a, uval, v[k], w[k]);
                stage(st, p, v[k], s.next, &a.ctr[C_NEXT], lane);
            }
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, edges, reqb, verts);
}

// ---------------------------------------------------------------------------
// V4: one 256-thread workgroup per frontier vertex (for hub lists).
// ---------------------------------------------------------------------------
template <class ColT, int A>
__global__ __launch_bounds__(kBlock) void k_block(ScanArgs s, OpArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(s.col);
    uint64_t edges = 0, reqb = 0, verts = 0;
    for (uint64_t q = blockIdx.x; q < s.n; q += gridDim.x) {
        const uint32_t u = uniform32(frontier_at(s, uint32_t(q)));
        const uint64_t b = uniform64(s.row_ptr[u]), e = uniform64(s.row_ptr[u + 1]);
        if (b == e) continue;
        const uint32_t uval = uniform32(source_value<A>(a, u));
        if (lane == 0 && wid == 0) {
            edges += e - b;
            reqb += request_bytes(b, e, s.col_bytes, s.req_unit);
            verts += 1;
        }
        const uint64_t start = b & ~s.align_mask;
        for (uint64_t j0 = start; j0 < e; j0 += uint64_t(kBlock) * 2) {
            uint32_t v[2], w[2];
            bool ok[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint64_t j = j0 + uint64_t(k) * kBlock + uint64_t(wid) * kWave + lane;
                ok[k] = (j >= b) && (j < e);
                v[k] = 0;
                w[k] = 0;
                if (ok[k]) {
                    v[k] = load_col(col, j);
                    if (A == A_SSSP) w[k] = s.w[j];
                }
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const bool p = ok[k] && visit<A>(a, uval, v[k], w[k]);
                stage(st, p, v[k], s.next, &a.ctr[C_NEXT], lane);
            }
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, edges, reqb, verts);
}

// ---------------------------------------------------------------------------
// V0: one thread per frontier vertex, element by element (Sec. 4.2 naive).
// V1: one 16-lane group per frontier vertex, start aligned to the group span.
// The wave loops until no lane of it has work, so staging stays uniform.
// ---------------------------------------------------------------------------
template <class ColT, int A, int G>
__global__ __launch_bounds__(kBlock) void k_group(ScanArgs s, OpArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(s.col);
    constexpr int kGroups = kWave / G;
    const int g = lane / G, gl = lane % G;
    uint64_t edges = 0, reqb = 0, verts = 0;
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t q0 = (uint64_t(blockIdx.x) * kWavesPerBlock + wid) * kGroups; q0 < s.n;
         q0 += nw * kGroups) {
        const uint64_t q = q0 + g;
        const bool has = q < s.n;
        uint32_t u = 0;
        uint64_t b = 0, e = 0;
        if (has) {
            u = frontier_at(s, uint32_t(q));
            b = s.row_ptr[u];
            e = s.row_ptr[u + 1];
        }
        uint32_t uval = 0;
        if (has && b < e) uval = source_value<A>(a, u);
        if (gl == 0 && b < e) {
            edges += e - b;
            reqb += request_bytes(b, e, s.col_bytes, s.req_unit);
            verts += 1;
        }
        // G == 1: no rounding (thread walks its own list); G == 16: round to the group span.
        const uint64_t start = (G == 1) ? b : (b & ~uint64_t(G - 1));
        for (uint64_t j = start + gl; __ballot(j < e) != 0; j += G) {
            const bool ok = (j >= b) && (j < e);
            uint32_t v = 0, w = 0;
            if (ok) {
                v = load_col(col, j);
                if (A == A_SSSP) w = s.w[j];
            }
            const bool p = ok && visit<A>(a, uval, v, w);
            stage(st, p, v, s.next, &a.ctr[C_NEXT], lane);
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, edges, reqb, verts);
}

// ---------------------------------------------------------------------------
// V5: edge-balanced.  Every frontier list is cut into aligned chunks of one
// wave load (64 elements, first chunk starting at the rounded-down start);
// chunk_scan[q] is the first chunk of entry q.  Waves take runs of
// kChunksPerWave consecutive chunks, so a hub is spread over many waves and
// many small lists share one wave.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t chunk_count(uint64_t b, uint64_t e, uint64_t mask) {
    if (b == e) return 0;
    const uint64_t start = b & ~mask;
    return (e - start + kWave - 1) / kWave;
}

// First q with chunk_scan[q + 1] > k  (chunk_scan has n + 1 entries).
__device__ __forceinline__ uint32_t find_entry(const uint64_t *scan, uint32_t n, uint64_t k) {
    uint32_t lo = 0, hi = n;  // answer in [0, n)
    while (lo + 1 < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (scan[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

template <class ColT, int A>
__global__ __launch_bounds__(kBlock) void k_balanced(ScanArgs s, OpArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(s.col);
    uint64_t edges = 0, reqb = 0, verts = 0;
    const uint64_t total = s.chunk_scan[s.n];
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t k0 = (uint64_t(blockIdx.x) * kWavesPerBlock + wid) * kChunksPerWave; k0 < total;
         k0 += nw * kChunksPerWave) {
        const uint64_t kend = k0 + kChunksPerWave < total ? k0 + kChunksPerWave : total;
        uint32_t q = uniform32(find_entry(s.chunk_scan, s.n, k0));
        uint64_t qfirst = uniform64(s.chunk_scan[q]), qnext = uniform64(s.chunk_scan[q + 1]);
        uint32_t u = uniform32(frontier_at(s, q));
        uint64_t b = uniform64(s.row_ptr[u]), e = uniform64(s.row_ptr[u + 1]);
        uint32_t uval = uniform32(source_value<A>(a, u));
        for (uint64_t kb = k0; kb < kend; kb += kUnroll) {
            uint32_t v[kUnroll], w[kUnroll], uv[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int i = 0; i < kUnroll; ++i) {
                const uint64_t kk = kb + i;
                ok[i] = false;
                v[i] = 0;
                w[i] = 0;
                uv[i] = uval;
                if (kk < kend) {
                    while (kk >= qnext) {  // next entry that owns chunks (uniform)
                        ++q;
                        qfirst = qnext;
                        qnext = uniform64(s.chunk_scan[q + 1]);
                        if (qnext > qfirst) {
                            u = uniform32(frontier_at(s, q));
                            b = uniform64(s.row_ptr[u]);
                            e = uniform64(s.row_ptr[u + 1]);
                            uval = uniform32(source_value<A>(a, u));
                        }
                    }
                    uv[i] = uval;
                    if (kk == qfirst && lane == 0) {
                        edges += e - b;
                        reqb += request_bytes(b, e, s.col_bytes, s.req_unit);
                        verts += 1;
                    }
                    const uint64_t j = (b & ~s.align_mask) + (kk - qfirst) * kWave + lane;
                    ok[i] = (j >= b) && (j < e);
                    if (ok[i]) {
                        v[i] = load_col(col, j);
                        if (A == A_SSSP) w[i] = s.w[j];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < kUnroll; ++i) {
                const bool p = ok[i] && visit<A>(a, uv[i], v[i], w[i]);
                stage(st, p, v[i], s.next, &a.ctr[C_NEXT], lane);
            }
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, edges, reqb, verts);
}

// ---- V5 prefix scan of per-entry chunk counts (reduce, scan partials, scan) ----
constexpr int kScanItems = 16;                  // entries per thread
constexpr int kScanTile = kBlock * kScanItems;  // entries per block

__device__ __forceinline__ uint64_t entry_chunks(const ScanArgs &s, uint32_t q) {
    if (q >= s.n) return 0;
    const uint32_t u = frontier_at(s, q);
    return chunk_count(s.row_ptr[u], s.row_ptr[u + 1], s.align_mask);
}

__device__ uint64_t block_exclusive_scan(uint64_t x, uint64_t *total) {
    __shared__ uint64_t s_w[kWavesPerBlock];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    uint64_t inc = x;
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t lo = __shfl_up(uint32_t(inc), o), hi = __shfl_up(uint32_t(inc >> 32), o);
        if (lane >= o) inc += (uint64_t(hi) << 32) | lo;
    }
    if (lane == kWave - 1) s_w[wid] = inc;
    __syncthreads();
    uint64_t wbase = 0, tot = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
        if (w < wid) wbase += s_w[w];
        tot += s_w[w];
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - x;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(ScanArgs s, uint64_t *block_sums) {
    uint64_t sum = 0;
    const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
    for (int i = 0; i < kScanItems; ++i) sum += entry_chunks(s, uint32_t(base + i));
    uint64_t tot;
    (void)block_exclusive_scan(sum, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_partials(uint64_t *block_sums, uint32_t nb) {
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nb; b0 += kBlock) {
        const uint32_t i = b0 + threadIdx.x;
        const uint64_t x = i < nb ? block_sums[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan(x, &tot);
        const uint64_t carry = s_carry;
        if (i < nb) block_sums[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_write(ScanArgs s, const uint64_t *block_sums,
                                                       uint64_t *scan) {
    uint64_t c[kScanItems];
    uint64_t sum = 0;
    const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
    for (int i = 0; i < kScanItems; ++i) {
        c[i] = entry_chunks(s, uint32_t(base + i));
        sum += c[i];
    }
    uint64_t tot;
    uint64_t run = block_sums[blockIdx.x] + block_exclusive_scan(sum, &tot);
    for (int i = 0; i < kScanItems; ++i) {
        const uint64_t q = base + i;
        if (q <= s.n) scan[q] = run;  // entry n receives the grand total
        run += c[i];
    }
}

// ---------------------------------------------------------------------------
// initialisation kernels
// ---------------------------------------------------------------------------
__global__ void k_fill(uint32_t *a, uint64_t n, uint32_t value) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        a[i] = value;
}

__global__ void k_iota(uint32_t *a, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        a[i] = uint32_t(i);
}

__global__ void k_seed_source(uint32_t *state, uint32_t *bitmap, uint32_t *queue, uint32_t src,
                              int mark) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        state[src] = 0;
        if (mark) bitmap[src >> 5] |= 1u << (src & 31u);
        queue[0] = src;
    }
}

// SSSP: a vertex that saw an overflowing relaxation and never got a finite
// distance is reachable only by paths longer than 0xFFFFFFFE.
__global__ void k_overflow_check(const uint32_t *dist, const uint32_t *marks, uint64_t V,
                                 unsigned long long *ctr) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V;
         i += uint64_t(gridDim.x) * blockDim.x)
        if (((marks[i >> 5] >> (i & 31u)) & 1u) && dist[i] == 0xFFFFFFFFu)
            atomicOr(&ctr[C_OVERFLOW], 2ull);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static unsigned fill_grid(uint64_t n) {
    uint64_t g = (n + kBlock - 1) / kBlock;
    return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(g, 4096)));
}

static emogi_status_t ensure_pool(emogi_graph_s *g, int algo) {
    Pool &p = g->pool;
    const uint64_t V = std::max<uint64_t>(g->V, 1);
    auto dalloc = [&](void **ptr, size_t bytes) -> emogi_status_t {
        if (*ptr) return EMOGI_OK;
        if (hipMalloc(ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            set_error("hipMalloc of %zu bytes for traversal state failed", bytes);
            return EMOGI_E_OOM_DEVICE;
        }
        return EMOGI_OK;
    };
    emogi_status_t st;
    for (int i = 0; i < 2; ++i)
        if ((st = dalloc(reinterpret_cast<void **>(&p.queue[i]), V * sizeof(uint32_t))) != EMOGI_OK)
            return st;
    if ((st = dalloc(reinterpret_cast<void **>(&p.bitmap), ((V + 31) / 32) * sizeof(uint32_t))) != EMOGI_OK)
        return st;
    if (algo != A_BFS &&
        (st = dalloc(reinterpret_cast<void **>(&p.stamp), V * sizeof(uint32_t))) != EMOGI_OK)
        return st;
    if ((st = dalloc(reinterpret_cast<void **>(&p.counters), C_COUNT * sizeof(unsigned long long))) != EMOGI_OK)
        return st;
    if (!p.host_counters) {
        if (hipHostMalloc(reinterpret_cast<void **>(&p.host_counters), C_COUNT * sizeof(unsigned long long),
                          hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p.host_counters = nullptr;
            set_error("pinned counter allocation failed");
            return EMOGI_E_OOM_HOST;
        }
    }
    return EMOGI_OK;
}

static emogi_status_t ensure_scan(emogi_graph_s *g, uint64_t n) {
    Pool &p = g->pool;
    if (p.chunk_scan && p.chunk_cap >= n) return EMOGI_OK;
    if (p.chunk_scan) (void)hipFree(p.chunk_scan);
    if (p.block_sums) (void)hipFree(p.block_sums);
    p.chunk_scan = nullptr;
    p.block_sums = nullptr;
    const uint64_t cap = std::max<uint64_t>(g->V, 1);
    const uint64_t nb = (cap + kScanTile) / kScanTile + 1;
    if (hipMalloc(&p.chunk_scan, (cap + 1 + kScanTile) * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&p.block_sums, nb * sizeof(uint64_t)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc for the balanced-variant scan failed");
        return EMOGI_E_OOM_DEVICE;
    }
    p.chunk_cap = cap;
    return EMOGI_OK;
}

template <class ColT, int A>
static void launch_variant(int var, const ScanArgs &s, const OpArgs &a, hipStream_t stream) {
    const uint64_t n = s.n;
    auto grid_for = [&](uint64_t per_block) {
        uint64_t b = (n + per_block - 1) / per_block;
        return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(b, kMaxGrid)));
    };
    switch (var) {
    case EMOGI_V0_THREAD:
        hipLaunchKernelGGL((k_group<ColT, A, 1>), dim3(grid_for(kBlock)), dim3(kBlock), 0, stream, s, a);
        break;
    case EMOGI_V1_GROUP16:
        hipLaunchKernelGGL((k_group<ColT, A, 16>), dim3(grid_for(kBlock / 16)), dim3(kBlock), 0, stream, s, a);
        break;
    case EMOGI_V2_WAVE:
        hipLaunchKernelGGL((k_wave<ColT, A, false>), dim3(grid_for(kWavesPerBlock)), dim3(kBlock), 0, stream, s, a);
        break;
    case EMOGI_V3_WAVE_ALIGNED:
        hipLaunchKernelGGL((k_wave<ColT, A, true>), dim3(grid_for(kWavesPerBlock)), dim3(kBlock), 0, stream, s, a);
        break;
    case EMOGI_V4_BLOCK:
        hipLaunchKernelGGL((k_block<ColT, A>), dim3(grid_for(1)), dim3(kBlock), 0, stream, s, a);
        break;
    default:
        hipLaunchKernelGGL((k_balanced<ColT, A>), dim3(kMaxGrid), dim3(kBlock), 0, stream, s, a);
        break;
    }
}

// The built-in rule of thumb (also the learned scheduler's fallback).
int heuristic_variant(const emogi_graph_s *g, uint64_t n) {
    if (n >= 2048) return EMOGI_V5_BALANCED;
    if (g->max_degree > 4096) return EMOGI_V5_BALANCED;
    return EMOGI_V3_WAVE_ALIGNED;
}

int choose_variant(emogi_graph_s *g, int algo, uint64_t n, const uint32_t *queue, hipStream_t stream,
                   float *features);

// Probe mode: save (restore=false) or restore (restore=true) the state a
// level step modifies, so every variant can be timed on the same level.
static emogi_status_t snapshot(emogi_graph_s *g, int algo, uint32_t *out, hipStream_t stream,
                               bool restore) {
    Pool &p = g->pool;
    const uint64_t V = std::max<uint64_t>(g->V, 1), words = (V + 31) / 32;
    if (!p.snap_state) {
        if (hipMalloc(&p.snap_state, V * 4) != hipSuccess || hipMalloc(&p.snap_stamp, V * 4) != hipSuccess ||
            hipMalloc(&p.snap_bitmap, words * 4) != hipSuccess) {
            (void)hipGetLastError();
            set_error("probe snapshot allocation failed");
            return EMOGI_E_OOM_DEVICE;
        }
    }
    auto cp = [&](void *live, void *snap, size_t bytes) {
        return restore ? hipMemcpyAsync(live, snap, bytes, hipMemcpyDeviceToDevice, stream)
                       : hipMemcpyAsync(snap, live, bytes, hipMemcpyDeviceToDevice, stream);
    };
    EMOGI_HIP_TRY(cp(out, p.snap_state, V * 4), EMOGI_E_HIP);
    if (algo != A_CC) EMOGI_HIP_TRY(cp(p.bitmap, p.snap_bitmap, words * 4), EMOGI_E_HIP);
    if (algo != A_BFS) EMOGI_HIP_TRY(cp(p.stamp, p.snap_stamp, V * 4), EMOGI_E_HIP);
    return EMOGI_OK;
}

static emogi_status_t traverse(emogi_graph_s *g, int algo, uint64_t src, uint32_t *out,
                               hipStream_t stream) {
    if (!g || !out) {
        set_error("null graph or output");
        return EMOGI_E_INVALID;
    }
    if (algo != A_CC && src >= g->V) {
        set_error("source %llu out of range (V = %llu)", (unsigned long long)src,
                  (unsigned long long)g->V);
        return EMOGI_E_INVALID;
    }
    if (algo == A_SSSP && !g->weights) {
        set_error("SSSP needs edge weights");
        return EMOGI_E_INVALID;
    }
    if (algo == A_CC && !(g->flags & EMOGI_F_SYMMETRIC)) {
        set_error("CC needs a graph created with EMOGI_F_SYMMETRIC");
        return EMOGI_E_NOT_SYMMETRIC;
    }
    {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, out) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            set_error("output must be device memory");
            return EMOGI_E_INVALID;
        }
    }
    emogi_status_t st = ensure_pool(g, algo);
    if (st != EMOGI_OK) return st;
    Pool &p = g->pool;
    const uint64_t V = g->V;
    emogi_stats_t &S = g->stats;
    memset(&S, 0, sizeof(S));
    S.request_unit = g->request_unit;

    EMOGI_HIP_TRY(hipEventRecord(g->ev_begin, stream), EMOGI_E_HIP);
    // ---- initial active set (Algorithm 1, set_initial_active_vertex) ----
    uint64_t n;
    bool identity = false;
    if (V > 0) {
        if (algo == A_CC) {
            hipLaunchKernelGGL(k_iota, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V);
            EMOGI_HIP_TRY(hipMemsetAsync(p.stamp, 0, V * sizeof(uint32_t), stream), EMOGI_E_HIP);
            n = V;
            identity = true;  // every vertex starts active (Sec. 5.4)
        } else {
            hipLaunchKernelGGL(k_fill, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V, 0xFFFFFFFFu);
            EMOGI_HIP_TRY(hipMemsetAsync(p.bitmap, 0, ((V + 31) / 32) * sizeof(uint32_t), stream),
                          EMOGI_E_HIP);
            if (algo == A_SSSP)
                EMOGI_HIP_TRY(hipMemsetAsync(p.stamp, 0, V * sizeof(uint32_t), stream), EMOGI_E_HIP);
            hipLaunchKernelGGL(k_seed_source, dim3(1), dim3(64), 0, stream, out, p.bitmap, p.queue[0],
                               uint32_t(src), algo == A_BFS ? 1 : 0);
            n = 1;
        }
        EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
    } else {
        n = 0;
    }

    uint64_t cap = V + 2;
    if (const char *env = getenv("EMOGI_MAX_ITERS")) cap = std::min<uint64_t>(cap, strtoull(env, nullptr, 10));
    const uint32_t align_elems = std::max<uint32_t>(1, g->request_unit / g->col_bytes);
    int cur = 0;
    uint32_t iter = 0;
    bool overflow_seen = false;
    while (n > 0) {
        if (iter >= cap) {
            (void)hipStreamSynchronize(stream);
            set_error("iteration cap %llu reached", (unsigned long long)cap);
            return EMOGI_E_NOCONVERGE;
        }
        const uint32_t *queue = identity ? nullptr : p.queue[cur];
        // One level with variant `v`: counters cleared, (V5) chunk scan, the
        // scan kernel between two events, counters copied back, host waits.
        auto run_level = [&](int v, float *ms_out) -> emogi_status_t {
            ScanArgs s;
            s.queue = queue;
            s.n = uint32_t(n);
            s.row_ptr = g->row_ptr;
            s.col = g->col;
            s.w = g->weights;
            s.next = p.queue[identity ? 0 : cur ^ 1];
            s.align_mask = uint64_t(align_elems) - 1;
            s.req_unit = g->request_unit;
            s.col_bytes = g->col_bytes;
            s.chunk_scan = nullptr;
            OpArgs a;
            a.state = out;
            a.bitmap = p.bitmap;
            a.stamp = p.stamp;
            a.tag = iter + 1;  // BFS: level of the next frontier; SSSP/CC: round
            a.V = uint32_t(V);
            a.ctr = p.counters;
            EMOGI_HIP_TRY(hipMemsetAsync(p.counters, 0, C_COUNT * sizeof(unsigned long long), stream),
                          EMOGI_E_HIP);
            if (v == EMOGI_V5_BALANCED) {
                emogi_status_t e2 = ensure_scan(g, n);
                if (e2 != EMOGI_OK) return e2;
                const unsigned nb = unsigned((n + kScanTile) / kScanTile);  // covers entry n too
                hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums);
                hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, stream, p.block_sums, nb);
                hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums,
                                   p.chunk_scan);
                s.chunk_scan = p.chunk_scan;
            }
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k0, stream), EMOGI_E_HIP);
            const int key = algo * 2 + (g->col_bytes == 8 ? 1 : 0);
            switch (key) {
            case 0: launch_variant<uint32_t, A_BFS>(v, s, a, stream); break;
            case 1: launch_variant<uint64_t, A_BFS>(v, s, a, stream); break;
            case 2: launch_variant<uint32_t, A_SSSP>(v, s, a, stream); break;
            case 3: launch_variant<uint64_t, A_SSSP>(v, s, a, stream); break;
            case 4: launch_variant<uint32_t, A_CC>(v, s, a, stream); break;
            default: launch_variant<uint64_t, A_CC>(v, s, a, stream); break;
            }
            EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k1, stream), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipMemcpyAsync(p.host_counters, p.counters, C_COUNT * sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, stream),
                          EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipEventElapsedTime(ms_out, g->ev_k0, g->ev_k1), EMOGI_E_HIP);
            return EMOGI_OK;
        };
        float feats[16];
        const bool want_feats = g->record_features && iter < EMOGI_MAX_LEVEL_STATS;
        int var = choose_variant(g, algo, n, queue, stream, want_feats ? feats : nullptr);
        if (var < 0) {
            set_error("scheduler kernels failed");
            return EMOGI_E_HIP;
        }
        if (want_feats) memcpy(S.level_features[iter], feats, sizeof(feats));
        if (g->sched_mode == EMOGI_SCHED_PROBE) {
            // Time every variant on the same level state, then run the fastest.
            if ((st = snapshot(g, algo, out, stream, false)) != EMOGI_OK) return st;
            float best = 1e30f;
            for (int v = 0; v < EMOGI_NUM_VARIANTS; ++v) {
                if (v > 0 && (st = snapshot(g, algo, out, stream, true)) != EMOGI_OK) return st;
                float pm = 0.f;
                if ((st = run_level(v, &pm)) != EMOGI_OK) return st;
                if (iter < EMOGI_MAX_LEVEL_STATS) S.level_probe_ms[iter][v] = pm;
                if (pm < best) {
                    best = pm;
                    var = v;
                }
            }
            if ((st = snapshot(g, algo, out, stream, true)) != EMOGI_OK) return st;
        }
        float ms = 0.f;
        if ((st = run_level(var, &ms)) != EMOGI_OK) return st;
        const unsigned long long *hc = p.host_counters;
        if (iter < EMOGI_MAX_LEVEL_STATS) {
            S.level_variant[iter] = uint8_t(var);
            S.level_frontier[iter] = uint32_t(n);
            S.level_ms[iter] = ms;
            S.level_edges[iter] = hc[C_EDGES];
            S.level_count = iter + 1;
        }
        S.variant_hist[var] += 1;
        S.expand_ms += ms;
        S.expand_launches += 1;
        S.edges_scanned += hc[C_EDGES];
        S.request_bytes += hc[C_REQBYTES];
        S.vertices_expanded += hc[C_VERTS];
        if (hc[C_OVERFLOW]) overflow_seen = true;
        n = hc[C_NEXT];
        if (identity) {
            identity = false;
            cur = 0;
        } else {
            cur ^= 1;
        }
        ++iter;
    }
    S.iterations = iter;
    S.useful_link_bytes = S.edges_scanned * (g->col_bytes + (algo == A_SSSP ? 4u : 0u));
    if (overflow_seen) {
        EMOGI_HIP_TRY(hipMemsetAsync(p.counters, 0, C_COUNT * sizeof(unsigned long long), stream),
                      EMOGI_E_HIP);
        hipLaunchKernelGGL(k_overflow_check, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, p.bitmap,
                           V, p.counters);
        EMOGI_HIP_TRY(hipMemcpyAsync(p.host_counters, p.counters, C_COUNT * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, stream),
                      EMOGI_E_HIP);
    }
    EMOGI_HIP_TRY(hipEventRecord(g->ev_end, stream), EMOGI_E_HIP);
    EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
    float total = 0.f;
    EMOGI_HIP_TRY(hipEventElapsedTime(&total, g->ev_begin, g->ev_end), EMOGI_E_HIP);
    S.total_ms = total;
    if (overflow_seen && (p.host_counters[C_OVERFLOW] & 2ull)) {
        set_error("a reachable vertex's distance exceeds 0xFFFFFFFE");
        return EMOGI_E_OVERFLOW;
    }
    return EMOGI_OK;
}

}  // namespace emogi

using namespace emogi;

extern "C" {

emogi_status_t emogi_bfs(emogi_graph_t g, uint64_t src, uint32_t *levels, void *stream) {
    return traverse(g, A_BFS, src, levels, static_cast<hipStream_t>(stream));
}

emogi_status_t emogi_sssp(emogi_graph_t g, uint64_t src, uint32_t *dist, void *stream) {
    return traverse(g, A_SSSP, src, dist, static_cast<hipStream_t>(stream));
}

emogi_status_t emogi_cc(emogi_graph_t g, uint32_t *labels, void *stream) {
    return traverse(g, A_CC, 0, labels, static_cast<hipStream_t>(stream));
}

}  // extern "C"
