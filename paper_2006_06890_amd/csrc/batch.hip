// Batched multi-source BFS and SSSP: up to 64 sources traverse together and
// every neighbour list read from the (zero-copy) edge list serves all sources
// that are active at that vertex.  The paper runs 64 sources per graph one at
// a time and averages them (Sec. 5.2); on a link-bound path the list reads
// are the cost, so sharing them is the MI355X-side win.
//
// Per vertex, one 64-bit mask says which sources have it in the current
// frontier (and for BFS which sources have visited it).  A level step is:
//   expand the short-list queue (a wave per vertex, start aligned to R,
//   Sec. 4.3.2) and the hub queue (a workgroup per vertex); pushes are
//   ballot-compacted through LDS segments; then clear the expanded masks and
//   advance the level.
// Steps read queue lengths from device memory, so several are captured into
// one hipGraph and replayed without a host round trip per level; a step whose
// frontier is empty does nothing, so over-running the last level is harmless.
#include "internal.h"
#include "packed.h"
#include "tier.h"
#include "wave.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

namespace emogi {

enum BatchCounter : int {
    B_Q0 = 0, B_Q1 = 1,  // short-list queue lengths (by parity)
    B_H0 = 2, B_H1 = 3,  // hub queue lengths (by parity)
    B_LEVEL = 4,         // number of non-empty steps executed
    B_OVF = 5,           // SSSP: an overflowing relaxation happened / a distance overflowed
    B_EDGES = 6,         // sum of degrees of expanded vertices
    B_TIER = 7,          // of those, edges read from the HBM tier
    B_READY = 8,         // SSSP bands: 1 when this step expanded a vertex (some source inside the band)
    B_BMIN = 9,          // SSSP: 2^32 - smallest distance left pending beyond the band (0: none)
    B_SPLIT = 10,        // SSSP: the band's upper end, shared by all sources
    B_REFILL = 11,       // SSSP: 1 when the next step starts by listing waiting sources
    B_PKB = 12,          // packed lists: encoded bytes of the lists expanded
    B_COUNT = 13
};

constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kBUnroll = 4;

struct BatchArgs {
    const uint64_t *row_ptr;
    const void *col;
    const uint32_t *w;
    unsigned long long *front, *next;  // masks: current and next frontier
    unsigned long long *vis;           // BFS
    unsigned long long *ovf;           // SSSP
    unsigned long long *wait;          // SSSP: sources waiting for a later band, per vertex
    uint32_t *out;                     // BFS: levels [n][V]; SSSP: dist [V][64]
    const uint32_t *q, *h;             // current short / hub queues
    uint32_t *nq, *nh;                 // next short / hub queues
    unsigned long long *ctr;
    int cur;                           // parity of the current queues
    uint32_t n;                        // number of sources
    uint64_t V;
    uint64_t align_mask;
    uint32_t hub_degree;
    TierView tier;                     // HBM copies of hub lists (tier.bits null: none)
    uint32_t delta;                    // SSSP band width (0: one band)
    const uint32_t *pk;                // packed lists (EMOGI_F_PACK), or null
    const uint64_t *pk_off;
    const uint8_t *pk_width, *pk_wwidth;
};

// A packed list's blocks (wave-uniform): first word, gap and weight widths,
// words per full block, and the encoded bytes a scan of it reads (its
// weights only when the scan uses them).
struct PackedList {
    uint64_t w0;
    uint32_t w, ww, full;
    uint64_t bytes;
};

__device__ __forceinline__ PackedList packed_list(const BatchArgs &a, uint32_t u, uint64_t d, bool weights) {
    PackedList L;
    L.w0 = uniform64(a.pk_off[u]);
    L.w = uniform32(a.pk_width[u]);
    L.ww = a.pk_wwidth ? uniform32(a.pk_wwidth[u]) : 0u;
    L.full = packed_block_words(L.w, L.ww);
    const uint64_t words = uniform64(a.pk_off[u + 1]) - L.w0;
    L.bytes = 4 * (weights ? words : words - packed_weight_words(d, L.ww));
    return L;
}


// Folds a kernel's expanded-edge counts into the batch counters.
__device__ __forceinline__ void batch_count(const BatchArgs &a, int lane, uint64_t edges, uint64_t tedges,
                                            uint64_t pkb) {
    edges = wave_sum64(edges);
    tedges = wave_sum64(tedges);
    pkb = wave_sum64(pkb);
    if (lane == 0 && edges) atomicAdd(&a.ctr[B_EDGES], (unsigned long long)edges);
    if (lane == 0 && tedges) atomicAdd(&a.ctr[B_TIER], (unsigned long long)tedges);
    if (lane == 0 && pkb) atomicAdd(&a.ctr[B_PKB], (unsigned long long)pkb);
}

// Pushes v (when `push`) to the short or hub queue by its degree.
__device__ __forceinline__ void push_vertex(const BatchArgs &a, Stage &st, bool push, uint32_t v,
                                            int lane) {
    bool hub = false;
    if (push) hub = (a.row_ptr[v + 1] - a.row_ptr[v]) > a.hub_degree;
    stage(st, push && !hub, v, a.nq, &a.ctr[B_Q0 + (a.cur ^ 1)], lane);
    if (push && hub) {
        const uint32_t i = uint32_t(atomicAdd(&a.ctr[B_H0 + (a.cur ^ 1)], 1ull));
        a.nh[i] = v;
    }
}

// SSSP bands for a batch: a source whose distance at u is not below the
// shared split waits — its bit moves to wait[u] and u is not re-queued for
// it; the smallest waiting distance decides the next split when a step finds
// nothing inside the band (the next step then lists the waiting sources that
// the new band covers, k_brefill).  Returns the mask of sources ready to
// expand u.  Uniform per wave; `lead` marks the one wave (of a workgroup)
// that records the waits.
__device__ __forceinline__ unsigned long long sssp_ready(const BatchArgs &a, uint32_t u, unsigned long long fm,
                                                         uint32_t du, int lane, bool lead) {
    if (!a.delta) return fm;  // one band: every pending source expands
    const uint32_t split = uint32_t(a.ctr[B_SPLIT]);
    const bool pend = (fm >> lane) & 1ull;
    const unsigned long long rm = __ballot(pend && du < split);
    const unsigned long long wait = fm & ~rm;
    if (wait && lead) {
        uint32_t m = (pend && du >= split) ? du : kInf;
        for (int o = 32; o > 0; o >>= 1) m = min(m, uint32_t(__shfl_xor(m, o)));
        if (lane == 0) {
            atomicMax(&a.ctr[B_BMIN], 0x100000000ull - m);
            atomicOr(&a.wait[u], wait);
        }
    }
    if (rm && lead && lane == 0) {
        a.ctr[B_READY] = 1ull;
        if (a.wait[u] & rm) atomicAnd(&a.wait[u], ~rm);  // expanded now: no longer waiting
    }
    return rm;
}

// First kernel of every SSSP step: after a band change (ctr[B_REFILL]) the
// waiting sources now below the split join the current frontier masks and
// their vertices the current queues; the sources still waiting give the
// smallest waiting distance again.  Does nothing otherwise.
__global__ __launch_bounds__(kBlock) void k_brefill(BatchArgs a) {
    if (a.ctr[B_REFILL] == 0) return;
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const uint32_t split = uint32_t(a.ctr[B_SPLIT]);
    uint32_t *q = const_cast<uint32_t *>(a.q);
    uint32_t m = kInf;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t v0 = uint64_t(blockIdx.x) * blockDim.x + uint64_t(wid) * kWave; v0 < a.V; v0 += stride) {
        const uint64_t mine = v0 + lane;
        const unsigned long long wv = mine < a.V ? a.wait[mine] : 0ull;
        for (unsigned long long todo = __ballot(wv != 0ull); todo; todo &= todo - 1) {
            const int k = __builtin_ctzll(todo);
            const uint32_t u = uint32_t(v0 + k);
            const unsigned long long wu = uniform64(__shfl(wv, k));
            const bool w8 = (wu >> lane) & 1ull;
            const uint32_t du = w8 ? a.out[uint64_t(u) * 64 + lane] : kInf;
            const unsigned long long rm = __ballot(w8 && du < split);
            if (w8 && du >= split) m = min(m, du);
            bool push = false, hub = false;
            if (rm && lane == 0) {
                atomicAnd(&a.wait[u], ~rm);
                push = atomicOr(const_cast<unsigned long long *>(&a.front[u]), rm) == 0ull;
                hub = (a.row_ptr[u + 1] - a.row_ptr[u]) > a.hub_degree;
            }
            push = __shfl(int(push), 0) != 0;
            hub = __shfl(int(hub), 0) != 0;
            stage(st, push && !hub && lane == 0, u, q, &a.ctr[B_Q0 + a.cur], lane);
            if (push && hub && lane == 0) {
                const uint32_t i = uint32_t(atomicAdd(&a.ctr[B_H0 + a.cur], 1ull));
                const_cast<uint32_t *>(a.h)[i] = u;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) m = min(m, uint32_t(__shfl_xor(m, o)));
    if (lane == 0 && m != kInf) atomicMax(&a.ctr[B_BMIN], 0x100000000ull - m);
    finish_queue(st, q, &a.ctr[B_Q0 + a.cur], lane, wid);
}

// BFS step for one neighbour v of a vertex whose frontier mask is fm.
__device__ __forceinline__ bool bfs_visit(const BatchArgs &a, unsigned long long fm, uint32_t v,
                                          uint32_t level) {
    if (v >= a.V) return false;
    const unsigned long long m = fm & ~a.vis[v];
    if (!m) return false;
    const unsigned long long newly = m & ~atomicOr(&a.vis[v], m);
    if (!newly) return false;
    for (unsigned long long b = newly; b; b &= b - 1) {
        const int s = __builtin_ctzll(b);
        a.out[uint64_t(s) * a.V + v] = level;
    }
    return atomicOr(&a.next[v], newly) == 0ull;
}

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_bbfs_short(BatchArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(a.col);
    const uint64_t n = a.ctr[B_Q0 + a.cur];
    const uint32_t level = uint32_t(a.ctr[B_LEVEL]) + 1;
    uint64_t edges = 0, tedges = 0, pkb = 0;
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t q = uint64_t(blockIdx.x) * kWavesPerBlock + wid; q < n; q += nw) {
        const uint32_t u = uniform32(a.q[q]);
        const uint64_t b = uniform64(a.row_ptr[u]), e = uniform64(a.row_ptr[u + 1]);
        const unsigned long long fm = uniform64(a.front[u]);
        if constexpr (kPacked<ColT>) {
            // one decoded block of 64 ids at a time
            const PackedList L = packed_list(a, u, e - b, false);
            if (lane == 0) {
                edges += e - b;
                pkb += L.bytes;
            }
            for (uint64_t k = 0; k * kWave < e - b; ++k) {
                const uint64_t rest = e - b - k * kWave;
                const uint32_t cnt = rest < uint64_t(kWave) ? uint32_t(rest) : uint32_t(kWave);
                const uint32_t v = packed_block(a.pk, L.w0 + k * L.full, L.w, L.ww, cnt, lane, nullptr);
                const bool p = uint32_t(lane) < cnt && bfs_visit(a, fm, v, level);
                push_vertex(a, st, p, v, lane);
            }
        } else {
            const ListSrc<ColT> src = list_src(a.tier, col, a.w, u, b);
            if (lane == 0) {
                edges += e - b;
                if (src.tier) tedges += e - b;
            }
            for (uint64_t j0 = b & ~a.align_mask; j0 < e; j0 += uint64_t(kWave) * kBUnroll) {
                uint32_t v[kBUnroll];
                bool ok[kBUnroll];
#pragma unroll
                for (int k = 0; k < kBUnroll; ++k) {
                    const uint64_t j = j0 + uint64_t(k) * kWave + lane;
                    ok[k] = j >= b && j < e;
                    v[k] = ok[k] ? uint32_t(src.col[j - src.shift]) : 0u;
                }
#pragma unroll
                for (int k = 0; k < kBUnroll; ++k) {
                    const bool p = ok[k] && bfs_visit(a, fm, v[k], level);
                    push_vertex(a, st, p, v[k], lane);
                }
            }
        }
    }
    finish_queue(st, a.nq, &a.ctr[B_Q0 + (a.cur ^ 1)], lane, wid);
    batch_count(a, lane, edges, tedges, pkb);
}

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_bbfs_hub(BatchArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(a.col);
    const uint64_t n = a.ctr[B_H0 + a.cur];
    const uint32_t level = uint32_t(a.ctr[B_LEVEL]) + 1;
    uint64_t edges = 0, tedges = 0, pkb = 0;
    for (uint64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const uint32_t u = uniform32(a.h[q]);
        const uint64_t b = uniform64(a.row_ptr[u]), e = uniform64(a.row_ptr[u + 1]);
        const unsigned long long fm = uniform64(a.front[u]);
        if constexpr (kPacked<ColT>) {
            // the workgroup's waves take the list's blocks in turn
            const PackedList L = packed_list(a, u, e - b, false);
            if (lane == 0 && wid == 0) {
                edges += e - b;
                pkb += L.bytes;
            }
            for (uint64_t k = wid; k * kWave < e - b; k += kWavesPerBlock) {
                const uint64_t rest = e - b - k * kWave;
                const uint32_t cnt = rest < uint64_t(kWave) ? uint32_t(rest) : uint32_t(kWave);
                const uint32_t v = packed_block(a.pk, L.w0 + k * L.full, L.w, L.ww, cnt, lane, nullptr);
                const bool p = uint32_t(lane) < cnt && bfs_visit(a, fm, v, level);
                push_vertex(a, st, p, v, lane);
            }
        } else {
            const ListSrc<ColT> src = list_src(a.tier, col, a.w, u, b);
            if (lane == 0 && wid == 0) {
                edges += e - b;
                if (src.tier) tedges += e - b;
            }
            for (uint64_t j0 = b & ~a.align_mask; j0 < e; j0 += uint64_t(kBlock) * 2) {
                uint32_t v[2];
                bool ok[2];
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const uint64_t j = j0 + uint64_t(k) * kBlock + uint64_t(wid) * kWave + lane;
                    ok[k] = j >= b && j < e;
                    v[k] = ok[k] ? uint32_t(src.col[j - src.shift]) : 0u;
                }
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const bool p = ok[k] && bfs_visit(a, fm, v[k], level);
                    push_vertex(a, st, p, v[k], lane);
                }
            }
        }
    }
    finish_queue(st, a.nq, &a.ctr[B_Q0 + (a.cur ^ 1)], lane, wid);
    batch_count(a, lane, edges, tedges, pkb);
}

// SSSP: lane s of the wave is source s.  The wave loads 64 (neighbour,
// weight) pairs of u's list, then walks them one at a time; each lane relaxes
// its own source's distance row dist[v][s] (a 256-byte coalesced access).
__device__ __forceinline__ void sssp_relax_chunk(const BatchArgs &a, Stage &st, int lane,
                                                 unsigned long long fm, uint32_t du,
                                                 uint32_t vl, uint32_t wl, bool okl) {
    const bool mine = ((fm >> lane) & 1ull) && du != kInf;
    uint64_t todo = __ballot(okl);
    while (todo) {
        // up to kBUnroll edges: load their distance rows first, then relax
        int ks[kBUnroll];
        uint32_t vs[kBUnroll], cur[kBUnroll];
        uint64_t nd[kBUnroll];
        int cnt = 0;
#pragma unroll
        for (int i = 0; i < kBUnroll; ++i) {
            ks[i] = -1;
            if (todo) {
                const int k = __builtin_ctzll(todo);
                todo &= todo - 1;
                ks[i] = k;
                cnt = i + 1;
            }
        }
#pragma unroll
        for (int i = 0; i < kBUnroll; ++i) {
            vs[i] = 0;
            cur[i] = 0;
            nd[i] = 0;
            if (i < cnt) {
                vs[i] = __builtin_amdgcn_readlane(vl, ks[i]);
                const uint32_t w = __builtin_amdgcn_readlane(wl, ks[i]);
                nd[i] = uint64_t(du) + w;
                if (mine && vs[i] < a.V) cur[i] = a.out[uint64_t(vs[i]) * 64 + lane];
            }
        }
#pragma unroll
        for (int i = 0; i < kBUnroll; ++i) {
            if (i >= cnt) continue;
            const uint32_t v = vs[i];
            bool imp = false;
            if (mine && v < a.V) {
                if (nd[i] > 0xFFFFFFFEull) {
                    atomicOr(&a.ovf[v], 1ull << lane);
                    atomicOr(&a.ctr[B_OVF], 1ull);
                } else if (uint32_t(nd[i]) < cur[i]) {
                    imp = atomicMin(&a.out[uint64_t(v) * 64 + lane], uint32_t(nd[i])) > uint32_t(nd[i]);
                }
            }
            const uint64_t nb = __ballot(imp);
            bool push = false;
            if (nb && lane == 0) push = atomicOr(&a.next[v], (unsigned long long)nb) == 0ull;
            push_vertex(a, st, push, v, lane);
        }
    }
}

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_bsssp_short(BatchArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(a.col);
    const uint64_t n = a.ctr[B_Q0 + a.cur];
    uint64_t edges = 0, tedges = 0, pkb = 0;
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t q = uint64_t(blockIdx.x) * kWavesPerBlock + wid; q < n; q += nw) {
        const uint32_t u = uniform32(a.q[q]);
        const uint64_t b = uniform64(a.row_ptr[u]), e = uniform64(a.row_ptr[u + 1]);
        const uint32_t du = a.out[uint64_t(u) * 64 + lane];
        const unsigned long long fm = sssp_ready(a, u, uniform64(a.front[u]), du, lane, true);
        if (!fm) continue;
        if constexpr (kPacked<ColT>) {
            const PackedList L = packed_list(a, u, e - b, true);
            if (lane == 0) {
                edges += e - b;
                pkb += L.bytes;
            }
            for (uint64_t k = 0; k * kWave < e - b; ++k) {
                const uint64_t rest = e - b - k * kWave;
                const uint32_t cnt = rest < uint64_t(kWave) ? uint32_t(rest) : uint32_t(kWave);
                uint32_t wl = 0;
                const uint32_t vl = packed_block(a.pk, L.w0 + k * L.full, L.w, L.ww, cnt, lane, &wl);
                sssp_relax_chunk(a, st, lane, fm, du, vl, wl, uint32_t(lane) < cnt);
            }
        } else {
            const ListSrc<ColT> src = list_src(a.tier, col, a.w, u, b);
            if (lane == 0) {
                edges += e - b;
                if (src.tier) tedges += e - b;
            }
            for (uint64_t j0 = b & ~a.align_mask; j0 < e; j0 += kWave) {
                const uint64_t j = j0 + lane;
                const bool ok = j >= b && j < e;
                const uint32_t vl = ok ? uint32_t(src.col[j - src.shift]) : 0u;
                const uint32_t wl = ok ? src.w[j - src.shift] : 0u;
                sssp_relax_chunk(a, st, lane, fm, du, vl, wl, ok);
            }
        }
    }
    finish_queue(st, a.nq, &a.ctr[B_Q0 + (a.cur ^ 1)], lane, wid);
    batch_count(a, lane, edges, tedges, pkb);
}

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_bsssp_hub(BatchArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(a.col);
    const uint64_t n = a.ctr[B_H0 + a.cur];
    uint64_t edges = 0, tedges = 0, pkb = 0;
    for (uint64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const uint32_t u = uniform32(a.h[q]);
        const uint64_t b = uniform64(a.row_ptr[u]), e = uniform64(a.row_ptr[u + 1]);
        const uint32_t du = a.out[uint64_t(u) * 64 + lane];
        const unsigned long long fm = sssp_ready(a, u, uniform64(a.front[u]), du, lane, wid == 0);
        if (!fm) continue;
        if constexpr (kPacked<ColT>) {
            const PackedList L = packed_list(a, u, e - b, true);
            if (lane == 0 && wid == 0) {
                edges += e - b;
                pkb += L.bytes;
            }
            for (uint64_t k = wid; k * kWave < e - b; k += kWavesPerBlock) {
                const uint64_t rest = e - b - k * kWave;
                const uint32_t cnt = rest < uint64_t(kWave) ? uint32_t(rest) : uint32_t(kWave);
                uint32_t wl = 0;
                const uint32_t vl = packed_block(a.pk, L.w0 + k * L.full, L.w, L.ww, cnt, lane, &wl);
                sssp_relax_chunk(a, st, lane, fm, du, vl, wl, uint32_t(lane) < cnt);
            }
        } else {
            const ListSrc<ColT> src = list_src(a.tier, col, a.w, u, b);
            if (lane == 0 && wid == 0) {
                edges += e - b;
                if (src.tier) tedges += e - b;
            }
            for (uint64_t j0 = (b & ~a.align_mask) + uint64_t(wid) * kWave; j0 < e; j0 += kBlock) {
                const uint64_t j = j0 + lane;
                const bool ok = j >= b && j < e;
                const uint32_t vl = ok ? uint32_t(src.col[j - src.shift]) : 0u;
                const uint32_t wl = ok ? src.w[j - src.shift] : 0u;
                sssp_relax_chunk(a, st, lane, fm, du, vl, wl, ok);
            }
        }
    }
    finish_queue(st, a.nq, &a.ctr[B_Q0 + (a.cur ^ 1)], lane, wid);
    batch_count(a, lane, edges, tedges, pkb);
}

// Clears the masks of the vertices just expanded (they become the next
// step's "next" masks) and, in block 0, nothing else: counters move in k_btick.
__global__ __launch_bounds__(kBlock) void k_bclear(BatchArgs a) {
    const uint64_t ns = a.ctr[B_Q0 + a.cur], nh = a.ctr[B_H0 + a.cur];
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ns + nh; i += stride) {
        const uint32_t u = i < ns ? a.q[i] : a.h[i - ns];
        a.front[u] = 0ull;
    }
}

// End of a step.  BFS, and SSSP in one band: a step with a non-empty queue is
// a level / round.  SSSP in bands: a step that expanded something is a round;
// one that only deferred sources opens the next band at the smallest waiting
// distance + delta and has the next step list the waiting sources first.
__global__ void k_btick(unsigned long long *ctr, int cur, int sssp, uint32_t delta) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (!sssp || !delta) {
            if (ctr[B_Q0 + cur] + ctr[B_H0 + cur] > 0) ctr[B_LEVEL] += 1;
        } else {
            ctr[B_REFILL] = 0;  // consumed by this step's k_brefill
            if (ctr[B_READY] > 0) {
                ctr[B_LEVEL] += 1;
            } else if (delta && ctr[B_BMIN] != 0) {
                const unsigned long long next = (0x100000000ull - ctr[B_BMIN]) + delta;
                ctr[B_SPLIT] = next < 0xFFFFFFFFull ? next : 0xFFFFFFFFull;
                ctr[B_REFILL] = 1;
                ctr[B_BMIN] = 0;  // k_brefill recomputes it for the sources left waiting
            }
        }
        ctr[B_READY] = 0;
        ctr[B_Q0 + cur] = 0;
        ctr[B_H0 + cur] = 0;
    }
}

__global__ void k_bfill64(unsigned long long *a, uint64_t n) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        a[i] = 0ull;
}

__global__ void k_bfill32(uint32_t *a, uint64_t n, uint32_t value) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        a[i] = value;
}

// Seeds: source s starts at srcs[s] with level / distance 0.
__global__ void k_bseed(BatchArgs a, const uint64_t *srcs, int sssp) {
    const uint32_t s = threadIdx.x;
    if (blockIdx.x != 0 || s >= a.n) return;
    const uint32_t v = uint32_t(srcs[s]);
    const unsigned long long bit = 1ull << s;
    if (sssp) {
        a.out[uint64_t(v) * 64 + s] = 0;
        if (s == 0) a.ctr[B_SPLIT] = a.delta ? a.delta : kInf;
    }
    else {
        a.out[uint64_t(s) * a.V + v] = 0;
        atomicOr(&a.vis[v], bit);
    }
    if (atomicOr(&a.front[v], bit) == 0ull) {
        const bool hub = (a.row_ptr[v + 1] - a.row_ptr[v]) > a.hub_degree;
        const uint32_t i = uint32_t(atomicAdd(&a.ctr[hub ? B_H0 : B_Q0], 1ull));
        (hub ? const_cast<uint32_t *>(a.h) : const_cast<uint32_t *>(a.q))[i] = v;
    }
}

// dist[V][64] -> out[s][V] through a 64x64 LDS tile.
__global__ __launch_bounds__(256) void k_btranspose(const uint32_t *dist, uint32_t *out, uint64_t V,
                                                    uint32_t n) {
    __shared__ uint32_t tile[64][65];
    const uint64_t v0 = uint64_t(blockIdx.x) * 64;
    for (int r = threadIdx.x / 64; r < 64; r += 4) {
        const uint64_t v = v0 + r;
        tile[r][threadIdx.x % 64] = v < V ? dist[v * 64 + threadIdx.x % 64] : kInf;
    }
    __syncthreads();
    for (int s = threadIdx.x / 64; s < int(n); s += 4) {
        const uint64_t v = v0 + threadIdx.x % 64;
        if (v < V) out[uint64_t(s) * V + v] = tile[threadIdx.x % 64][s];
    }
}

// A distance that saw an overflowing relaxation and stayed infinite overflowed.
__global__ void k_boverflow(const uint32_t *dist, const unsigned long long *ovf, uint64_t V,
                            uint32_t n, unsigned long long *ctr) {
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < V;
         v += uint64_t(gridDim.x) * blockDim.x) {
        const unsigned long long m = ovf[v];
        for (unsigned long long b = m; b; b &= b - 1) {
            const int s = __builtin_ctzll(b);
            if (uint32_t(s) < n && dist[v * 64 + s] == kInf) atomicOr(&ctr[B_OVF], 2ull);
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static unsigned grid_for(uint64_t n) {
    return unsigned(std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 8192)));
}

static emogi_status_t ensure_batch(emogi_graph_s *g, bool sssp) {
    BatchPool &b = g->batch;
    const uint64_t V = std::max<uint64_t>(g->V, 1);
    auto dalloc = [&](void **p, size_t bytes) -> emogi_status_t {
        if (*p) return EMOGI_OK;
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            set_error("hipMalloc of %zu bytes for batched traversal failed", bytes);
            return EMOGI_E_OOM_DEVICE;
        }
        return EMOGI_OK;
    };
    emogi_status_t st;
    for (int i = 0; i < 2; ++i) {
        if ((st = dalloc(reinterpret_cast<void **>(&b.mask[i]), V * 8)) != EMOGI_OK) return st;
        if ((st = dalloc(reinterpret_cast<void **>(&b.hub[i]), V * 4)) != EMOGI_OK) return st;
        if ((st = dalloc(reinterpret_cast<void **>(&g->pool.queue[i]), V * 4)) != EMOGI_OK) return st;
    }
    if ((st = dalloc(reinterpret_cast<void **>(&b.ctr), B_COUNT * 8)) != EMOGI_OK) return st;
    if ((st = dalloc(reinterpret_cast<void **>(&b.srcs), 64 * 8)) != EMOGI_OK) return st;
    if (sssp) {
        if ((st = dalloc(reinterpret_cast<void **>(&b.ovf), V * 8)) != EMOGI_OK) return st;
        if ((st = dalloc(reinterpret_cast<void **>(&b.wait), V * 8)) != EMOGI_OK) return st;
        if ((st = dalloc(reinterpret_cast<void **>(&b.dist), V * 64 * 4)) != EMOGI_OK) return st;
    } else {
        if ((st = dalloc(reinterpret_cast<void **>(&b.vis), V * 8)) != EMOGI_OK) return st;
    }
    if (!b.host_ctr && hipHostMalloc(reinterpret_cast<void **>(&b.host_ctr), B_COUNT * 8,
                                     hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        b.host_ctr = nullptr;
        set_error("pinned counter allocation failed");
        return EMOGI_E_OOM_HOST;
    }
    if (!b.stream && hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        b.stream = nullptr;
        set_error("hipStreamCreate failed");
        return EMOGI_E_HIP;
    }
    return EMOGI_OK;
}

template <class ColT>
static void launch_step(const BatchArgs &a, bool sssp, unsigned grid, hipStream_t s) {
    if (sssp) {
        if (a.delta) hipLaunchKernelGGL(k_brefill, dim3(grid), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_bsssp_short<ColT>, dim3(grid), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_bsssp_hub<ColT>, dim3(grid), dim3(kBlock), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_bbfs_short<ColT>, dim3(grid), dim3(kBlock), 0, s, a);
        hipLaunchKernelGGL(k_bbfs_hub<ColT>, dim3(grid), dim3(kBlock), 0, s, a);
    }
    hipLaunchKernelGGL(k_bclear, dim3(grid), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_btick, dim3(1), dim3(64), 0, s, a.ctr, a.cur, sssp ? 1 : 0, a.delta);
}

static emogi_status_t run_batch(emogi_graph_s *g, bool sssp, const uint64_t *srcs, uint32_t n,
                                uint32_t *out, hipStream_t caller) {
    if (!g || !srcs || !out || n == 0 || n > 64) {
        set_error("batched traversal needs 1..64 sources and an output");
        return EMOGI_E_INVALID;
    }
    for (uint32_t i = 0; i < n; ++i)
        if (srcs[i] >= g->V) {
            set_error("source %llu out of range", (unsigned long long)srcs[i]);
            return EMOGI_E_INVALID;
        }
    if (sssp && !g->weights && !g->packed.wwidth) {
        set_error("SSSP needs edge weights");
        return EMOGI_E_INVALID;
    }
    {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, out) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            set_error("output must be device memory");
            return EMOGI_E_INVALID;
        }
    }
    emogi_status_t st = ensure_batch(g, sssp);
    if (st != EMOGI_OK) return st;
    BatchPool &b = g->batch;
    const emogi_batch_params_t P = g->batch_params;
    const uint64_t V = g->V;
    hipStream_t s = b.stream;
    const auto t0 = std::chrono::steady_clock::now();
    EMOGI_HIP_TRY(hipStreamSynchronize(caller), EMOGI_E_HIP);

    BatchArgs a;
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.w = g->weights;
    a.vis = b.vis;
    a.ovf = b.ovf;
    a.wait = b.wait;
    a.out = sssp ? b.dist : out;
    a.ctr = b.ctr;
    a.n = n;
    a.V = V;
    a.align_mask = std::max<uint32_t>(1, g->request_unit / g->col_bytes) - 1;
    a.tier = tier_view(g);
    a.hub_degree = P.hub_degree;
    a.delta = sssp ? P.sssp_delta : 0;
    a.pk = g->packed.stream;
    a.pk_off = g->packed.off;
    a.pk_width = g->packed.width;
    a.pk_wwidth = g->packed.wwidth;
    // ---- init ----
    EMOGI_HIP_TRY(hipMemcpyAsync(b.srcs, srcs, n * sizeof(uint64_t), hipMemcpyHostToDevice, s), EMOGI_E_HIP);
    hipLaunchKernelGGL(k_bfill64, dim3(grid_for(B_COUNT)), dim3(256), 0, s, b.ctr, uint64_t(B_COUNT));
    for (int i = 0; i < 2; ++i)
        hipLaunchKernelGGL(k_bfill64, dim3(grid_for(V)), dim3(256), 0, s, b.mask[i], V);
    if (sssp) {
        hipLaunchKernelGGL(k_bfill64, dim3(grid_for(V)), dim3(256), 0, s, b.ovf, V);
        hipLaunchKernelGGL(k_bfill64, dim3(grid_for(V)), dim3(256), 0, s, b.wait, V);
        hipLaunchKernelGGL(k_bfill32, dim3(grid_for(V * 64)), dim3(256), 0, s, b.dist, V * 64, kInf);
    } else {
        hipLaunchKernelGGL(k_bfill64, dim3(grid_for(V)), dim3(256), 0, s, b.vis, V);
        hipLaunchKernelGGL(k_bfill32, dim3(grid_for(uint64_t(n) * V)), dim3(256), 0, s, out,
                           uint64_t(n) * V, kInf);
    }
    {
        BatchArgs seed = a;
        seed.front = b.mask[0];
        seed.q = g->pool.queue[0];
        seed.h = b.hub[0];
        hipLaunchKernelGGL(k_bseed, dim3(1), dim3(64), 0, s, seed, b.srcs, sssp ? 1 : 0);
    }
    EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);

    // ---- the two step shapes (parity 0 and 1) ----
    BatchArgs step[2];
    for (int c = 0; c < 2; ++c) {
        step[c] = a;
        step[c].cur = c;
        step[c].front = b.mask[c];
        step[c].next = b.mask[c ^ 1];
        step[c].q = g->pool.queue[c];
        step[c].h = b.hub[c];
        step[c].nq = g->pool.queue[c ^ 1];
        step[c].nh = b.hub[c ^ 1];
    }
    const unsigned grid = 256u * std::max(1u, std::min(8u, P.blocks_per_cu));
    const uint32_t K = std::max(2u, std::min(32u, P.steps_per_graph & ~1u));
    const bool u64col = g->col_bytes == 8;
    auto enqueue_steps = [&]() {
        for (uint32_t k = 0; k < K; ++k) {
            if (g->packed.stream) launch_step<PackedCol>(step[k & 1], sssp, grid, s);
            else if (u64col) launch_step<uint64_t>(step[k & 1], sssp, grid, s);
            else launch_step<uint32_t>(step[k & 1], sssp, grid, s);
        }
    };
    hipGraphExec_t exec = nullptr;
    if (P.use_graph) {
        hipGraph_t graph = nullptr;
        EMOGI_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), EMOGI_E_HIP);
        enqueue_steps();
        hipError_t ce = hipStreamEndCapture(s, &graph);
        if (ce != hipSuccess || !graph) {
            (void)hipGetLastError();
            set_error("hipGraph capture of the level steps failed");
            return EMOGI_E_HIP;
        }
        ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ce != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipGraphInstantiate failed");
            return EMOGI_E_HIP;
        }
    }
    // rounds: each expands at least one vertex for one source, and with
    // bands the sources' rounds interleave, so the bound scales with n
    uint64_t cap = (V + 2) * (sssp ? n : 1);
    if (const char *env = getenv("EMOGI_MAX_ITERS")) cap = std::min<uint64_t>(cap, strtoull(env, nullptr, 10));
    uint64_t steps = 0;
    emogi_status_t rc = EMOGI_OK;
    for (;;) {
        if (exec) {
            if (hipGraphLaunch(exec, s) != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipGraphLaunch failed");
                rc = EMOGI_E_HIP;
                break;
            }
        } else {
            enqueue_steps();
        }
        steps += K;
        if (hipMemcpyAsync(b.host_ctr, b.ctr, B_COUNT * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            (void)hipGetLastError();
            set_error("batched step failed");
            rc = EMOGI_E_HIP;
            break;
        }
        // K is even: parity 0 is current; SSSP is done when nothing waits either
        if (b.host_ctr[B_Q0] + b.host_ctr[B_H0] == 0 && b.host_ctr[B_REFILL] == 0 && b.host_ctr[B_BMIN] == 0) break;
        // a step that expands nothing opens a band; its listing step finds
        // the smallest waiting distance anew, so at most two such steps come
        // in a row and steps stay below three times the rounds
        if (b.host_ctr[B_LEVEL] >= cap || steps >= 3 * cap + K) {
            set_error("iteration cap %llu reached", (unsigned long long)cap);
            rc = EMOGI_E_NOCONVERGE;
            break;
        }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (rc != EMOGI_OK) return rc;
    const uint64_t levels = b.host_ctr[B_LEVEL], edges = b.host_ctr[B_EDGES];
    bool overflow = false;
    if (sssp) {
        if (b.host_ctr[B_OVF]) {
            hipLaunchKernelGGL(k_boverflow, dim3(grid_for(V)), dim3(256), 0, s, b.dist, b.ovf, V, n, b.ctr);
            EMOGI_HIP_TRY(hipMemcpyAsync(b.host_ctr, b.ctr, B_COUNT * 8, hipMemcpyDeviceToHost, s), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipStreamSynchronize(s), EMOGI_E_HIP);
            overflow = (b.host_ctr[B_OVF] & 2ull) != 0;
        }
        hipLaunchKernelGGL(k_btranspose, dim3(unsigned((V + 63) / 64)), dim3(256), 0, s, b.dist, out, V, n);
        EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
    }
    EMOGI_HIP_TRY(hipStreamSynchronize(s), EMOGI_E_HIP);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    emogi_stats_t &S = g->stats;
    memset(&S, 0, sizeof(S));
    S.iterations = uint32_t(levels);
    S.edges_scanned = edges;
    S.tier_edges = b.host_ctr[B_TIER];
    if (g->packed.stream) {
        S.weights_read = 0;  // weights come packed inside the blocks
        S.useful_link_bytes = b.host_ctr[B_PKB];
    } else {
        S.weights_read = sssp ? edges - S.tier_edges : 0;  // every weight of a scanned list
        S.useful_link_bytes = (edges - S.tier_edges) * g->col_bytes + S.weights_read * 4;
    }
    S.total_ms = ms;
    S.expand_ms = ms;
    S.expand_launches = uint32_t(steps);
    S.request_unit = g->request_unit;
    if (overflow) {
        set_error("a reachable vertex's distance exceeds 0xFFFFFFFE");
        return EMOGI_E_OVERFLOW;
    }
    return EMOGI_OK;
}

}  // namespace emogi

using namespace emogi;

extern "C" {

emogi_status_t emogi_bfs_batch(emogi_graph_t g, const uint64_t *srcs, uint32_t n, uint32_t *out,
                               void *stream) {
    return run_batch(g, false, srcs, n, out, static_cast<hipStream_t>(stream));
}

emogi_status_t emogi_sssp_batch(emogi_graph_t g, const uint64_t *srcs, uint32_t n, uint32_t *out,
                                void *stream) {
    return run_batch(g, true, srcs, n, out, static_cast<hipStream_t>(stream));
}

emogi_status_t emogi_set_batch_params(emogi_graph_t g, const emogi_batch_params_t *p) {
    if (!g || !p || p->blocks_per_cu < 1 || p->blocks_per_cu > 8 || p->steps_per_graph < 2 ||
        p->steps_per_graph > 32 || (p->steps_per_graph & 1u)) {
        set_error("batch params: blocks_per_cu 1..8, steps_per_graph even in 2..32");
        return EMOGI_E_INVALID;
    }
    g->batch_params = *p;
    return EMOGI_OK;
}

emogi_status_t emogi_get_batch_params(emogi_graph_t g, emogi_batch_params_t *p) {
    if (!g || !p) {
        set_error("null argument");
        return EMOGI_E_INVALID;
    }
    *p = g->batch_params;
    return EMOGI_OK;
}

emogi_status_t emogi_autotune_batch(emogi_graph_t g, int algo, const uint64_t *srcs, uint32_t n,
                                    uint32_t *out, void *stream, emogi_batch_params_t *best,
                                    emogi_batch_trial_t *table, uint32_t table_len) {
    if (!g || (algo != 0 && algo != 1)) {
        set_error("autotune: algo must be 0 (BFS) or 1 (SSSP)");
        return EMOGI_E_INVALID;
    }
    // Candidate grid: hub threshold x level steps per replay x occupancy.
    const uint32_t hubs[] = {256, 1024, 8192};
    const uint32_t ks[] = {2, 8};
    const uint32_t bpc[] = {4, 8};
    emogi_batch_params_t keep = g->batch_params, win = keep;
    float win_ms = 1e30f;
    uint32_t t = 0;
    for (uint32_t h : hubs)
        for (uint32_t k : ks)
            for (uint32_t c : bpc) {
                g->batch_params = emogi_batch_params_t{h, k, c, 1, keep.sssp_delta};
                emogi_status_t st = run_batch(g, algo == 1, srcs, n, out, static_cast<hipStream_t>(stream));
                if (st != EMOGI_OK) {
                    g->batch_params = keep;
                    return st;
                }
                const float ms = float(g->stats.total_ms);
                if (table && t < table_len) table[t] = emogi_batch_trial_t{g->batch_params, ms};
                ++t;
                if (ms < win_ms) {
                    win_ms = ms;
                    win = g->batch_params;
                }
            }
    g->batch_params = win;
    if (best) *best = win;
    return EMOGI_OK;
}

}  // extern "C"
