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
#include "packed.h"
#include "tier.h"
#include "wave.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace emogi {

enum Algo { A_BFS = 0, A_SSSP = 1, A_CC = 2, A_LINK = 3 };  // A_LINK: CC union-find hooking pass

constexpr int kUnroll = 4;        // loads in flight per lane in the wave variants
constexpr int kChunksPerWave = 8; // V5: consecutive aligned chunks per wave visit
constexpr int kMaxGrid = 256 * 8; // 8 blocks of 4 waves on each of the 256 CUs

// Per-wave statistics of a scan, folded into the level's counters once per
// block (lane 0 of a list or chunk adds to most fields; see count_list).
struct Tally {
    uint64_t edges = 0;   // ids of the expanded lists
    uint64_t reqb = 0;    // those lists rounded out to the request unit
    uint64_t verts = 0;   // expanded vertices
    uint64_t tedges = 0;  // ids read from the HBM tier
    uint64_t wlink = 0;   // SSSP: weights read over the host link
    uint64_t pkb = 0;     // packed lists: encoded bytes scanned
    uint64_t isect = 0;   // 32-byte sectors of ids read over the host link
    uint64_t wsect = 0;   // 32-byte sectors of weights read over the host link
};

__device__ __forceinline__ void add_counter(unsigned long long *ctr, int c, uint64_t x) {
    x = wave_sum64(x);
    if (lane_id() == 0 && x) atomicAdd(&ctr[c], (unsigned long long)x);
}

__device__ __forceinline__ void flush_tally(const Tally &t, unsigned long long *ctr) {
    add_counter(ctr, C_EDGES, t.edges);
    add_counter(ctr, C_REQBYTES, t.reqb);
    add_counter(ctr, C_VERTS, t.verts);
    add_counter(ctr, C_TIER, t.tedges);
    add_counter(ctr, C_WLINK, t.wlink);
    add_counter(ctr, C_PKBYTES, t.pkb);
    add_counter(ctr, C_IDSECT, t.isect);
    add_counter(ctr, C_WSECT, t.wsect);
}

// End of a scan block: flush the staged frontier and fold the statistics.
__device__ __forceinline__ void finish_block(Stage &st, uint32_t *next, unsigned long long *ctr, int lane, int wid,
                                             const Tally &t) {
    finish_queue(st, next, &ctr[C_NEXT], lane, wid);
    flush_tally(t, ctr);
}

// Number of 32-byte sectors holding the 4-byte elements of the lanes in m,
// lane l's element at byte address base + 4 l (consecutive lanes, so the
// mask shifted by base's position inside its sector has one byte per sector).
__device__ __forceinline__ uint32_t sectors_of(uint64_t m, uint64_t base) {
    if (!m) return 0;
    const uint32_t off = uint32_t(base >> 2) & 7u;
    const uint64_t hi = off ? (m >> (64 - off)) : 0;
    uint64_t x = m << off;
    x |= x >> 4;
    x |= x >> 2;
    x |= x >> 1;
    return uint32_t(__popcll(x & 0x0101010101010101ull)) + (hi ? 1u : 0u);
}

// Per-list statistics: every expanded list counts its edges; a list read over
// the host link also counts its request-granular bytes, a tier list its edges.
__device__ __forceinline__ void count_list(bool tier, uint64_t b, uint64_t e, uint32_t cb, uint32_t R, Tally &t);

// ---------------------------------------------------------------------------
// Application step per neighbour (Algorithm 1's workload + condition).
// ---------------------------------------------------------------------------
struct OpArgs {
    uint32_t *state;    // levels / dist / labels (the caller's output array)
    uint32_t *bitmap;   // BFS visited bits; SSSP overflow marks
    uint32_t *stamp;    // CC label propagation: last round in which v was pushed
    uint32_t tag;       // BFS: level of the next frontier; CC: round number
    uint32_t V;         // neighbour ids at or above V are ignored (malformed input)
    uint32_t *nextbits; // ordered frontier: next frontier as a bitmap (null: LDS-staged queue);
                        // SSSP: vertices improved below the split this round
    uint32_t split;     // SSSP: improvements at or above it wait for a later band ...
    uint32_t *farbits;  // ... marked here
    uint32_t wmin;      // SSSP: no edge weight is smaller
    unsigned long long *ctr;
    const uint8_t *inmin = nullptr;  // SSSP: per target, no weight of an edge into it is smaller
};

template <int A>
__device__ __forceinline__ uint32_t source_value(const OpArgs &a, uint32_t u) {
    if (A == A_BFS) return 0u;
    if (A == A_LINK) return u;
    return a.state[u];
}

__device__ __forceinline__ uint32_t load_parent(const uint32_t *parent, uint32_t x) {
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Union of the trees of a and b in a parent forest where every parent id is
// at most its child's id: a root is only ever hooked below a smaller id, so
// the root of each finished tree is the smallest id of its component.  The
// larger of the two current roots strictly decreases every round, so the
// loop ends (the hooking step of Afforest, Sutton et al. 2018).
__device__ __forceinline__ void uf_link(uint32_t *parent, uint32_t a, uint32_t b) {
    uint32_t p1 = load_parent(parent, a), p2 = load_parent(parent, b);
    while (p1 != p2) {
        const uint32_t high = p1 > p2 ? p1 : p2, low = p1 > p2 ? p2 : p1;
        const uint32_t ph = load_parent(parent, high);
        if (ph == low) break;
        if (ph == high && atomicCAS(&parent[high], high, low) == high) break;
        p1 = load_parent(parent, load_parent(parent, high));
        p2 = load_parent(parent, low);
    }
}

// Returns 1 when v joins the next frontier, 2 when an SSSP improvement waits
// for a later band, else 0; SSSP adds kWeightRead when it read the weight.
constexpr int kWeightRead = 4;

template <int A, bool kGivenWeight = false>
__device__ __forceinline__ int visit(const OpArgs &a, uint32_t uval, uint32_t v, const uint32_t *wp,
                                     uint32_t wv = 0) {
    if (v >= a.V) return 0;
    if (A == A_BFS) {
        // BFS: an unvisited neighbour is visited at the next level.
        uint32_t word = v >> 5, bit = 1u << (v & 31u);
        if (a.bitmap[word] & bit) return 0;
        uint32_t old = atomicOr(&a.bitmap[word], bit);
        if (old & bit) return 0;
        a.state[v] = a.tag;
        return 1;
    } else if (A == A_SSSP) {
        // SSSP: relax the edge; an improved vertex joins the next round when
        // its distance is inside the band, otherwise it waits, marked.  The
        // weight is read (over the host link) only when the edge can improve
        // v: with dist(v) <= dist(u) + the smallest weight of an edge into v
        // it cannot.  Both bounds are HBM reads issued together.
        // (kGivenWeight: the weight wv came in a packed block with the id.)
        const uint32_t cur = a.state[v];
        uint64_t nd;
        int flag = 0;
        if constexpr (!kGivenWeight) {
            const uint32_t lo = a.inmin ? max(a.wmin, uint32_t(a.inmin[v])) : a.wmin;
            const uint64_t floor_nd = uint64_t(uval) + lo;
            if (floor_nd <= 0xFFFFFFFEull && cur <= floor_nd) return 0;
            nd = uint64_t(uval) + *wp;
            flag = kWeightRead;
        } else {
            nd = uint64_t(uval) + wv;
        }
        if (nd > 0xFFFFFFFEull) {
            atomicOr(&a.bitmap[v >> 5], 1u << (v & 31u));
            atomicOr(&a.ctr[C_OVERFLOW], 1ull);
            return flag;
        }
        if (cur <= uint32_t(nd)) return flag;
        uint32_t old = atomicMin(&a.state[v], uint32_t(nd));
        if (old <= uint32_t(nd)) return flag;
        return flag | (uint32_t(nd) < a.split ? 1 : 2);
    } else if (A == A_LINK) {
        uf_link(a.state, uval, v);
        return 0;
    } else {
        // CC: push the smaller label; a lowered vertex is re-activated once per round.
        if (a.state[v] <= uval) return 0;
        uint32_t old = atomicMin(&a.state[v], uval);
        if (old <= uval) return 0;
        return atomicExch(&a.stamp[v], a.tag) != a.tag ? 1 : 0;
    }
}

// Hands a visit result to the next-frontier staging.
// Uniform: every lane of the wave calls it.
template <int A>
__device__ __forceinline__ void emit(Stage &st, int r, uint32_t v, uint32_t *next, const OpArgs &a,
                                     int lane) {
    const uint32_t bit = 1u << (v & 31u);
    if (a.nextbits) {
        // ordered frontier: mark; a listing pass later lists the marks in id order
        if (r == 1 && !(a.nextbits[v >> 5] & bit)) atomicOr(&a.nextbits[v >> 5], bit);
    } else {
        stage(st, r == 1, v, next, &a.ctr[C_NEXT], lane);
    }
    if (A == A_SSSP && r == 2 && !(a.farbits[v >> 5] & bit)) atomicOr(&a.farbits[v >> 5], bit);
}

struct ScanArgs {
    const uint32_t *queue;  // null: the frontier is every vertex 0..n-1
    uint32_t n;
    const unsigned long long *n_dev;  // when set, the frontier length is *n_dev (left on
                                      // the device by the previous level) instead of n
    const uint64_t *row_ptr;
    const void *col;
    const uint32_t *w;
    uint32_t *next;
    uint64_t align_mask;    // elements per request unit - 1
    uint32_t req_unit;      // bytes
    uint32_t col_bytes;
    const uint64_t *chunk_scan;  // V5 only
    TierView tier;               // HBM copies of hub lists (tier.bits null: none)
    const uint32_t *pk = nullptr;        // packed lists (EMOGI_F_PACK; col is then unused)
    const uint64_t *pk_off = nullptr;    // word offset of each packed list (V + 1)
    const uint8_t *pk_width = nullptr;   // gap width of each packed list, bits
    const uint8_t *pk_wwidth = nullptr;  // weight width of each packed list, bits (null: no weights)
};

// V5 chunks loaded per group.  A packed block is a short read, so packed
// scans keep twice as many in flight per wave; so does SSSP, whose chunks
// wait on a second link read (the weights) after the first: eight chunks in
// flight at 4 waves per SIMD measured 2 % faster at R-MAT 26 than four at 6
// waves (609 against 621 ms), and as fast as two at 8 waves (with spills).
template <class ColT, int A = A_BFS>
constexpr int kGroupChunks = (kPacked<ColT> || A == A_SSSP) ? 8 : 4;

__device__ __forceinline__ uint64_t request_bytes(uint64_t s, uint64_t e, uint32_t cb, uint32_t R) {
    uint64_t first = (s * cb) / R, last = (e * cb + R - 1) / R;
    return (last - first) * R;
}

__device__ __forceinline__ void count_list(bool tier, uint64_t b, uint64_t e, uint32_t cb, uint32_t R, Tally &t) {
    t.edges += e - b;
    t.verts += 1;
    if (tier) {
        t.tedges += e - b;
    } else {
        t.reqb += request_bytes(b, e, cb, R);
        t.isect += request_bytes(b, e, cb, 32) / 32;
    }
}

// A packed list [b, e) in words [w0, w1) counts its edges, its encoded
// bytes (without its weight words unless the scan uses the weights), and
// its words rounded out to the request unit.  Its 32-byte sectors are
// counted per block as the blocks are read (count_packed_block).
__device__ __forceinline__ void count_packed(uint64_t b, uint64_t e, uint64_t w0, uint64_t w1, uint32_t ww,
                                             bool weights, uint32_t R, Tally &t) {
    const uint64_t d = e - b, nb = (d + 63) / 64, last = d - (nb - 1) * 64;
    const uint64_t wwords = (nb - 1) * 2 * uint64_t(ww) + (last * ww + 31) / 32;
    t.edges += d;
    t.verts += 1;
    t.reqb += request_bytes(w0, w1, 4, R);
    t.pkb += (w1 - w0 - (weights ? 0 : wwords)) * 4;
}

__device__ __forceinline__ uint32_t frontier_at(const ScanArgs &s, uint32_t q) {
    return s.queue ? s.queue[q] : q;
}

// The kernel's view of the scan arguments with the frontier length resolved.
__device__ __forceinline__ ScanArgs resolved(const ScanArgs &s0) {
    ScanArgs s = s0;
    if (s0.n_dev) s.n = uint32_t(*s0.n_dev);
    return s;
}

// ---------------------------------------------------------------------------
// V2/V3: one wave per frontier vertex.  V3 rounds the start down to the
// request unit and masks the lanes below the true start (Sec. 4.3.2).
// ---------------------------------------------------------------------------
template <class ColT, int A, bool ALIGN>
__global__ __launch_bounds__(kBlock) void k_wave(ScanArgs s0, OpArgs a) {
    const ScanArgs s = resolved(s0);
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(s.col);
    Tally t;
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t q = uint64_t(blockIdx.x) * kWavesPerBlock + wid; q < s.n; q += nw) {
        const uint32_t u = uniform32(frontier_at(s, uint32_t(q)));
        const uint64_t b = uniform64(s.row_ptr[u]), e = uniform64(s.row_ptr[u + 1]);
        if (b == e) continue;
        const uint32_t uval = uniform32(source_value<A>(a, u));
        const ListSrc<ColT> src = list_src(s.tier, col, s.w, u, b);
        if (lane == 0) count_list(src.tier, b, e, s.col_bytes, s.req_unit, t);
        const uint64_t start = ALIGN ? (b & ~s.align_mask) : b;
        for (uint64_t j0 = start; j0 < e; j0 += uint64_t(kWave) * kUnroll) {
            uint32_t v[kUnroll];
            const uint32_t *wp[kUnroll];
            bool ok[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const uint64_t j = j0 + uint64_t(k) * kWave + lane;
                ok[k] = (j >= b) && (j < e);
                v[k] = 0;
                wp[k] = (A == A_SSSP) ? src.w + (j - src.shift) : nullptr;
                if (ok[k]) v[k] = load_col(src.col, j - src.shift);
            }
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                const int r = ok[k] ? visit<A>(a, uval, v[k], wp[k]) : 0;
                if (A == A_SSSP && !src.tier) {
                    const uint64_t m = __ballot(r & kWeightRead);
                    if (lane == 0) {
                        t.wlink += __popcll(m);
                        t.wsect += sectors_of(m, reinterpret_cast<uint64_t>(src.w + (j0 + uint64_t(k) * kWave - src.shift)));
                    }
                }
                emit<A>(st, r & 3, v[k], s.next, a, lane);
            }
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, t);
}

// ---------------------------------------------------------------------------
// V4: one 256-thread workgroup per frontier vertex (for hub lists).
// ---------------------------------------------------------------------------
template <class ColT, int A>
__global__ __launch_bounds__(kBlock) void k_block(ScanArgs s0, OpArgs a) {
    const ScanArgs s = resolved(s0);
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(s.col);
    Tally t;
    for (uint64_t q = blockIdx.x; q < s.n; q += gridDim.x) {
        const uint32_t u = uniform32(frontier_at(s, uint32_t(q)));
        const uint64_t b = uniform64(s.row_ptr[u]), e = uniform64(s.row_ptr[u + 1]);
        if (b == e) continue;
        const uint32_t uval = uniform32(source_value<A>(a, u));
        const ListSrc<ColT> src = list_src(s.tier, col, s.w, u, b);
        if (lane == 0 && wid == 0) count_list(src.tier, b, e, s.col_bytes, s.req_unit, t);
        const uint64_t start = b & ~s.align_mask;
        for (uint64_t j0 = start; j0 < e; j0 += uint64_t(kBlock) * 2) {
            uint32_t v[2];
            const uint32_t *wp[2];
            bool ok[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const uint64_t j = j0 + uint64_t(k) * kBlock + uint64_t(wid) * kWave + lane;
                ok[k] = (j >= b) && (j < e);
                v[k] = 0;
                wp[k] = (A == A_SSSP) ? src.w + (j - src.shift) : nullptr;
                if (ok[k]) v[k] = load_col(src.col, j - src.shift);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int r = ok[k] ? visit<A>(a, uval, v[k], wp[k]) : 0;
                if (A == A_SSSP && !src.tier) {
                    const uint64_t m = __ballot(r & kWeightRead);
                    if (lane == 0) {
                        t.wlink += __popcll(m);
                        t.wsect += sectors_of(m, reinterpret_cast<uint64_t>(
                                                     src.w + (j0 + uint64_t(k) * kBlock + uint64_t(wid) * kWave - src.shift)));
                    }
                }
                emit<A>(st, r & 3, v[k], s.next, a, lane);
            }
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, t);
}

// ---------------------------------------------------------------------------
// V0: one thread per frontier vertex, element by element (Sec. 4.2 naive).
// V1: one 16-lane group per frontier vertex, start aligned to the group span.
// The wave loops until no lane of it has work, so staging stays uniform.
// ---------------------------------------------------------------------------
template <class ColT, int A, int G>
__global__ __launch_bounds__(kBlock) void k_group(ScanArgs s0, OpArgs a) {
    const ScanArgs s = resolved(s0);
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    const ColT *col = static_cast<const ColT *>(s.col);
    constexpr int kGroups = kWave / G;
    const int g = lane / G, gl = lane % G;
    Tally t;
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
        ListSrc<ColT> src{col, s.w, 0, false};
        if (has && b < e) {
            uval = source_value<A>(a, u);
            src = list_src(s.tier, col, s.w, u, b);
        }
        if (gl == 0 && b < e) count_list(src.tier, b, e, s.col_bytes, s.req_unit, t);
        // G == 1: no rounding (thread walks its own list); G == 16: round to the group span.
        const uint64_t start = (G == 1) ? b : (b & ~uint64_t(G - 1));
        for (uint64_t j = start + gl; __ballot(j < e) != 0; j += G) {
            const bool ok = (j >= b) && (j < e);
            uint32_t v = 0;
            if (ok) v = load_col(src.col, j - src.shift);
            const int r = ok ? visit<A>(a, uval, v, A == A_SSSP ? src.w + (j - src.shift) : nullptr) : 0;
            if ((r & kWeightRead) && !src.tier) {
                // lists of different lanes (groups) lie apart: one sector per
                // weight (an upper bound when neighbouring lists share one)
                ++t.wlink;
                ++t.wsect;
            }
            emit<A>(st, r & 3, v, s.next, a, lane);
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, t);
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

// The chunks one wave owns: runs of kChunksPerWave consecutive chunks, one
// run per grid stride.  All fields are wave-uniform.
template <class ColT>
struct ChunkCursor {
    uint64_t run0, kb, kend;           // current run [run0, kend), next chunk kb
    uint64_t stride, total;            // run stride of the grid, chunks of the level
    uint32_t q;                        // frontier entry owning chunk kb (or an earlier one)
    uint64_t qfirst, qnext;            // its chunk range
    uint32_t u, uval;
    uint64_t b, e;
    ListSrc<ColT> src;
    uint64_t pw0, pw1;       // packed: the list's words [pw0, pw1)
    uint32_t pwidth, pfull;  // packed: gap width, words per full block
    uint32_t wwidth;         // packed: weight width (0: no weights)
};

// U chunks' neighbours (and weights), loaded, not yet visited.
template <int U>
struct ChunkGroup {
    uint32_t v[U];
    bool ok[U];
    // wave-uniform per chunk: the source value, where lane 0's weight is
    // (SSSP reads lane l's at wbase + l only if needed), and the tier flag
    uint32_t uv[U];
    uint64_t wbase[U];
    bool tier[U];
    // packed lists: v[i] and wv[i] hold the lane's word of the block's id
    // and weight parts until the loads are back; shape[i] is the block's gap
    // width (bits 0-7), weight width (8-15) and id count (16-23)
    uint32_t shape[U];
    uint32_t wv[U];
};

template <class ColT, int A>
__device__ __forceinline__ void enter_entry(ChunkCursor<ColT> &c, const ScanArgs &s, const OpArgs &a) {
    c.u = uniform32(frontier_at(s, c.q));
    c.b = uniform64(s.row_ptr[c.u]);
    c.e = uniform64(s.row_ptr[c.u + 1]);
    c.uval = uniform32(source_value<A>(a, c.u));
    c.src = list_src(s.tier, static_cast<const ColT *>(s.col), s.w, c.u, c.b);
    if constexpr (kPacked<ColT>) {
        c.pw0 = uniform64(s.pk_off[c.u]);
        c.pw1 = uniform64(s.pk_off[c.u + 1]);
        c.pwidth = uniform32(s.pk_width[c.u]);
        c.wwidth = s.pk_wwidth ? uniform32(s.pk_wwidth[c.u]) : 0u;
        c.pfull = packed_block_words(c.pwidth, c.wwidth);
    }
}

template <class ColT, int A>
__device__ __forceinline__ void open_run(ChunkCursor<ColT> &c, const ScanArgs &s, const OpArgs &a, uint64_t k0) {
    if (k0 >= c.total) {
        c.kb = c.kend = c.total;
        return;
    }
    c.run0 = c.kb = k0;
    c.kend = k0 + kChunksPerWave < c.total ? k0 + kChunksPerWave : c.total;
    c.q = uniform32(find_entry(s.chunk_scan, s.n, k0));
    c.qfirst = uniform64(s.chunk_scan[c.q]);
    c.qnext = uniform64(s.chunk_scan[c.q + 1]);
    enter_entry<ColT, A>(c, s, a);
}

// Issues the loads of the next U chunks (those left in the run) and
// moves the cursor past them, to the next run when this one is done.
template <class ColT, int A>
__device__ __forceinline__ void load_group(ChunkCursor<ColT> &c, ChunkGroup<kGroupChunks<ColT, A>> &g, const ScanArgs &s,
                                           const OpArgs &a, int lane, Tally &t) {
    constexpr int U = kGroupChunks<ColT, A>;
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const uint64_t kk = c.kb + i;
        g.ok[i] = false;
        g.v[i] = 0;
        g.wbase[i] = 0;
        g.tier[i] = false;
        g.uv[i] = c.uval;
        if constexpr (kPacked<ColT>) {
            g.shape[i] = 0;
            g.wv[i] = 0;
        }
        if (kk < c.kend) {
            while (kk >= c.qnext) {  // next entry that owns chunks (uniform)
                ++c.q;
                c.qfirst = c.qnext;
                c.qnext = uniform64(s.chunk_scan[c.q + 1]);
                if (c.qnext > c.qfirst) enter_entry<ColT, A>(c, s, a);
            }
            g.uv[i] = c.uval;
            if (kk == c.qfirst && lane == 0) {
                if constexpr (kPacked<ColT>)
                    count_packed(c.b, c.e, c.pw0, c.pw1, c.wwidth, A == A_SSSP, s.req_unit, t);
                else
                    count_list(c.src.tier, c.b, c.e, s.col_bytes, s.req_unit, t);
            }
            const uint64_t j0 = uniform64((c.b & ~s.align_mask) + (kk - c.qfirst) * kWave);
            const uint64_t j = j0 + lane;
            g.ok[i] = (j >= c.b) && (j < c.e);
            if (A == A_SSSP) g.wbase[i] = uniform64(reinterpret_cast<uint64_t>(c.src.w + (j0 - c.src.shift)));
            g.tier[i] = c.src.tier;
            if constexpr (kPacked<ColT>) {
                // block kk - qfirst of the list (chunks of a packed list are its
                // blocks: align_mask is 0): lane l loads word l of the block's
                // ids and, for SSSP, word l of its weights (which follow the
                // ids), each word once
                const uint32_t cnt = uint32_t(c.e - j0 < uint64_t(kWave) ? c.e - j0 : uint64_t(kWave));
                const uint64_t idb = c.pw0 + (kk - c.qfirst) * c.pfull;
                const uint32_t idw = packed_id_words(cnt, c.pwidth);
                if (lane == 0) t.isect += request_bytes(idb, idb + idw, 4, 32) / 32;  // 32-byte sectors
                if (uint32_t(lane) < idw) g.v[i] = s.pk[idb + lane];
                if (A == A_SSSP && c.wwidth) {
                    const uint64_t wtb = idb + idw;
                    const uint32_t wwd = packed_block_weight_words(cnt, c.wwidth);
                    // the sectors the weight words add to the id words' ones
                    if (lane == 0)
                        t.wsect += request_bytes(idb, wtb + wwd, 4, 32) / 32 - request_bytes(idb, wtb, 4, 32) / 32;
                    if (uint32_t(lane) < wwd) g.wv[i] = s.pk[wtb + lane];
                }
                g.shape[i] = c.pwidth | (c.wwidth << 8) | (cnt << 16);
            } else {
                if (g.ok[i]) g.v[i] = load_col(c.src.col, j - c.src.shift);
            }
        }
    }
    if constexpr (kPacked<ColT>) {
        // decode from the words the lanes hold (lane moves, no memory access)
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t w = g.shape[i] & 0xFFu, ww = (g.shape[i] >> 8) & 0xFFu, cnt = g.shape[i] >> 16;
            g.v[i] = packed_ids(g.v[i], w, cnt, lane);
            if (A == A_SSSP) g.wv[i] = packed_weights(g.wv[i], ww, lane);
        }
    }
    c.kb += U;
    if (c.kb >= c.kend) open_run<ColT, A>(c, s, a, c.run0 + c.stride);
}

// V5 main loop: load U chunks, then visit their neighbours.  (Keeping
// the next group's loads in flight during the visits measured no faster:
// vector loads return in issue order, so the visits' HBM loads wait for them.)
template <class ColT, int A>
__device__ __forceinline__ void balanced_body(const ScanArgs &s0, const OpArgs &a,
                                              uint32_t (*seg)[kSegCap]) {
    constexpr int U = kGroupChunks<ColT, A>;
    const ScanArgs s = resolved(s0);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Stage st{seg[wid], 0};
    Tally t;
    ChunkCursor<ColT> c;
    c.total = s.chunk_scan[s.n];
    c.stride = uint64_t(gridDim.x) * kWavesPerBlock * kChunksPerWave;
    open_run<ColT, A>(c, s, a, (uint64_t(blockIdx.x) * kWavesPerBlock + wid) * kChunksPerWave);
    while (c.kb < c.kend) {
        ChunkGroup<U> g;
        load_group<ColT, A>(c, g, s, a, lane, t);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            int r = 0;
            if (g.ok[i]) {
                if constexpr (kPacked<ColT>)
                    r = visit<A, true>(a, g.uv[i], g.v[i], nullptr, g.wv[i]);
                else
                    r = visit<A>(a, g.uv[i], g.v[i], reinterpret_cast<const uint32_t *>(g.wbase[i]) + lane);
            }
            if (A == A_SSSP && !kPacked<ColT> && !g.tier[i]) {
                const uint64_t m = __ballot(r & kWeightRead);
                if (lane == 0) {
                    t.wlink += __popcll(m);
                    t.wsect += sectors_of(m, g.wbase[i]);
                }
            }
            emit<A>(st, r & 3, g.v[i], s.next, a, lane);
        }
    }
    finish_block(st, s.next, a.ctr, lane, wid, t);
}

template <class ColT, int A>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_balanced(ScanArgs s0,
                                                                                           OpArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    balanced_body<ColT, A>(s0, a, seg);
}

// V5 over packed lists, a kernel of its own: the decoding sets its register
// use (SSSP 120 VGPRs, 4 waves per SIMD; BFS 86, 5 waves), uncapped.
template <int A>
__global__ __launch_bounds__(kBlock) void k_balanced_packed(ScanArgs s0, OpArgs a) {
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    balanced_body<PackedCol, A>(s0, a, seg);
}

// ---------------------------------------------------------------------------
// Bottom-up BFS levels (direction-optimizing BFS).  The paper's Sec. 6 notes
// that a pull over incoming lists reads memory the way the push over
// outgoing lists does; on an undirected graph a vertex's list is also its
// list of incoming edges.  The current frontier is a bitmap (fbits); every
// unvisited vertex with edges reads its own list until it meets a frontier
// vertex, which puts it in the next level (there is no race: only the
// vertex itself decides).  The reads are small and mostly one per vertex,
// in vertex order, so they reach the host link as a dense stream of 32-byte
// requests.
//   k_bu_probe: a wave owns tiles of 64 consecutive vertices (two bitmap
//     words, written back whole, without atomics).  Its candidates are
//     compacted in LDS and served kBuLanes = 32 / sizeof(id) lanes each: a
//     step reads the 32-byte sector of the list that holds the next ids,
//     at most kBuProbeSectors steps; a candidate that neither found a
//     frontier neighbour nor ran out of ids is queued for
//   k_bu_rest: a wave per queued vertex, 64-id loads from where the probe
//     stopped, leaving at the first frontier neighbour.
// ---------------------------------------------------------------------------
constexpr int kBuProbeSectors = 2;
// Ids of a packed list the bottom-up probe decodes per unvisited vertex.
constexpr int kBuPackedProbeIds = 8;

struct BuArgs {
    const uint64_t *row_ptr;
    const void *col;
    TierView tier;
    uint64_t V;
    const uint32_t *fbits;    // the current frontier
    uint32_t *visited;        // BFS visited bits
    uint32_t *nextbits;       // the next frontier (marked here)
    uint32_t *level;          // levels (the caller's output)
    uint32_t tag;             // level of the next frontier
    uint32_t *rest;           // vertices left by the probe (k_bu_probe writes, k_bu_rest reads)
    unsigned long long *ctr;  // C_NEXT, C_FEDGES, C_REST, C_EDGES (ids examined), C_IDSECT,
                              // C_REQBYTES (sectors x 32), C_TIER, C_VERTS (candidates),
                              // C_PKBYTES (packed: encoded bytes read)
    const uint32_t *pk = nullptr;        // packed lists (EMOGI_F_PACK), or null
    const uint64_t *pk_off = nullptr;
    const uint8_t *pk_width = nullptr, *pk_wwidth = nullptr;
};

__device__ __forceinline__ bool in_frontier(const uint32_t *fbits, uint64_t V, uint32_t x) {
    return x < V && ((fbits[x >> 5] >> (x & 31u)) & 1u);
}

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_bu_probe(BuArgs s) {
    constexpr int G = 32 / int(sizeof(ColT));  // lanes per candidate: one sector of ids
    constexpr int S = kWave / G;               // candidates served per step
    __shared__ uint32_t cand[kWavesPerBlock][kWave];
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    __shared__ uint32_t found_w[kWavesPerBlock][2];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int slot = lane / G, gl = lane % G;
    const uint64_t gmask = ((uint64_t(1) << G) - 1) << (slot * G);
    Stage st{seg[wid], 0};
    Tally t;
    uint64_t nfound = 0, fedges = 0;
    const ColT *col = static_cast<const ColT *>(s.col);
    const uint64_t words = (s.V + 31) / 32, tiles = (s.V + 63) / 64;
    for (uint64_t tile = uint64_t(blockIdx.x) * kWavesPerBlock + wid; tile < tiles;
         tile += uint64_t(gridDim.x) * kWavesPerBlock) {
        const uint64_t w0 = 2 * tile;
        const uint32_t vis0 = s.visited[w0], vis1 = w0 + 1 < words ? s.visited[w0 + 1] : ~0u;
        const uint64_t vis = uint64_t(vis0) | (uint64_t(vis1) << 32);
        if (vis == ~uint64_t(0)) continue;  // (uniform) nothing left in the tile
        const uint64_t v = tile * 64 + lane;
        bool c = v < s.V && !((vis >> lane) & 1u);
        if (c) c = s.row_ptr[v + 1] > s.row_ptr[v];
        const uint64_t cm = __ballot(c);
        if (!cm) continue;
        if (c) cand[wid][rank_below(cm)] = uint32_t(v);
        if (lane < 2) found_w[wid][lane] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t nc = uint32_t(__popcll(cm));
        if (lane == 0) t.verts += nc;
        for (uint32_t r0 = 0; r0 < nc; r0 += S) {
            const uint32_t k = r0 + slot;
            const bool has = k < nc;
            uint32_t x = 0;
            uint64_t b = 0, e = 0;
            if (has) {
                x = cand[wid][k];
                b = s.row_ptr[x];
                e = s.row_ptr[x + 1];
            }
            const ListSrc<ColT> src = has ? list_src(s.tier, col, static_cast<const uint32_t *>(nullptr), x, b)
                                          : ListSrc<ColT>{col, nullptr, 0, false};
            const uint64_t j0 = b & ~uint64_t(G - 1);
            bool hit = false, more = has;
            for (int step = 0; step < kBuProbeSectors; ++step) {
                const uint64_t j = j0 + uint64_t(step) * G + gl;
                const bool ok = more && j >= b && j < e;
                uint32_t nb = 0;
                if (ok) nb = load_col(src.col, j - src.shift);
                const uint64_t fm = __ballot(ok && in_frontier(s.fbits, s.V, nb));
                const uint64_t om = __ballot(ok);
                if (gl == 0 && more) {
                    const uint32_t n_ok = uint32_t(__popcll(om & gmask));
                    t.edges += n_ok;
                    if (src.tier) t.tedges += n_ok;
                    else {
                        t.isect += 1;
                        t.reqb += 32;
                    }
                }
                if (fm & gmask) {
                    hit = true;
                    more = false;
                } else if (j0 + uint64_t(step + 1) * G >= e) {
                    more = false;
                }
                if (__ballot(more) == 0) break;
            }
            if (gl == 0 && hit) {
                s.level[x] = s.tag;
                atomicOr(&found_w[wid][(x & 63u) >> 5], 1u << (x & 31u));
                fedges += e - b;
            }
            // a candidate with ids left over goes to the wave-per-vertex pass
            stage(st, gl == 0 && more, x, s.rest, &s.ctr[C_REST], lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t f0 = found_w[wid][0], f1 = found_w[wid][1];
        if (lane == 0 && (f0 | f1)) {
            nfound += __popc(f0) + __popc(f1);
            // the wave owns both words of its tile during this kernel
            if (f0) {
                s.visited[w0] = vis0 | f0;
                s.nextbits[w0] |= f0;
            }
            if (f1) {
                s.visited[w0 + 1] = vis1 | f1;
                s.nextbits[w0 + 1] |= f1;
            }
        }
    }
    finish_queue(st, s.rest, &s.ctr[C_REST], lane, wid);
    flush_tally(t, s.ctr);
    add_counter(s.ctr, C_NEXT, nfound);
    add_counter(s.ctr, C_FEDGES, fedges);
}

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_bu_rest(BuArgs s) {
    constexpr int G = 32 / int(sizeof(ColT));
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Tally t;
    uint64_t nfound = 0, fedges = 0;
    const ColT *col = static_cast<const ColT *>(s.col);
    const uint64_t n = s.ctr[C_REST];
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t q = uint64_t(blockIdx.x) * kWavesPerBlock + wid; q < n; q += nw) {
        const uint32_t x = uniform32(s.rest[q]);
        const uint64_t b = uniform64(s.row_ptr[x]), e = uniform64(s.row_ptr[x + 1]);
        const ListSrc<ColT> src = list_src(s.tier, col, static_cast<const uint32_t *>(nullptr), x, b);
        // the probe read the sectors up to `from`
        const uint64_t from = (b & ~uint64_t(G - 1)) + uint64_t(kBuProbeSectors) * G;
        bool hit = false;
        for (uint64_t j0 = from & ~uint64_t(kWave - 1); j0 < e && !hit; j0 += kWave) {
            const uint64_t j = j0 + lane;
            const bool ok = j >= from && j < e;
            uint32_t nb = 0;
            if (ok) nb = load_col(src.col, j - src.shift);
            const uint64_t om = __ballot(ok);
            hit = __ballot(ok && in_frontier(s.fbits, s.V, nb)) != 0;
            if (lane == 0) {
                t.edges += __popcll(om);
                if (src.tier) {
                    t.tedges += __popcll(om);
                } else {
                    const uint64_t lo = j0 > from ? j0 : from, hi = j0 + kWave < e ? j0 + kWave : e;
                    const uint64_t sec = request_bytes(lo, hi, sizeof(ColT), 32) / 32;
                    t.isect += sec;
                    t.reqb += 32 * sec;
                }
            }
        }
        if (hit && lane == 0) {
            s.level[x] = s.tag;
            atomicOr(&s.visited[x >> 5], 1u << (x & 31u));
            atomicOr(&s.nextbits[x >> 5], 1u << (x & 31u));
            nfound += 1;
            fedges += e - b;
        }
    }
    flush_tally(t, s.ctr);
    add_counter(s.ctr, C_NEXT, nfound);
    add_counter(s.ctr, C_FEDGES, fedges);
}

// Bottom-up levels over packed lists.  The first G ids of a list are its
// first word and the next G - 1 gaps, at most G words (w <= 32 bits a gap):
//   k_bu_probe_packed<G>: tiles and candidates as in k_bu_probe; G lanes per
//     candidate load those words (lane j word j, fewer for narrow gaps),
//     gather each gap from its words' lanes and restore the ids by a prefix
//     sum inside the G lanes; a candidate with no frontier neighbour among
//     them and more ids is queued for
//   k_bu_rest_packed<G>: a wave per queued vertex decodes the list's blocks
//     in turn (block 0 again, its first G ids skipped), leaving at the first
//     frontier neighbour.

// Inclusive prefix sum inside each group of G (8 or 16) lanes (every lane
// calls it): DPP row shifts by 1, 2, 4 (and 8), an added value kept only
// where it comes from the same group.
template <int G>
__device__ __forceinline__ uint32_t group_prefix_sum(uint32_t x, int lane) {
    static_assert(G == 8 || G == 16, "groups of 8 or 16 lanes");
    constexpr int kRowShr = 0x110;
    const uint32_t gl = uint32_t(lane) & uint32_t(G - 1);
    uint32_t y = uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 1, 0xf, 0xf, true));
    x += gl >= 1u ? y : 0u;
    y = uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 2, 0xf, 0xf, true));
    x += gl >= 2u ? y : 0u;
    y = uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 4, 0xf, 0xf, true));
    x += gl >= 4u ? y : 0u;
    if constexpr (G == 16) {
        y = uint32_t(__builtin_amdgcn_update_dpp(0, int(x), kRowShr + 8, 0xf, 0xf, true));
        x += gl >= 8u ? y : 0u;
    }
    return x;
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_bu_probe_packed(BuArgs s) {
    constexpr int S = kWave / G;  // candidates served per step
    __shared__ uint32_t cand[kWavesPerBlock][kWave];
    __shared__ uint32_t seg[kWavesPerBlock][kSegCap];
    __shared__ uint32_t found_w[kWavesPerBlock][2];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int slot = lane / G, gl = lane % G;
    const uint64_t gmask = ((uint64_t(1) << G) - 1) << (slot * G);
    Stage st{seg[wid], 0};
    Tally t;
    uint64_t nfound = 0, fedges = 0;
    const uint64_t words = (s.V + 31) / 32, tiles = (s.V + 63) / 64;
    for (uint64_t tile = uint64_t(blockIdx.x) * kWavesPerBlock + wid; tile < tiles;
         tile += uint64_t(gridDim.x) * kWavesPerBlock) {
        const uint64_t w0 = 2 * tile;
        const uint32_t vis0 = s.visited[w0], vis1 = w0 + 1 < words ? s.visited[w0 + 1] : ~0u;
        const uint64_t vis = uint64_t(vis0) | (uint64_t(vis1) << 32);
        if (vis == ~uint64_t(0)) continue;  // (uniform) nothing left in the tile
        const uint64_t v = tile * 64 + lane;
        bool c = v < s.V && !((vis >> lane) & 1u);
        if (c) c = s.row_ptr[v + 1] > s.row_ptr[v];
        const uint64_t cm = __ballot(c);
        if (!cm) continue;
        if (c) cand[wid][rank_below(cm)] = uint32_t(v);
        if (lane < 2) found_w[wid][lane] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t nc = uint32_t(__popcll(cm));
        if (lane == 0) t.verts += nc;
        for (uint32_t r0 = 0; r0 < nc; r0 += S) {
            const uint32_t k = r0 + slot;
            const bool has = k < nc;
            uint32_t x = 0, w = 0, n = 0, nw = 0;
            uint64_t b = 0, e = 0, pw0 = 0;
            if (has) {
                x = cand[wid][k];
                b = s.row_ptr[x];
                e = s.row_ptr[x + 1];
                pw0 = s.pk_off[x];
                w = s.pk_width[x];
                n = e - b < uint64_t(G) ? uint32_t(e - b) : uint32_t(G);  // ids probed (>= 1)
                nw = packed_id_words(n, w);                                  // their words (<= G)
            }
            const uint32_t word = uint32_t(gl) < nw ? s.pk[pw0 + gl] : 0u;
            // gap gl of the group's list (lane gl >= 1) from the group's lanes
            const uint32_t gap = lane_field(word, uint32_t(slot * G + 1), uint32_t(gl) - 1u, w);
            const bool ok = uint32_t(gl) < n;
            const uint32_t id = group_prefix_sum<G>(gl == 0 ? word : (ok ? gap : 0u), lane);
            const uint64_t fm = __ballot(ok && in_frontier(s.fbits, s.V, id));
            const bool hit = (fm & gmask) != 0;
            if (gl == 0 && has) {
                t.edges += n;
                const uint64_t sec = request_bytes(pw0, pw0 + nw, 4, 32) / 32;
                t.isect += sec;
                t.reqb += 32 * sec;
                t.pkb += 4 * nw;
                if (hit) {
                    s.level[x] = s.tag;
                    atomicOr(&found_w[wid][(x & 63u) >> 5], 1u << (x & 31u));
                    fedges += e - b;
                }
            }
            // a candidate with ids left over goes to the wave-per-vertex pass
            stage(st, gl == 0 && has && !hit && e - b > uint64_t(G), x, s.rest, &s.ctr[C_REST], lane);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t f0 = found_w[wid][0], f1 = found_w[wid][1];
        if (lane == 0 && (f0 | f1)) {
            nfound += __popc(f0) + __popc(f1);
            // the wave owns both words of its tile during this kernel
            if (f0) {
                s.visited[w0] = vis0 | f0;
                s.nextbits[w0] |= f0;
            }
            if (f1) {
                s.visited[w0 + 1] = vis1 | f1;
                s.nextbits[w0 + 1] |= f1;
            }
        }
    }
    finish_queue(st, s.rest, &s.ctr[C_REST], lane, wid);
    flush_tally(t, s.ctr);
    add_counter(s.ctr, C_NEXT, nfound);
    add_counter(s.ctr, C_FEDGES, fedges);
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_bu_rest_packed(BuArgs s) {
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    Tally t;
    uint64_t nfound = 0, fedges = 0;
    const uint64_t n = s.ctr[C_REST];
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t q = uint64_t(blockIdx.x) * kWavesPerBlock + wid; q < n; q += nw) {
        const uint32_t x = uniform32(s.rest[q]);
        const uint64_t b = uniform64(s.row_ptr[x]), e = uniform64(s.row_ptr[x + 1]);
        const uint64_t pw0 = uniform64(s.pk_off[x]);
        const uint32_t w = uniform32(s.pk_width[x]);
        const uint32_t full = packed_block_words(w, s.pk_wwidth ? uniform32(s.pk_wwidth[x]) : 0u);
        bool hit = false;
        for (uint64_t k = 0; k * kWave < e - b && !hit; ++k) {
            const uint64_t rest = e - b - k * kWave;
            const uint32_t cnt = rest < uint64_t(kWave) ? uint32_t(rest) : uint32_t(kWave);
            const uint64_t idb = pw0 + k * full;
            const uint32_t id = packed_block(s.pk, idb, w, 0, cnt, lane, nullptr);
            // block 0's first ids were probed already
            const bool ok = uint32_t(lane) < cnt && (k > 0 || lane >= G);
            const uint64_t om = __ballot(ok);
            hit = __ballot(ok && in_frontier(s.fbits, s.V, id)) != 0;
            if (lane == 0) {
                const uint32_t idw = packed_id_words(cnt, w);
                const uint64_t sec = request_bytes(idb, idb + idw, 4, 32) / 32;
                t.edges += __popcll(om);
                t.isect += sec;
                t.reqb += 32 * sec;
                t.pkb += 4 * idw;
            }
        }
        if (hit && lane == 0) {
            s.level[x] = s.tag;
            atomicOr(&s.visited[x >> 5], 1u << (x & 31u));
            atomicOr(&s.nextbits[x >> 5], 1u << (x & 31u));
            nfound += 1;
            fedges += e - b;
        }
    }
    flush_tally(t, s.ctr);
    add_counter(s.ctr, C_NEXT, nfound);
    add_counter(s.ctr, C_FEDGES, fedges);
}

// ---------------------------------------------------------------------------
// PageRank (the fourth EMOGI workload, Sec. 5.1): every iteration streams
// all neighbour lists, like CC's first round.  Pull form on an undirected
// graph in fixed point (emogi_pagerank): the chunks of vertex u's list are
// dealt out as in V5; each wave sums the contributions c of a chunk's
// neighbours and adds the chunk's sum to acc[u].  The sums are integers, so
// the result does not depend on the order in which chunks finish.
// ---------------------------------------------------------------------------
struct PrArgs {
    const uint64_t *contrib;  // c(v) = floor(pr(v) / deg(v)) of the current iteration
    unsigned long long *acc;  // per-vertex sums for the next iteration (zero on entry)
    unsigned long long *ctr;  // C_EDGES, C_REQBYTES, C_VERTS, C_TIER
};

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_pr_pull(ScanArgs s, PrArgs pa) {
    constexpr int U = kGroupChunks<ColT>;
    const int lane = lane_id();
    OpArgs a{};  // the cursor reads only source_value<A_LINK>, which is the vertex id
    Tally t;
    ChunkCursor<ColT> c;
    c.total = s.chunk_scan[s.n];
    c.stride = uint64_t(gridDim.x) * kWavesPerBlock * kChunksPerWave;
    open_run<ColT, A_LINK>(c, s, a, (uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave) * kChunksPerWave);
    while (c.kb < c.kend) {
        ChunkGroup<U> g;
        load_group<ColT, A_LINK>(c, g, s, a, lane, t);
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint64_t x = (g.ok[i] && g.v[i] < s.n) ? pa.contrib[g.v[i]] : 0ull;
            const uint64_t sum = wave_sum64(x);
            if (lane == 0 && sum) atomicAdd(&pa.acc[g.uv[i]], (unsigned long long)sum);
        }
    }
    flush_tally(t, pa.ctr);
}

// pr(v) = base + floor(d * acc(v) / 2^F); acc(v) = 0; c(v) = floor(pr(v) / deg(v)).
__global__ void k_pr_finish(const uint64_t *row_ptr, uint64_t V, uint64_t base, uint64_t d, uint32_t F,
                            unsigned long long *acc, uint64_t *pr, uint64_t *contrib) {
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < V;
         v += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t sum = acc[v];
        acc[v] = 0;
        const uint64_t lo = d * sum, hi = __umul64hi(d, sum);
        const uint64_t x = base + ((hi << (64 - F)) | (lo >> F));
        pr[v] = x;
        const uint64_t deg = row_ptr[v + 1] - row_ptr[v];
        contrib[v] = deg ? x / deg : 0;
    }
}

// pr(v) = floor(2^F / V), c(v) = floor(pr(v) / deg(v)), acc(v) = 0.
__global__ void k_pr_init(const uint64_t *row_ptr, uint64_t V, uint64_t p0, unsigned long long *acc, uint64_t *pr,
                          uint64_t *contrib) {
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < V;
         v += uint64_t(gridDim.x) * blockDim.x) {
        acc[v] = 0;
        pr[v] = p0;
        const uint64_t deg = row_ptr[v + 1] - row_ptr[v];
        contrib[v] = deg ? p0 / deg : 0;
    }
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

__global__ __launch_bounds__(kBlock) void k_scan_reduce(ScanArgs s0, uint64_t *block_sums) {
    const ScanArgs s = resolved(s0);
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

__global__ __launch_bounds__(kBlock) void k_scan_write(ScanArgs s0, const uint64_t *block_sums,
                                                       uint64_t *scan) {
    const ScanArgs s = resolved(s0);
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

__device__ __forceinline__ void push_ballot(bool p, uint32_t v, uint32_t *dst, unsigned long long *count,
                                            int lane) {
    const uint64_t m = __ballot(p);
    if (!m) return;
    uint32_t base = 0;
    if (lane == 0) base = uint32_t(atomicAdd(count, (unsigned long long)__popcll(m)));
    base = __shfl(base, 0);
    if (p) dst[base + rank_below(m)] = v;
}

// ---------------------------------------------------------------------------
// Ordered frontier: the next frontier is collected as a bitmap during the
// scan and listed here in ascending id order (so the next level reads
// neighbour lists in edge-array order), clearing the listed marks.
// SSSP bands (dist != null): a marked vertex is listed only when its distance
// is below `split`; the others stay marked for a later band, and the smallest
// of their distances d is kept, as 2^32 - d by atomicMax, in ctr[C_BANDMIN].
// also_clear (optional): the listed vertices' bits are cleared there too.
// ---------------------------------------------------------------------------
constexpr int kBitsPerThread = 16;                     // words per thread
constexpr int kBitsTile = kBlock * kBitsPerThread;     // words per block

__device__ __forceinline__ uint32_t band_select(uint32_t w, uint64_t word, const uint32_t *dist, uint32_t split,
                                                uint32_t &rest_min) {
    if (!dist) return w;
    uint32_t m = 0;
    for (uint32_t x = w; x; x &= x - 1) {
        const int b = __ffs(x) - 1;
        const uint32_t d = dist[word * 32 + b];
        if (d < split) m |= 1u << b;
        else rest_min = min(rest_min, d);
    }
    return m;
}

// A thread's kBitsPerThread consecutive words of a mark bitmap: four 16-byte
// loads when all of them lie inside it (the start is 64-byte aligned), else
// word by word up to the end.
__device__ __forceinline__ void load_mark_words(const uint32_t *bits, uint64_t base, uint64_t words,
                                                uint32_t (&w)[kBitsPerThread]) {
    static_assert(kBitsPerThread == 16, "four uint4 loads per thread");
    if (base + kBitsPerThread <= words) {
        const uint4 *p = reinterpret_cast<const uint4 *>(bits + base);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 x = p[q];
            w[4 * q] = x.x;
            w[4 * q + 1] = x.y;
            w[4 * q + 2] = x.z;
            w[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kBitsPerThread; ++i) w[i] = base + i < words ? bits[base + i] : 0u;
    }
}

__global__ __launch_bounds__(kBlock) void k_bits_count(const uint32_t *bits, uint64_t words, const uint32_t *dist,
                                                        uint32_t split, uint64_t *block_sums,
                                                        unsigned long long *ctr) {
    uint64_t c = 0;
    uint32_t rest = 0xFFFFFFFFu;
    const uint64_t base = uint64_t(blockIdx.x) * kBitsTile + uint64_t(threadIdx.x) * kBitsPerThread;
    uint32_t wd[kBitsPerThread];
    load_mark_words(bits, base, words, wd);
#pragma unroll
    for (int i = 0; i < kBitsPerThread; ++i)
        if (wd[i]) c += __popc(band_select(wd[i], base + i, dist, split, rest));
    uint64_t tot;
    (void)block_exclusive_scan(c, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
    if (dist) {
        for (int o = 32; o > 0; o >>= 1) rest = min(rest, uint32_t(__shfl_xor(rest, o)));
        if (lane_id() == 0 && rest != 0xFFFFFFFFu) atomicMax(&ctr[C_BANDMIN], 0x100000000ull - rest);
    }
}

__global__ __launch_bounds__(kBlock) void k_bits_write(uint32_t *bits, uint64_t words, const uint32_t *dist,
                                                        uint32_t split, const uint64_t *block_offsets, uint32_t nb,
                                                        uint32_t *queue, uint32_t *also_clear,
                                                        unsigned long long *ctr) {
    const uint64_t base = uint64_t(blockIdx.x) * kBitsTile + uint64_t(threadIdx.x) * kBitsPerThread;
    uint32_t sel[kBitsPerThread];
    uint32_t rest = 0xFFFFFFFFu;  // not used here: k_bits_count reported it
    uint64_t c = 0;
    load_mark_words(bits, base, words, sel);
#pragma unroll
    for (int i = 0; i < kBitsPerThread; ++i) {
        if (sel[i]) sel[i] = band_select(sel[i], base + i, dist, split, rest);
        c += __popc(sel[i]);
    }
    uint64_t tot;
    uint64_t pos = block_offsets[blockIdx.x] + block_exclusive_scan(c, &tot);
#pragma unroll
    for (int i = 0; i < kBitsPerThread; ++i) {
        uint32_t w = sel[i];
        if (!w) continue;
        bits[base + i] &= ~w;  // this thread alone owns the word during the listing
        if (also_clear) also_clear[base + i] &= ~w;
        while (w) {
            const int b = __ffs(w) - 1;
            w &= w - 1;
            queue[pos++] = uint32_t((base + i) * 32 + b);
        }
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) ctr[C_NEXT] = block_offsets[blockIdx.x] + tot;
}

// ---------------------------------------------------------------------------
// CC by sampled union-find (the labels equal min-label propagation's: every
// tree's root is its component's smallest id).
//   1. hook every vertex to its first kCcSample neighbours (reads a prefix
//      of each list: one small request per vertex), or, on graphs without
//      hubs, hook the whole lists of an id range of vertices (see traverse);
//   2. compress; the most frequent root among sampled vertices is taken as
//      the large component C;
//   3. scan the whole lists of the vertices outside C only: an edge with one
//      end in C is also in the other end's list, so no edge that could join
//      two trees is skipped (symmetric graphs only);
//   4. compress again: label = root.
// ---------------------------------------------------------------------------
constexpr int kCcSample = 2;
constexpr int kCcProbe = 1024;

template <class ColT>
__global__ __launch_bounds__(kBlock) void k_cc_sample(const uint64_t *row_ptr, const ColT *col, uint64_t V,
                                                      TierView tier, uint32_t *parent, unsigned long long *ctr) {
    Tally t;
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < V;
         v += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t b = row_ptr[v], e = row_ptr[v + 1];
        const uint64_t n = e - b < kCcSample ? e - b : kCcSample;
        if (n == 0) continue;
        const ListSrc<ColT> src = list_src(tier, col, static_cast<const uint32_t *>(nullptr), uint32_t(v), b);
        ColT nb[kCcSample];
        for (uint64_t r = 0; r < n; ++r) nb[r] = src.col[b + r - src.shift];
        for (uint64_t r = 0; r < n; ++r)
            if (uint64_t(nb[r]) < V) uf_link(parent, uint32_t(v), uint32_t(nb[r]));
        t.edges += n;
        if (src.tier) {
            t.tedges += n;
        } else {
            // a prefix read is its own short request: whole sectors
            const uint64_t sec = request_bytes(b, b + n, sizeof(ColT), 32) / 32;
            t.isect += sec;
            t.reqb += 32 * sec;
        }
    }
    flush_tally(t, ctr);
}

// Sampled hooking on packed lists: the first two ids of block 0 of each
// list, its first word and the gap at the start of the next word.  Both
// words are loaded before the first hook, so the two host reads of a thread
// overlap instead of waiting on the hook's HBM atomics.
__global__ __launch_bounds__(kBlock) void k_cc_sample_packed(const uint64_t *row_ptr, const uint32_t *pk,
                                                             const uint64_t *pk_off, const uint8_t *pk_width,
                                                             uint64_t V, uint32_t *parent,
                                                             unsigned long long *ctr) {
    static_assert(kCcSample == 2, "the sample is a list's first word and the gap after it");
    uint64_t edges = 0, pkb = 0, isect = 0;
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < V;
         v += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t d = row_ptr[v + 1] - row_ptr[v];
        if (d == 0) continue;
        const uint64_t w0 = pk_off[v];
        const uint32_t w = pk_width[v];
        const bool second = d > 1;
        const uint32_t words = second && w ? 2u : 1u;  // a zero gap width stores no gap words
        const uint32_t x0 = pk[w0];
        const uint32_t g1 = words == 2u ? pk[w0 + 1] : 0u;
        pkb += 4 * words;
        isect += request_bytes(w0, w0 + words, 4, 32) / 32;
        if (x0 < V) uf_link(parent, uint32_t(v), x0);
        if (second) {
            const uint32_t x1 = x0 + packed_field(g1, 0u, 0u, w);
            if (x1 < V) uf_link(parent, uint32_t(v), x1);
        }
        edges += second ? 2 : 1;
    }
    add_counter(ctr, C_EDGES, edges);
    add_counter(ctr, C_PKBYTES, pkb);
    add_counter(ctr, C_IDSECT, isect);
    add_counter(ctr, C_REQBYTES, 32 * isect);
}

__global__ void k_compress(uint32_t *parent, uint64_t V) {
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < V;
         v += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t r = parent[v];
        while (parent[r] != r) r = parent[r];
        parent[v] = r;
    }
}

// Roots of kCcProbe pseudo-randomly chosen vertices (SplitMix64 of the index).
__global__ void k_cc_probe(const uint32_t *parent, uint64_t V, uint32_t *roots) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kCcProbe) return;
    uint64_t z = (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    roots[i] = parent[z % V];
}

// Vertices with edges whose root is not `big`, in id order per wave.
__global__ __launch_bounds__(kBlock) void k_cc_outside(const uint32_t *parent, const uint64_t *row_ptr,
                                                        uint64_t V, uint32_t big, uint32_t *queue,
                                                        unsigned long long *ctr) {
    const int lane = lane_id();
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i0 = uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u); i0 < V; i0 += stride) {
        const uint64_t v = i0 + lane;
        const bool p = v < V && parent[v] != big && row_ptr[v + 1] > row_ptr[v];
        push_ballot(p, uint32_t(v), queue, &ctr[C_NEXT], lane);
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

// Size and degree sum of a frontier held as marks (C_NEXT, C_FEDGES).
__global__ __launch_bounds__(kBlock) void k_marks_tally(const uint32_t *bits, uint64_t words, const uint64_t *row_ptr,
                                                         unsigned long long *ctr) {
    uint64_t cnt = 0, deg = 0;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t w = bits[i];
        cnt += __popc(w);
        while (w) {
            const uint64_t v = i * 32 + uint64_t(__ffs(w) - 1);
            w &= w - 1;
            deg += row_ptr[v + 1] - row_ptr[v];
        }
    }
    add_counter(ctr, C_NEXT, cnt);
    add_counter(ctr, C_FEDGES, deg);
}

// Sum of the out-degrees of the vertices with a finite value (C_FEDGES).
__global__ __launch_bounds__(kBlock) void k_reached_edges(const uint32_t *state, const uint64_t *row_ptr, uint64_t V,
                                                           unsigned long long *ctr) {
    uint64_t deg = 0;
    for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < V; v += uint64_t(gridDim.x) * blockDim.x)
        if (state[v] != 0xFFFFFFFFu) deg += row_ptr[v + 1] - row_ptr[v];
    add_counter(ctr, C_FEDGES, deg);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static unsigned fill_grid(uint64_t n) {
    uint64_t g = (n + kBlock - 1) / kBlock;
    return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(g, 4096)));
}

// Clears device words with a kernel (every buffer cleared here is whole
// 32-bit words); errors surface at the caller's next launch check.
static void zero_async(void *ptr, size_t bytes, hipStream_t stream) {
    const uint64_t words = bytes / 4;
    hipLaunchKernelGGL(k_fill, dim3(fill_grid(words)), dim3(kBlock), 0, stream, static_cast<uint32_t *>(ptr), words,
                       0u);
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
    if (algo == A_CC &&
        (st = dalloc(reinterpret_cast<void **>(&p.stamp), V * sizeof(uint32_t))) != EMOGI_OK)
        return st;
    if (algo == A_CC &&
        (st = dalloc(reinterpret_cast<void **>(&p.cc_probe), kCcProbe * sizeof(uint32_t))) != EMOGI_OK)
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

bool sched_needs_features(const emogi_graph_s *g);

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

// Packed lists are scanned by V5 only (their chunks are their blocks).
template <int A>
static void launch_packed(const ScanArgs &s, const OpArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL((k_balanced_packed<A>), dim3(kMaxGrid), dim3(kBlock), 0, stream, s, a);
}

// Points a scan at the graph's packed lists (no-op for plain lists).
static void use_packed(ScanArgs &s, const emogi_graph_s *g) {
    if (!g->packed.stream) return;
    s.pk = g->packed.stream;
    s.pk_off = g->packed.off;
    s.pk_width = g->packed.width;
    s.pk_wwidth = g->packed.wwidth;
    s.align_mask = 0;
}

// Levels per host wait for BFS: the setting, or (0) 8 on graphs of fewer
// than 2^24 edges and 1 above (measured on R-MAT 16/18/20: batches win up to
// scale 18; at scale 20 the ordered per-level frontier is worth more than the
// saved waits); always 1 when per-level features are recorded or every
// variant is timed.  The learned scheduler keeps the batches: the host does
// not see a batch's frontiers, so the batch rule picks their variant and the
// network decides the levels that run one per host wait.
static uint32_t level_batch(const emogi_graph_s *g) {
    if (g->record_features || g->sched_mode == EMOGI_SCHED_PROBE || g->packed.stream) return 1;
    if (g->level_batch) return g->level_batch;
    return g->E < (uint64_t(1) << 24) ? 8u : 1u;
}

// Whether BFS may run bottom-up levels (see emogi_set_direction): a vertex's
// list must also list its incoming edges (symmetric graphs), and the
// direction is picked per level on the host from the ordered frontier.
static bool direction_allowed(const emogi_graph_s *g) {
    return g->direction != EMOGI_DIR_TOP_DOWN && (g->flags & EMOGI_F_SYMMETRIC) && g->ordered_frontier &&
           g->sched_mode != EMOGI_SCHED_PROBE && g->V > 0 && level_batch(g) == 1;
}

// Direction of the next level (true: bottom-up), from the level just run
// (bottom-up or not, its frontier size n) and the next frontier (n_next
// vertices whose lists hold m_next edges); `explored` is the degree sum of
// every vertex reached so far.  Beamer, Asanovic and Patterson (SC 2012):
// go bottom-up when the next frontier's edges exceed the edges still
// unexplored / alpha while the frontier grows; come back when it shrinks
// below (vertices with edges) / beta.
static bool choose_bottom_up(const emogi_graph_s *g, bool bu, uint64_t n, uint64_t n_next, uint64_t m_next,
                             uint64_t explored) {
    if (g->direction == EMOGI_DIR_BOTTOM_UP) return true;
    if (!bu) {
        const uint64_t unexplored = g->E > explored ? g->E - explored : 0;
        return n_next > n && m_next * uint64_t(g->dir_alpha) > unexplored;
    }
    return !(n_next < n && n_next * uint64_t(g->dir_beta) < g->nonisolated);
}

static emogi_status_t ensure_level_blocks(emogi_graph_s *g, uint32_t lb) {
    Pool &p = g->pool;
    if (p.level_ctr && p.level_cap >= lb) return EMOGI_OK;
    if (p.level_ctr) (void)hipFree(p.level_ctr);
    if (p.level_host) (void)hipHostFree(p.level_host);
    p.level_ctr = nullptr;
    p.level_host = nullptr;
    p.level_cap = 0;
    const size_t bytes = size_t(lb) * C_COUNT * sizeof(unsigned long long);
    if (hipMalloc(reinterpret_cast<void **>(&p.level_ctr), bytes) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&p.level_host), bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("level-batch counter allocation failed");
        return EMOGI_E_OOM_DEVICE;
    }
    p.level_cap = lb;
    return EMOGI_OK;
}

// The built-in rule of thumb (also the learned scheduler's fallback).
int heuristic_variant(const emogi_graph_s *g, uint64_t n) {
    if (n >= 2048) return EMOGI_V5_BALANCED;
    if (g->max_degree > 4096) return EMOGI_V5_BALANCED;
    return EMOGI_V3_WAVE_ALIGNED;
}

int choose_variant(emogi_graph_s *g, int algo, uint64_t n, const uint32_t *queue, hipStream_t stream,
                   float *features, int *by_network);
emogi_status_t sched_begin(emogi_graph_s *g, hipStream_t stream);
emogi_status_t sched_prefetch(emogi_graph_s *g, int algo, const uint32_t *queue, unsigned long long *counters,
                              hipStream_t stream);
int choose_prefetched(const emogi_graph_s *g, uint64_t n, const unsigned long long *hc, float *features,
                      int *by_network);

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
    if (algo == A_CC && p.stamp) EMOGI_HIP_TRY(cp(p.stamp, p.snap_stamp, V * 4), EMOGI_E_HIP);
    if (algo == A_SSSP) {
        // marks of improved vertices waiting for a later band survive the listing
        if ((!p.snap_nextbits && hipMalloc(&p.snap_nextbits, words * 4) != hipSuccess) ||
            (!p.snap_farbits && hipMalloc(&p.snap_farbits, words * 4) != hipSuccess)) {
            (void)hipGetLastError();
            set_error("probe snapshot allocation failed");
            return EMOGI_E_OOM_DEVICE;
        }
        EMOGI_HIP_TRY(cp(p.nextbits, p.snap_nextbits, words * 4), EMOGI_E_HIP);
        EMOGI_HIP_TRY(cp(p.farbits, p.snap_farbits, words * 4), EMOGI_E_HIP);
    }
    return EMOGI_OK;
}

// Adds a level's (or a pass's) device counters to the traversal statistics.
static void absorb_counters(emogi_stats_t &S, const unsigned long long *hc) {
    S.edges_scanned += hc[C_EDGES];
    S.tier_edges += hc[C_TIER];
    S.request_bytes += hc[C_REQBYTES];
    S.vertices_expanded += hc[C_VERTS];
    S.weights_read += hc[C_WLINK];
    S.id_sector_bytes += 32 * hc[C_IDSECT];
    S.weight_sector_bytes += 32 * hc[C_WSECT];
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
    if (algo == A_SSSP && !g->weights && !g->packed.wwidth) {
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
    int kalgo = algo;  // the operation the scan kernels run (A_LINK for sampled CC)
    uint64_t packed_bytes = 0;  // encoded bytes of the packed lists scanned
    if (V > 0) {
        if (algo == A_CC && g->cc_sampled) {
            // sampled union-find: hook, compress, find the large tree, then one
            // full pass over the lists of the vertices outside it
            hipLaunchKernelGGL(k_iota, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V);
            zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
            // the sampling pass reads lists over the link like a level does:
            // its time counts in expand_ms (its chunk prefix in prep_ms)
            EMOGI_HIP_TRY(hipEventRecord(g->ev_s0, stream), EMOGI_E_HIP);
            bool sample_prefix = false;  // ev_k0 recorded between the prefix and the hooking scan
            const uint64_t davg = std::max<uint64_t>(1, g->E / V);
            if (g->max_degree <= 4 * davg) {
                // Lists of about equal length (no hubs): a read of each list's
                // first ids costs one small host-link request per vertex, so
                // instead hook the whole lists of the vertices in an id range
                // that holds a fraction f of the edges (one sequential read).
                // A vertex stays unhooked with probability (1-f)^(d+1) and is
                // then read in full by step 3; f = ln(d+1)/(d+1) balances the two.
                const double f = std::min(0.5, std::log(double(davg) + 1.0) / (double(davg) + 1.0));
                const uint64_t target = uint64_t(f * double(g->E));
                uint64_t lo = 0, hi = V;  // first vertex v1 with row_ptr[v1] >= target
                while (lo < hi) {
                    const uint64_t mid = lo + (hi - lo) / 2;
                    uint64_t x = 0;
                    EMOGI_HIP_TRY(hipMemcpy(&x, g->row_ptr + mid, sizeof(x), hipMemcpyDeviceToHost), EMOGI_E_HIP);
                    if (x < target) lo = mid + 1; else hi = mid;
                }
                if (lo > 0) {
                    if ((st = ensure_scan(g, V)) != EMOGI_OK) return st;
                    ScanArgs s{};
                    s.queue = nullptr;  // vertices 0 .. lo-1
                    s.n = uint32_t(lo);
                    s.n_dev = nullptr;
                    s.row_ptr = g->row_ptr;
                    s.col = g->col;
                    s.align_mask = uint64_t(std::max<uint32_t>(1, g->request_unit / g->col_bytes)) - 1;
                    s.req_unit = g->request_unit;
                    s.col_bytes = g->col_bytes;
                    s.tier = tier_view(g);
                    use_packed(s, g);
                    const unsigned nb = unsigned((lo + kScanTile) / kScanTile);
                    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums);
                    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, stream, p.block_sums, nb);
                    hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums,
                                       p.chunk_scan);
                    s.chunk_scan = p.chunk_scan;
                    EMOGI_HIP_TRY(hipEventRecord(g->ev_k0, stream), EMOGI_E_HIP);
                    sample_prefix = true;
                    OpArgs a{};
                    a.state = out;
                    a.V = uint32_t(V);
                    a.ctr = p.counters;
                    a.split = 0xFFFFFFFFu;
                    if (g->packed.stream)
                        launch_packed<A_LINK>(s, a, stream);
                    else if (g->col_bytes == 8)
                        launch_variant<uint64_t, A_LINK>(EMOGI_V5_BALANCED, s, a, stream);
                    else
                        launch_variant<uint32_t, A_LINK>(EMOGI_V5_BALANCED, s, a, stream);
                }
            } else if (g->packed.stream) {
                hipLaunchKernelGGL(k_cc_sample_packed, dim3(kMaxGrid), dim3(kBlock), 0, stream, g->row_ptr,
                                   g->packed.stream, g->packed.off, g->packed.width, V, out, p.counters);
            } else if (g->col_bytes == 8) {
                hipLaunchKernelGGL(k_cc_sample<uint64_t>, dim3(kMaxGrid), dim3(kBlock), 0, stream, g->row_ptr,
                                   static_cast<const uint64_t *>(g->col), V, tier_view(g), out, p.counters);
            } else {
                hipLaunchKernelGGL(k_cc_sample<uint32_t>, dim3(kMaxGrid), dim3(kBlock), 0, stream, g->row_ptr,
                                   static_cast<const uint32_t *>(g->col), V, tier_view(g), out, p.counters);
            }
            EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k1, stream), EMOGI_E_HIP);
            hipLaunchKernelGGL(k_compress, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V);
            hipLaunchKernelGGL(k_cc_probe, dim3((kCcProbe + 255) / 256), dim3(256), 0, stream, out, V,
                               p.cc_probe);
            std::vector<uint32_t> roots(kCcProbe);
            EMOGI_HIP_TRY(hipMemcpyAsync(roots.data(), p.cc_probe, kCcProbe * sizeof(uint32_t),
                                         hipMemcpyDeviceToHost, stream),
                          EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipMemcpyAsync(p.host_counters, p.counters, C_COUNT * sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, stream),
                          EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
            {
                float total_ms = 0.f, prep = 0.f;
                EMOGI_HIP_TRY(hipEventElapsedTime(&total_ms, g->ev_s0, g->ev_k1), EMOGI_E_HIP);
                if (sample_prefix) EMOGI_HIP_TRY(hipEventElapsedTime(&prep, g->ev_s0, g->ev_k0), EMOGI_E_HIP);
                S.expand_ms += total_ms;
                S.prep_ms += prep;
                S.expand_launches += 1;
            }
            absorb_counters(S, p.host_counters);
            packed_bytes += p.host_counters[C_PKBYTES];
            std::sort(roots.begin(), roots.end());
            uint32_t big = roots[0], best = 0;
            for (size_t i = 0, j; i < roots.size(); i = j) {
                for (j = i; j < roots.size() && roots[j] == roots[i]; ++j) {}
                if (j - i > best) {
                    best = uint32_t(j - i);
                    big = roots[i];
                }
            }
            zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
            hipLaunchKernelGGL(k_cc_outside, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, g->row_ptr, V, big,
                               p.queue[0], p.counters);
            EMOGI_HIP_TRY(hipMemcpyAsync(p.host_counters, p.counters, C_COUNT * sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, stream),
                          EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
            n = p.host_counters[C_NEXT];
            kalgo = A_LINK;
        } else if (algo == A_CC) {
            hipLaunchKernelGGL(k_iota, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V);
            zero_async(p.stamp, V * sizeof(uint32_t), stream);
            n = V;
            identity = true;  // every vertex starts active (Sec. 5.4)
        } else {
            hipLaunchKernelGGL(k_fill, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V, 0xFFFFFFFFu);
            zero_async(p.bitmap, ((V + 31) / 32) * sizeof(uint32_t), stream);
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
    // Round list starts so each wave load covers whole request units of every
    // array it reads: SSSP also reads the 4-byte weights at the same indices,
    // so it aligns to R / 4 elements (8-byte ids then span two units).
    const uint32_t elem_bytes = (algo == A_SSSP) ? 4u : g->col_bytes;
    const uint32_t align_elems = std::max<uint32_t>(1, g->request_unit / elem_bytes);
    int cur = 0;
    uint32_t iter = 0;
    bool overflow_seen = false;
    // The next frontier is listed from a bitmap (ordered) for BFS and CC label
    // propagation when asked, and always for SSSP, whose marks also hold the
    // improved vertices that wait for a later distance band.
    const bool ordered = (g->ordered_frontier || algo == A_SSSP) && kalgo != A_LINK && V > 0;
    if (ordered) {
        if ((st = ensure_scan(g, V)) != EMOGI_OK) return st;
        if (!p.nextbits && hipMalloc(&p.nextbits, ((V + 31) / 32) * sizeof(uint32_t)) != hipSuccess) {
            (void)hipGetLastError();
            p.nextbits = nullptr;
            set_error("hipMalloc of the ordered-frontier bitmap failed");
            return EMOGI_E_OOM_DEVICE;
        }
        zero_async(p.nextbits, ((V + 31) / 32) * sizeof(uint32_t), stream);
        if (algo == A_SSSP) {
            if (!p.farbits && hipMalloc(&p.farbits, ((V + 31) / 32) * sizeof(uint32_t)) != hipSuccess) {
                (void)hipGetLastError();
                p.farbits = nullptr;
                set_error("hipMalloc of the SSSP band bitmap failed");
                return EMOGI_E_OOM_DEVICE;
            }
            zero_async(p.farbits, ((V + 31) / 32) * sizeof(uint32_t), stream);
        }
    }
    // SSSP distance bands (Sec. 5.1 leaves the SSSP algorithm open; this is a
    // near-far worklist): an improvement below `split` joins the next round
    // (marked in nextbits), one at or above it waits (marked in farbits).
    // When a round lists nothing, the split moves to the smallest waiting
    // distance + delta and the waiting vertices below it are listed.
    // delta = 0: one band, plain label correcting.
    const uint32_t delta = g->sssp_delta;
    uint32_t split = (algo == A_SSSP && delta > 0) ? delta : 0xFFFFFFFFu;
    const uint64_t words = (V + 31) / 32;
    const unsigned nbw = unsigned((words + kBitsTile - 1) / kBitsTile);
    // Lists the marks in `bits` (with `dist`: those below `cut`) into `queue`
    // in id order, also clearing them in `also_clear`; the count lands in
    // counters[C_NEXT], the smallest distance left marked in C_BANDMIN.
    auto list_marks = [&](uint32_t *bits, const uint32_t *dist, uint32_t cut, uint32_t *queue,
                          uint32_t *also_clear) {
        hipLaunchKernelGGL(k_bits_count, dim3(nbw), dim3(kBlock), 0, stream, bits, words, dist, cut,
                           p.block_sums, p.counters);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, stream, p.block_sums, nbw);
        hipLaunchKernelGGL(k_bits_write, dim3(nbw), dim3(kBlock), 0, stream, bits, words, dist, cut,
                           p.block_sums, nbw, queue, also_clear, p.counters);
    };
    auto sync_counters = [&]() -> emogi_status_t {
        EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
        EMOGI_HIP_TRY(hipMemcpyAsync(p.host_counters, p.counters, C_COUNT * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, stream),
                      EMOGI_E_HIP);
        EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
        return EMOGI_OK;
    };
    // The scheduler's features and pick for the next frontier are computed
    // behind each level (and behind an SSSP band step's listing) and come
    // back with its counters (have_pick); the first frontier is scored on its
    // own.
    // (BFS with bottom-up levels scores each top-down frontier on its own)
    const bool prefetch = V > 0 && sched_needs_features(g) && !(algo == A_BFS && direction_allowed(g));
    bool have_pick = false;
    if (prefetch && (st = sched_begin(g, stream)) != EMOGI_OK) return st;

    // BFS level batches: on small graphs the host's wait after each level
    // costs more than the level, so `lb` levels are enqueued at once.  Each
    // level has its own counter block; its kernels read the frontier length
    // the previous level left there and do nothing once it is zero, so
    // enqueuing past the last level is harmless.  The host waits once per
    // batch.  The variant is fixed for the batch (the host cannot see the
    // frontiers), pushes go through the LDS-staged queue.
    const uint32_t lb = (algo == A_BFS && V > 0) ? level_batch(g) : 1;
    if (lb > 1) {
        if ((st = ensure_level_blocks(g, lb)) != EMOGI_OK) return st;
        const int m = g->sched_mode;
        // without a fixed variant: a workgroup per vertex on small graphs (no
        // prefix kernels per level; measured fastest on R-MAT 16 and 18), else V5
        const int var = (m >= 0 && m < EMOGI_NUM_VARIANTS) ? m
                        : g->E < (uint64_t(1) << 24) ? int(EMOGI_V4_BLOCK) : heuristic_variant(g, V);
        const unsigned nb_max = unsigned((V + kScanTile) / kScanTile);
        if (var == EMOGI_V5_BALANCED && (st = ensure_scan(g, V)) != EMOGI_OK) return st;
        while (n > 0) {
            if (iter >= cap) {
                (void)hipStreamSynchronize(stream);
                set_error("iteration cap %llu reached", (unsigned long long)cap);
                return EMOGI_E_NOCONVERGE;
            }
            const uint32_t k = uint32_t(std::min<uint64_t>(lb, cap - iter));  // the cap holds exactly
            zero_async(p.level_ctr, size_t(k) * C_COUNT * sizeof(unsigned long long), stream);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k0, stream), EMOGI_E_HIP);
            for (uint32_t i = 0; i < k; ++i) {
                ScanArgs s;
                s.queue = p.queue[cur];
                s.n = i == 0 ? uint32_t(n) : uint32_t(V);  // later levels: V only sizes the grids
                s.n_dev = i == 0 ? nullptr : &p.level_ctr[(i - 1) * C_COUNT + C_NEXT];
                s.row_ptr = g->row_ptr;
                s.col = g->col;
                s.w = g->weights;
                s.next = p.queue[cur ^ 1];
                s.align_mask = uint64_t(align_elems) - 1;
                s.req_unit = g->request_unit;
                s.col_bytes = g->col_bytes;
                s.chunk_scan = nullptr;
                s.tier = tier_view(g);
                OpArgs a;
                a.state = out;
                a.bitmap = p.bitmap;
                a.stamp = nullptr;
                a.tag = iter + i + 1;
                a.V = uint32_t(V);
                a.ctr = &p.level_ctr[i * C_COUNT];
                a.nextbits = nullptr;
                a.split = 0xFFFFFFFFu;
                a.farbits = nullptr;
                a.wmin = 0;
                if (var == EMOGI_V5_BALANCED) {
                    const unsigned nb = i == 0 ? unsigned((n + kScanTile) / kScanTile) : nb_max;
                    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums);
                    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, stream, p.block_sums, nb);
                    hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums,
                                       p.chunk_scan);
                    s.chunk_scan = p.chunk_scan;
                }
                if (g->col_bytes == 8)
                    launch_variant<uint64_t, A_BFS>(var, s, a, stream);
                else
                    launch_variant<uint32_t, A_BFS>(var, s, a, stream);
                cur ^= 1;
            }
            EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k1, stream), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipMemcpyAsync(p.level_host, p.level_ctr, size_t(k) * C_COUNT * sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, stream),
                          EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
            float ms = 0.f;
            EMOGI_HIP_TRY(hipEventElapsedTime(&ms, g->ev_k0, g->ev_k1), EMOGI_E_HIP);
            S.expand_ms += ms;
            uint32_t ran = 0;
            for (uint32_t i = 0; i < k && n > 0; ++i, ++ran) {
                const unsigned long long *hc = &p.level_host[i * C_COUNT];
                if (iter < EMOGI_MAX_LEVEL_STATS) {
                    S.level_variant[iter] = uint8_t(var);
                    S.level_frontier[iter] = uint32_t(n);
                    S.level_edges[iter] = hc[C_EDGES];
                    S.level_count = iter + 1;
                }
                S.variant_hist[var] += 1;
                S.expand_launches += 1;
                absorb_counters(S, hc);
                n = hc[C_NEXT];
                ++iter;
            }
            // the batch's time, shared evenly by the levels that had work
            for (uint32_t i = 0; i < ran; ++i)
                if (iter - ran + i < EMOGI_MAX_LEVEL_STATS) S.level_ms[iter - ran + i] = ms / float(ran);
        }
    }
    // Direction-optimizing BFS (emogi_set_direction): `bu` says the current
    // frontier is held as the bitmap fbits and the level runs bottom-up.
    // The next frontier is always collected as marks (nextbits); after each
    // level one pass counts them and sums their degrees, the host picks the
    // next level's direction, and the marks are either listed into the queue
    // (top-down) or become the frontier bitmap (bottom-up).
    const bool do_bfs = algo == A_BFS && ordered && direction_allowed(g);
    if (do_bfs && !p.fbits) {
        if (hipMalloc(&p.fbits, words * sizeof(uint32_t)) != hipSuccess) {
            (void)hipGetLastError();
            p.fbits = nullptr;
            set_error("hipMalloc of the bottom-up frontier bitmap failed");
            return EMOGI_E_OOM_DEVICE;
        }
    }
    bool bu = false;
    uint64_t explored = 0;  // degree sum of the vertices reached so far
    const int colkind = g->col_bytes == 8 ? 1 : 0;
    while (true) {
        if (n == 0) {
            // SSSP: the band is exhausted; open the next one at the smallest
            // waiting distance (a pass that lists nothing and keeps the
            // minimum), or stop when nothing waits
            have_pick = false;
            if (algo != A_SSSP || split == 0xFFFFFFFFu) break;
            zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
            hipLaunchKernelGGL(k_bits_count, dim3(nbw), dim3(kBlock), 0, stream, p.farbits, words, out, 0u,
                               p.block_sums, p.counters);
            if ((st = sync_counters()) != EMOGI_OK) return st;
            const unsigned long long bm = p.host_counters[C_BANDMIN];
            if (bm == 0) break;
            const uint64_t m = 0x100000000ull - bm;
            split = uint32_t(std::min<uint64_t>(std::max<uint64_t>(m + delta, split), 0xFFFFFFFFull));
            zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
            list_marks(p.farbits, out, split, p.queue[cur], nullptr);
            if (prefetch) {
                // the band's first frontier is scored behind its listing and its
                // pick comes back with the counters
                emogi_status_t e3 = sched_prefetch(g, algo, p.queue[cur], p.counters, stream);
                if (e3 != EMOGI_OK) return e3;
            }
            if ((st = sync_counters()) != EMOGI_OK) return st;
            n = p.host_counters[C_NEXT];
            have_pick = prefetch;
            continue;
        }
        if (iter >= cap) {
            (void)hipStreamSynchronize(stream);
            set_error("iteration cap %llu reached", (unsigned long long)cap);
            return EMOGI_E_NOCONVERGE;
        }
        const uint32_t *queue = identity ? nullptr : p.queue[cur];
        // One level with variant `v`: counters cleared, (V5) chunk prefix
        // between ev_s0 and ev_k0, the scan kernel between ev_k0 and ev_k1,
        // counters copied back, host waits.  *ms_out: the scan kernel,
        // *prep_out: the prefix.
        auto run_level = [&](int v, float *ms_out, float *prep_out) -> emogi_status_t {
            ScanArgs s;
            s.queue = queue;
            s.n = uint32_t(n);
            s.n_dev = nullptr;
            s.row_ptr = g->row_ptr;
            s.col = g->col;
            s.w = g->weights;
            s.next = p.queue[identity ? 0 : cur ^ 1];
            s.align_mask = uint64_t(align_elems) - 1;
            s.req_unit = g->request_unit;
            s.col_bytes = g->col_bytes;
            s.chunk_scan = nullptr;
            s.tier = tier_view(g);
            use_packed(s, g);
            OpArgs a;
            a.state = out;
            a.bitmap = p.bitmap;
            a.stamp = p.stamp;
            a.tag = iter + 1;  // BFS: level of the next frontier; SSSP/CC: round
            a.V = uint32_t(V);
            a.ctr = p.counters;
            a.nextbits = ordered ? p.nextbits : nullptr;
            a.split = split;
            a.farbits = p.farbits;
            a.wmin = g->min_weight;
            a.inmin = g->in_min;
            zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_s0, stream), EMOGI_E_HIP);
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
            const int key = g->packed.stream ? 8 + kalgo : kalgo * 2 + colkind;
            switch (key) {
            case 8 + A_BFS: launch_packed<A_BFS>(s, a, stream); break;
            case 8 + A_SSSP: launch_packed<A_SSSP>(s, a, stream); break;
            case 8 + A_CC: launch_packed<A_CC>(s, a, stream); break;
            case 8 + A_LINK: launch_packed<A_LINK>(s, a, stream); break;
            case 0: launch_variant<uint32_t, A_BFS>(v, s, a, stream); break;
            case 1: launch_variant<uint64_t, A_BFS>(v, s, a, stream); break;
            case 2: launch_variant<uint32_t, A_SSSP>(v, s, a, stream); break;
            case 3: launch_variant<uint64_t, A_SSSP>(v, s, a, stream); break;
            case 4: launch_variant<uint32_t, A_CC>(v, s, a, stream); break;
            case 5: launch_variant<uint64_t, A_CC>(v, s, a, stream); break;
            case 6: launch_variant<uint32_t, A_LINK>(v, s, a, stream); break;
            default: launch_variant<uint64_t, A_LINK>(v, s, a, stream); break;
            }
            EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k1, stream), EMOGI_E_HIP);
            if (ordered && !do_bfs) {
                list_marks(p.nextbits, nullptr, 0xFFFFFFFFu, s.next, algo == A_SSSP ? p.farbits : nullptr);
                EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            }
            if (prefetch) {
                emogi_status_t e3 = sched_prefetch(g, algo, s.next, p.counters, stream);
                if (e3 != EMOGI_OK) return e3;
            }
            EMOGI_HIP_TRY(hipMemcpyAsync(p.host_counters, p.counters, C_COUNT * sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, stream),
                          EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipEventElapsedTime(ms_out, g->ev_k0, g->ev_k1), EMOGI_E_HIP);
            *prep_out = 0.f;
            if (v == EMOGI_V5_BALANCED) EMOGI_HIP_TRY(hipEventElapsedTime(prep_out, g->ev_s0, g->ev_k0), EMOGI_E_HIP);
            return EMOGI_OK;
        };
        // One bottom-up level: the probe over every vertex tile, then a wave
        // per vertex the probe left; *ms_out: both kernels.
        auto run_bottom_up = [&](float *ms_out) -> emogi_status_t {
            BuArgs b;
            b.row_ptr = g->row_ptr;
            b.col = g->col;
            b.tier = tier_view(g);
            b.V = V;
            b.fbits = p.fbits;
            b.visited = p.bitmap;
            b.nextbits = p.nextbits;
            b.level = out;
            b.tag = iter + 1;
            b.rest = p.queue[cur ^ 1];
            b.ctr = p.counters;
            zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
            const uint64_t tiles = (V + 63) / 64;
            const unsigned grid = unsigned(std::max<uint64_t>(
                1, std::min<uint64_t>((tiles + kWavesPerBlock - 1) / kWavesPerBlock, kMaxGrid)));
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k0, stream), EMOGI_E_HIP);
            if (g->packed.stream) {
                b.pk = g->packed.stream;
                b.pk_off = g->packed.off;
                b.pk_width = g->packed.width;
                b.pk_wwidth = g->packed.wwidth;
                hipLaunchKernelGGL(k_bu_probe_packed<kBuPackedProbeIds>, dim3(grid), dim3(kBlock), 0, stream, b);
                hipLaunchKernelGGL(k_bu_rest_packed<kBuPackedProbeIds>, dim3(kMaxGrid), dim3(kBlock), 0, stream, b);
            } else if (colkind) {
                hipLaunchKernelGGL(k_bu_probe<uint64_t>, dim3(grid), dim3(kBlock), 0, stream, b);
                hipLaunchKernelGGL(k_bu_rest<uint64_t>, dim3(kMaxGrid), dim3(kBlock), 0, stream, b);
            } else {
                hipLaunchKernelGGL(k_bu_probe<uint32_t>, dim3(grid), dim3(kBlock), 0, stream, b);
                hipLaunchKernelGGL(k_bu_rest<uint32_t>, dim3(kMaxGrid), dim3(kBlock), 0, stream, b);
            }
            EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k1, stream), EMOGI_E_HIP);
            if ((st = sync_counters()) != EMOGI_OK) return st;
            EMOGI_HIP_TRY(hipEventElapsedTime(ms_out, g->ev_k0, g->ev_k1), EMOGI_E_HIP);
            return EMOGI_OK;
        };
        float ms = 0.f, prep = 0.f;
        int var = 0;
        if (bu) {
            if ((st = run_bottom_up(&ms)) != EMOGI_OK) return st;
            S.bottom_up_levels += 1;
        } else {
            float feats[16];
            const bool want_feats = g->record_features && iter < EMOGI_MAX_LEVEL_STATS;
            int by_net = 0;
            var = have_pick ? choose_prefetched(g, n, p.host_counters, want_feats ? feats : nullptr, &by_net)
                            : choose_variant(g, algo, n, queue, stream, want_feats ? feats : nullptr, &by_net);
            if (var < 0) {
                set_error("scheduler kernels failed");
                return EMOGI_E_HIP;
            }
            if (want_feats) memcpy(S.level_features[iter], feats, sizeof(feats));
            if (g->packed.stream) {
                var = EMOGI_V5_BALANCED;  // the one variant that decodes packed lists
                by_net = 0;
            }
            if (g->sched_mode == EMOGI_SCHED_PROBE && !g->packed.stream) {
                // Time every variant on the same level state (its preparation
                // kernels included), then run the fastest.
                if ((st = snapshot(g, algo, out, stream, false)) != EMOGI_OK) return st;
                float best = 1e30f;
                for (int v = 0; v < EMOGI_NUM_VARIANTS; ++v) {
                    if (v > 0 && (st = snapshot(g, algo, out, stream, true)) != EMOGI_OK) return st;
                    float pm = 0.f, pp = 0.f;
                    if ((st = run_level(v, &pm, &pp)) != EMOGI_OK) return st;
                    if (iter < EMOGI_MAX_LEVEL_STATS) S.level_probe_ms[iter][v] = pm + pp;
                    if (pm + pp < best) {
                        best = pm + pp;
                        var = v;
                    }
                }
                if ((st = snapshot(g, algo, out, stream, true)) != EMOGI_OK) return st;
            }
            if ((st = run_level(var, &ms, &prep)) != EMOGI_OK) return st;
            have_pick = prefetch;
            S.variant_hist[var] += 1;
            S.levels_by_network += by_net ? 1 : 0;
        }
        const unsigned long long *hc = p.host_counters;
        if (iter < EMOGI_MAX_LEVEL_STATS) {
            S.level_variant[iter] = bu ? uint8_t(EMOGI_NUM_VARIANTS) : uint8_t(var);
            S.level_direction[iter] = bu ? 1 : 0;
            S.level_frontier[iter] = uint32_t(n);
            S.level_ms[iter] = ms;
            S.level_edges[iter] = hc[C_EDGES];
            S.level_count = iter + 1;
        }
        S.expand_ms += ms + prep;
        S.prep_ms += prep;
        S.expand_launches += 1;
        absorb_counters(S, hc);
        packed_bytes += hc[C_PKBYTES];
        if (hc[C_OVERFLOW]) overflow_seen = true;
        if (do_bfs) {
            if (iter == 0) explored = hc[C_EDGES];  // the source's list (a top-down level)
            uint64_t n_next = hc[C_NEXT], m_next = hc[C_FEDGES];
            if (!bu) {
                // a top-down level left marks only: count them, sum their degrees
                zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
                hipLaunchKernelGGL(k_marks_tally, dim3(fill_grid(words)), dim3(kBlock), 0, stream, p.nextbits, words,
                                   g->row_ptr, p.counters);
                if ((st = sync_counters()) != EMOGI_OK) return st;
                n_next = p.host_counters[C_NEXT];
                m_next = p.host_counters[C_FEDGES];
            }
            explored += m_next;
            const bool next_bu = n_next > 0 && choose_bottom_up(g, bu, n, n_next, m_next, explored);
            if (next_bu) {
                std::swap(p.fbits, p.nextbits);
                zero_async(p.nextbits, words * sizeof(uint32_t), stream);
            } else if (n_next > 0) {
                list_marks(p.nextbits, nullptr, 0xFFFFFFFFu, p.queue[cur ^ 1], nullptr);
                EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            }
            n = n_next;
            bu = next_bu;
            cur ^= 1;
            ++iter;
            continue;
        }
        n = hc[C_NEXT];
        if (identity) {
            identity = false;
            cur = 0;
        } else {
            cur ^= 1;
        }
        ++iter;
    }
    if (kalgo == A_LINK)
        hipLaunchKernelGGL(k_compress, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V);
    S.iterations = iter;
    // ids of every list read over the link (packed: their encoded bytes);
    // SSSP weights only where read
    S.useful_link_bytes = (g->packed.stream ? packed_bytes : (S.edges_scanned - S.tier_edges) * g->col_bytes) +
                          S.weights_read * 4;
    // the TEPS numerator: a top-down BFS expands every reached vertex once;
    // bottom-up levels sum the found vertices' degrees instead; SSSP adds up
    // the reached vertices' degrees in one pass; CC counts every edge
    if (algo == A_BFS) {
        S.reached_edges = do_bfs ? explored : S.edges_scanned;
    } else if (algo == A_SSSP && V > 0) {
        zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
        hipLaunchKernelGGL(k_reached_edges, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, g->row_ptr, V,
                           p.counters);
        if ((st = sync_counters()) != EMOGI_OK) return st;
        S.reached_edges = p.host_counters[C_FEDGES];
    } else if (algo == A_CC) {
        S.reached_edges = g->E;
    }
    if (overflow_seen) {
        zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
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

static emogi_status_t pagerank(emogi_graph_s *g, uint32_t iters, uint32_t F, uint64_t d, uint64_t *out,
                               hipStream_t stream) {
    if (!g || !out) {
        set_error("null graph or output");
        return EMOGI_E_INVALID;
    }
    if (!(g->flags & EMOGI_F_SYMMETRIC)) {
        set_error("PageRank (pull form) needs a graph created with EMOGI_F_SYMMETRIC");
        return EMOGI_E_NOT_SYMMETRIC;
    }
    if (F < 1 || F > 62 || d >= (uint64_t(1) << F)) {
        set_error("PageRank needs 1 <= frac_bits <= 62 and damping_fixed < 2^frac_bits");
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
    emogi_status_t st = ensure_pool(g, A_BFS);
    if (st != EMOGI_OK) return st;
    Pool &p = g->pool;
    const uint64_t V = g->V;
    emogi_stats_t &S = g->stats;
    memset(&S, 0, sizeof(S));
    S.request_unit = g->request_unit;
    uint64_t packed_bytes = 0;
    EMOGI_HIP_TRY(hipEventRecord(g->ev_begin, stream), EMOGI_E_HIP);
    if (V > 0) {
        for (void **b : {reinterpret_cast<void **>(&p.pr_acc), reinterpret_cast<void **>(&p.pr_contrib)})
            if (!*b && hipMalloc(b, V * sizeof(uint64_t)) != hipSuccess) {
                (void)hipGetLastError();
                *b = nullptr;
                set_error("hipMalloc of the PageRank buffers failed");
                return EMOGI_E_OOM_DEVICE;
            }
        if ((st = ensure_scan(g, V)) != EMOGI_OK) return st;
        const uint64_t one = uint64_t(1) << F;
        ScanArgs s{};
        s.queue = nullptr;  // every vertex, in id order
        s.n = uint32_t(V);
        s.n_dev = nullptr;
        s.row_ptr = g->row_ptr;
        s.col = g->col;
        s.w = nullptr;
        s.next = nullptr;
        s.align_mask = uint64_t(std::max<uint32_t>(1, g->request_unit / g->col_bytes)) - 1;
        s.req_unit = g->request_unit;
        s.col_bytes = g->col_bytes;
        s.tier = tier_view(g);
        use_packed(s, g);
        const unsigned nb = unsigned((V + kScanTile) / kScanTile);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kBlock), 0, stream, p.block_sums, nb);
        hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(kBlock), 0, stream, s, p.block_sums, p.chunk_scan);
        s.chunk_scan = p.chunk_scan;
        hipLaunchKernelGGL(k_pr_init, dim3(fill_grid(V)), dim3(kBlock), 0, stream, g->row_ptr, V, one / V,
                           p.pr_acc, out, p.pr_contrib);
        EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
        PrArgs pa{p.pr_contrib, p.pr_acc, p.counters};
        for (uint32_t t = 0; t < iters; ++t) {
            zero_async(p.counters, C_COUNT * sizeof(unsigned long long), stream);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k0, stream), EMOGI_E_HIP);
            if (g->packed.stream)
                hipLaunchKernelGGL(k_pr_pull<PackedCol>, dim3(kMaxGrid), dim3(kBlock), 0, stream, s, pa);
            else if (g->col_bytes == 8)
                hipLaunchKernelGGL(k_pr_pull<uint64_t>, dim3(kMaxGrid), dim3(kBlock), 0, stream, s, pa);
            else
                hipLaunchKernelGGL(k_pr_pull<uint32_t>, dim3(kMaxGrid), dim3(kBlock), 0, stream, s, pa);
            EMOGI_HIP_TRY(hipEventRecord(g->ev_k1, stream), EMOGI_E_HIP);
            hipLaunchKernelGGL(k_pr_finish, dim3(fill_grid(V)), dim3(kBlock), 0, stream, g->row_ptr, V, (one - d) / V,
                               d, F, p.pr_acc, out, p.pr_contrib);
            EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipMemcpyAsync(p.host_counters, p.counters, C_COUNT * sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, stream),
                          EMOGI_E_HIP);
            EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
            float ms = 0.f;
            EMOGI_HIP_TRY(hipEventElapsedTime(&ms, g->ev_k0, g->ev_k1), EMOGI_E_HIP);
            const unsigned long long *hc = p.host_counters;
            if (t < EMOGI_MAX_LEVEL_STATS) {
                S.level_variant[t] = uint8_t(EMOGI_V5_BALANCED);
                S.level_frontier[t] = uint32_t(V);
                S.level_ms[t] = ms;
                S.level_edges[t] = hc[C_EDGES];
                S.level_count = t + 1;
            }
            S.variant_hist[EMOGI_V5_BALANCED] += 1;
            S.expand_ms += ms;
            S.expand_launches += 1;
            absorb_counters(S, hc);
            packed_bytes += hc[C_PKBYTES];
        }
    }
    S.iterations = iters;
    S.reached_edges = g->E;
    S.useful_link_bytes = g->packed.stream ? packed_bytes : (S.edges_scanned - S.tier_edges) * g->col_bytes;
    EMOGI_HIP_TRY(hipEventRecord(g->ev_end, stream), EMOGI_E_HIP);
    EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
    float total = 0.f;
    EMOGI_HIP_TRY(hipEventElapsedTime(&total, g->ev_begin, g->ev_end), EMOGI_E_HIP);
    S.total_ms = total;
    return EMOGI_OK;
}

// Bytes of device scratch bfs_in_scratch needs for V vertices: two frontier
// queues (V ids each), the visited bitmap and one counter block per level of
// a batch, each part starting on a 256-byte boundary.
static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
constexpr uint32_t kScratchLevels = 8;  // levels enqueued per host wait

uint64_t bfs_scratch_bytes(uint64_t V) {
    const uint64_t v = std::max<uint64_t>(V, 1);
    return 2 * align256(v * 4) + align256(((v + 31) / 32) * 4) +
           align256(uint64_t(kScratchLevels) * C_COUNT * sizeof(unsigned long long));
}

// BFS whose every device buffer lives in `scratch` (bytes >= bfs_scratch_bytes(V)):
// the same level kernels as emogi_bfs, with kScratchLevels levels enqueued per
// host wait (each level reads the frontier length the previous one left on
// the device, as in emogi_bfs's level batches), top-down, pushes through the
// LDS-staged queue, the variant fixed for the traversal (a fixed scheduler
// variant V0..V4 if set, else a workgroup per vertex).  Allocates nothing: the
// counters come back through a host array on this thread's stack.
// Stats: levels, variants, frontiers, edges, link bytes and times.
emogi_status_t bfs_in_scratch(emogi_graph_s *g, uint64_t src, uint32_t *out, void *scratch, uint64_t bytes,
                              hipStream_t stream) {
    if (!g || !out || !scratch) {
        set_error("null graph, output or scratch");
        return EMOGI_E_INVALID;
    }
    if (src >= g->V) {
        set_error("source %llu out of range (V = %llu)", (unsigned long long)src, (unsigned long long)g->V);
        return EMOGI_E_INVALID;
    }
    if (g->packed.stream) {
        set_error("packed lists are scanned by the edge-balanced variant, whose chunk prefix has no room here");
        return EMOGI_E_UNSUPPORTED;
    }
    {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, out) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            set_error("output must be device memory");
            return EMOGI_E_INVALID;
        }
    }
    const uint64_t V = g->V;
    if (bytes < bfs_scratch_bytes(V)) {
        set_error("BFS over %llu vertices needs %llu scratch bytes, %llu available", (unsigned long long)V,
                  (unsigned long long)bfs_scratch_bytes(V), (unsigned long long)bytes);
        return EMOGI_E_INVALID;
    }
    char *base = static_cast<char *>(scratch);
    uint32_t *queue[2];
    queue[0] = reinterpret_cast<uint32_t *>(base);
    queue[1] = reinterpret_cast<uint32_t *>(base + align256(V * 4));
    uint32_t *bitmap = reinterpret_cast<uint32_t *>(base + 2 * align256(V * 4));
    unsigned long long *ctr =
        reinterpret_cast<unsigned long long *>(base + 2 * align256(V * 4) + align256(((V + 31) / 32) * 4));
    unsigned long long host[kScratchLevels * C_COUNT];

    emogi_stats_t &S = g->stats;
    memset(&S, 0, sizeof(S));
    S.request_unit = g->request_unit;
    const int m = g->sched_mode;
    const int var = (m >= 0 && m < int(EMOGI_V5_BALANCED)) ? m : int(EMOGI_V4_BLOCK);
    const uint32_t align_elems = std::max<uint32_t>(1, g->request_unit / g->col_bytes);

    EMOGI_HIP_TRY(hipEventRecord(g->ev_begin, stream), EMOGI_E_HIP);
    hipLaunchKernelGGL(k_fill, dim3(fill_grid(V)), dim3(kBlock), 0, stream, out, V, 0xFFFFFFFFu);
    zero_async(bitmap, ((V + 31) / 32) * sizeof(uint32_t), stream);
    hipLaunchKernelGGL(k_seed_source, dim3(1), dim3(64), 0, stream, out, bitmap, queue[0], uint32_t(src), 1);
    EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);

    uint64_t n = 1, iter = 0;
    const uint64_t cap = V + 2;  // a BFS has at most V levels with work
    int cur = 0;
    while (n > 0) {
        if (iter >= cap) {
            (void)hipStreamSynchronize(stream);
            set_error("iteration cap %llu reached", (unsigned long long)cap);
            return EMOGI_E_NOCONVERGE;
        }
        const uint32_t k = uint32_t(std::min<uint64_t>(kScratchLevels, cap - iter));
        zero_async(ctr, size_t(k) * C_COUNT * sizeof(unsigned long long), stream);
        EMOGI_HIP_TRY(hipEventRecord(g->ev_k0, stream), EMOGI_E_HIP);
        for (uint32_t i = 0; i < k; ++i) {
            ScanArgs s;
            s.queue = queue[cur];
            s.n = i == 0 ? uint32_t(n) : uint32_t(V);  // later levels: V only sizes the grids
            s.n_dev = i == 0 ? nullptr : &ctr[(i - 1) * C_COUNT + C_NEXT];
            s.row_ptr = g->row_ptr;
            s.col = g->col;
            s.w = g->weights;
            s.next = queue[cur ^ 1];
            s.align_mask = uint64_t(align_elems) - 1;
            s.req_unit = g->request_unit;
            s.col_bytes = g->col_bytes;
            s.chunk_scan = nullptr;
            s.tier = tier_view(g);
            OpArgs a;
            a.state = out;
            a.bitmap = bitmap;
            a.stamp = nullptr;
            a.tag = uint32_t(iter + i + 1);
            a.V = uint32_t(V);
            a.ctr = &ctr[i * C_COUNT];
            a.nextbits = nullptr;
            a.split = 0xFFFFFFFFu;
            a.farbits = nullptr;
            a.wmin = 0;
            if (g->col_bytes == 8)
                launch_variant<uint64_t, A_BFS>(var, s, a, stream);
            else
                launch_variant<uint32_t, A_BFS>(var, s, a, stream);
            cur ^= 1;
        }
        EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
        EMOGI_HIP_TRY(hipEventRecord(g->ev_k1, stream), EMOGI_E_HIP);
        EMOGI_HIP_TRY(hipMemcpyAsync(host, ctr, size_t(k) * C_COUNT * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, stream),
                      EMOGI_E_HIP);
        EMOGI_HIP_TRY(hipStreamSynchronize(stream), EMOGI_E_HIP);
        float ms = 0.f;
        EMOGI_HIP_TRY(hipEventElapsedTime(&ms, g->ev_k0, g->ev_k1), EMOGI_E_HIP);
        S.expand_ms += ms;
        uint32_t ran = 0;
        for (uint32_t i = 0; i < k && n > 0; ++i, ++ran) {
            const unsigned long long *hc = &host[i * C_COUNT];
            if (iter < EMOGI_MAX_LEVEL_STATS) {
                S.level_variant[iter] = uint8_t(var);
                S.level_frontier[iter] = uint32_t(n);
                S.level_edges[iter] = hc[C_EDGES];
                S.level_count = uint32_t(iter + 1);
            }
            S.variant_hist[var] += 1;
            S.expand_launches += 1;
            absorb_counters(S, hc);
            n = hc[C_NEXT];
            ++iter;
        }
        for (uint32_t i = 0; i < ran; ++i)
            if (iter - ran + i < EMOGI_MAX_LEVEL_STATS) S.level_ms[iter - ran + i] = ms / float(ran);
    }
    S.iterations = uint32_t(iter);
    S.useful_link_bytes = (S.edges_scanned - S.tier_edges) * g->col_bytes;
    S.reached_edges = S.edges_scanned;  // top-down BFS scans each reached vertex's list once
    EMOGI_HIP_TRY(hipEventRecord(g->ev_end, stream), EMOGI_E_HIP);
    EMOGI_HIP_TRY(hipEventSynchronize(g->ev_end), EMOGI_E_HIP);
    float total = 0.f;
    EMOGI_HIP_TRY(hipEventElapsedTime(&total, g->ev_begin, g->ev_end), EMOGI_E_HIP);
    S.total_ms = total;
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

emogi_status_t emogi_pagerank(emogi_graph_t g, uint32_t iters, uint32_t frac_bits, uint64_t damping_fixed,
                              uint64_t *scores, void *stream) {
    return pagerank(g, iters, frac_bits, damping_fixed, scores, static_cast<hipStream_t>(stream));
}

}  // extern "C"
