// Internal definitions of the zero-copy traversal library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/emogi.h"

namespace emogi {

// Thread-local message of the last failing call.
void set_error(const char *fmt, ...);

#define EMOGI_HIP_TRY(expr, code)                                                  \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            (void)hipGetLastError();                                               \
            ::emogi::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                               \
            return (code);                                                         \
        }                                                                          \
    } while (0)

// Device counters written by the scan kernels; copied to host once per level.
enum Counter : int {
    C_NEXT = 0,      // entries pushed to the next frontier
    C_EDGES = 1,     // sum of degrees of expanded vertices
    C_REQBYTES = 2,  // request-granular link bytes of those lists
    C_OVERFLOW = 3,  // SSSP: some relaxation exceeded 0xFFFFFFFE
    C_VERTS = 4,     // expanded vertices
    C_BANDMIN = 5,   // SSSP: 2^32 - (smallest distance of a marked vertex left for a later band), 0: none
    C_CHOICE = 6,    // scheduler: variant picked for the next frontier (low 32 bits)
    C_FEAT = 7,      // scheduler: the next frontier's 16 features (fp32, 8 slots)
    C_TIER = 15,     // edges of expanded vertices whose lists were read from the HBM tier
    C_WLINK = 16,    // SSSP: weights read over the host link
    C_PKBYTES = 17,  // packed lists: encoded bytes of the lists scanned
    C_FEDGES = 18,   // sum of degrees of the next frontier (listing pass or bottom-up finds)
    C_REST = 19,     // bottom-up: vertices left for the wave-per-vertex pass
    C_IDSECT = 20,   // 32-byte sectors of neighbour ids read over the host link
    C_WSECT = 21,    // SSSP: 32-byte sectors of weights read over the host link
    C_COUNT = 22
};

// Degree bins of the scheduler's frontier histogram: <=1, [2,4), [4,8),
// [8,16), [16,64), [64,256), [256,4096), >=4096.  The histogram is 8 counts
// then the degree sum (9 x u64).
constexpr int kHistBins = 8;
__device__ __forceinline__ int degree_bin(uint64_t d) {
    return d <= 1 ? 0 : d < 4 ? 1 : d < 8 ? 2 : d < 16 ? 3 : d < 64 ? 4 : d < 256 ? 5 : d < 4096 ? 6 : 7;
}

// HBM tier of neighbour lists (device arrays; see tier.h).
struct Tier {
    uint32_t *bits = nullptr;   // V bits
    uint32_t *ids = nullptr;    // tier vertices, ascending
    uint64_t *start = nullptr;  // n + 1 offsets into col / w
    void *col = nullptr;
    uint32_t *w = nullptr;
    uint32_t n = 0;
    uint64_t elems = 0;         // list elements held
    uint64_t bytes = 0;         // device bytes of col + w
};

// Packed neighbour lists (EMOGI_F_PACK).  Each list is cut into blocks of
// 64 ids; a block is its first id as a whole word, then the gaps to the next
// ids (at most 63) at the list's gap width w, then (with weights) the
// block's weights at the list's weight width ww, each part bit-packed into
// whole words.  Every block but a list's last is full, so block k of list u
// starts at word off[u] + k * (1 + ceil(63 w / 32) + 2 ww).
struct Packed {
    uint32_t *stream = nullptr;  // the blocks of all lists, as the GPU addresses them
    void *pinned = nullptr;      // host allocation behind stream (zero-copy placement)
    bool on_device = false;      // stream is in HBM
    uint64_t *off = nullptr;     // HBM, V + 1 word offsets
    uint8_t *width = nullptr;    // HBM, V gap widths in bits (0..32)
    uint8_t *wwidth = nullptr;   // HBM, V weight widths in bits (0..32), or null: no weights
    uint64_t words = 0;          // stream length
    uint64_t wwords = 0;         // of which weight words
};

struct Pool {
    uint32_t *queue[2] = {nullptr, nullptr}; // frontier ids, V entries each
    uint32_t *bitmap = nullptr;               // BFS visited / SSSP overflow marks
    uint32_t *stamp = nullptr;                // CC label propagation: round in which v was last pushed
    uint64_t *chunk_scan = nullptr;           // V5: exclusive scan of per-entry chunk counts
    uint64_t *block_sums = nullptr;           // V5: scan partials
    unsigned long long *counters = nullptr;   // C_COUNT device counters
    unsigned long long *host_counters = nullptr; // pinned mirror
    float *features = nullptr;                // scheduler features (device)
    uint32_t *degree_hist = nullptr;          // scheduler degree histogram (device)
    uint32_t *snap_state = nullptr;           // probe mode: saved state of a level
    uint32_t *snap_stamp = nullptr;
    uint32_t *snap_bitmap = nullptr;
    uint32_t *snap_nextbits = nullptr;        // probe mode: saved SSSP marks
    uint32_t *farbits = nullptr;              // SSSP: improved beyond the band, not yet expanded
    uint32_t *snap_farbits = nullptr;
    uint32_t *cc_probe = nullptr;             // CC: roots of probed vertices
    uint32_t *nextbits = nullptr;             // ordered frontier bitmap (SSSP: improved, not yet expanded)
    uint32_t *fbits = nullptr;                // bottom-up BFS: the current frontier as a bitmap
    unsigned long long *pr_acc = nullptr;     // PageRank: per-vertex sums of the iteration
    uint64_t *pr_contrib = nullptr;           // PageRank: floor(score / degree) per vertex
    unsigned long long *level_ctr = nullptr;  // BFS level batches: one counter block per level
    unsigned long long *level_host = nullptr; // pinned mirror
    uint32_t level_cap = 0;
    size_t chunk_cap = 0;
};

// State of batched multi-source traversals (up to 64 sources, one bit each).
struct BatchPool {
    unsigned long long *mask[2] = {nullptr, nullptr}; // frontier masks (current / next) per vertex
    unsigned long long *vis = nullptr;    // BFS: sources that reached v
    unsigned long long *ovf = nullptr;    // SSSP: sources whose relaxation into v overflowed
    unsigned long long *wait = nullptr;   // SSSP: sources waiting for a later band at v
    uint32_t *dist = nullptr;             // SSSP: distances, vertex-major [V][64]
    uint32_t *hub[2] = {nullptr, nullptr};// queues of long lists (workgroup per vertex)
    unsigned long long *ctr = nullptr;    // queue lengths, level, flags
    unsigned long long *host_ctr = nullptr;
    uint64_t *srcs = nullptr;             // device copy of the sources
    hipStream_t stream = nullptr;         // private stream for capture and replay
};

}  // namespace emogi

struct emogi_graph_s {
    uint64_t V = 0, E = 0;
    uint32_t col_bytes = 4;
    uint32_t flags = 0;
    emogi_placement_t placement = EMOGI_PLACE_HOST_ZERO_COPY;
    int device = 0;

    uint64_t *row_ptr = nullptr;   // device (HBM)
    void *col = nullptr;           // device-dereferenceable edge list
    uint32_t *weights = nullptr;   // device-dereferenceable weights or null
    // ownership of the edge storage
    enum Kind { NONE, DEVICE, PINNED, MANAGED, BORROWED } col_kind = NONE, w_kind = NONE;

    uint32_t request_unit = 256;
    uint32_t sssp_delta = 3;       // near-far band width; 0 = plain label correcting
    bool cc_sampled = true;        // CC by sampled union-find (else min-label propagation)
    bool ordered_frontier = true;  // list each next frontier in ascending id order
    uint32_t level_batch = 0;      // BFS levels per host wait (0: automatic)
    int sched_mode = EMOGI_SCHED_HEURISTIC;
    bool record_features = false;  // store per-level frontier features in the stats
    float *mlp_params = nullptr;   // device, 5638 floats, or null
    float *mlp_range = nullptr;    // device, 16 lower then 16 upper feature bounds, or null
    uint64_t max_degree = 0;
    uint32_t min_weight = 0;       // smallest edge weight (a bound for skipping weight reads)
    uint8_t *in_min = nullptr;     // device, per vertex: smallest weight of an edge into it,
                                   // saturated at 255 (a tighter bound of the same kind)
    double in_min_ms = 0;          // time of the pass that computed in_min (0: not computed)
    uint64_t nonisolated = 0;      // vertices with at least one edge
    int direction = EMOGI_DIR_AUTO; // BFS level direction policy (emogi_set_direction)
    uint32_t dir_alpha = 14, dir_beta = 24;

    emogi::Pool pool;
    emogi::BatchPool batch;
    emogi::Tier tier;
    emogi::Packed packed;           // set for EMOGI_F_PACK graphs (col is then null)
    emogi_batch_params_t batch_params{1024, 4, 8, 1, 0};
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr;
    hipEvent_t ev_s0 = nullptr;     // before a level's preparation kernels (V5 chunk prefix)
    emogi_stats_t stats{};
};

namespace emogi {
void tier_release(emogi_graph_s *g);  // frees the HBM tier (tier.hip)
}  // namespace emogi
