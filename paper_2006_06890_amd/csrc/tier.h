// HBM tier of neighbour lists: a copy, in GPU memory, of the lists (and
// weights) of the highest-degree vertices, so a scan of such a list does not
// cross the host link.  This is the caching of graph data in GPU memory that
// EMOGI names as a way to cut host-link traffic further (Sec. 6); MI355X's
// 288 GB of HBM leaves room for it beside the vertex state.  Results do not
// depend on it: a tier list is a byte copy of the list it stands for.
#pragma once

#include "internal.h"

namespace emogi {

// Device view of the tier, passed by value to the scan kernels.
struct TierView {
    const uint32_t *bits;   // one bit per vertex: its list is in the tier (null: no tier)
    const uint32_t *ids;    // tier vertices, ascending
    const uint64_t *start;  // tier offset of each tier vertex's first element (n + 1 entries)
    const void *col;        // tier neighbour ids (same width as the edge list)
    const uint32_t *w;      // tier weights, or null
    uint32_t n;             // tier vertices
};

// Where the elements of vertex u's list [b, e) are read from: element j sits at
// col[j - shift] (and w[j - shift]); for a tier vertex col/w are the tier's.
template <class ColT>
struct ListSrc {
    const ColT *col;
    const uint32_t *w;
    uint64_t shift;
    bool tier;
};

template <class ColT>
__device__ __forceinline__ ListSrc<ColT> list_src(const TierView &t, const ColT *col, const uint32_t *w,
                                                  uint32_t u, uint64_t b) {
    if (t.bits && ((t.bits[u >> 5] >> (u & 31u)) & 1u)) {
        uint32_t lo = 0, hi = t.n;  // ids[lo] <= u < ids[hi]; u is among ids
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (t.ids[mid] <= u) lo = mid; else hi = mid;
        }
        // tier lists are laid out in id order, so start[lo] <= b and the shift is >= 0
        return ListSrc<ColT>{static_cast<const ColT *>(t.col), t.w, b - t.start[lo], true};
    }
    return ListSrc<ColT>{col, w, 0, false};
}

inline TierView tier_view(const ::emogi_graph_s *g) {
    TierView t{};
    if (g->tier.n) {
        t.bits = g->tier.bits;
        t.ids = g->tier.ids;
        t.start = g->tier.start;
        t.col = g->tier.col;
        t.w = g->tier.w;
        t.n = g->tier.n;
    }
    return t;
}

}  // namespace emogi
