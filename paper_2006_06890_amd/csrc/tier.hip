// HBM tier of neighbour lists: which lists are copied into GPU memory, the
// copy itself, and its C ABI entry point.  The scan kernels find a tier list
// through tier.h; every traversal result is unchanged by the tier.
//
// Selection: vertices in order of decreasing degree (ties: ascending id), the
// longest prefix of that order whose lists (and weights) fit the budget.  On
// skewed graphs a small budget holds a large share of the edges: R-MAT puts a
// quarter of its edges in the lists of about 0.1 % of the vertices.
#include "internal.h"
#include "tier.h"
#include "wave.h"

#include <algorithm>
#include <vector>

namespace emogi {

void tier_release(emogi_graph_s *g) {
    Tier &t = g->tier;
    for (void *x : {(void *)t.bits, (void *)t.ids, (void *)t.start, t.col, (void *)t.w})
        if (x) (void)hipFree(x);
    t = Tier{};
}

// One wave per tier vertex: copy its list (and weights) from the edge list.
template <class ColT>
__global__ __launch_bounds__(kBlock) void k_tier_fill(const uint64_t *row_ptr, const ColT *col, const uint32_t *w,
                                                      const uint32_t *ids, const uint64_t *start, uint32_t n,
                                                      ColT *tcol, uint32_t *tw) {
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const uint64_t nw = uint64_t(gridDim.x) * kWavesPerBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kWavesPerBlock + wid; i < n; i += nw) {
        const uint32_t u = ids[i];
        const uint64_t b = row_ptr[u], e = row_ptr[u + 1], t0 = start[i];
        for (uint64_t j = b + lane; j < e; j += kWave) {
            tcol[t0 + (j - b)] = col[j];
            if (tw) tw[t0 + (j - b)] = w[j];
        }
    }
}

__global__ void k_tier_bits(const uint32_t *ids, uint32_t n, uint32_t *bits) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        atomicOr(&bits[ids[i] >> 5], 1u << (ids[i] & 31u));
}

// Tier vertices for a budget, ascending; *elems gets their total degree.
static std::vector<uint32_t> select_tier(const std::vector<uint64_t> &rp, uint64_t elem_bytes, uint64_t budget,
                                         uint64_t max_degree, uint64_t *elems) {
    const uint64_t V = rp.size() - 1;
    std::vector<uint64_t> cnt(max_degree + 1, 0);
    for (uint64_t v = 0; v < V; ++v) cnt[rp[v + 1] - rp[v]] += 1;
    // walk degrees downwards: every vertex of degree >= full fits; `take` more of degree `part`
    uint64_t acc = 0, full = max_degree + 1, part = 0, take = 0;
    for (uint64_t d = max_degree; d >= 1; --d) {
        if (!cnt[d]) continue;
        const uint64_t per = d * elem_bytes;
        if (acc + cnt[d] * per <= budget) {
            acc += cnt[d] * per;
            full = d;
            continue;
        }
        part = d;
        take = (budget - acc) / per;
        break;
    }
    std::vector<uint32_t> ids;
    uint64_t total = 0, taken = 0;
    for (uint64_t v = 0; v < V; ++v) {
        const uint64_t d = rp[v + 1] - rp[v];
        if (d == 0) continue;
        if (d >= full || (d == part && taken < take)) {
            if (d == part && d < full) ++taken;
            ids.push_back(uint32_t(v));
            total += d;
        }
    }
    *elems = total;
    return ids;
}

}  // namespace emogi

using namespace emogi;

extern "C" {

emogi_status_t emogi_set_hbm_tier(emogi_graph_t g, uint64_t budget_bytes, uint64_t *tier_vertices,
                                  uint64_t *tier_bytes) {
    if (!g) {
        set_error("null graph");
        return EMOGI_E_INVALID;
    }
    if (g->packed.stream) {
        set_error("the HBM tier copies plain lists; this graph's lists are packed");
        return EMOGI_E_UNSUPPORTED;
    }
    EMOGI_HIP_TRY(hipDeviceSynchronize(), EMOGI_E_HIP);
    tier_release(g);
    if (tier_vertices) *tier_vertices = 0;
    if (tier_bytes) *tier_bytes = 0;
    if (budget_bytes == 0 || g->V == 0 || g->E == 0) return EMOGI_OK;

    const uint64_t V = g->V, eb = g->col_bytes + (g->weights ? 4u : 0u);
    std::vector<uint64_t> rp(V + 1);
    EMOGI_HIP_TRY(hipMemcpy(rp.data(), g->row_ptr, (V + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost), EMOGI_E_HIP);
    uint64_t elems = 0;
    std::vector<uint32_t> ids = select_tier(rp, eb, budget_bytes, g->max_degree, &elems);
    if (ids.empty()) return EMOGI_OK;
    const uint32_t n = uint32_t(ids.size());
    std::vector<uint64_t> start(n + 1, 0);
    for (uint32_t i = 0; i < n; ++i) start[i + 1] = start[i] + (rp[ids[i] + 1] - rp[ids[i]]);

    Tier &t = g->tier;
    const uint64_t words = (V + 31) / 32;
    const uint64_t need = words * 4 + uint64_t(n) * 4 + (uint64_t(n) + 1) * 8 + elems * eb;
    size_t free_b = 0, total_b = 0;
    EMOGI_HIP_TRY(hipMemGetInfo(&free_b, &total_b), EMOGI_E_HIP);
    if (need + (size_t(256) << 20) > free_b) {
        set_error("HBM tier of %llu bytes does not fit (%zu bytes free)", (unsigned long long)need, free_b);
        return EMOGI_E_OOM_DEVICE;
    }
    auto dalloc = [&](void **p, size_t bytes) {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return false;
        }
        return true;
    };
    if (!dalloc(reinterpret_cast<void **>(&t.bits), words * 4) || !dalloc(reinterpret_cast<void **>(&t.ids), n * 4ull) ||
        !dalloc(reinterpret_cast<void **>(&t.start), (n + 1ull) * 8) || !dalloc(&t.col, elems * g->col_bytes) ||
        (g->weights && !dalloc(reinterpret_cast<void **>(&t.w), elems * 4))) {
        tier_release(g);
        set_error("hipMalloc for the HBM tier failed");
        return EMOGI_E_OOM_DEVICE;
    }
    auto fail = [&](hipError_t e) {
        (void)hipGetLastError();
        tier_release(g);
        set_error("HBM tier set-up failed: %s", hipGetErrorString(e));
        return EMOGI_E_HIP;
    };
    hipError_t e;
    if ((e = hipMemset(t.bits, 0, words * 4)) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(t.ids, ids.data(), n * 4ull, hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(t.start, start.data(), (n + 1ull) * 8, hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
    const unsigned grid = unsigned(std::max<uint64_t>(1, std::min<uint64_t>((n + 3) / 4, 8192)));
    hipLaunchKernelGGL(k_tier_bits, dim3(std::min<unsigned>(grid, 1024)), dim3(256), 0, nullptr, t.ids, n, t.bits);
    if (g->col_bytes == 8)
        hipLaunchKernelGGL(k_tier_fill<uint64_t>, dim3(grid), dim3(kBlock), 0, nullptr, g->row_ptr,
                           static_cast<const uint64_t *>(g->col), g->weights, t.ids, t.start, n,
                           static_cast<uint64_t *>(t.col), t.w);
    else
        hipLaunchKernelGGL(k_tier_fill<uint32_t>, dim3(grid), dim3(kBlock), 0, nullptr, g->row_ptr,
                           static_cast<const uint32_t *>(g->col), g->weights, t.ids, t.start, n,
                           static_cast<uint32_t *>(t.col), t.w);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e);
    t.n = n;
    t.elems = elems;
    t.bytes = elems * eb;
    if (tier_vertices) *tier_vertices = n;
    if (tier_bytes) *tier_bytes = t.bytes;
    return EMOGI_OK;
}

}  // extern "C"
