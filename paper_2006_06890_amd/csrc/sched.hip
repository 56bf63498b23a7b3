// Per-level choice of the access variant.
//
// EMOGI fixes the worker at one warp per vertex and notes (Sec. 4.3.1) that a
// finer worker only pays when the graph is in GPU memory with low degrees;
// Sec. 5.3.1 shows alignment pays least on uniformly low-degree graphs.  So no
// variant wins on every frontier.  The scheduler reads 16 features of the
// current frontier and picks one of the six result-identical variants, either
// by a fixed rule or by a 16-64-64-6 MLP whose inference runs in one wave here.
// The features are computed on the GPU from the frontier queue and row_ptr.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace emogi {

int heuristic_variant(const emogi_graph_s *g, uint64_t n);

constexpr int kNIn = 16, kNH = 64, kNOut = 6;
constexpr int kNParams = kNH * kNIn + kNH + kNH * kNH + kNH + kNOut * kNH + kNOut;  // 5638

// acc[0..7]: degree histogram of the frontier, acc[8]: sum of degrees.
// The frontier length is n, or *n_dev when n_dev is set (a frontier the
// previous level has just written, whose length the host does not know yet).
// A block adds to acc only the counts it found (small frontiers leave most
// blocks idle and touch acc from few blocks).
__global__ __launch_bounds__(256) void k_frontier_hist(const uint32_t *queue, uint64_t n,
                                                       const unsigned long long *n_dev,
                                                       const uint64_t *row_ptr,
                                                       unsigned long long *acc) {
    __shared__ unsigned long long s_acc[kHistBins + 1];
    if (n_dev) n = *n_dev;
    if (threadIdx.x < kHistBins + 1) s_acc[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long local[kHistBins + 1] = {};
    for (uint64_t q = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
         q += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t u = queue ? queue[q] : uint32_t(q);
        const uint64_t d = row_ptr[u + 1] - row_ptr[u];
        local[degree_bin(d)] += 1;
        local[kHistBins] += d;
    }
    for (int i = 0; i < kHistBins + 1; ++i)
        if (local[i]) atomicAdd(&s_acc[i], local[i]);
    __syncthreads();
    if (threadIdx.x < kHistBins + 1 && s_acc[threadIdx.x]) atomicAdd(&acc[threadIdx.x], s_acc[threadIdx.x]);
}

struct FeatureConsts {
    float n, V, E, col8, weights, zero_copy, managed;
};

// One workgroup of 256 threads: the 16 features from the histogram, then
// z = W3 relu(W2 relu(W1 x + b1) + b2) + b3, argmax over the eligible
// variants (the straggler guard below) into *choice.  The
// parameters are first copied into LDS with coalesced loads (all in flight
// at once), so the layers wait on one global round trip, not one per input;
// the 64x64 layer uses four threads per unit.  The choice is -1 without
// weights, or when a feature lies outside the range the network was trained
// on (range: 16 lower, then 16 upper bounds; null: no check), so the caller
// falls back to the heuristic.  Also stores the features for harvesting, and
// clears the histogram for its next use.  n_dev as above.
__global__ __launch_bounds__(256) void k_mlp_pick(unsigned long long *acc, FeatureConsts c,
                                                  const unsigned long long *n_dev, const float *params,
                                                  const float *range, int *choice, float *feat_out) {
    __shared__ float P[kNParams];
    __shared__ float x[kNIn], h1[kNH], part[4][kNH], h2[kNH], z[kNOut];
    const int t = threadIdx.x;
    if (params) {
#pragma unroll 8
        for (int i = t; i < kNParams; i += 256) P[i] = params[i];
    }
    if (n_dev) c.n = float(*n_dev);
    if (t == 0) {
        const float sumdeg = float(acc[kHistBins]);
        x[0] = log2f(1.f + c.n) / 32.f;
        x[1] = c.n / fmaxf(c.V, 1.f);
        x[2] = log2f(1.f + sumdeg) / 40.f;
        x[3] = sumdeg / fmaxf(c.E, 1.f);
        for (int b = 0; b < kHistBins; ++b) x[4 + b] = float(acc[b]) / fmaxf(c.n, 1.f);
        x[12] = c.col8;
        x[13] = c.weights;
        x[14] = c.zero_copy;
        x[15] = c.managed;
    }
    __syncthreads();
    if (t < kHistBins + 1) acc[t] = 0;
    if (t < kNIn && feat_out) feat_out[t] = x[t];
    const int outside = range && t < kNIn && (x[t] < range[t] || x[t] > range[kNIn + t]);
    if (__syncthreads_or(outside) || !params) {  // (uniform) no pick outside the trained range
        if (t == 0) *choice = -1;
        return;
    }
    const float *W1 = P, *b1 = W1 + kNH * kNIn, *W2 = b1 + kNH, *b2 = W2 + kNH * kNH, *W3 = b2 + kNH,
                *b3 = W3 + kNOut * kNH;
    if (t < kNH) {
        float a = b1[t];
#pragma unroll
        for (int k = 0; k < kNIn; ++k) a += W1[t * kNIn + k] * x[k];
        h1[t] = fmaxf(a, 0.f);
    }
    __syncthreads();
    {
        const int o = t % kNH, qr = t / kNH;  // unit o, inputs [16 qr, 16 qr + 16)
        float a = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) a += W2[o * kNH + qr * 16 + k] * h1[qr * 16 + k];
        part[qr][o] = a;
    }
    __syncthreads();
    if (t < kNH) h2[t] = fmaxf(b2[t] + ((part[0][t] + part[1][t]) + (part[2][t] + part[3][t])), 0.f);
    __syncthreads();
    if (t < kNOut) {
        float a = b3[t];
#pragma unroll 16
        for (int k = 0; k < kNH; ++k) a += W3[t * kNH + k] * h2[k];
        z[t] = a;
    }
    __syncthreads();
    if (t == 0) {
        // Straggler guard: a worker narrower than the frontier's longest list
        // reads that list alone while the rest of the level waits, so a variant
        // is eligible only if every list fits it: a thread (V0) below 16 ids,
        // a 16-lane group (V1) below 64, a wave (V2, V3) below 4096; the
        // workgroup (V4) and the edge-balanced scan (V5) always are.
        // (x[4 + b] > 0: some frontier vertex has a degree in bin b.)
        bool long_at[kHistBins + 1];  // some list in bin b or above
        long_at[kHistBins] = false;
        for (int b = kHistBins - 1; b >= 0; --b) long_at[b] = long_at[b + 1] || x[4 + b] > 0.f;
        const bool eligible[kNOut] = {!long_at[4], !long_at[5], !long_at[7], !long_at[7], true, true};
        int best = -1;
        for (int j = 0; j < kNOut; ++j)
            if (eligible[j] && (best < 0 || z[j] > z[best])) best = j;
        *choice = best;
    }
}

// Scratch for the scheduler: acc (9 u64), choice (int) and features (16 f32).
struct SchedScratch {
    unsigned long long *acc;
    int *choice;
    float *feat;
};

static emogi_status_t sched_scratch(emogi_graph_s *g, SchedScratch *s) {
    Pool &p = g->pool;
    if (!p.degree_hist) {
        // layout: [acc: 9 x u64][pad][choice: int][pad][features: 16 f32]
        if (hipMalloc(&p.degree_hist, 256) != hipSuccess) {
            (void)hipGetLastError();
            p.degree_hist = nullptr;
            set_error("scheduler scratch allocation failed");
            return EMOGI_E_OOM_DEVICE;
        }
        // k_mlp_pick leaves the histogram cleared after every pick
        EMOGI_HIP_TRY(hipMemset(p.degree_hist, 0, 256), EMOGI_E_HIP);
    }
    char *base = reinterpret_cast<char *>(p.degree_hist);
    s->acc = reinterpret_cast<unsigned long long *>(base);
    s->choice = reinterpret_cast<int *>(base + 96);
    s->feat = reinterpret_cast<float *>(base + 128);
    return EMOGI_OK;
}

// Frontier features (and the MLP's pick when weights are loaded).
// Returns the variant, or -1 on a HIP failure.
static FeatureConsts feature_consts(const emogi_graph_s *g, int algo, uint64_t n) {
    FeatureConsts c;
    c.n = float(n);
    c.V = float(g->V);
    c.E = float(g->E);
    c.col8 = g->col_bytes == 8 ? 1.f : 0.f;
    c.weights = algo == 1 ? 1.f : 0.f;
    c.zero_copy = g->placement == EMOGI_PLACE_HOST_ZERO_COPY ? 1.f : 0.f;
    c.managed = g->placement == EMOGI_PLACE_MANAGED ? 1.f : 0.f;
    return c;
}

static int learned_pick(emogi_graph_s *g, int algo, uint64_t n, const uint32_t *queue,
                        hipStream_t stream, float *features_host, int *by_network) {
    SchedScratch s;
    if (sched_scratch(g, &s) != EMOGI_OK) return -1;
    const unsigned grid = unsigned(std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 1024)));
    hipLaunchKernelGGL(k_frontier_hist, dim3(grid), dim3(256), 0, stream, queue, n,
                       static_cast<const unsigned long long *>(nullptr), g->row_ptr, s.acc);
    hipLaunchKernelGGL(k_mlp_pick, dim3(1), dim3(256), 0, stream, s.acc, feature_consts(g, algo, n),
                       static_cast<const unsigned long long *>(nullptr), g->mlp_params, g->mlp_range, s.choice,
                       s.feat);
    // choice (byte 96) and features (bytes 128..191) in one copy
    unsigned char h[96];
    if (hipMemcpyAsync(h, s.choice, sizeof(h), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    int choice;
    memcpy(&choice, h, sizeof(int));
    if (features_host) memcpy(features_host, h + 32, kNIn * sizeof(float));
    if (!g->mlp_params || choice < 0 || choice >= kNOut) return heuristic_variant(g, n);  // also: outside range
    *by_network = 1;
    return choice;
}

// Whether the scheduler needs the frontier's features at all.
bool sched_needs_features(const emogi_graph_s *g) {
    return g->record_features || (g->sched_mode == EMOGI_SCHED_LEARNED && g->mlp_params);
}

// Clears the histogram before a traversal that uses sched_prefetch.
emogi_status_t sched_begin(emogi_graph_s *g, hipStream_t stream) {
    SchedScratch s;
    emogi_status_t st = sched_scratch(g, &s);
    if (st != EMOGI_OK) return st;
    EMOGI_HIP_TRY(hipMemsetAsync(s.acc, 0, 128, stream), EMOGI_E_HIP);
    return EMOGI_OK;
}

// Features and pick for the frontier a level has just written (its length is
// counters[C_NEXT] on the device), enqueued behind that level: the results
// land in the counter block the level copies back anyway, so the choice costs
// no extra host round trip.  The histogram is left cleared by k_mlp_pick.
emogi_status_t sched_prefetch(emogi_graph_s *g, int algo, const uint32_t *queue, unsigned long long *counters,
                              hipStream_t stream) {
    SchedScratch s;
    emogi_status_t st = sched_scratch(g, &s);
    if (st != EMOGI_OK) return st;
    const unsigned grid = unsigned(std::max<uint64_t>(1, std::min<uint64_t>((g->V + 255) / 256, 1024)));
    hipLaunchKernelGGL(k_frontier_hist, dim3(grid), dim3(256), 0, stream, queue, uint64_t(0),
                       static_cast<const unsigned long long *>(&counters[C_NEXT]), g->row_ptr, s.acc);
    hipLaunchKernelGGL(k_mlp_pick, dim3(1), dim3(256), 0, stream, s.acc, feature_consts(g, algo, 0),
                       static_cast<const unsigned long long *>(&counters[C_NEXT]), g->mlp_params, g->mlp_range,
                       reinterpret_cast<int *>(&counters[C_CHOICE]), reinterpret_cast<float *>(&counters[C_FEAT]));
    EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
    return EMOGI_OK;
}

// Variant for a frontier whose pick and features sched_prefetch computed
// (hc: the host copy of the counter block).  Same rule as choose_variant.
// *by_network is set to 1 when the network's pick is used.
int choose_prefetched(const emogi_graph_s *g, uint64_t n, const unsigned long long *hc, float *features,
                      int *by_network) {
    *by_network = 0;
    if (features) memcpy(features, &hc[C_FEAT], kNIn * sizeof(float));
    const int m = g->sched_mode;
    if (m >= 0 && m < EMOGI_NUM_VARIANTS) return m;
    if (m == EMOGI_SCHED_LEARNED && g->mlp_params) {
        const int c = int(uint32_t(hc[C_CHOICE] & 0xFFFFFFFFull));
        if (c >= 0 && c < kNOut) {
            *by_network = 1;
            return c;
        }
    }
    return heuristic_variant(g, n);
}

// Variant for the level; fills `features` (16 floats) when non-null.
// Returns -1 when the scheduler's kernels fail.
int choose_variant(emogi_graph_s *g, int algo, uint64_t n, const uint32_t *queue, hipStream_t stream,
                   float *features, int *by_network) {
    const int m = g->sched_mode;
    int learned = -2, net = 0;
    *by_network = 0;
    // a one-vertex frontier (the source) has nothing to schedule: unless its
    // features are recorded, it takes the heuristic without a host round trip
    if (!features && m == EMOGI_SCHED_LEARNED && n <= 1) return heuristic_variant(g, n);
    if (features || (m == EMOGI_SCHED_LEARNED && g->mlp_params)) {
        learned = learned_pick(g, algo, n, queue, stream, features, &net);
        if (learned < 0) return -1;
    }
    if (m >= 0 && m < EMOGI_NUM_VARIANTS) return m;
    if (m == EMOGI_SCHED_LEARNED && g->mlp_params) {
        *by_network = net;
        return learned;
    }
    return heuristic_variant(g, n);
}

}  // namespace emogi

using namespace emogi;

extern "C" {

emogi_status_t emogi_set_scheduler_weights(emogi_graph_t g, const float *params, size_t count) {
    if (!g) {
        set_error("null graph");
        return EMOGI_E_INVALID;
    }
    if (!params) {
        if (g->mlp_params) (void)hipFree(g->mlp_params);
        g->mlp_params = nullptr;
        return EMOGI_OK;
    }
    if (count != size_t(kNParams)) {
        set_error("expected %d scheduler parameters, got %zu", kNParams, count);
        return EMOGI_E_INVALID;
    }
    if (!g->mlp_params) {
        if (hipMalloc(&g->mlp_params, kNParams * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            g->mlp_params = nullptr;
            set_error("hipMalloc for scheduler weights failed");
            return EMOGI_E_OOM_DEVICE;
        }
    }
    EMOGI_HIP_TRY(hipMemcpy(g->mlp_params, params, kNParams * sizeof(float), hipMemcpyHostToDevice),
                  EMOGI_E_HIP);
    return EMOGI_OK;
}

emogi_status_t emogi_set_scheduler_range(emogi_graph_t g, const float *lo, const float *hi) {
    if (!g || (!lo) != (!hi)) {
        set_error("scheduler range needs both bounds or neither");
        return EMOGI_E_INVALID;
    }
    if (!lo) {
        if (g->mlp_range) (void)hipFree(g->mlp_range);
        g->mlp_range = nullptr;
        return EMOGI_OK;
    }
    if (!g->mlp_range) {
        if (hipMalloc(&g->mlp_range, 2 * kNIn * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            g->mlp_range = nullptr;
            set_error("hipMalloc for the scheduler range failed");
            return EMOGI_E_OOM_DEVICE;
        }
    }
    EMOGI_HIP_TRY(hipMemcpy(g->mlp_range, lo, kNIn * sizeof(float), hipMemcpyHostToDevice), EMOGI_E_HIP);
    EMOGI_HIP_TRY(hipMemcpy(g->mlp_range + kNIn, hi, kNIn * sizeof(float), hipMemcpyHostToDevice), EMOGI_E_HIP);
    return EMOGI_OK;
}

}  // extern "C"
