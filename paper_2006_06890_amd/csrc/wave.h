// Wave64 helpers shared by the traversal kernels: lane ids, uniform values,
// and per-wave LDS staging of frontier pushes (ballot + mbcnt compaction).
#pragma once

#include "internal.h"

namespace emogi {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kSegCap = 512;      // LDS staging entries per wave

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}
__device__ __forceinline__ uint32_t uniform32(uint32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(x));
    uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(x >> 32));
    return (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = __shfl_xor(uint32_t(x), o), hi = __shfl_xor(uint32_t(x >> 32), o);
        x += (uint64_t(hi) << 32) | lo;
    }
    return x;
}

template <class ColT>
__device__ __forceinline__ uint32_t load_col(const ColT *col, uint64_t i) {
    return uint32_t(col[i]);
}

// ---------------------------------------------------------------------------
// Per-wave LDS staging of next-frontier entries.
// All 64 lanes must call stage()/flush() together (uniform control flow).
// ---------------------------------------------------------------------------
struct Stage {
    uint32_t *seg;  // this wave's LDS segment
    uint32_t cnt;   // entries staged (same value in every lane)
};

__device__ __forceinline__ void flush(Stage &st, uint32_t *next, unsigned long long *count, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t base = 0;
    if (lane == 0) base = uint32_t(atomicAdd(count, (unsigned long long)st.cnt));
    base = __shfl(base, 0);
    for (uint32_t i = lane; i < st.cnt; i += kWave) next[base + i] = st.seg[i];
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    st.cnt = 0;
}

__device__ __forceinline__ void stage(Stage &st, bool push, uint32_t v, uint32_t *next,
                                      unsigned long long *count, int lane) {
    uint64_t m = __ballot(push);
    if (m == 0) return;
    uint32_t c = uint32_t(__popcll(m));
    if (st.cnt + c > uint32_t(kSegCap)) flush(st, next, count, lane);
    if (push) st.seg[st.cnt + rank_below(m)] = v;
    st.cnt += c;
}

// End of a block: one global reservation for all staged entries, then the
// waves copy their segments out.
__device__ __forceinline__ void finish_queue(Stage &st, uint32_t *next, unsigned long long *count,
                                             int lane, int wid) {
    __shared__ uint32_t s_cnt[kWavesPerBlock];
    __shared__ uint32_t s_off[kWavesPerBlock];
    __shared__ uint32_t s_base;
    if (lane == 0) s_cnt[wid] = st.cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            s_off[w] = tot;
            tot += s_cnt[w];
        }
        s_base = tot ? uint32_t(atomicAdd(count, (unsigned long long)tot)) : 0u;
    }
    __syncthreads();
    uint32_t base = s_base + s_off[wid];
    for (uint32_t i = lane; i < st.cnt; i += kWave) next[base + i] = st.seg[i];
    st.cnt = 0;
}

}  // namespace emogi
