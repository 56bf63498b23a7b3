// Host-link calibration: the MI355X counterpart of the paper's toy 1-D copy
// study (Sec. 3.3, Fig. 4).  The paper copies a large zero-copy array into GPU
// memory with strided, merged+aligned and merged+misaligned access and finds
// that merged, aligned requests reach the bulk-copy rate.  Here the same
// experiment measures, on pinned host memory:
//   * the bulk copy rate (hipMemcpy host->device), the denominator the paper
//     uses (Sec. 5.3.2);
//   * the kernel read rate of a sequential wave-merged scan;
//   * random block reads for block sizes 32..4096 B, aligned and shifted by
//     32 B, from which the request unit R is the smallest aligned block that
//     reaches the copy rate within a tolerance (Sec. 4.3.2 aligns list starts
//     to it);
//   * the round-trip latency of a dependent pointer chase (Little's law,
//     Sec. 3.3, turns it into the outstanding requests needed).
#include "internal.h"

#include <algorithm>
#include <cstring>

namespace emogi {

// Each wave reads whole 64*W-byte chunks, grid-stride; the sum is kept live.
template <int W>
__global__ __launch_bounds__(256) void k_seq_read(const uint8_t *__restrict__ src, uint64_t chunks,
                                                  unsigned long long *sink) {
    const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
    const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) / 64;
    const int lane = threadIdx.x & 63;
    unsigned long long acc = 0;
    for (uint64_t c = wave; c < chunks; c += nwaves) {
        const uint8_t *p = src + c * (64ull * W) + lane * W;
        if (W == 4) acc += *reinterpret_cast<const uint32_t *>(p);
        else if (W == 8) acc += *reinterpret_cast<const uint64_t *>(p);
        else {
            const uint4 v = *reinterpret_cast<const uint4 *>(p);
            acc += v.x + v.y + v.z + v.w;
        }
    }
    if (acc == 0x9E3779B97F4A7C15ull) sink[0] = acc;
}

// Each wave reads `per_wave` blocks of B bytes at pseudo-random slots of the
// buffer: slot * A + shift, with 4-byte lanes.  Slots are < nslots, so every
// read stays inside [0, nslots * A + shift + B) which the host checks fits.
__global__ __launch_bounds__(256) void k_rand_read(const uint8_t *__restrict__ src, uint64_t nslots,
                                                   uint32_t B, uint32_t A, uint32_t shift,
                                                   uint32_t per_wave, uint64_t seed,
                                                   unsigned long long *sink) {
    const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x & 63;
    unsigned long long acc = 0;
    const uint32_t lanes_needed = B / 4;
    for (uint32_t k = 0; k < per_wave; ++k) {
        uint64_t z = seed + (wave * per_wave + k + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const uint64_t base = (z % nslots) * A + shift;
        for (uint32_t l = lane; l < lanes_needed; l += 64)
            acc += *reinterpret_cast<const uint32_t *>(src + base + 4ull * l);
    }
    if (acc == 0x9E3779B97F4A7C15ull) sink[0] = acc;
}

// One thread follows `hops` dependent links through the buffer.
__global__ void k_chase(const uint64_t *__restrict__ next, uint64_t start, uint32_t hops,
                        unsigned long long *sink) {
    uint64_t i = start;
    for (uint32_t h = 0; h < hops; ++h) i = next[i];
    sink[0] = i;
}

}  // namespace emogi

using namespace emogi;

extern "C" {

emogi_status_t emogi_calibrate_link(size_t bytes, emogi_link_profile_t *out) {
    if (!out || bytes < (size_t(64) << 20)) {
        set_error("calibration needs an output struct and at least 64 MiB");
        return EMOGI_E_INVALID;
    }
    bytes &= ~size_t(4095);
    memset(out, 0, sizeof(*out));
    void *h = nullptr, *d = nullptr;
    unsigned long long *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    emogi_status_t st = EMOGI_OK;
    auto cleanup = [&]() {
        if (h) (void)hipHostFree(h);
        if (d) (void)hipFree(d);
        if (sink) (void)hipFree(sink);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipHostMalloc(&h, bytes, hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        h = nullptr;
        set_error("pinned allocation of %zu bytes failed", bytes);
        return EMOGI_E_OOM_HOST;
    }
    if (hipMalloc(&d, bytes) != hipSuccess || hipMalloc(&sink, 64) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("device allocation for calibration failed");
        return EMOGI_E_OOM_DEVICE;
    }
    void *hd = nullptr;
    if (hipHostGetDevicePointer(&hd, h, 0) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("hipHostGetDevicePointer failed");
        return EMOGI_E_HIP;
    }
    // Pointer-chase ring: slot k (one per 64 KiB, so every hop is a new page)
    // links to slot (k + step) mod n with gcd(step, n) = 1, one cycle over all n.
    memset(h, 0, bytes);
    const uint64_t stride = (uint64_t(64) << 10) / 8, nslot = bytes / 8 / stride;
    {
        uint64_t *ring = static_cast<uint64_t *>(h);
        uint64_t step = 2654435761ull % nslot;
        auto gcd = [](uint64_t a, uint64_t b) { while (b) { uint64_t t = a % b; a = b; b = t; } return a; };
        while (step == 0 || gcd(step, nslot) != 1) step = (step + 1) % nslot;
        for (uint64_t k = 0; k < nslot; ++k) ring[k * stride] = ((k + step) % nslot) * stride;
    }
    auto time_ms = [&](auto launch) -> float {
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, 0);
            launch();
            (void)hipEventRecord(e1, 0);
            if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms);
        }
        return best;
    };
    // 1. bulk copy rate
    float ms = time_ms([&] { (void)hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, 0); });
    out->memcpy_GBps = ms > 0 ? bytes / (ms * 1e6) : 0;
    // 2. sequential wave-merged kernel reads, 4/8/16-byte lanes
    const uint8_t *src = static_cast<const uint8_t *>(hd);
    const int widths[3] = {4, 8, 16};
    for (int i = 0; i < 3; ++i) {
        const uint64_t chunks = bytes / (64ull * widths[i]);
        ms = time_ms([&] {
            if (widths[i] == 4) hipLaunchKernelGGL(k_seq_read<4>, dim3(8192), dim3(256), 0, 0, src, chunks, sink);
            if (widths[i] == 8) hipLaunchKernelGGL(k_seq_read<8>, dim3(8192), dim3(256), 0, 0, src, chunks, sink);
            if (widths[i] == 16) hipLaunchKernelGGL(k_seq_read<16>, dim3(8192), dim3(256), 0, 0, src, chunks, sink);
        });
        out->seq_read_GBps[i] = ms > 0 ? chunks * 64.0 * widths[i] / (ms * 1e6) : 0;
    }
    // 3. random block reads, aligned and shifted by 32 bytes
    const double seq_best = std::max({out->seq_read_GBps[0], out->seq_read_GBps[1], out->seq_read_GBps[2]});
    out->request_unit = 0;
    for (int i = 0; i < EMOGI_CALIB_BLOCKS; ++i) {
        const uint32_t B = 32u << i;  // 32 .. 4096
        out->block_bytes[i] = B;
        const uint32_t per_wave = std::max(1u, 16384u / B);
        const dim3 grid(4096);
        const uint64_t waves = uint64_t(grid.x) * 4;
        for (int sh = 0; sh < 2; ++sh) {
            const uint32_t shift = sh ? 32 : 0;
            const uint64_t nslots = (bytes - B - 64) / B;  // keeps slot*B + shift + B inside the buffer
            ms = time_ms([&] {
                hipLaunchKernelGGL(k_rand_read, grid, dim3(256), 0, 0, src, nslots, B, B, shift, per_wave,
                                   uint64_t(1234 + i), sink);
            });
            const double gbps = ms > 0 ? double(waves) * per_wave * B / (ms * 1e6) : 0;
            if (sh) out->rand_shift32_GBps[i] = gbps;
            else out->rand_aligned_GBps[i] = gbps;
        }
        if (!out->request_unit && out->rand_aligned_GBps[i] >= 0.9 * seq_best) out->request_unit = B;
    }
    if (!out->request_unit) out->request_unit = 256;
    // 4. dependent-load latency
    {
        const uint32_t hops = uint32_t(std::min<uint64_t>(4096, nslot));
        ms = time_ms([&] { hipLaunchKernelGGL(k_chase, dim3(1), dim3(1), 0, 0,
                                              static_cast<const uint64_t *>(hd), 0ull, hops, sink); });
        out->latency_us = ms > 0 ? ms * 1e3 / hops : 0;
    }
    if (hipGetLastError() != hipSuccess) st = EMOGI_E_HIP;
    out->buffer_bytes = bytes;
    cleanup();
    if (st != EMOGI_OK) set_error("a calibration kernel failed");
    return st;
}

}  // extern "C"
