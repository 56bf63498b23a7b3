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
//     Sec. 3.3, turns it into the outstanding requests needed), and the
//     rate against the number of waves in flight, each with one R-byte
//     block outstanding, whose knee that law predicts;
//   * R-byte blocks started at offsets 0..R past a request boundary;
//   * coherent against non-coherent pinning;
//   * the GPU-memory read and copy rates, the bound of the vertex state.
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

// Little's-law sweep: each wave reads `per_wave` random aligned B-byte
// blocks, one at a time: the next block's address depends on a word of the
// previous block (always 0 here: the words read are below 2^31, but the
// compiler cannot know), so a wave never has two blocks in flight and the
// launch's waves are the outstanding requests.
__global__ __launch_bounds__(256) void k_wave_read(const uint8_t *__restrict__ src, uint64_t nslots, uint32_t B,
                                                   uint32_t per_wave, uint64_t seed, unsigned long long *sink) {
    const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x & 63;
    unsigned long long acc = 0;
    uint64_t dep = 0;
    const uint32_t lanes_needed = B / 4;
#pragma unroll 1
    for (uint32_t k = 0; k < per_wave; ++k) {
        uint64_t z = seed + (wave * per_wave + k + 1) * 0x9E3779B97F4A7C15ull + dep;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const uint64_t base = (z % nslots) * B;
        uint32_t first = 0;
        for (uint32_t l = lane; l < lanes_needed; l += 64) {
            const uint32_t x = *reinterpret_cast<const uint32_t *>(src + base + 4ull * l);
            acc += x;
            if (l == uint32_t(lane)) first = x;
        }
        dep = uint64_t(__shfl(int(first), 0)) >> 31;
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
    void *h = nullptr, *d = nullptr, *hn = nullptr, *d2 = nullptr;
    unsigned long long *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    emogi_status_t st = EMOGI_OK;
    auto cleanup = [&]() {
        if (h) (void)hipHostFree(h);
        if (hn) (void)hipHostFree(hn);
        if (d) (void)hipFree(d);
        if (d2) (void)hipFree(d2);
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
    // the non-coherent arm is measured when its buffer can be had (fields stay 0 otherwise)
    if (hipHostMalloc(&hn, bytes, hipHostMallocMapped | hipHostMallocNonCoherent) != hipSuccess) {
        (void)hipGetLastError();
        hn = nullptr;
    }
    if (hipMalloc(&d, bytes) != hipSuccess || hipMalloc(&d2, bytes) != hipSuccess ||
        hipMalloc(&sink, 64) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("device allocation for calibration failed");
        return EMOGI_E_OOM_DEVICE;
    }
    void *hd = nullptr, *hnd = nullptr;
    if (hipHostGetDevicePointer(&hd, h, 0) != hipSuccess ||
        (hn && hipHostGetDevicePointer(&hnd, hn, 0) != hipSuccess)) {
        (void)hipGetLastError();
        cleanup();
        set_error("hipHostGetDevicePointer failed");
        return EMOGI_E_HIP;
    }
    // Pointer-chase ring: slot k (one per 64 KiB, so every hop is a new page)
    // links to slot (k + step) mod n with gcd(step, n) = 1, one cycle over all n.
    memset(h, 0, bytes);
    if (hn) memset(hn, 0, bytes);
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
    const uint32_t R = out->request_unit;
    // 3b. waves in flight (Little's law): random aligned R-byte blocks, one
    // in flight per wave, 16 .. 8192 waves (all resident at once)
    {
        const uint64_t nslots = (bytes - R - 64) / R;
        double best = 0;
        for (int i = 0; i < EMOGI_CALIB_WAVES; ++i) {
            const uint32_t W = 16u << i;
            const uint32_t per_wave = uint32_t(std::max<uint64_t>(4, (uint64_t(64) << 20) / (uint64_t(W) * R)));
            ms = time_ms([&] {
                hipLaunchKernelGGL(k_wave_read, dim3(W / 4), dim3(256), 0, 0, src, nslots, R, per_wave,
                                   uint64_t(777 + i), sink);
            });
            out->waves[i] = W;
            out->waves_GBps[i] = ms > 0 ? double(W) * per_wave * R / (ms * 1e6) : 0;
            best = std::max(best, out->waves_GBps[i]);
        }
        for (int i = 0; i < EMOGI_CALIB_WAVES; ++i)
            if (out->waves_GBps[i] >= 0.9 * best) {
                out->knee_waves = out->waves[i];
                break;
            }
    }
    // 3c. R-byte blocks starting `off` past an R boundary (off = 0 .. R)
    {
        const uint32_t step = std::max(16u, R / 16);
        const uint64_t nslots = (bytes - 2ull * R - 64) / R;  // slot*R + off + R stays inside the buffer
        const uint32_t per_wave = std::max(1u, 16384u / R);
        for (int k = 0; k < EMOGI_CALIB_OFFSETS; ++k) {
            const uint32_t off = std::min(R, k * step);
            ms = time_ms([&] {
                hipLaunchKernelGGL(k_rand_read, dim3(4096), dim3(256), 0, 0, src, nslots, R, R, off, per_wave,
                                   uint64_t(4321 + k), sink);
            });
            out->offset_bytes[k] = off;
            out->offset_GBps[k] = ms > 0 ? 4096.0 * 4 * per_wave * R / (ms * 1e6) : 0;
        }
    }
    // 3d. the same reads from a non-coherent pinned buffer, and the coherent
    // one again with the same launch for a side-by-side pair
    if (hn) {
        const uint8_t *nsrc = static_cast<const uint8_t *>(hnd);
        ms = time_ms([&] { (void)hipMemcpyAsync(d, hn, bytes, hipMemcpyHostToDevice, 0); });
        out->nc_memcpy_GBps = ms > 0 ? bytes / (ms * 1e6) : 0;
        const uint64_t chunks = bytes / (64ull * 16);
        ms = time_ms([&] { hipLaunchKernelGGL(k_seq_read<16>, dim3(8192), dim3(256), 0, 0, nsrc, chunks, sink); });
        out->nc_seq_read_GBps = ms > 0 ? chunks * 64.0 * 16 / (ms * 1e6) : 0;
        const uint64_t nslots = (bytes - R - 64) / R;
        const uint32_t per_wave = std::max(1u, 16384u / R);
        for (int c = 0; c < 2; ++c) {
            const uint8_t *p = c ? src : nsrc;
            ms = time_ms([&] {
                hipLaunchKernelGGL(k_rand_read, dim3(4096), dim3(256), 0, 0, p, nslots, R, R, 0u, per_wave,
                                   uint64_t(99), sink);
            });
            (c ? out->coh_rand_GBps : out->nc_rand_GBps) = ms > 0 ? 4096.0 * 4 * per_wave * R / (ms * 1e6) : 0;
        }
    }
    // 3e. GPU memory: wave-merged read of a device buffer, device-to-device copy
    {
        (void)hipMemsetAsync(d, 1, bytes, 0);
        const uint64_t chunks = bytes / (64ull * 16);
        const uint8_t *dsrc = static_cast<const uint8_t *>(d);
        ms = time_ms([&] { hipLaunchKernelGGL(k_seq_read<16>, dim3(8192), dim3(256), 0, 0, dsrc, chunks, sink); });
        out->hbm_read_GBps = ms > 0 ? chunks * 64.0 * 16 / (ms * 1e6) : 0;
        ms = time_ms([&] { (void)hipMemcpyAsync(d2, d, bytes, hipMemcpyDeviceToDevice, 0); });
        out->hbm_copy_GBps = ms > 0 ? 2.0 * bytes / (ms * 1e6) : 0;
    }
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
