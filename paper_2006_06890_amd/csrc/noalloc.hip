// BFS for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the frontier
// queues, visited bitmap and level counters live in one file-scope device
// array instead of the graph's lazily allocated pool.
//
// Host code must not pass `scratch` itself to a kernel or a copy: in host code
// the name stands for a host-side shadow, not a device address.  Its device
// address is looked up once per device with hipGetSymbolAddress (each GPU
// holds its own copy of the array) and only that address is used.
#include "internal.h"

#include <mutex>

namespace emogi {
uint64_t bfs_scratch_bytes(uint64_t V);
emogi_status_t bfs_in_scratch(emogi_graph_s *g, uint64_t src, uint32_t *out, void *scratch, uint64_t bytes,
                              hipStream_t stream);
}  // namespace emogi

using namespace emogi;

// Sized for graphs of up to 2^22 vertices: two queues of 2^22 ids (16 MiB
// each), the 512 KiB visited bitmap and the level counters.
constexpr uint64_t kMaxVertices = uint64_t(1) << 22;
constexpr uint64_t kScratchBytes = 34ull << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// Device address of this device's scratch array (looked up on first use).
emogi_status_t scratch_on(int dev, void **ptr) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the scratch table covers", dev, kMaxDevices);
        return EMOGI_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the BFS scratch array failed: %s", hipGetErrorString(e));
            return EMOGI_E_HIP;
        }
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    return EMOGI_OK;
}

}  // namespace

extern "C" {

emogi_status_t emogi_bfs_noalloc(emogi_graph_t g, uint64_t src, uint32_t *levels, void *stream) {
    if (!g || !levels) {
        set_error("null graph or output");
        return EMOGI_E_INVALID;
    }
    if (g->V > kMaxVertices || bfs_scratch_bytes(g->V) > kScratchBytes) {
        set_error("emogi_bfs_noalloc handles at most %llu vertices; this graph has %llu",
                  (unsigned long long)kMaxVertices, (unsigned long long)g->V);
        return EMOGI_E_INVALID;
    }
    int dev = -1;
    EMOGI_HIP_TRY(hipGetDevice(&dev), EMOGI_E_HIP);
    if (dev != g->device) {
        set_error("emogi_bfs_noalloc: device %d is current, the graph lives on device %d", dev, g->device);
        return EMOGI_E_INVALID;
    }
    void *ptr = nullptr;
    emogi_status_t st = scratch_on(dev, &ptr);
    if (st != EMOGI_OK) return st;
    return bfs_in_scratch(g, src, levels, ptr, kScratchBytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"
