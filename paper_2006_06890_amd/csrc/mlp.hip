// Training kernels of the per-level variant scheduler (16 -> 64 -> 64 -> 6,
// ReLU, softmax cross-entropy, Adam), fp32 on the vector ALUs.
//
// Parameters are one flat vector in the order W1[64][16], b1[64], W2[64][64],
// b2[64], W3[6][64], b3[6] (row-major): the layout the inference kernel in
// sched.hip reads.  Batch sums run in a fixed order (one thread per
// parameter walks the batch), so gradients are deterministic.  The network is
// ~11 kFLOP per sample: nothing here is worth a matrix-core tile.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace emogi {

constexpr int kIn = 16, kH = 64, kOut = 6;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;
static_assert(kParams == 5638, "parameter count");

// One 64-thread block per sample: pre-activations A1, A2 and logits Z.
__global__ __launch_bounds__(64) void k_mlp_fwd(const float *__restrict__ p, const float *__restrict__ X,
                                                uint32_t B, float *A1, float *A2, float *Z) {
    __shared__ float x[kIn], h1[kH], h2[kH];
    const uint32_t b = blockIdx.x;
    const int t = threadIdx.x;
    if (b >= B) return;
    if (t < kIn) x[t] = X[uint64_t(b) * kIn + t];
    __syncthreads();
    float a = p[oB1 + t];
    for (int k = 0; k < kIn; ++k) a += p[oW1 + t * kIn + k] * x[k];
    A1[uint64_t(b) * kH + t] = a;
    h1[t] = fmaxf(a, 0.f);
    __syncthreads();
    a = p[oB2 + t];
    for (int k = 0; k < kH; ++k) a += p[oW2 + t * kH + k] * h1[k];
    A2[uint64_t(b) * kH + t] = a;
    h2[t] = fmaxf(a, 0.f);
    __syncthreads();
    if (t < kOut) {
        a = p[oB3 + t];
        for (int k = 0; k < kH; ++k) a += p[oW3 + t * kH + k] * h2[k];
        Z[uint64_t(b) * kOut + t] = a;
    }
}

// dZ = (softmax(Z) - onehot(y)) / B ; per-sample loss = logsumexp(Z) - Z[y].
__global__ void k_mlp_xent(const float *Z, const int32_t *y, uint32_t B, float *dZ, float *loss_b) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float *z = Z + uint64_t(b) * kOut;
    float m = z[0];
    for (int k = 1; k < kOut; ++k) m = fmaxf(m, z[k]);
    float s = 0.f;
    for (int k = 0; k < kOut; ++k) s += expf(z[k] - m);
    const int yb = y[b];
    for (int k = 0; k < kOut; ++k) {
        const float pk = expf(z[k] - m) / s;
        dZ[uint64_t(b) * kOut + k] = (pk - (k == yb ? 1.f : 0.f)) / float(B);
    }
    loss_b[b] = (m + logf(s)) - z[yb];
}

// Mean of the per-sample losses in a fixed order (one block).
__global__ void k_mlp_mean(const float *loss_b, uint32_t B, float *loss) {
    __shared__ float part[256];
    float s = 0.f;
    for (uint32_t i = threadIdx.x; i < B; i += 256) s += loss_b[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int i = 0; i < 256; ++i) t += part[i];
        *loss = t / float(B);
    }
}

// Back through the hidden layers, one block per sample: dA2, dA1.
__global__ __launch_bounds__(64) void k_mlp_bwd_hidden(const float *__restrict__ p, const float *A1,
                                                       const float *A2, const float *dZ, uint32_t B,
                                                       float *dA1, float *dA2) {
    __shared__ float dz[kOut], da2[kH];
    const uint32_t b = blockIdx.x;
    const int t = threadIdx.x;
    if (b >= B) return;
    if (t < kOut) dz[t] = dZ[uint64_t(b) * kOut + t];
    __syncthreads();
    float g = 0.f;
    for (int k = 0; k < kOut; ++k) g += dz[k] * p[oW3 + k * kH + t];
    g = A2[uint64_t(b) * kH + t] > 0.f ? g : 0.f;
    dA2[uint64_t(b) * kH + t] = g;
    da2[t] = g;
    __syncthreads();
    g = 0.f;
    for (int k = 0; k < kH; ++k) g += da2[k] * p[oW2 + k * kH + t];
    dA1[uint64_t(b) * kH + t] = A1[uint64_t(b) * kH + t] > 0.f ? g : 0.f;
}

// One thread per parameter: its batch sum, in batch order.
__global__ void k_mlp_wgrad(const float *X, const float *A1, const float *A2, const float *dZ,
                            const float *dA1, const float *dA2, uint32_t B, float *grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    float s = 0.f;
    if (i < oB1) {
        const int j = (i - oW1) / kIn, k = (i - oW1) % kIn;
        for (uint32_t b = 0; b < B; ++b) s += dA1[uint64_t(b) * kH + j] * X[uint64_t(b) * kIn + k];
    } else if (i < oW2) {
        const int j = i - oB1;
        for (uint32_t b = 0; b < B; ++b) s += dA1[uint64_t(b) * kH + j];
    } else if (i < oB2) {
        const int j = (i - oW2) / kH, k = (i - oW2) % kH;
        for (uint32_t b = 0; b < B; ++b) s += dA2[uint64_t(b) * kH + j] * fmaxf(A1[uint64_t(b) * kH + k], 0.f);
    } else if (i < oW3) {
        const int j = i - oB2;
        for (uint32_t b = 0; b < B; ++b) s += dA2[uint64_t(b) * kH + j];
    } else if (i < oB3) {
        const int j = (i - oW3) / kH, k = (i - oW3) % kH;
        for (uint32_t b = 0; b < B; ++b) s += dZ[uint64_t(b) * kOut + j] * fmaxf(A2[uint64_t(b) * kH + k], 0.f);
    } else {
        const int j = i - oB3;
        for (uint32_t b = 0; b < B; ++b) s += dZ[uint64_t(b) * kOut + j];
    }
    grad[i] = s;
}

// Adam (Kingma & Ba 2015, Algorithm 1), step t >= 1.
__global__ void k_mlp_adam(float *p, const float *g, float *m, float *v, uint32_t t, float lr, float b1,
                           float b2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    const float mi = b1 * m[i] + (1.f - b1) * g[i];
    const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(b1, float(t))), vh = vi / (1.f - powf(b2, float(t)));
    p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Device scratch for a batch of B samples.
struct MlpScratch {
    float *A1 = nullptr, *A2 = nullptr, *Z = nullptr, *dZ = nullptr, *dA1 = nullptr, *dA2 = nullptr,
          *loss_b = nullptr;
    uint32_t cap = 0;
    void release() {
        for (float *q : {A1, A2, Z, dZ, dA1, dA2, loss_b})
            if (q) (void)hipFree(q);
        *this = MlpScratch();
    }
    bool ensure(uint32_t B) {
        if (B <= cap) return true;
        release();
        const size_t h = size_t(B) * kH * 4, o = size_t(B) * kOut * 4;
        if (hipMalloc(&A1, h) != hipSuccess || hipMalloc(&A2, h) != hipSuccess ||
            hipMalloc(&Z, o) != hipSuccess || hipMalloc(&dZ, o) != hipSuccess ||
            hipMalloc(&dA1, h) != hipSuccess || hipMalloc(&dA2, h) != hipSuccess ||
            hipMalloc(&loss_b, size_t(B) * 4) != hipSuccess) {
            (void)hipGetLastError();
            release();
            return false;
        }
        cap = B;
        return true;
    }
};

static emogi_status_t loss_grad(MlpScratch &sc, const float *p, const float *X, const int32_t *y,
                                uint32_t B, float *grad, float *loss, hipStream_t s) {
    if (!sc.ensure(B)) {
        set_error("scheduler training scratch allocation failed");
        return EMOGI_E_OOM_DEVICE;
    }
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, s, p, X, B, sc.A1, sc.A2, sc.Z);
    hipLaunchKernelGGL(k_mlp_xent, dim3((B + 255) / 256), dim3(256), 0, s, sc.Z, y, B, sc.dZ, sc.loss_b);
    if (loss) hipLaunchKernelGGL(k_mlp_mean, dim3(1), dim3(256), 0, s, sc.loss_b, B, loss);
    hipLaunchKernelGGL(k_mlp_bwd_hidden, dim3(B), dim3(64), 0, s, p, sc.A1, sc.A2, sc.dZ, B, sc.dA1, sc.dA2);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((kParams + 255) / 256), dim3(256), 0, s, X, sc.A1, sc.A2, sc.dZ,
                       sc.dA1, sc.dA2, B, grad);
    EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
    return EMOGI_OK;
}

}  // namespace emogi

using namespace emogi;

extern "C" {

emogi_status_t emogi_mlp_forward(const float *params, const float *X, uint32_t B, float *Z, void *stream) {
    if (!params || !X || !Z || B == 0) {
        set_error("emogi_mlp_forward: null argument or empty batch");
        return EMOGI_E_INVALID;
    }
    MlpScratch sc;
    if (!sc.ensure(B)) {
        set_error("scratch allocation failed");
        return EMOGI_E_OOM_DEVICE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, s, params, X, B, sc.A1, sc.A2, Z);
    hipError_t e = hipStreamSynchronize(s);
    sc.release();
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("forward kernel failed");
        return EMOGI_E_HIP;
    }
    return EMOGI_OK;
}

emogi_status_t emogi_mlp_loss_grad(const float *params, const float *X, const int32_t *y, uint32_t B,
                                   float *grad, float *loss, void *stream) {
    if (!params || !X || !y || !grad || B == 0) {
        set_error("emogi_mlp_loss_grad: null argument or empty batch");
        return EMOGI_E_INVALID;
    }
    MlpScratch sc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    emogi_status_t st = loss_grad(sc, params, X, y, B, grad, loss, s);
    hipError_t e = hipStreamSynchronize(s);
    sc.release();
    if (st != EMOGI_OK) return st;
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("gradient kernels failed");
        return EMOGI_E_HIP;
    }
    return EMOGI_OK;
}

emogi_status_t emogi_mlp_adam_step(float *params, const float *grad, float *m, float *v, uint32_t t,
                                   float lr, float beta1, float beta2, float eps, void *stream) {
    if (!params || !grad || !m || !v || t == 0) {
        set_error("emogi_mlp_adam_step: null argument or t == 0");
        return EMOGI_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, params, grad, m, v, t, lr,
                       beta1, beta2, eps);
    EMOGI_HIP_TRY(hipGetLastError(), EMOGI_E_HIP);
    return EMOGI_OK;
}

emogi_status_t emogi_mlp_train(const float *X, const int32_t *y, uint32_t N, const emogi_train_config_t *cfg,
                               float *params, float *loss_history) {
    if (!X || !y || !cfg || !params || N == 0 || cfg->batch == 0) {
        set_error("emogi_mlp_train: null argument or empty data");
        return EMOGI_E_INVALID;
    }
    for (uint32_t i = 0; i < N; ++i)
        if (y[i] < 0 || y[i] >= kOut) {
            set_error("label %d out of range", y[i]);
            return EMOGI_E_INVALID;
        }
    const uint32_t B = std::min(cfg->batch, N);
    float *dX = nullptr, *dP = nullptr, *dG = nullptr, *dM = nullptr, *dV = nullptr, *dLoss = nullptr;
    float *bX = nullptr;
    int32_t *dY = nullptr, *bY = nullptr;
    MlpScratch sc;
    hipStream_t s = nullptr;
    emogi_status_t st = EMOGI_OK;
    auto cleanup = [&]() {
        for (void *q : {(void *)dX, (void *)dP, (void *)dG, (void *)dM, (void *)dV, (void *)dLoss,
                        (void *)bX, (void *)dY, (void *)bY})
            if (q) (void)hipFree(q);
        sc.release();
        if (s) (void)hipStreamDestroy(s);
    };
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(&dX, size_t(N) * kIn * 4) != hipSuccess || hipMalloc(&dY, size_t(N) * 4) != hipSuccess ||
        hipMalloc(&bX, size_t(B) * kIn * 4) != hipSuccess || hipMalloc(&bY, size_t(B) * 4) != hipSuccess ||
        hipMalloc(&dP, kParams * 4) != hipSuccess || hipMalloc(&dG, kParams * 4) != hipSuccess ||
        hipMalloc(&dM, kParams * 4) != hipSuccess || hipMalloc(&dV, kParams * 4) != hipSuccess ||
        hipMalloc(&dLoss, 4) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("training allocation failed");
        return EMOGI_E_OOM_DEVICE;
    }
    std::vector<float> zero(kParams, 0.f);
    if (hipMemcpy(dX, X, size_t(N) * kIn * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dY, y, size_t(N) * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dP, params, kParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dM, zero.data(), kParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dV, zero.data(), kParams * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        set_error("training upload failed");
        return EMOGI_E_HIP;
    }
    // Seeded shuffle per epoch (SplitMix64 counter stream, Fisher-Yates on the host).
    std::vector<uint32_t> order(N);
    std::vector<float> hx(size_t(B) * kIn);
    std::vector<int32_t> hy(B);
    uint32_t t = 0;
    uint64_t ctr = 0;
    auto rnd = [&]() {
        uint64_t z = cfg->seed + (++ctr) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (uint32_t ep = 0; ep < cfg->epochs && st == EMOGI_OK; ++ep) {
        for (uint32_t i = 0; i < N; ++i) order[i] = i;
        for (uint32_t i = N - 1; i > 0; --i) std::swap(order[i], order[rnd() % (uint64_t(i) + 1)]);
        double ep_loss = 0.0;
        uint32_t nb = 0;
        for (uint32_t b0 = 0; b0 + B <= N && st == EMOGI_OK; b0 += B) {
            for (uint32_t k = 0; k < B; ++k) {
                memcpy(&hx[size_t(k) * kIn], X + size_t(order[b0 + k]) * kIn, kIn * 4);
                hy[k] = y[order[b0 + k]];
            }
            if (hipMemcpyAsync(bX, hx.data(), size_t(B) * kIn * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(bY, hy.data(), size_t(B) * 4, hipMemcpyHostToDevice, s) != hipSuccess) {
                st = EMOGI_E_HIP;
                break;
            }
            st = loss_grad(sc, dP, bX, bY, B, dG, dLoss, s);
            if (st != EMOGI_OK) break;
            ++t;
            hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, dP, dG, dM, dV, t,
                               cfg->lr, cfg->beta1, cfg->beta2, cfg->eps);
            float hl = 0.f;
            if (hipMemcpyAsync(&hl, dLoss, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                st = EMOGI_E_HIP;
                break;
            }
            ep_loss += hl;
            ++nb;
        }
        if (loss_history) loss_history[ep] = nb ? float(ep_loss / nb) : 0.f;
    }
    if (st == EMOGI_OK && hipMemcpy(params, dP, kParams * 4, hipMemcpyDeviceToHost) != hipSuccess)
        st = EMOGI_E_HIP;
    if (st == EMOGI_E_HIP) {
        (void)hipGetLastError();
        set_error("training step failed");
    }
    cleanup();
    return st;
}

}  // extern "C"
