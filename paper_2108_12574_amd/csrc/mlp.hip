// Skeleton-rank predictor: a 3-layer MLP (width 64) from box features to
// log2(k + 1), k the rank the pivoted QR of the box's ID will find.  Weights are
// used rounded to bfloat16 (nearest, ties to even); activations and sums are
// FP32.  Training: mean-squared-error gradient by backpropagation (the weight
// gradient is taken at the rounded weights and applied to the FP32 master
// weights) and Adam.  All reductions over samples run in a fixed order.
#include <cstdint>
#include <mutex>

#include "internal.h"

namespace cbd {

constexpr int kF = kMlpFeatures, kH = kMlpWidth;
constexpr int oW1 = 0, ob1 = kH * kF, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kH;
constexpr int kMlpThreads = 256;

__device__ __forceinline__ float bf16_round(float w) {
    uint32_t u = __float_as_uint(w);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    return __uint_as_float(u);
}

// Rounded weights and biases staged in LDS.
struct MlpLds {
    float W1[kH * kF], b1[kH], W2[kH * kH], b2[kH], W3[kH], b3;
};

__device__ void stage_params(const float* __restrict__ p, MlpLds& s) {
    for (int e = threadIdx.x; e < kH * kF; e += blockDim.x) s.W1[e] = bf16_round(p[oW1 + e]);
    for (int e = threadIdx.x; e < kH * kH; e += blockDim.x) s.W2[e] = bf16_round(p[oW2 + e]);
    for (int e = threadIdx.x; e < kH; e += blockDim.x) {
        s.b1[e] = p[ob1 + e];
        s.b2[e] = p[ob2 + e];
        s.W3[e] = bf16_round(p[oW3 + e]);
    }
    if (threadIdx.x == 0) s.b3 = p[ob3];
    __syncthreads();
}

// One thread per sample; z1, z2 (n x kH each) are kept for the backward pass when act != NULL.
__global__ __launch_bounds__(kMlpThreads) void k_mlp_forward(const float* __restrict__ p, int n,
                                                             const float* __restrict__ X,
                                                             float* __restrict__ y, float* __restrict__ z1o,
                                                             float* __restrict__ z2o) {
    __shared__ MlpLds s;
    stage_params(p, s);
    const int i = blockIdx.x * kMlpThreads + threadIdx.x;
    if (i >= n) return;
    float x[kF];
#pragma unroll
    for (int f = 0; f < kF; ++f) x[f] = X[(long)i * kF + f];
    float h1[kH];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        float z = s.b1[o];
#pragma unroll
        for (int f = 0; f < kF; ++f) z = fmaf(s.W1[o * kF + f], x[f], z);
        if (z1o) z1o[(long)i * kH + o] = z;
        h1[o] = z > 0.f ? z : 0.f;
    }
    float out = s.b3;
    for (int o = 0; o < kH; ++o) {
        float z = s.b2[o];
#pragma unroll
        for (int c = 0; c < kH; ++c) z = fmaf(s.W2[o * kH + c], h1[c], z);
        if (z2o) z2o[(long)i * kH + o] = z;
        out = fmaf(s.W3[o], z > 0.f ? z : 0.f, out);
    }
    y[i] = out;
}

// Per-sample deltas: dy = 2 (y - t)/n, dz2 = dy W3 * [z2 > 0], dz1 = (W2^T dz2) * [z1 > 0].
__global__ __launch_bounds__(kMlpThreads) void k_mlp_deltas(const float* __restrict__ p, int n,
                                                            const float* __restrict__ y,
                                                            const float* __restrict__ t,
                                                            const float* __restrict__ z1,
                                                            const float* __restrict__ z2,
                                                            float* __restrict__ dy, float* __restrict__ dz1,
                                                            float* __restrict__ dz2) {
    __shared__ MlpLds s;
    stage_params(p, s);
    const int i = blockIdx.x * kMlpThreads + threadIdx.x;
    if (i >= n) return;
    const float g = 2.f * (y[i] - t[i]) / (float)n;
    dy[i] = g;
    float d2[kH];
#pragma unroll
    for (int o = 0; o < kH; ++o) {
        d2[o] = z2[(long)i * kH + o] > 0.f ? g * s.W3[o] : 0.f;
        dz2[(long)i * kH + o] = d2[o];
    }
    for (int c = 0; c < kH; ++c) {
        float a = 0.f;
#pragma unroll
        for (int o = 0; o < kH; ++o) a = fmaf(s.W2[o * kH + c], d2[o], a);
        dz1[(long)i * kH + c] = z1[(long)i * kH + c] > 0.f ? a : 0.f;
    }
}

__device__ __forceinline__ float block_sum_f(float v, float* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float r = 0.f;
    for (int w = 0; w < kMlpThreads / 64; ++w) r += red[w];
    return r;
}

// Weight gradients, summed over samples in a fixed order.  Block o < kH: row o of
// W1 and W2 (and b1[o], b2[o]); block kH: W3, b3 and the loss.
__global__ __launch_bounds__(kMlpThreads) void k_mlp_grads(int n, const float* __restrict__ X,
                                                           const float* __restrict__ y,
                                                           const float* __restrict__ t,
                                                           const float* __restrict__ z1,
                                                           const float* __restrict__ z2,
                                                           const float* __restrict__ dy,
                                                           const float* __restrict__ dz1,
                                                           const float* __restrict__ dz2,
                                                           float* __restrict__ grad, float* __restrict__ loss) {
    __shared__ float red[kMlpThreads / 64];
    const int o = blockIdx.x;
    if (o < kH) {
        float a2[kH], a1[kF], bb1 = 0.f, bb2 = 0.f;
#pragma unroll
        for (int c = 0; c < kH; ++c) a2[c] = 0.f;
#pragma unroll
        for (int f = 0; f < kF; ++f) a1[f] = 0.f;
        for (int i = threadIdx.x; i < n; i += kMlpThreads) {
            const float d2 = dz2[(long)i * kH + o], d1 = dz1[(long)i * kH + o];
            bb2 += d2;
            bb1 += d1;
#pragma unroll
            for (int c = 0; c < kH; ++c) {
                const float h = z1[(long)i * kH + c];
                a2[c] = fmaf(d2, h > 0.f ? h : 0.f, a2[c]);
            }
#pragma unroll
            for (int f = 0; f < kF; ++f) a1[f] = fmaf(d1, X[(long)i * kF + f], a1[f]);
        }
        for (int c = 0; c < kH; ++c) {
            const float r = block_sum_f(a2[c], red);
            if (threadIdx.x == 0) grad[oW2 + o * kH + c] = r;
        }
        for (int f = 0; f < kF; ++f) {
            const float r = block_sum_f(a1[f], red);
            if (threadIdx.x == 0) grad[oW1 + o * kF + f] = r;
        }
        const float r1 = block_sum_f(bb1, red);
        const float r2 = block_sum_f(bb2, red);
        if (threadIdx.x == 0) {
            grad[ob1 + o] = r1;
            grad[ob2 + o] = r2;
        }
    } else {
        float a3[kH], bb3 = 0.f, ls = 0.f;
#pragma unroll
        for (int c = 0; c < kH; ++c) a3[c] = 0.f;
        for (int i = threadIdx.x; i < n; i += kMlpThreads) {
            const float g = dy[i];
            bb3 += g;
            const float r = y[i] - t[i];
            ls = fmaf(r, r, ls);
#pragma unroll
            for (int c = 0; c < kH; ++c) {
                const float h = z2[(long)i * kH + c];
                a3[c] = fmaf(g, h > 0.f ? h : 0.f, a3[c]);
            }
        }
        for (int c = 0; c < kH; ++c) {
            const float r = block_sum_f(a3[c], red);
            if (threadIdx.x == 0) grad[oW3 + c] = r;
        }
        const float r3 = block_sum_f(bb3, red);
        const float rl = block_sum_f(ls, red);
        if (threadIdx.x == 0) {
            grad[ob3] = r3;
            if (loss) loss[0] = rl / (float)n;
        }
    }
}

__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int np, float lr, float c1, float c2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < np; e += gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.f - b1) * ge;
        const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
    }
}

void launch_mlp_forward(const float* p, int n, const float* X, float* y, float* z1, float* z2,
                        hipStream_t s) {
    if (n <= 0) return;
    CBD_LAUNCH(k_mlp_forward, dim3((n + kMlpThreads - 1) / kMlpThreads), dim3(kMlpThreads), 0, s, p,
                       n, X, y, z1, z2);
}

void launch_mlp_loss_grad(const float* p, int n, const float* X, const float* t, float* grad, float* loss,
                          float* ws, hipStream_t s) {
    float* y = ws;
    float* dy = y + n;
    float* z1 = dy + n;
    float* z2 = z1 + (long)n * kH;
    float* dz1 = z2 + (long)n * kH;
    float* dz2 = dz1 + (long)n * kH;
    const int blocks = (n + kMlpThreads - 1) / kMlpThreads;
    CBD_LAUNCH(k_mlp_forward, dim3(blocks), dim3(kMlpThreads), 0, s, p, n, X, y, z1, z2);
    CBD_LAUNCH(k_mlp_deltas, dim3(blocks), dim3(kMlpThreads), 0, s, p, n, y, t, z1, z2, dy, dz1, dz2);
    CBD_LAUNCH(k_mlp_grads, dim3(kH + 1), dim3(kMlpThreads), 0, s, n, X, y, t, z1, z2, dy, dz1, dz2,
                       grad, loss);
}

// Library-owned scratch of the loss/gradient for callers that cannot allocate device
// memory: (2 + 4 kH) floats per sample for up to kMlpStaticMax samples, one copy per
// device, held until the process ends.  Host code never passes the array's name to a
// kernel: it uses the device address that hipGetSymbolAddress returns, once per
// device with that device current.
__device__ __align__(256) float scratch[(size_t)(2 + 4 * kH) * kMlpStaticMax];

float* mlp_static_scratch() {
    static std::mutex mx;
    static float* addr[64] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mx);
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        addr[dev] = (float*)p;
    }
    return addr[dev];
}

void launch_mlp_adam(float* p, const float* g, float* m, float* v, int step, float lr, hipStream_t s) {
    const float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
    CBD_LAUNCH(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, p, g, m, v, kMlpParams,
                       lr, c1, c2);
}

}  // namespace cbd
