// Selector network on the GPU: forward, backward (chain rule) and Adam for
// a perceptron with two hidden ReLU layers,
//   y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,
//   loss = sum(mask * (y - t)^2) / sum(mask).
// Parameters are packed {W1[H*F], b1[H], W2[H*H], b2[H], W3[K*H], b3[K]}.
// One 64-lane wave per sample; per-parameter gradients are sums over the
// batch in sample order (deterministic).
#include <algorithm>
#include <mutex>

#include "common.h"

namespace alto {
namespace {

constexpr int kT = 256;
constexpr int kMaxH = 256;

struct Packing {
    int64_t W1, b1, W2, b2, W3, b3, total;
};

Packing pack(int F, int H, int K) {
    Packing p;
    p.W1 = 0;
    p.b1 = p.W1 + (int64_t)H * F;
    p.W2 = p.b1 + H;
    p.b2 = p.W2 + (int64_t)H * H;
    p.W3 = p.b2 + H;
    p.b3 = p.W3 + (int64_t)K * H;
    p.total = p.b3 + K;
    return p;
}

__global__ __launch_bounds__(kT) void fwd_k(int B, int F, int H, int K, const float *__restrict__ prm, Packing pk,
                                            const float *__restrict__ x, float *__restrict__ h1,
                                            float *__restrict__ h2, float *__restrict__ y) {
    __shared__ float s1[kT / 64][kMaxH];
    __shared__ float s2[kT / 64][kMaxH];
    const int w = threadIdx.x / 64, lane = __lane_id();
    const int b = blockIdx.x * (kT / 64) + w;
    const bool live = b < B;
    const float *xb = x + (int64_t)(live ? b : 0) * F;
    for (int j = lane; live && j < H; j += 64) {
        float a = prm[pk.b1 + j];
        for (int f = 0; f < F; f++) a += prm[pk.W1 + (int64_t)j * F + f] * xb[f];
        a = a > 0.f ? a : 0.f;
        s1[w][j] = a;
        h1[(int64_t)b * H + j] = a;
    }
    __syncthreads();
    for (int j = lane; live && j < H; j += 64) {
        float a = prm[pk.b2 + j];
        for (int q = 0; q < H; q++) a += prm[pk.W2 + (int64_t)j * H + q] * s1[w][q];
        a = a > 0.f ? a : 0.f;
        s2[w][j] = a;
        h2[(int64_t)b * H + j] = a;
    }
    __syncthreads();
    for (int k = lane; live && k < K; k += 64) {
        float a = prm[pk.b3 + k];
        for (int q = 0; q < H; q++) a += prm[pk.W3 + (int64_t)k * H + q] * s2[w][q];
        y[(int64_t)b * K + k] = a;
    }
}

// stats[0] = sum(mask), stats[1] = sum(mask*(y-t)^2); loss = stats[1]/stats[0]
__global__ __launch_bounds__(kT) void loss_k(int64_t n, const float *__restrict__ y, const float *__restrict__ t,
                                             const float *__restrict__ mask, float *__restrict__ stats,
                                             float *__restrict__ loss) {
    __shared__ float r0[kT / 64], r1[kT / 64];
    float c = 0.f, l = 0.f;
    for (int64_t e = threadIdx.x; e < n; e += kT) {
        const float m = mask[e], d = y[e] - t[e];
        c += m;
        l += m * d * d;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        c += __shfl_xor(c, off);
        l += __shfl_xor(l, off);
    }
    if (__lane_id() == 0) {
        r0[threadIdx.x / 64] = c;
        r1[threadIdx.x / 64] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.f, z = 0.f;
        for (int q = 0; q < kT / 64; q++) {
            a += r0[q];
            z += r1[q];
        }
        stats[0] = a;
        stats[1] = z;
        if (loss) *loss = a > 0.f ? z / a : 0.f;
    }
}

__global__ __launch_bounds__(kT) void delta_k(int B, int H, int K, const float *__restrict__ prm, Packing pk,
                                              const float *__restrict__ y, const float *__restrict__ t,
                                              const float *__restrict__ mask, const float *__restrict__ stats,
                                              const float *__restrict__ h1, const float *__restrict__ h2,
                                              float *__restrict__ dy, float *__restrict__ d2, float *__restrict__ d1) {
    __shared__ float sdy[kT / 64][64];
    __shared__ float sd2[kT / 64][kMaxH];
    const int w = threadIdx.x / 64, lane = __lane_id();
    const int b = blockIdx.x * (kT / 64) + w;
    const bool live = b < B;
    const float cnt = stats[0];
    for (int k = lane; live && k < K; k += 64) {
        const int64_t e = (int64_t)b * K + k;
        const float g = cnt > 0.f ? 2.f * mask[e] * (y[e] - t[e]) / cnt : 0.f;
        dy[e] = g;
        sdy[w][k] = g;
    }
    __syncthreads();
    for (int q = lane; live && q < H; q += 64) {
        float g = 0.f;
        for (int k = 0; k < K; k++) g += prm[pk.W3 + (int64_t)k * H + q] * sdy[w][k];
        g = h2[(int64_t)b * H + q] > 0.f ? g : 0.f;
        d2[(int64_t)b * H + q] = g;
        sd2[w][q] = g;
    }
    __syncthreads();
    for (int q = lane; live && q < H; q += 64) {
        float g = 0.f;
        for (int j = 0; j < H; j++) g += prm[pk.W2 + (int64_t)j * H + q] * sd2[w][j];
        d1[(int64_t)b * H + q] = h1[(int64_t)b * H + q] > 0.f ? g : 0.f;
    }
}

// One thread per parameter: sum over samples in order.
__global__ __launch_bounds__(kT) void wgrad_k(int B, int F, int H, int K, Packing pk, const float *__restrict__ x,
                                              const float *__restrict__ h1, const float *__restrict__ h2,
                                              const float *__restrict__ dy, const float *__restrict__ d2,
                                              const float *__restrict__ d1, float *__restrict__ g) {
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= pk.total) return;
    float s = 0.f;
    if (p < pk.b1) {
        const int64_t j = p / F, f = p % F;
        for (int b = 0; b < B; b++) s += d1[(int64_t)b * H + j] * x[(int64_t)b * F + f];
    } else if (p < pk.W2) {
        const int64_t j = p - pk.b1;
        for (int b = 0; b < B; b++) s += d1[(int64_t)b * H + j];
    } else if (p < pk.b2) {
        const int64_t j = (p - pk.W2) / H, q = (p - pk.W2) % H;
        for (int b = 0; b < B; b++) s += d2[(int64_t)b * H + j] * h1[(int64_t)b * H + q];
    } else if (p < pk.W3) {
        const int64_t j = p - pk.b2;
        for (int b = 0; b < B; b++) s += d2[(int64_t)b * H + j];
    } else if (p < pk.b3) {
        const int64_t k = (p - pk.W3) / H, q = (p - pk.W3) % H;
        for (int b = 0; b < B; b++) s += dy[(int64_t)b * K + k] * h2[(int64_t)b * H + q];
    } else {
        const int64_t k = p - pk.b3;
        for (int b = 0; b < B; b++) s += dy[(int64_t)b * K + k];
    }
    g[p] = s;
}

__global__ __launch_bounds__(kT) void adam_k(int64_t P, float *__restrict__ w, const float *__restrict__ g,
                                             float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                             float b2, float eps, float c1, float c2) {
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// per-process scratch for activations and deltas (grown on demand)
std::mutex g_mu;
float *g_ws = nullptr;
size_t g_ws_bytes = 0;

int scratch(size_t bytes, float **out) {
    if (g_ws_bytes < bytes) {
        if (g_ws) ALTO_HIP(hipFree(g_ws));
        g_ws = nullptr;
        g_ws_bytes = 0;
        ALTO_HIP(hipMalloc(&g_ws, bytes));
        g_ws_bytes = bytes;
    }
    *out = g_ws;
    return ALTO_OK;
}

int check(int B, int F, int H, int K, const void *params, const void *x) {
    if (B < 1 || F < 1 || H < 1 || K < 1 || H > kMaxH || K > 64)
        return set_error(ALTO_E_INVAL, "MLP sizes: B, F >= 1, 1 <= H <= 256, 1 <= K <= 64");
    if (!params || !x) return set_error(ALTO_E_INVAL, "null parameter or input");
    return ALTO_OK;
}

}  // namespace

int mlp_forward(int B, int F, int H, int K, const float *params, const float *x, const float *t, const float *mask,
                float *y, float *loss, hipStream_t s) {
    int rc = check(B, F, H, K, params, x);
    if (rc) return rc;
    if (!y) return set_error(ALTO_E_INVAL, "null output");
    if (loss && (!t || !mask)) return set_error(ALTO_E_INVAL, "loss needs targets and mask");
    std::lock_guard<std::mutex> lk(g_mu);
    float *ws;
    rc = scratch(sizeof(float) * ((size_t)2 * B * H + 2), &ws);
    if (rc) return rc;
    const Packing pk = pack(F, H, K);
    const unsigned grid = (unsigned)((B + kT / 64 - 1) / (kT / 64));
    fwd_k<<<grid, kT, 0, s>>>(B, F, H, K, params, pk, x, ws, ws + (size_t)B * H, y);
    if (loss) loss_k<<<1, kT, 0, s>>>((int64_t)B * K, y, t, mask, ws + (size_t)2 * B * H, loss);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int mlp_backward(int B, int F, int H, int K, const float *params, const float *x, const float *t, const float *mask,
                 float *grads, float *loss, hipStream_t s) {
    int rc = check(B, F, H, K, params, x);
    if (rc) return rc;
    if (!t || !mask || !grads) return set_error(ALTO_E_INVAL, "null targets, mask or gradient buffer");
    std::lock_guard<std::mutex> lk(g_mu);
    float *ws;
    const size_t BH = (size_t)B * H, BK = (size_t)B * K;
    rc = scratch(sizeof(float) * (4 * BH + 2 * BK + 2), &ws);
    if (rc) return rc;
    float *h1 = ws, *h2 = h1 + BH, *d2 = h2 + BH, *d1 = d2 + BH, *y = d1 + BH, *dy = y + BK, *stats = dy + BK;
    const Packing pk = pack(F, H, K);
    const unsigned grid = (unsigned)((B + kT / 64 - 1) / (kT / 64));
    fwd_k<<<grid, kT, 0, s>>>(B, F, H, K, params, pk, x, h1, h2, y);
    loss_k<<<1, kT, 0, s>>>((int64_t)BK, y, t, mask, stats, loss);
    delta_k<<<grid, kT, 0, s>>>(B, H, K, params, pk, y, t, mask, stats, h1, h2, dy, d2, d1);
    wgrad_k<<<(unsigned)((pk.total + kT - 1) / kT), kT, 0, s>>>(B, F, H, K, pk, x, h1, h2, dy, d2, d1, grads);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int mlp_adam(int64_t P, float *params, const float *grads, float *m, float *v, float lr, float b1, float b2, float eps,
             int t, hipStream_t s) {
    if (P < 1 || !params || !grads || !m || !v || t < 1) return set_error(ALTO_E_INVAL, "bad Adam arguments");
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    adam_k<<<(unsigned)((P + kT - 1) / kT), kT, 0, s>>>(P, params, grads, m, v, lr, b1, b2, eps, c1, c2);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

}  // namespace alto
