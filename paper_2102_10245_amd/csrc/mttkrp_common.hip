// Host helpers and small kernels shared by the MTTKRP launchers: the
// reduction of per-XCD output replicas and the XCC id probe.
#include <mutex>
#include <vector>

#include "mttkrp_impl.h"

namespace alto {

namespace {

__global__ __launch_bounds__(256) void replica_reduce4_k(float4 *__restrict__ out, const float4 *__restrict__ rep,
                                                         uint64_t stride4, int nrep, uint64_t n4) {
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (uint64_t)gridDim.x * 256) {
        float4 s = out[e];
        for (int x = 0; x < nrep; x++) {
            const float4 r = rep[(uint64_t)x * stride4 + e];
            s.x += r.x;
            s.y += r.y;
            s.z += r.z;
            s.w += r.w;
        }
        out[e] = s;
    }
}

__global__ __launch_bounds__(256) void replica_reduce1_k(float *__restrict__ out, const float *__restrict__ rep,
                                                         uint64_t stride, int nrep, uint64_t n) {
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (uint64_t)gridDim.x * 256) {
        float s = out[e];
        for (int x = 0; x < nrep; x++) s += rep[(uint64_t)x * stride + e];
        out[e] = s;
    }
}

__global__ __launch_bounds__(64) void xcc_probe_k(uint32_t *ids) {
    if (threadIdx.x == 0) ids[blockIdx.x] = xcc_id();
}

std::mutex g_mu;
std::vector<int> g_xcc;  // per device, -1 = not probed

}  // namespace

int launch_replica_reduce(float *out, const float *rep, uint64_t stride, int nrep, uint64_t n, hipStream_t s) {
    if (n == 0 || nrep == 0) return ALTO_OK;
    const bool v4 = (n % 4 == 0) && (stride % 4 == 0) && (((uintptr_t)out | (uintptr_t)rep) % 16 == 0);
    const uint64_t work = v4 ? n / 4 : n;
    const unsigned grid = (unsigned)std::min<uint64_t>(4096, (work + 255) / 256);
    if (v4)
        replica_reduce4_k<<<grid, 256, 0, s>>>((float4 *)out, (const float4 *)rep, stride / 4, nrep, n / 4);
    else
        replica_reduce1_k<<<grid, 256, 0, s>>>(out, rep, stride, nrep, n);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int device_xcc_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_xcc.size() <= dev) g_xcc.resize(dev + 1, -1);
    if (g_xcc[dev] >= 0) return g_xcc[dev];
    g_xcc[dev] = 0;
    constexpr int kBlocks = 4096;
    uint32_t *d = nullptr;
    if (hipMalloc(&d, sizeof(uint32_t) * kBlocks) != hipSuccess) return 0;
    std::vector<uint32_t> h(kBlocks, 0);
    xcc_probe_k<<<kBlocks, 64, 0, 0>>>(d);
    if (hipGetLastError() == hipSuccess &&
        hipMemcpy(h.data(), d, sizeof(uint32_t) * kBlocks, hipMemcpyDeviceToHost) == hipSuccess) {
        uint32_t mx = 0;
        for (uint32_t v : h) mx = v > mx ? v : mx;
        g_xcc[dev] = mx < (uint32_t)kMaxReplicas ? (int)mx + 1 : 0;
    }
    (void)hipFree(d);
    return g_xcc[dev];
}

}  // namespace alto
