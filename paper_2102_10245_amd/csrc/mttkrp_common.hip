// Host helpers and small kernels shared by the MTTKRP launchers: adding the
// FP64 accumulator(s) of the atomic updates into the FP32 output, and the
// XCC id probe.
#include <mutex>
#include <vector>

#include "mttkrp_impl.h"

namespace alto {

namespace {

__global__ __launch_bounds__(256) void acc64_finish_k(float *__restrict__ out, const double *__restrict__ acc,
                                                      uint64_t stride, int nacc, uint64_t n) {
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (uint64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int x = 0; x < nacc; x++) s += acc[(uint64_t)x * stride + e];
        out[e] += (float)s;
    }
}

__global__ __launch_bounds__(64) void xcc_probe_k(uint32_t *ids) {
    if (threadIdx.x == 0) ids[blockIdx.x] = xcc_id();
}

std::mutex g_mu;
std::vector<int> g_xcc;  // per device, -1 = not probed

}  // namespace

int launch_acc64_finish(float *out, const double *acc, uint64_t stride, int nacc, uint64_t n, hipStream_t s) {
    if (n == 0) return ALTO_OK;
    const unsigned grid = (unsigned)std::min<uint64_t>(8192, (n + 255) / 256);
    acc64_finish_k<<<grid, 256, 0, s>>>(out, acc, stride, nacc < 1 ? 1 : nacc, n);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int device_xcc_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_xcc.size() <= dev) g_xcc.resize(dev + 1, -1);
    if (g_xcc[dev] >= 0) return g_xcc[dev];
    g_xcc[dev] = 1;
    constexpr int kBlocks = 4096;
    uint32_t *d = nullptr;
    if (hipMalloc(&d, sizeof(uint32_t) * kBlocks) != hipSuccess) return 1;
    std::vector<uint32_t> h(kBlocks, 0);
    xcc_probe_k<<<kBlocks, 64, 0, 0>>>(d);
    if (hipGetLastError() == hipSuccess &&
        hipMemcpy(h.data(), d, sizeof(uint32_t) * kBlocks, hipMemcpyDeviceToHost) == hipSuccess) {
        uint32_t mx = 0;
        for (uint32_t v : h) mx = v > mx ? v : mx;
        g_xcc[dev] = (int)mx + 1;
    }
    (void)hipFree(d);
    return g_xcc[dev];
}

}  // namespace alto
