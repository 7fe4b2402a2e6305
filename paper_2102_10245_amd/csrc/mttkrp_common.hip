// Host helpers and small kernels shared by the MTTKRP launchers: adding the
// FP64 accumulator of the atomic updates into the FP32 output.
#include "mttkrp_impl.h"

namespace alto {

namespace {

__global__ __launch_bounds__(256) void acc64_finish4_k(float4 *__restrict__ out, const double2 *__restrict__ acc,
                                                       uint64_t n4) {
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (uint64_t)gridDim.x * 256) {
        float4 o = out[e];
        const double2 a = acc[2 * e], b = acc[2 * e + 1];
        o.x += (float)a.x;
        o.y += (float)a.y;
        o.z += (float)b.x;
        o.w += (float)b.y;
        out[e] = o;
    }
}

__global__ __launch_bounds__(256) void acc64_finish1_k(float *__restrict__ out, const double *__restrict__ acc,
                                                       uint64_t n) {
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (uint64_t)gridDim.x * 256)
        out[e] += (float)acc[e];
}

}  // namespace

int launch_acc64_finish(float *out, const double *acc, uint64_t n, hipStream_t s) {
    if (n == 0) return ALTO_OK;
    const bool v4 = (n % 4 == 0) && ((uintptr_t)out % 16 == 0) && ((uintptr_t)acc % 16 == 0);
    const uint64_t work = v4 ? n / 4 : n;
    const unsigned grid = (unsigned)std::min<uint64_t>(4096, (work + 255) / 256);
    if (v4) acc64_finish4_k<<<grid, 256, 0, s>>>((float4 *)out, (const double2 *)acc, n / 4);
    else acc64_finish1_k<<<grid, 256, 0, s>>>(out, acc, n);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

}  // namespace alto
