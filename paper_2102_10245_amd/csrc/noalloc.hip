// alto_mttkrp_noalloc: the atomic-update MTTKRP over the tensor's current
// partition with its scratch buffer in one static device array, for callers
// that cannot allocate device memory.
//
// The atomic strategy accumulates its updates in an I_mode x R FP64 array
// (see mttkrp_k); here that array is `scratch`, a file-scope device array of
// kScratchBytes that every GPU the library runs on holds until the process
// ends.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress (when a tensor is built on the device, or at this
// entry point's first call there) and only that address is passed to
// kernels.  Clearing uses a fill kernel, so the call records no memset.
#include <mutex>
#include <vector>

#include "mttkrp_impl.h"

namespace alto {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;  // per device; nullptr until looked up

// Device address of `scratch` on the current device (looked up once).
int scratch_ptr(double **out) {
    int dev = 0;
    ALTO_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(ALTO_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return ALTO_OK;
}

template <typename T>
__global__ __launch_bounds__(256) void fill_zero_k(T *__restrict__ a, uint64_t n) {
    for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (uint64_t)gridDim.x * 256) a[e] = T(0);
}

template <typename T>
int launch_fill_zero(T *a, uint64_t n, hipStream_t s) {
    if (n == 0) return ALTO_OK;
    const unsigned grid = (unsigned)std::min<uint64_t>(4096, (n + 255) / 256);
    fill_zero_k<T><<<grid, 256, 0, s>>>(a, n);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

}  // namespace

// Set-up on the current device (called by alto_build): the scratch address.
int noalloc_prepare_device() {
    double *p = nullptr;
    return scratch_ptr(&p);
}

}  // namespace alto

using namespace alto;

extern "C" int alto_mttkrp_noalloc(const alto_tensor *t, const void *const *factors, int R, int prec, int mode,
                                   float *out, hipStream_t s) {
    int rc = check_mttkrp_args(t, factors, R, prec, mode, out);
    if (rc) return rc;
    if (!t->part) return set_error(ALTO_E_STATE, "tensor has no partition");
    const uint64_t outn = t->dims[mode] * (uint64_t)R;
    if (outn * sizeof(double) > kScratchBytes)
        return set_error(ALTO_E_INVAL, "alto_mttkrp_noalloc: I_mode * R * 8 bytes exceeds the " +
                                           std::to_string(kScratchBytes >> 20) + " MiB static scratch");
    double *acc = nullptr;
    rc = scratch_ptr(&acc);
    if (rc) return rc;
    rc = launch_fill_zero(out, outn, s);
    if (rc) return rc;
    if (t->nnz == 0) return ALTO_OK;
    rc = launch_fill_zero(acc, outn, s);
    if (rc) return rc;
    MtLaunch a;
    rc = fill_mt_launch(t, factors, R, prec, mode, false, &a);
    if (rc) return rc;
    a.out = out;
    a.acc64 = acc;
    a.acc_stride = outn;
    a.nacc = 1;
    a.list = nullptr;  // every segment, in order
    a.n_list = t->part->L;
    a.staged = 0;
    a.temp_rows = 0;
    rc = launch_mt(a, t->key_bits, prec, s);
    if (rc) return rc;
    return launch_acc64_finish(out, acc, outn, 1, outn, s);
}
