// Sparse tensor transposition on an ALTO tensor, one of the operations the
// ALTO paper's related-work section (sparse tensor operations) names as
// benefiting from the format: the nonzeros in lexicographic order of their
// coordinates taken in a given mode order.  The usual method sorts the
// nonzeros by their multi-mode coordinates; here each nonzero's linearized
// index is rewritten as the lexicographic index of the permuted coordinates
// (the same B bits, grouped mode by mode), and one stable LSD radix sort
// over those B bits orders them: ceil(B/8) passes over one word per
// nonzero, where a sort of the coordinates themselves would move N words
// and make 4N byte passes.
#include <algorithm>

#include "common.h"

namespace alto {
namespace {

constexpr int kTT = 256;

// Where mode `mode[j]` (j = 0 most significant) sits in the lexicographic
// index: bits [off[j], off[j] + bits[j]).
struct LexPlan {
    int N;
    int mode[kMaxModes];
    int off[kMaxModes];
    int bits[kMaxModes];
};

struct OutPtrs {
    uint32_t *p[kMaxModes];
};

// v (at most 32 bits wide) placed at bit `pos` of a key; for 128-bit keys a
// field may straddle the two words.
template <typename K>
__device__ __forceinline__ void put_field(K &k, uint32_t v, int pos) {
    k |= (K)v << pos;
}
template <>
__device__ __forceinline__ void put_field<u128>(u128 &k, uint32_t v, int pos) {
    if (pos >= 64) {
        k.hi |= (uint64_t)v << (pos - 64);
    } else {
        k.lo |= (uint64_t)v << pos;
        if (pos > 32) k.hi |= (uint64_t)v >> (64 - pos);
    }
}
template <typename K>
__device__ __forceinline__ uint32_t get_field(const K &k, int pos, int len) {
    return len == 0 ? 0u : (uint32_t)((k >> pos) & (K)((1ull << len) - 1));
}
template <>
__device__ __forceinline__ uint32_t get_field<u128>(const u128 &k, int pos, int len) {
    if (len == 0) return 0u;
    uint64_t w;
    if (pos >= 64) w = k.hi >> (pos - 64);
    else if (pos == 0) w = k.lo;
    else w = (k.lo >> pos) | (k.hi << (64 - pos));
    return (uint32_t)(w & ((1ull << len) - 1));
}

template <typename K>
__global__ __launch_bounds__(kTT) void lexkey_k(const K *__restrict__ keys, int64_t n, RunTable tab, LexPlan p,
                                                K *__restrict__ out) {
    for (int64_t x = (int64_t)blockIdx.x * kTT + threadIdx.x; x < n; x += (int64_t)gridDim.x * kTT) {
        const K key = keys[x];
        K lk = KeyOps<K>::zero();
        for (int j = 0; j < p.N; j++)
            if (p.bits[j]) put_field(lk, extract_mode(key, tab, p.mode[j]), p.off[j]);
        out[x] = lk;
    }
}

template <typename K>
__global__ __launch_bounds__(kTT) void lexdecode_k(const K *__restrict__ lkeys, const float *__restrict__ vin,
                                                   int64_t n, LexPlan p, OutPtrs outp, float *__restrict__ vout) {
    for (int64_t x = (int64_t)blockIdx.x * kTT + threadIdx.x; x < n; x += (int64_t)gridDim.x * kTT) {
        const K lk = lkeys[x];
        for (int j = 0; j < p.N; j++) outp.p[j][x] = get_field(lk, p.off[j], p.bits[j]);
        vout[x] = vin[x];
    }
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(8192, (n + kTT - 1) / kTT)); }

template <typename K>
int run_transpose(const alto_tensor *t, const LexPlan &p, uint32_t *const *coords_out, float *vals_out,
                  hipStream_t s) {
    const int64_t n = t->nnz;
    const size_t kb = sizeof(K);
    const size_t sort_ws = radix_sort_scratch(t->key_bits, n);
    char *base = nullptr;
    const size_t a_keys = (kb * n + 255) & ~(size_t)255, a_vals = (sizeof(float) * n + 255) & ~(size_t)255;
    ALTO_HIP(hipMalloc(&base, 2 * a_keys + 2 * a_vals + sort_ws));
    K *k0 = (K *)base, *k1 = (K *)(base + a_keys);
    float *v0 = (float *)(base + 2 * a_keys), *v1 = (float *)(base + 2 * a_keys + a_vals);
    void *ws = base + 2 * a_keys + 2 * a_vals;
    auto fail = [&](int rc) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(base);
        return rc;
    };
    lexkey_k<K><<<grid_of(n), kTT, 0, s>>>((const K *)t->keys, n, t->tab, p, k0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(hip_error(e, "lexkey_k"));
    e = hipMemcpyAsync(v0, t->vals, sizeof(float) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return fail(hip_error(e, "hipMemcpyAsync(values)"));
    bool in_alt = false;
    int rc = radix_sort(t->key_bits, t->B, n, k0, v0, k1, v1, ws, sort_ws, &in_alt, s);
    if (rc) return fail(rc);
    OutPtrs outp{};
    for (int j = 0; j < p.N; j++) outp.p[j] = coords_out[j];
    lexdecode_k<K><<<grid_of(n), kTT, 0, s>>>(in_alt ? k1 : k0, in_alt ? v1 : v0, n, p, outp, vals_out);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(hip_error(e, "lexdecode_k"));
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(hip_error(e, "hipStreamSynchronize"));
    return fail(ALTO_OK);
}

}  // namespace
}  // namespace alto

using namespace alto;

extern "C" int alto_transpose(const alto_tensor *t, const int *perm, uint32_t *const *coords_out, float *vals_out,
                              hipStream_t s) {
    if (!t || !perm || !coords_out || (t->nnz > 0 && !vals_out)) return set_error(ALTO_E_INVAL, "null argument");
    LexPlan p{};
    p.N = t->N;
    bool seen[kMaxModes] = {};
    for (int j = 0; j < t->N; j++) {
        if (perm[j] < 0 || perm[j] >= t->N || seen[perm[j]])
            return set_error(ALTO_E_INVAL, "perm is not a permutation of 0..N-1");
        seen[perm[j]] = true;
        if (t->nnz > 0 && !coords_out[j]) return set_error(ALTO_E_INVAL, "null coordinate output");
    }
    int off = t->B;
    for (int j = 0; j < t->N; j++) {
        p.mode[j] = perm[j];
        p.bits[j] = t->nbits[perm[j]];
        off -= p.bits[j];
        p.off[j] = off;
    }
    if (t->nnz == 0) return ALTO_OK;
    if (t->key_bits == 32) return run_transpose<uint32_t>(t, p, coords_out, vals_out, s);
    if (t->key_bits == 64) return run_transpose<uint64_t>(t, p, coords_out, vals_out, s);
    return run_transpose<u128>(t, p, coords_out, vals_out, s);
}
