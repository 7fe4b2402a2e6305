// Incremental format generation: append a batch of COO nonzeros to a built
// ALTO tensor.  Streaming tensor decomposition (which the ALTO paper names
// as an application of its cheap format generation) grows a tensor batch by
// batch and refits the factors after each; rebuilding the whole tensor each
// time would linearize and radix-sort every nonzero again.  Here only the
// batch is linearized and sorted; it is then merged with the tensor's sorted
// index in one pass (merge path: every thread finds where its output range
// splits the two inputs by binary search, then merges that range), repeated
// coordinates are summed, and the partition is rebuilt.  The result equals a
// build of the old COO input followed by the batch, bit for bit.
#include <algorithm>

#include "common.h"

namespace alto {
namespace {

constexpr int kMT = 256;
constexpr int kMItems = 8;  // outputs per thread

template <typename K>
__device__ __forceinline__ bool key_le(const K &a, const K &b) {
    return a <= b;
}
template <>
__device__ __forceinline__ bool key_le<u128>(const u128 &a, const u128 &b) {
    return a.hi < b.hi || (a.hi == b.hi && a.lo <= b.lo);
}

// Stable merge of sorted a[na] (first on ties) and b[nb] into out[na + nb].
template <typename K>
__global__ __launch_bounds__(kMT) void merge_k(const K *__restrict__ a, const float *__restrict__ av, int64_t na,
                                               const K *__restrict__ b, const float *__restrict__ bv, int64_t nb,
                                               K *__restrict__ out, float *__restrict__ ov) {
    const int64_t n = na + nb;
    const int64_t d0 = ((int64_t)blockIdx.x * kMT + threadIdx.x) * kMItems;
    if (d0 >= n) return;
    // co-rank: the number i of a-elements among the first d0 outputs
    int64_t lo = d0 > nb ? d0 - nb : 0, hi = d0 < na ? d0 : na;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (key_le(a[mid], b[d0 - mid - 1])) lo = mid + 1;
        else hi = mid;
    }
    int64_t i = lo, j = d0 - lo;
    const int64_t d1 = d0 + kMItems < n ? d0 + kMItems : n;
    for (int64_t d = d0; d < d1; d++) {
        if (i < na && (j >= nb || key_le(a[i], b[j]))) {
            out[d] = a[i];
            ov[d] = av[i];
            i++;
        } else {
            out[d] = b[j];
            ov[d] = bv[j];
            j++;
        }
    }
}

int launch_merge(int key_bits, const void *a, const float *av, int64_t na, const void *b, const float *bv,
                 int64_t nb, void *out, float *ov, hipStream_t s) {
    const int64_t n = na + nb;
    if (n == 0) return ALTO_OK;
    const unsigned grid = (unsigned)((n + (int64_t)kMT * kMItems - 1) / ((int64_t)kMT * kMItems));
#define ALTO_MERGE(K) \
    merge_k<K><<<grid, kMT, 0, s>>>((const K *)a, av, na, (const K *)b, bv, nb, (K *)out, ov)
    if (key_bits == 32) ALTO_MERGE(uint32_t);
    else if (key_bits == 64) ALTO_MERGE(uint64_t);
    else ALTO_MERGE(u128);
#undef ALTO_MERGE
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

}  // namespace
}  // namespace alto

using namespace alto;

extern "C" int alto_append(alto_tensor *t, const uint32_t *const *coords, const float *vals, int64_t nnz,
                           hipStream_t s) {
    if (!t) return set_error(ALTO_E_INVAL, "null tensor handle");
    if (nnz < 0) return set_error(ALTO_E_INVAL, "nnz must be >= 0");
    if (nnz == 0) return ALTO_OK;
    if (!coords || !vals) return set_error(ALTO_E_INVAL, "null coords or vals");
    for (int n = 0; n < t->N; n++)
        if (!coords[n]) return set_error(ALTO_E_INVAL, "null coordinate pointer");
    const size_t kb = (size_t)t->key_bits / 8;
    const int64_t na = t->nnz, n_all = na + nnz;
    void *bkeys = nullptr, *bkeys_alt = nullptr, *mkeys = nullptr, *dims_d = nullptr;
    float *bvals = nullptr, *bvals_alt = nullptr, *mvals = nullptr;
    int *flag = nullptr;
    double *sums = nullptr;
    auto done = [&](int code) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(bkeys);
        (void)hipFree(bkeys_alt);
        (void)hipFree(bvals);
        (void)hipFree(bvals_alt);
        (void)hipFree(mkeys);
        (void)hipFree(mvals);
        (void)hipFree(dims_d);
        (void)hipFree(flag);
        (void)hipFree(sums);
        return code;
    };
#define ALTO_TRY(call)                                        \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return done(hip_error(e_, #call)); \
    } while (0)
    // a tensor built empty has no byte tables yet
    if (!t->ctab && !t->h_ctab.empty()) {
        ALTO_TRY(hipMalloc(&t->ctab, t->h_ctab.size()));
        ALTO_TRY(hipMemcpyAsync(t->ctab, t->h_ctab.data(), t->h_ctab.size(), hipMemcpyHostToDevice, s));
    }
    if (!t->etab && !t->h_etab.empty()) {
        ALTO_TRY(hipMalloc(&t->etab, t->h_etab.size()));
        ALTO_TRY(hipMemcpyAsync(t->etab, t->h_etab.data(), t->h_etab.size(), hipMemcpyHostToDevice, s));
    }
    // linearize and order the batch alone
    ALTO_TRY(hipMalloc(&bkeys, kb * nnz));
    ALTO_TRY(hipMalloc(&bkeys_alt, kb * nnz));
    ALTO_TRY(hipMalloc(&bvals, sizeof(float) * nnz));
    ALTO_TRY(hipMalloc(&bvals_alt, sizeof(float) * nnz));
    ALTO_TRY(hipMalloc(&dims_d, sizeof(uint64_t) * kMaxModes));
    ALTO_TRY(hipMalloc(&flag, sizeof(int)));
    ALTO_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
    ALTO_TRY(hipMemcpyAsync(dims_d, t->dims, sizeof(uint64_t) * kMaxModes, hipMemcpyHostToDevice, s));
    ALTO_TRY(hipMemcpyAsync(bvals, vals, sizeof(float) * nnz, hipMemcpyDeviceToDevice, s));
    CoordPtrs cp{};
    for (int n = 0; n < t->N; n++) cp.p[n] = coords[n];
    int rc = launch_encode(t->key_bits, cp, (const uint64_t *)dims_d, nnz, t->tab, t->etab, bkeys, flag, s);
    if (rc) return done(rc);
    int hflag = 0;
    ALTO_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ALTO_TRY(hipStreamSynchronize(s));
    if (hflag) return done(set_error(ALTO_E_RANGE, "a coordinate is not below its dimension"));
    rc = ensure_workspace(t, std::max(radix_sort_scratch(t->key_bits, nnz), coalesce_scratch(n_all)));
    if (rc) return done(rc);
    bool in_alt = false;
    rc = radix_sort(t->key_bits, t->B, nnz, bkeys, bvals, bkeys_alt, bvals_alt, t->ws, t->ws_bytes, &in_alt, s);
    if (rc) return done(rc);
    if (in_alt) {
        std::swap(bkeys, bkeys_alt);
        std::swap(bvals, bvals_alt);
    }
    // helper-flag bits would change the order of the merge: clear them
    // (they describe the old partition anyway)
    if (t->flags_in_keys) {
        rc = launch_mask_keys(t->key_bits, t->keys, na, t->B, t->keys, s);
        if (rc) return done(rc);
        t->flags_in_keys = false;
        for (int n = 0; n < t->N; n++) t->flag_L[n] = t->flag_NG[n] = 0;
    }
    // merge behind the tensor's nonzeros (which came first in input order)
    ALTO_TRY(hipMalloc(&mkeys, kb * n_all));
    ALTO_TRY(hipMalloc(&mvals, sizeof(float) * n_all));
    rc = launch_merge(t->key_bits, t->keys, t->vals, na, bkeys, bvals, nnz, mkeys, mvals, s);
    if (rc) return done(rc);
    // sum repeated coordinates (the batch's own and those already present)
    (void)hipFree(bkeys_alt);
    (void)hipFree(bvals_alt);
    bkeys_alt = nullptr;
    bvals_alt = nullptr;
    int64_t nu = n_all;
    void *ckeys = nullptr;
    float *cvals = nullptr;
    ALTO_TRY(hipMalloc(&ckeys, kb * n_all));
    ALTO_TRY(hipMalloc(&cvals, sizeof(float) * n_all));
    bkeys_alt = ckeys;  // freed by done() unless kept
    bvals_alt = cvals;
    rc = coalesce(t->key_bits, n_all, mkeys, mvals, ckeys, cvals, t->ws, t->ws_bytes, &nu, s);
    if (rc) return done(rc);
    // the merged (and coalesced) arrays become the tensor's
    ALTO_TRY(hipStreamSynchronize(s));
    (void)hipFree(t->keys);
    (void)hipFree(t->vals);
    if (nu != n_all) {
        t->keys = ckeys;
        t->vals = cvals;
        bkeys_alt = nullptr;
        bvals_alt = nullptr;
    } else {
        t->keys = mkeys;
        t->vals = mvals;
        mkeys = nullptr;
        mvals = nullptr;
    }
    t->nnz = nu;
    t->nnz_in += nnz;
    ALTO_TRY(hipMalloc(&sums, sizeof(double) * 1025));
    rc = launch_sumsq(t->vals, t->nnz, sums, s);
    if (rc) return done(rc);
    ALTO_TRY(hipMemcpyAsync(&t->norm2, sums + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
    ALTO_TRY(hipStreamSynchronize(s));
#undef ALTO_TRY
    // every partition, segment-local order and timed plan described the old
    // tensor; the new one gets a partition with the same number of segments
    const int L = t->part ? t->part->L_req : 0;
    t->part.reset();
    t->spare.clear();
    t->tuned.clear();
    rc = make_partition(t, L, s);
    if (rc) return done(rc);
    rc = compute_row_features(t, s);
    return done(rc);
}
