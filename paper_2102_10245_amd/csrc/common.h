// Internal declarations shared by the libalto sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "alto.h"

namespace alto {

constexpr int kMaxModes = ALTO_MAX_MODES;
constexpr int kMaxRuns = 40;  // runs of consecutive index bits per mode (<= 32 bits + word splits)

// ---------------------------------------------------------------- keys
// A linearized index (Section 3.1) of 32, 64 or 128 bits.
struct u128 {
    uint64_t lo, hi;
};

template <typename K>
struct KeyOps;

template <>
struct KeyOps<uint32_t> {
    static constexpr int kBits = 32;
    __device__ __forceinline__ static uint32_t field(uint32_t k, int pos, int len) {
        return (k >> pos) & (uint32_t)((1ull << len) - 1);
    }
    __device__ __forceinline__ static void deposit(uint32_t &k, uint32_t v, int pos) { k |= v << pos; }
    __device__ __forceinline__ static uint32_t digit(uint32_t k, int shift) { return (k >> shift) & 0xffu; }
    __device__ __forceinline__ static bool eq(uint32_t a, uint32_t b) { return a == b; }
    __device__ __forceinline__ static uint32_t zero() { return 0u; }
};

template <>
struct KeyOps<uint64_t> {
    static constexpr int kBits = 64;
    __device__ __forceinline__ static uint32_t field(uint64_t k, int pos, int len) {
        return (uint32_t)((k >> pos) & ((1ull << len) - 1));
    }
    __device__ __forceinline__ static void deposit(uint64_t &k, uint32_t v, int pos) { k |= (uint64_t)v << pos; }
    __device__ __forceinline__ static uint32_t digit(uint64_t k, int shift) { return (uint32_t)(k >> shift) & 0xffu; }
    __device__ __forceinline__ static bool eq(uint64_t a, uint64_t b) { return a == b; }
    __device__ __forceinline__ static uint64_t zero() { return 0ull; }
};

template <>
struct KeyOps<u128> {
    static constexpr int kBits = 128;
    // runs never straddle bit 64 (the host splits them)
    __device__ __forceinline__ static uint32_t field(const u128 &k, int pos, int len) {
        const uint64_t w = pos < 64 ? k.lo : k.hi;
        return (uint32_t)((w >> (pos & 63)) & ((1ull << len) - 1));
    }
    __device__ __forceinline__ static void deposit(u128 &k, uint32_t v, int pos) {
        if (pos < 64) k.lo |= (uint64_t)v << pos;
        else k.hi |= (uint64_t)v << (pos - 64);
    }
    __device__ __forceinline__ static uint32_t digit(const u128 &k, int shift) {
        const uint64_t w = shift < 64 ? k.lo : k.hi;
        return (uint32_t)(w >> (shift & 63)) & 0xffu;
    }
    __device__ __forceinline__ static bool eq(const u128 &a, const u128 &b) { return a.lo == b.lo && a.hi == b.hi; }
    __device__ __forceinline__ static u128 zero() { return u128{0ull, 0ull}; }
    __device__ __forceinline__ static uint64_t lo_word(const u128 &k) { return k.lo; }
    __device__ __forceinline__ static uint64_t hi_word(const u128 &k) { return k.hi; }
};

// Bit runs of every mode: run r of mode n moves `len` consecutive bits from
// index position `kpos` to coordinate position `cpos` (packed kpos | cpos<<8 | len<<16).
struct RunTable {
    int N;
    int nruns[kMaxModes];
    uint32_t run[kMaxModes][kMaxRuns];
    // Compact form: mode n's coordinate is bits [coff[n], coff[n] + b_n) of
    // the word that the byte tables assemble (64 bits at most for indices of
    // at most 64 bits; for 128-bit indices a {lo, hi} pair of 64-bit words,
    // which a coordinate may straddle).
    uint32_t coff[kMaxModes];
    uint32_t cmask[kMaxModes];
    // 128-bit indices: index bytes covered by the byte tables
    int tbytes128;
    // Linearization by deposit tables: byte j of mode n's coordinate selects
    // entry eoff[n] + 256 j + byte, which holds that byte's bits at their
    // index positions (ebytes[n] = ceil(b_n / 8) bytes per coordinate).
    // etab_entries = 0: no tables, the bit runs deposit.
    uint32_t eoff[kMaxModes];
    uint8_t ebytes[kMaxModes];
    int etab_entries;
};

// largest deposit tables staged in LDS by the encode kernel
constexpr size_t kEncodeTableMax = 64 * 1024;

__device__ __forceinline__ int run_kpos(uint32_t r) { return (int)(r & 0xffu); }
__device__ __forceinline__ int run_cpos(uint32_t r) { return (int)((r >> 8) & 0xffu); }
__device__ __forceinline__ int run_len(uint32_t r) { return (int)((r >> 16) & 0xffu); }

// De-linearize one mode: bit-level scatter of the mode's index bits.
template <typename K>
__device__ __forceinline__ uint32_t extract_mode(const K &key, const RunTable &tab, int n) {
    uint32_t c = 0;
    const int nr = tab.nruns[n];
    for (int q = 0; q < nr; q++) {
        const uint32_t r = tab.run[n][q];
        c |= KeyOps<K>::field(key, run_kpos(r), run_len(r)) << run_cpos(r);
    }
    return c;
}

// De-linearize all modes at once (indices of at most 64 bits).  Byte j of the
// index, with value v, contributes table entry lt[j*256 + v]: the bits of v
// moved to their places in the compact word, where the modes' coordinates sit
// back to back.  The OR over the index bytes is a bit-level scatter of every
// mode in one pass (Section 3.1's de-linearization).
template <typename K>
__device__ __forceinline__ K compact_index(const K key, const K *lt) {
    K c = 0;
#pragma unroll
    for (int j = 0; j < (int)sizeof(K); j++) c |= lt[j * 256 + (int)((key >> (8 * j)) & 0xffu)];
    return c;
}

// entries of the byte tables of a key width (0: the width has none)
__host__ __device__ constexpr int byte_table_entries(int key_bits) { return key_bits <= 64 ? key_bits / 8 * 256 : 0; }

struct CoordPtrs {
    const uint32_t *p[kMaxModes];
};

// Segment lists of one MTTKRP plan: segments run with atomics, and staged
// segments bucketed by the LDS rows their mode interval needs.
struct SegLists {
    static constexpr int kBuckets = 3;
    int32_t *d = nullptr;  // device: atomic list, then bucket 0, 1, 2
    int n_atomic = 0;
    int n_bucket[kBuckets] = {};
    int w_bucket[kBuckets] = {};
};

// ---------------------------------------------------------------- tensor
// One cut of the ordered tensor into L equal-nonzero line segments, with
// everything derived from it: mode intervals, per-row coverage, MTTKRP plans
// and segment-local mode orders.  Owns its device memory.
struct Partition {
    int L = 0;
    int L_req = 0;  // the segment count asked for (L is capped at nnz)
    int64_t *d_seg = nullptr;         // L+1
    uint32_t *d_ivl = nullptr;        // L*N*2
    uint32_t *d_cov[kMaxModes] = {};  // per mode, I_n
    std::vector<int64_t> h_seg;
    std::vector<uint32_t> h_ivl;
    // plans keyed by (mode, strategy, LDS row capacity)
    std::map<uint64_t, SegLists> lists;
    // segment-local mode orders: index and values reordered inside each
    // segment by one mode's coordinate
    void *okeys[kMaxModes] = {};  // compact words for keys of at most 64 bits
    float *ovals[kMaxModes] = {};
    Partition() = default;
    Partition(const Partition &) = delete;
    Partition &operator=(const Partition &) = delete;
    ~Partition() {
        (void)hipFree(d_seg);
        (void)hipFree(d_ivl);
        for (int n = 0; n < kMaxModes; n++) {
            (void)hipFree(d_cov[n]);
            (void)hipFree(okeys[n]);
            (void)hipFree(ovals[n]);
        }
        for (auto &kv : lists) (void)hipFree(kv.second.d);
    }
};

}  // namespace alto

struct alto_tensor {
    int device = 0;
    int N = 0;
    uint64_t dims[alto::kMaxModes] = {};
    int nbits[alto::kMaxModes] = {};
    uint64_t mask_lo[alto::kMaxModes] = {}, mask_hi[alto::kMaxModes] = {};
    int B = 0;
    int key_bits = 64;
    alto::RunTable tab{};
    int64_t nnz_in = 0, nnz = 0;
    void *keys = nullptr;  // device, nnz * key_bits/8
    void *ctab = nullptr;  // device byte tables of the compact form
    std::vector<uint8_t> h_ctab;  // their host image (source of the upload)
    void *etab = nullptr;  // device deposit tables of the linearization
    std::vector<uint8_t> h_etab;  // their host image
    float *vals = nullptr; // device, nnz
    double norm2 = 0.0;
    // the current partition, and recently used ones (so that alternating
    // segment counts between modes costs nothing after first use)
    std::unique_ptr<alto::Partition> part;
    std::vector<std::unique_ptr<alto::Partition>> spare;
    // reusable device workspace (grown on demand)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // FP64 accumulator of the atomic updates of the linearized-order
    // strategies, I_mode x R doubles (grown on demand)
    double *acc64 = nullptr;
    size_t acc64_bytes = 0;
    // plans found by timing every candidate, for (mode, R, prec) outside the
    // selector's training range (see tuned_key)
    std::map<uint64_t, alto_exec> tuned;
    // Helper flags (Section 3.3): index bit flag_bit[n] (one of the spare
    // bits at or above B; -1: none) marks the nonzeros whose mode-n row no
    // other lane group touches, so their atomic-strategy updates are plain
    // writes.  Valid for the current index order cut into flag_L segments of
    // flag_NG lane groups each (flag_L = 0: not computed).
    int flag_bit[alto::kMaxModes] = {-1, -1, -1, -1, -1, -1, -1, -1};
    int flag_L[alto::kMaxModes] = {};
    int flag_NG[alto::kMaxModes] = {};
    bool flags_in_keys = false;  // some flag bit may be set in keys
    // selector features from the row counts of evenly spaced nonzeros (set
    // by alto_build and alto_append): per mode, log2 of the
    // hottest row's count over the count a uniform mode would give, and log2
    // of the fraction of distinct rows in the sample
    float row_hot[alto::kMaxModes] = {};
    float row_distinct[alto::kMaxModes] = {};
};

namespace alto {

// error state (api.hip)
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
#define ALTO_HIP(call)                                            \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::alto::hip_error(e_, #call); \
    } while (0)

// ---------------------------------------------------------------- launchers
// build.hip
int launch_encode(int key_bits, const CoordPtrs &c, const uint64_t *dims, int64_t n, const RunTable &tab,
                  const void *etab, void *keys, int *d_flag, hipStream_t s);
int radix_sort(int key_bits, int nbits, int64_t n, void *keys, float *vals, void *keys_alt, float *vals_alt,
               void *scratch, size_t scratch_bytes, bool *result_in_alt, hipStream_t s);
size_t radix_sort_scratch(int key_bits, int64_t n);
int coalesce(int key_bits, int64_t n, const void *keys, const float *vals, void *keys_out, float *vals_out,
             void *scratch, size_t scratch_bytes, int64_t *n_unique, hipStream_t s);
size_t coalesce_scratch(int64_t n);
int launch_intervals(int key_bits, const void *keys, const int64_t *seg, int L, const RunTable &tab,
                     const void *ctab, uint32_t *ivl, hipStream_t s);
int coverage(int N, int L, const uint32_t *d_ivl, int mode, uint64_t dim, uint32_t *cov, void *scratch,
             size_t scratch_bytes, hipStream_t s);
size_t coverage_scratch(uint64_t dim);
int launch_sumsq(const float *vals, int64_t n, double *out, hipStream_t s);
// helper flags: bit `fbit` of every index := its row along `mode` is
// touched by its own lane-group range only (segments from seg, NG ranges
// each; owner: scratch of dim uint32)
int launch_owner_flags(int key_bits, void *keys, const int64_t *seg, int L, int NG, const RunTable &tab,
                       const void *ctab, int mode, uint32_t *owner, uint64_t dim, int fbit, hipStream_t s);
// index words -> compact words in place, and back (keys of at most 64 bits)
int launch_compact_keys(int key_bits, void *keys, int64_t n, const void *ctab, hipStream_t s);
int launch_expand_keys(int key_bits, const void *cw, int64_t n, const RunTable &tab, void *out, hipStream_t s);
// out[x] = bit fbit of index x
int launch_get_flags(int key_bits, const void *keys, int64_t n, int fbit, uint8_t *out, hipStream_t s);
// cnt[b] += 1 for every sampled nonzero (indices floor(k * M / S), k < S)
// whose mode-`mode` row r maps to bucket b = r (nb >= dims[mode]) or a hash
// of r (nb < dims[mode]); then res[0] = max(res[0], max cnt) and res[1] +=
// the number of nonzero buckets (res zeroed by the caller)
int launch_row_sample(int key_bits, const void *keys, int64_t S, int64_t M, const RunTable &tab,
                      const void *ctab, int mode, uint64_t dim, uint32_t nb, uint32_t *cnt, uint32_t *res,
                      hipStream_t s);
// the row features of every mode (t->row_hot, t->row_distinct); synchronizes s
int compute_row_features(alto_tensor *t, hipStream_t s);
// out = keys with every bit at or above B cleared (out may equal keys)
int launch_mask_keys(int key_bits, const void *keys, int64_t n, int B, void *out, hipStream_t s);
// segment-local order by `mode` (scratch: seg_order_scratch bytes)
size_t seg_order_scratch(int key_bits, int64_t n);
int launch_seg_order(int key_bits, const void *keys, const float *vals, const int64_t *seg, int L,
                     const RunTable &tab, const void *ctab, int mode, int nbits, void *scratch, int64_t n,
                     void *okeys, float *ovals, hipStream_t s);


// cpals.hip
int launch_gram(const void *A, int prec, uint64_t I, int R, double *G, double *partials, int nparts,
                hipStream_t s);
int cp_als_impl(alto_tensor *t, int R, int iters, int prec, void *const *factors, double *lambda,
                double *fit, const alto_exec *ex, hipStream_t s);
int launch_round_bf16(const double *in, uint16_t *out, int64_t n, hipStream_t s);

// mlp.hip
int mlp_forward(int B, int F, int H, int K, const float *params, const float *x, const float *t,
                const float *mask, float *y, float *loss, hipStream_t s);
int mlp_backward(int B, int F, int H, int K, const float *params, const float *x, const float *t,
                 const float *mask, float *grads, float *loss, hipStream_t s);
int mlp_adam(int64_t P, float *params, const float *grads, float *m, float *v, float lr, float b1, float b2,
             float eps, int t, hipStream_t s);

// selector.hip: where an automatic plan comes from
enum { kPlanRule = 0, kPlanNet = 1, kPlanOutside = 2, kPlanClose = 3 };
// the selector's (or, without weights, the reuse rule's) plan and its
// source; kPlanClose: the network's best prediction is within the margin
// (ALTO_SELECT_MARGIN, log2 time) of others, listed in *close (best first)
int select_plan(const alto_tensor *t, int mode, int R, int prec, alto_exec *out,
                std::vector<alto_exec> *close = nullptr);
// every (strategy, L) the selector chooses among
std::vector<alto_exec> selector_candidates();
inline uint64_t tuned_key(int mode, int R, int prec) {
    return (uint64_t)mode | ((uint64_t)R << 8) | ((uint64_t)prec << 20);
}

// api.hip: execution planning shared with cp_als
int plan_and_run_mttkrp(alto_tensor *t, const void *const *factors, int R, int prec, int mode, float *out,
                        const alto_exec *ex, hipStream_t s);
int ensure_workspace(alto_tensor *t, size_t bytes);
// make the partition into L segments current (0: 8 per compute unit)
int make_partition(alto_tensor *t, int L, hipStream_t s);

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

}  // namespace alto
