// C entry points of libalto: argument checks, the host side of format
// generation (bit layout, run tables, partition bounds) and MTTKRP planning.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"
#include "mttkrp_impl.h"

namespace alto {

namespace {
thread_local std::string g_err;
}

int set_error(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_error(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? ALTO_E_NOMEM : ALTO_E_HIP;
}

namespace {

int ceil_log2(uint64_t x) {
    int b = 0;
    while (b < 64 && (1ull << b) < x) b++;
    return b;
}

// Bit layout of Section 3.1: b_n = ceil(log2 I_n) bits per mode, given out
// level by level from the least significant bit; inside a level the shorter
// mode gets the lower bit (equal lengths: lower mode number first), so the
// top bits split the longest mode first.
int make_layout(alto_tensor *t, int key_bits_req) {
    const int N = t->N;
    int order[kMaxModes];
    int maxb = 0;
    for (int n = 0; n < N; n++) {
        t->nbits[n] = ceil_log2(t->dims[n]);
        maxb = std::max(maxb, t->nbits[n]);
        order[n] = n;
        t->mask_lo[n] = t->mask_hi[n] = 0;
    }
    std::stable_sort(order, order + N, [&](int a, int b) { return t->dims[a] < t->dims[b]; });
    int pos = 0;
    // bit positions of each mode, coordinate bit k -> index bit pos
    int where[kMaxModes][32];
    for (int lvl = 0; lvl < maxb; lvl++)
        for (int q = 0; q < N; q++) {
            const int n = order[q];
            if (t->nbits[n] <= lvl) continue;
            if (pos >= 128) return set_error(ALTO_E_TOO_WIDE, "linearized index needs more than 128 bits");
            where[n][lvl] = pos;
            if (pos < 64) t->mask_lo[n] |= 1ull << pos;
            else t->mask_hi[n] |= 1ull << (pos - 64);
            pos++;
        }
    t->B = pos;
    if (key_bits_req == 0) t->key_bits = pos <= 32 ? 32 : (pos <= 64 ? 64 : 128);
    else if (key_bits_req == 32 || key_bits_req == 64 || key_bits_req == 128) t->key_bits = key_bits_req;
    else return set_error(ALTO_E_INVAL, "key_bits must be 0, 32, 64 or 128");
    if (pos > t->key_bits)
        return set_error(ALTO_E_TOO_WIDE, "linearized index needs " + std::to_string(pos) + " bits, key has " +
                                              std::to_string(t->key_bits));
    // helper-flag bits: the spare index bits go to the longest modes first
    // (fewest nonzeros per row); a flagged row also needs a free bit 31
    {
        int by_len[kMaxModes];
        for (int n = 0; n < N; n++) {
            by_len[n] = n;
            t->flag_bit[n] = -1;
            t->flag_L[n] = t->flag_NG[n] = 0;
        }
        std::stable_sort(by_len, by_len + N, [&](int a, int b) { return t->dims[a] > t->dims[b]; });
        int next = pos;
        for (int q = 0; q < N && next < t->key_bits; q++)
            if (t->dims[by_len[q]] < 0x80000000ull) t->flag_bit[by_len[q]] = next++;
    }
    // runs of consecutive positions, split at the 64-bit word boundary
    t->tab.N = N;
    for (int n = 0; n < N; n++) {
        int nr = 0;
        int k = 0;
        while (k < t->nbits[n]) {
            const int kp = where[n][k];
            int len = 1;
            while (k + len < t->nbits[n] && where[n][k + len] == kp + len && (kp + len) != 64) len++;
            if (nr >= kMaxRuns) return set_error(ALTO_E_INVAL, "internal: too many bit runs");
            t->tab.run[n][nr++] = (uint32_t)kp | ((uint32_t)k << 8) | ((uint32_t)len << 16);
            k += len;
        }
        t->tab.nruns[n] = nr;
    }
    // deposit tables: the index bits of each byte value of each coordinate byte
    t->h_etab.clear();
    {
        int E = 0;
        for (int n = 0; n < N; n++) {
            t->tab.ebytes[n] = (uint8_t)((t->nbits[n] + 7) / 8);
            t->tab.eoff[n] = (uint32_t)E;
            E += t->tab.ebytes[n] * 256;
        }
        const size_t esz = (size_t)t->key_bits / 8;
        t->tab.etab_entries = (size_t)E * esz <= kEncodeTableMax ? E : 0;
        if (t->tab.etab_entries > 0) {
            t->h_etab.assign((size_t)E * esz, 0);
            for (int n = 0; n < N; n++)
                for (int j = 0; j < t->tab.ebytes[n]; j++)
                    for (int v = 0; v < 256; v++) {
                        uint64_t e[2] = {0, 0};
                        for (int b = 0; b < 8; b++) {
                            const int k = 8 * j + b;
                            if (k < t->nbits[n] && ((v >> b) & 1)) e[where[n][k] >> 6] |= 1ull << (where[n][k] & 63);
                        }
                        std::memcpy(&t->h_etab[((size_t)t->tab.eoff[n] + (size_t)j * 256 + v) * esz], e,
                                    esz);  // little-endian entry ({lo, hi} for 128 bits)
                    }
        }
    }
    // compact form: coordinate bit k of mode n lands at bit coff[n] + k
    int coff = 0;
    for (int n = 0; n < N; n++) {
        t->tab.coff[n] = (uint32_t)coff;
        t->tab.cmask[n] = t->nbits[n] >= 32 ? 0xffffffffu : (1u << t->nbits[n]) - 1u;
        coff += t->nbits[n];
    }
    t->h_ctab.clear();
    t->tab.tbytes128 = 0;
    if (t->key_bits == 128) {
        // 128-bit compact word {lo, hi}; a coordinate may straddle the halves
        int cmap[128];
        for (int p = 0; p < 128; p++) cmap[p] = -1;
        for (int n = 0; n < N; n++)
            for (int k = 0; k < t->nbits[n]; k++) cmap[where[n][k]] = (int)t->tab.coff[n] + k;
        const int nb = std::max(1, (pos + 7) / 8);
        t->tab.tbytes128 = nb;
        t->h_ctab.assign((size_t)nb * 256 * 16, 0);
        for (int j = 0; j < nb; j++)
            for (int v = 0; v < 256; v++) {
                uint64_t e[2] = {0, 0};
                for (int b = 0; b < 8; b++) {
                    const int c = cmap[8 * j + b];
                    if (((v >> b) & 1) && c >= 0) e[c >> 6] |= 1ull << (c & 63);
                }
                std::memcpy(&t->h_ctab[((size_t)j * 256 + v) * 16], e, 16);  // {lo, hi}
            }
    }
    if (t->key_bits <= 64) {
        int cmap[64];
        for (int p = 0; p < 64; p++) cmap[p] = -1;
        for (int n = 0; n < N; n++)
            for (int k = 0; k < t->nbits[n]; k++) cmap[where[n][k]] = (int)t->tab.coff[n] + k;
        const int kb = t->key_bits / 8;
        t->h_ctab.assign((size_t)byte_table_entries(t->key_bits) * kb, 0);
        for (int j = 0; j < kb; j++)
            for (int v = 0; v < 256; v++) {
                uint64_t e = 0;
                for (int b = 0; b < 8; b++)
                    if (((v >> b) & 1) && cmap[8 * j + b] >= 0) e |= 1ull << cmap[8 * j + b];
                std::memcpy(&t->h_ctab[((size_t)j * 256 + v) * kb], &e, kb);  // little-endian entry
            }
    }
    return ALTO_OK;
}

// Segment-local order by one mode: inside every line segment, a stable
// reordering of the nonzeros by their mode coordinate, written to arrays of
// its own (one workgroup per segment, see seg_order_k).  Built once per mode
// and partition.
int build_mode_order(alto_tensor *t, int mode, hipStream_t s) {
    Partition &P = *t->part;
    if (P.okeys[mode]) return ALTO_OK;
    const int64_t n = t->nnz;
    if ((uint64_t)(n + P.L - 1) / (uint64_t)std::max(1, P.L) > 0xffffffffull)
        return set_error(ALTO_E_INVAL, "segment-local orders need segments of fewer than 2^32 nonzeros");
    const size_t kb = (size_t)t->key_bits / 8;
    int rc = ensure_workspace(t, seg_order_scratch(t->key_bits, n));
    if (rc) return rc;
    // the order is recorded only once it has been launched, so a failure
    // leaves no half-built order behind
    void *ok = nullptr;
    float *ov = nullptr;
    hipError_t e = hipMalloc(&ok, kb * n);
    if (e == hipSuccess) e = hipMalloc(&ov, sizeof(float) * n);
    if (e != hipSuccess) {
        (void)hipFree(ok);
        return hip_error(e, "hipMalloc(segment-local order)");
    }
    rc = launch_seg_order(t->key_bits, t->keys, t->vals, P.d_seg, P.L, t->tab, t->ctab, mode, t->nbits[mode], t->ws,
                          n, ok, ov, s);
    if (rc) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(ok);
        (void)hipFree(ov);
        return rc;
    }
    if (t->key_bits <= 64) {
        rc = launch_compact_keys(t->key_bits, ok, n, t->ctab, s);
        if (rc) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(ok);
            (void)hipFree(ov);
            return rc;
        }
    }
    P.okeys[mode] = ok;
    P.ovals[mode] = ov;
    return ALTO_OK;
}

int cu_count() {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) return 256;
    return cu;
}

// Section 3.2: L equal-nonzero line segments, mode intervals, and the number
// of segments whose interval holds each output row.
int build_partition(alto_tensor *t, int Le, hipStream_t s, std::unique_ptr<Partition> *out) {
    auto pp = std::make_unique<Partition>();
    Partition &p = *pp;
    const int64_t M = t->nnz;
    p.L = Le;
    p.h_seg.resize(Le + 1);
    for (int l = 0; l <= Le; l++)
        p.h_seg[l] = Le == 0 ? 0 : (int64_t)(((unsigned __int128)l * (uint64_t)M) / (uint64_t)Le);
    ALTO_HIP(hipMalloc(&p.d_seg, sizeof(int64_t) * (Le + 1)));
    ALTO_HIP(hipMalloc(&p.d_ivl, sizeof(uint32_t) * std::max(1, Le * t->N * 2)));
    ALTO_HIP(hipMemcpyAsync(p.d_seg, p.h_seg.data(), sizeof(int64_t) * (Le + 1), hipMemcpyHostToDevice, s));
    int rc = launch_intervals(t->key_bits, t->keys, p.d_seg, Le, t->tab, t->ctab, p.d_ivl, s);
    if (rc) return rc;
    uint64_t maxdim = 0;
    for (int n = 0; n < t->N; n++) maxdim = std::max(maxdim, t->dims[n]);
    rc = ensure_workspace(t, coverage_scratch(maxdim));
    if (rc) return rc;
    for (int n = 0; n < t->N; n++) {
        ALTO_HIP(hipMalloc(&p.d_cov[n], sizeof(uint32_t) * t->dims[n]));
        rc = coverage(t->N, Le, p.d_ivl, n, t->dims[n], p.d_cov[n], t->ws, t->ws_bytes, s);
        if (rc) return rc;
    }
    p.h_ivl.resize((size_t)Le * t->N * 2);
    if (Le > 0)
        ALTO_HIP(hipMemcpyAsync(p.h_ivl.data(), p.d_ivl, sizeof(uint32_t) * p.h_ivl.size(), hipMemcpyDeviceToHost, s));
    ALTO_HIP(hipStreamSynchronize(s));
    *out = std::move(pp);
    return ALTO_OK;
}

constexpr size_t kSparePartitions = 3;

// Make the partition into L segments (L capped at nnz; 0 = 8 per compute
// unit) the current one: reuse a recent one or build it.
int select_partition(alto_tensor *t, int L, hipStream_t s) {
    if (L <= 0) L = 8 * cu_count();
    const int Le = t->nnz == 0 ? 0 : (int)std::min<int64_t>(L, t->nnz);
    if (t->part && t->part->L == Le) {
        t->part->L_req = L;
        return ALTO_OK;
    }
    for (size_t q = 0; q < t->spare.size(); q++)
        if (t->spare[q]->L == Le) {
            std::unique_ptr<Partition> p = std::move(t->spare[q]);
            t->spare.erase(t->spare.begin() + q);
            if (t->part) t->spare.push_back(std::move(t->part));
            t->part = std::move(p);
            t->part->L_req = L;
            return ALTO_OK;
        }
    std::unique_ptr<Partition> p;
    const int rc = build_partition(t, Le, s, &p);
    if (rc) return rc;
    if (t->part) {
        if (t->spare.size() >= kSparePartitions) {
            ALTO_HIP(hipStreamSynchronize(s));  // work queued on the evicted partition has finished
            t->spare.erase(t->spare.begin());
        }
        t->spare.push_back(std::move(t->part));
    }
    t->part = std::move(p);
    t->part->L_req = L;
    return ALTO_OK;
}

long env_long(const char *name, long dflt) {
    const char *e = getenv(name);
    return e && *e ? atol(e) : dflt;
}

// LDS budget of the Temp rows of a staged segment (one workgroup per CU at
// the top of the range, several below it).
size_t staged_lds_budget() {
    static size_t budget = (size_t)std::min<long>(140 * 1024, std::max<long>(4096, env_long("ALTO_STAGE_LDS_BYTES", 96 * 1024)));
    return budget;
}

// Workgroup size of launches that flush with atomics: enough waves for
// about eight per SIMD over the whole grid of L workgroups (1024 threads at
// L <= 512, 512 at L = 1024, 256 above).  ALTO_MT_THREADS (64..1024, a
// multiple of 64) overrides.
int atomic_threads(int L) {
    const long v = env_long("ALTO_MT_THREADS", 0);
    if (v >= 64 && v <= 1024 && v % 64 == 0) return (int)v;
    return L <= 512 ? 1024 : (L <= 1024 ? 512 : 256);
}

// workgroup size for a staged launch whose Temp takes `bytes` of LDS
int staged_threads(size_t bytes) { return bytes <= 40 * 1024 ? 256 : (bytes <= 80 * 1024 ? 512 : 1024); }

int build_lists(alto_tensor *t, int mode, int strategy, int R, int prec, SegLists **out) {
    (void)prec;
    const size_t budget = staged_lds_budget();
    const int cap_rows = strategy == ALTO_STRATEGY_STAGED ? (int)(budget / ((size_t)temp_stride(R) * 4)) : 0;
    const uint64_t key = ((uint64_t)mode << 40) | ((uint64_t)strategy << 32) | (uint64_t)(uint32_t)cap_rows;
    Partition &P = *t->part;
    auto it = P.lists.find(key);
    if (it != P.lists.end()) {
        *out = &it->second;
        return ALTO_OK;
    }
    const int L = P.L, N = t->N;
    std::vector<int32_t> atomic_l;
    std::vector<int32_t> bucket[SegLists::kBuckets];
    // bucket bounds: 1/8, 1/2 and all of the row capacity
    const int bound[SegLists::kBuckets] = {std::max(1, cap_rows / 8), std::max(1, cap_rows / 2), cap_rows};
    for (int l = 0; l < L; l++) {
        const uint32_t s0 = P.h_ivl[((size_t)l * N + mode) * 2 + 0];
        const uint32_t e0 = P.h_ivl[((size_t)l * N + mode) * 2 + 1];
        const uint64_t w = (uint64_t)e0 - s0 + 1;
        if (cap_rows == 0 || w > (uint64_t)cap_rows) {
            atomic_l.push_back(l);
            continue;
        }
        for (int b = 0; b < SegLists::kBuckets; b++)
            if (w <= (uint64_t)bound[b]) {
                bucket[b].push_back(l);
                break;
            }
    }
    SegLists sl;
    sl.n_atomic = (int)atomic_l.size();
    std::vector<int32_t> all(atomic_l);
    for (int b = 0; b < SegLists::kBuckets; b++) {
        sl.n_bucket[b] = (int)bucket[b].size();
        sl.w_bucket[b] = bound[b];
        all.insert(all.end(), bucket[b].begin(), bucket[b].end());
    }
    ALTO_HIP(hipMalloc(&sl.d, sizeof(int32_t) * std::max<size_t>(1, all.size())));
    if (!all.empty()) ALTO_HIP(hipMemcpy(sl.d, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice));
    auto ins = P.lists.emplace(key, sl);
    *out = &ins.first->second;
    return ALTO_OK;
}

int check_tensor(const alto_tensor *t) {
    if (!t) return set_error(ALTO_E_INVAL, "null tensor handle");
    return ALTO_OK;
}

}  // namespace

int make_partition(alto_tensor *t, int L, hipStream_t s) { return select_partition(t, L, s); }

int ensure_workspace(alto_tensor *t, size_t bytes) {
    if (t->ws_bytes >= bytes) return ALTO_OK;
    if (t->ws) ALTO_HIP(hipFree(t->ws));
    t->ws = nullptr;
    t->ws_bytes = 0;
    ALTO_HIP(hipMalloc(&t->ws, bytes));
    t->ws_bytes = bytes;
    return ALTO_OK;
}

// Selector features from row counts: at most 2^20 evenly spaced nonzeros
// of the tensor order, counted per mode into min(I_n, 2^24)
// buckets (rows of larger modes fold onto them by hashing).
int compute_row_features(alto_tensor *t, hipStream_t s) {
    for (int n = 0; n < t->N; n++) t->row_hot[n] = t->row_distinct[n] = 0.f;
    if (t->nnz == 0) return ALTO_OK;
    const int64_t S = std::min<int64_t>(t->nnz, (int64_t)1 << 20);
    uint64_t nb_max = 0;
    for (int n = 0; n < t->N; n++) nb_max = std::max<uint64_t>(nb_max, std::min<uint64_t>(t->dims[n], 1u << 24));
    int rc = ensure_workspace(t, sizeof(uint32_t) * (nb_max + 2 * kMaxModes));
    if (rc) return rc;
    uint32_t *res = (uint32_t *)t->ws;
    uint32_t *cnt = res + 2 * kMaxModes;
    ALTO_HIP(hipMemsetAsync(res, 0, sizeof(uint32_t) * 2 * kMaxModes, s));
    for (int n = 0; n < t->N; n++) {
        const uint32_t nb = (uint32_t)std::min<uint64_t>(t->dims[n], 1u << 24);
        ALTO_HIP(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * nb, s));
        rc = launch_row_sample(t->key_bits, t->keys, S, t->nnz, t->tab, t->ctab, n, t->dims[n], nb, cnt, res + 2 * n, s);
        if (rc) return rc;
    }
    uint32_t h[2 * kMaxModes];
    ALTO_HIP(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s));
    ALTO_HIP(hipStreamSynchronize(s));
    for (int n = 0; n < t->N; n++) {
        const double nb = (double)std::min<uint64_t>(t->dims[n], 1u << 24);
        t->row_hot[n] = (float)std::log2(std::max(1.0, (double)h[2 * n]) * (double)t->dims[n] / (double)S);
        t->row_distinct[n] = (float)std::log2(std::max(1.0, (double)h[2 * n + 1]) / std::min((double)S, nb));
    }
    return ALTO_OK;
}

// Exhaustive timing: run every candidate (strategy, L) once to build its
// plan and order, time a second run with events on the stream, keep the
// fastest.  The selector's fallback outside its training range.
int autotune(alto_tensor *t, const void *const *factors, int R, int prec, int mode, float *out, hipStream_t s,
             const std::vector<alto_exec> &cands, alto_exec *best) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ALTO_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_error(he, "hipEventCreate");
    }
    float best_ms = INFINITY;
    int rc = ALTO_OK;
    for (const alto_exec &c : cands) {
        rc = plan_and_run_mttkrp(t, factors, R, prec, mode, out, &c, s);
        if (rc) break;
        he = hipEventRecord(e0, s);
        if (he == hipSuccess) rc = plan_and_run_mttkrp(t, factors, R, prec, mode, out, &c, s);
        if (he == hipSuccess && !rc) he = hipEventRecord(e1, s);
        if (he == hipSuccess && !rc) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess && !rc) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) rc = hip_error(he, "timing a candidate plan");
        if (rc) break;
        if (ms < best_ms) {
            best_ms = ms;
            *best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int resolve_strategy(alto_tensor *t, const void *const *factors, int R, int prec, int mode, float *out,
                     const alto_exec *ex, hipStream_t s, alto_exec *res) {
    if (ex && (ex->strategy < 0 || ex->strategy > 3)) return set_error(ALTO_E_INVAL, "unknown strategy");
    if (ex && ex->num_segments < 0) return set_error(ALTO_E_INVAL, "num_segments must be >= 0");
    if (ex && ex->strategy != ALTO_STRATEGY_AUTO) {
        *res = *ex;
        return ALTO_OK;
    }
    alto_exec sel;
    std::vector<alto_exec> close;
    const int src = select_plan(t, mode, R, prec, &sel, &close);
    if (ex && ex->num_segments > 0) {
        sel.num_segments = ex->num_segments;  // a fixed L: the strategy as chosen
    } else if ((src == kPlanOutside || src == kPlanClose) && t->nnz > 0) {
        // time every candidate (outside the training range) or the close
        // ones, once per (mode, R, prec); the tensor keeps the fastest
        const uint64_t key = tuned_key(mode, R, prec);
        auto it = t->tuned.find(key);
        if (it == t->tuned.end()) {
            alto_exec best{};
            const int rc = autotune(t, factors, R, prec, mode, out, s,
                                    src == kPlanClose ? close : selector_candidates(), &best);
            if (rc) return rc;
            it = t->tuned.emplace(key, best).first;
        }
        sel = it->second;
    }
    *res = sel;
    return ALTO_OK;
}

int check_mttkrp_args(const alto_tensor *t, const void *const *factors, int R, int prec, int mode,
                      const float *out) {
    int rc = check_tensor(t);
    if (rc) return rc;
    if (mode < 0 || mode >= t->N) return set_error(ALTO_E_INVAL, "mode out of range");
    if (R < 1 || R > ALTO_MAX_RANK) return set_error(ALTO_E_INVAL, "R must be in 1..256");
    if (prec != ALTO_PREC_F32 && prec != ALTO_PREC_BF16) return set_error(ALTO_E_INVAL, "unknown precision");
    if (!out || !factors) return set_error(ALTO_E_INVAL, "null output or factor array");
    // row 2^32-1 would alias the kernels' "no row" marker
    if (t->dims[mode] > 0xffffffffull)
        return set_error(ALTO_E_INVAL, "MTTKRP output mode must have fewer than 2^32 rows");
    for (int m = 0; m < t->N; m++)
        if (m != mode && !factors[m]) return set_error(ALTO_E_INVAL, "null factor pointer");
    // rank-specialized kernels gather rows with 16-byte loads
    for (int m = 0; m < t->N; m++)
        if (m != mode && ((uintptr_t)factors[m] & 15u)) return set_error(ALTO_E_INVAL, "factor pointer not 16-byte aligned");
    if ((uintptr_t)out & 15u) return set_error(ALTO_E_INVAL, "output pointer not 16-byte aligned");
    return ALTO_OK;
}

int fill_mt_launch(const alto_tensor *t, const void *const *factors, int R, int prec, int mode, bool sorted,
                   MtLaunch *out) {
    MtLaunch &a = *out;
    a = MtLaunch{};
    a.dec.fbit = -1;
    a.keys = sorted ? t->part->okeys[mode] : t->keys;
    a.vals = sorted ? t->part->ovals[mode] : t->vals;
    a.seg = t->part->d_seg;
    a.ivl = t->part->d_ivl;
    a.cov = t->part->d_cov[mode];
    // the other modes first, in increasing order, then the output mode
    for (int m = 0, j = 0; m <= t->N; m++) {
        const int mm = m < t->N ? m : mode;
        if (m < t->N && m == mode) continue;
        if (m < t->N) a.fac.p[j] = factors[m];
        a.dec.om[j] = mm;
        a.dec.coff[j] = t->tab.coff[mm];
        a.dec.cmask[j] = t->tab.cmask[mm];
        j++;
    }
    a.R = R;
    a.N = t->N;
    a.mode = mode;
    a.tab = t->tab;
    a.ctab = t->ctab;
    a.dec.compact = sorted && t->key_bits <= 64;
    a.ordered = sorted;
    a.wide = false;
    const uint64_t fs = prec == ALTO_PREC_BF16 ? 2u : 4u;
    for (int m = 0; m < t->N; m++)
        if (m != mode && t->dims[m] * (uint64_t)R * fs > 0xffffffffull) a.wide = true;
    // Factor matrices of other modes small enough to sit in LDS (smallest
    // first, ALTO_STAGE_FACTOR_BYTES in total) are gathered from there; such
    // launches use 1024-thread workgroups so one copy serves 16 waves, which
    // pays only with segments long enough to keep 128 lane groups busy (on
    // the 4-mode tensor it wins at 71K nonzeros per segment and loses at 35K).
    a.dec.smask = 0;
    const int64_t seg_len = t->nnz / std::max(1, t->part->L);
    if ((R == 8 || R == 16 || R == 32 || R == 64) && seg_len >= 65536) {
        // what a 1024-thread launch needs besides: the flush queues (two rows
        // per lane group) and the byte tables
        const int vec = prec == ALTO_PREC_BF16 ? 8 : 4, gpw = 64 / (R / vec);
        const uint64_t queue = 16ull * 2 * gpw * (R + 1) * 4;
        const uint64_t table = t->key_bits <= 64 ? (uint64_t)(t->key_bits / 8) * 256 * (t->key_bits / 8)
                                                 : (uint64_t)t->tab.tbytes128 * 256 * 16;
        const uint64_t room = 160 * 1024 - std::min<uint64_t>(160 * 1024, queue + table + 512);
        const uint64_t budget =
            std::min<uint64_t>(room, (uint64_t)std::max<long>(0, env_long("ALTO_STAGE_FACTOR_BYTES", 64 * 1024)));
        int js[kMaxModes];
        for (int j = 0; j < t->N - 1; j++) js[j] = j;
        std::sort(js, js + t->N - 1, [&](int x, int y) { return t->dims[a.dec.om[x]] < t->dims[a.dec.om[y]]; });
        uint64_t used = 0;
        for (int q = 0; q < t->N - 1; q++) {
            const int j = js[q];
            const uint64_t bytes = t->dims[a.dec.om[j]] * (uint64_t)R * fs;
            if (used + bytes > budget) break;
            a.dec.smask |= 1u << j;
            a.dec.sbytes[j] = (uint32_t)bytes;
            used += bytes;
        }
    }
    a.threads = a.dec.smask ? 1024 : atomic_threads(t->part->L);
    if (!a.dec.smask && env_long("ALTO_MT_THREADS", 0) == 0) {
        // LDS per workgroup: the flush queues (two rows per lane group) and,
        // unless the keys are compact words, the byte tables (48 KB for a
        // 95-bit index).  Small workgroups with large tables leave a compute
        // unit few waves (two 256-thread workgroups: 8), so the workgroup
        // grows until LDS admits at least 16 waves per compute unit.
        const bool spec = R == 8 || R == 16 || R == 32 || R == 64;
        const int vec = prec == ALTO_PREC_BF16 ? 8 : 4;
        const uint64_t per_wave = spec ? 2ull * (64 / (R / vec)) * (R + 1) * 4 : 0;
        const uint64_t table = a.dec.compact ? 0
                               : t->key_bits <= 64 ? (uint64_t)(t->key_bits / 8) * 256 * (t->key_bits / 8)
                                                   : (uint64_t)t->tab.tbytes128 * 256 * 16;
        while (a.threads < 1024) {
            const uint64_t lds = (uint64_t)(a.threads / 64) * per_wave + table;
            const uint64_t wgs = lds ? (160 * 1024) / lds : 32;
            if (wgs * (uint64_t)(a.threads / 64) >= 16) break;
            a.threads *= 2;
        }
    }
    return ALTO_OK;
}

// Helper flags of `mode` (Section 3.3) for the current partition cut into
// NG lane groups per segment (the unit that walks its nonzeros in order):
// flag set iff every nonzero of the row lies in the same lane-group range.
// Only for modes of limited fiber reuse (nnz / I_mode <= 4, where the reuse
// rule picks atomics); computed once per (partition, NG) and kept in the
// index's spare bit.
int ensure_flags(alto_tensor *t, int mode, int NG, hipStream_t s) {
    Partition &P = *t->part;
    if (t->flag_bit[mode] < 0 || t->nnz == 0 || P.L == 0) return ALTO_OK;
    if ((double)t->nnz > 4.0 * (double)t->dims[mode]) return ALTO_OK;
    if (t->flag_L[mode] == P.L && t->flag_NG[mode] == NG) return ALTO_OK;
    if ((uint64_t)P.L * (uint64_t)NG >= 0xfffffffeull) return ALTO_OK;
    int rc = ensure_workspace(t, sizeof(uint32_t) * t->dims[mode]);
    if (rc) return rc;
    rc = launch_owner_flags(t->key_bits, t->keys, P.d_seg, P.L, NG, t->tab, t->ctab, mode, (uint32_t *)t->ws,
                            t->dims[mode], t->flag_bit[mode], s);
    if (rc) return rc;
    t->flags_in_keys = true;
    t->flag_L[mode] = P.L;
    t->flag_NG[mode] = NG;
    return ALTO_OK;
}

// Kernel timing for measurement (alto_timing_enable / alto_timing_read): an
// event pair per MTTKRP around its kernels, on the launch stream.
namespace {
using EventPair = std::pair<hipEvent_t, hipEvent_t>;
std::mutex g_tm_mu;
bool g_tm_on = false;
std::vector<EventPair> g_tm_pending, g_tm_free;

struct CallTimer {
    EventPair ev{nullptr, nullptr};
    bool active = false;
    CallTimer() = default;
    CallTimer(const CallTimer &) = delete;
    CallTimer &operator=(const CallTimer &) = delete;
    // a call that failed between begin and end gives its pair back unrecorded
    ~CallTimer() {
        if (!ev.first) return;
        if (active) {
            std::lock_guard<std::mutex> lk(g_tm_mu);
            g_tm_free.push_back(ev);
        }
    }
    int begin(hipStream_t s) {
        {
            std::lock_guard<std::mutex> lk(g_tm_mu);
            if (!g_tm_on) return ALTO_OK;
            if (!g_tm_free.empty()) {
                ev = g_tm_free.back();
                g_tm_free.pop_back();
            }
        }
        if (!ev.first) {
            ALTO_HIP(hipEventCreate(&ev.first));
            if (hipEventCreate(&ev.second) != hipSuccess) {
                (void)hipEventDestroy(ev.first);
                ev.first = nullptr;
                return set_error(ALTO_E_HIP, "hipEventCreate");
            }
        }
        active = true;  // from here the pair goes back to the pool on failure
        ALTO_HIP(hipEventRecord(ev.first, s));
        return ALTO_OK;
    }
    int end(hipStream_t s) {
        if (!active) return ALTO_OK;
        ALTO_HIP(hipEventRecord(ev.second, s));
        active = false;
        std::lock_guard<std::mutex> lk(g_tm_mu);
        g_tm_pending.push_back(ev);
        return ALTO_OK;
    }
};
}  // namespace

int plan_and_run_mttkrp(alto_tensor *t, const void *const *factors, int R, int prec, int mode, float *out,
                        const alto_exec *ex, hipStream_t s) {
    int rc = check_mttkrp_args(t, factors, R, prec, mode, out);
    if (rc) return rc;
    alto_exec plan;
    rc = resolve_strategy(t, factors, R, prec, mode, out, ex, s, &plan);
    if (rc) return rc;
    if (plan.num_segments > 0) {
        rc = select_partition(t, plan.num_segments, s);
        if (rc) return rc;
    }
    const uint64_t outn = t->dims[mode] * (uint64_t)R;
    ALTO_HIP(hipMemsetAsync(out, 0, sizeof(float) * outn, s));
    if (t->nnz == 0) return ALTO_OK;
    const bool sorted = plan.strategy == ALTO_STRATEGY_SORTED;
    if (sorted) {
        rc = build_mode_order(t, mode, s);
        if (rc) return rc;
    }
    SegLists *sl = nullptr;
    rc = build_lists(t, mode, sorted ? ALTO_STRATEGY_ATOMIC : plan.strategy, R, prec, &sl);
    if (rc) return rc;
    // the strategies that visit the nonzeros in linearized order accumulate
    // their atomic updates in FP64 (see mttkrp_k); the segment-local order
    // makes one FP32 atomic per (segment, row) run, directly into out
    const bool fp64 = !sorted;
    // per-XCD copies unless the output is large: the hot lines of a small or
    // skewed output would otherwise take the atomics of the whole GPU.  The
    // copies cost one clear and one read each (at most 0.1 ms at 256 MiB)
    const int nxcc = fp64 ? device_xcc_count() : 1;
    const int nacc = nxcc > 1 && (uint64_t)nxcc * outn * sizeof(double) <= ((uint64_t)256 << 20) ? nxcc : 1;
    const size_t acc_bytes = fp64 ? sizeof(double) * outn * nacc : 0;
    if (fp64 && t->acc64_bytes < acc_bytes) {
        if (t->acc64) ALTO_HIP(hipFree(t->acc64));
        t->acc64 = nullptr;
        t->acc64_bytes = 0;
        ALTO_HIP(hipMalloc(&t->acc64, acc_bytes));
        t->acc64_bytes = acc_bytes;
    }
    if (fp64) ALTO_HIP(hipMemsetAsync(t->acc64, 0, acc_bytes, s));
    MtLaunch a;
    rc = fill_mt_launch(t, factors, R, prec, mode, sorted, &a);
    if (rc) return rc;
    a.out = out;
    a.acc64 = fp64 ? t->acc64 : nullptr;
    a.acc_stride = outn;
    a.nacc = nacc;
    const int atomic_wg = a.threads;
    // helper flags for the launches that update the output with atomics on
    // the linearized order (ALTO_HELPER_FLAGS=0 turns them off)
    a.dec.fbit = -1;
    if (!sorted && sl->n_atomic > 0 && t->flag_bit[mode] >= 0 && env_long("ALTO_HELPER_FLAGS", 1) != 0) {
        const int G = mt_group_lanes(R, prec);
        rc = ensure_flags(t, mode, atomic_wg / G, s);
        if (rc) return rc;
        if (t->flag_L[mode] == t->part->L && t->flag_NG[mode] == atomic_wg / G) a.dec.fbit = t->flag_bit[mode];
    }
    auto run = [&](const int32_t *list, int n, int staged, int rows) -> int {
        a.list = list;
        a.n_list = n;
        a.staged = staged;
        a.temp_rows = rows;
        a.threads = staged ? staged_threads((size_t)rows * temp_stride(R) * 4) : atomic_wg;
        const int fbit = a.dec.fbit;
        if (staged) a.dec.fbit = -1;
        const int rc2 = launch_mt(a, t->key_bits, prec, s);
        a.dec.fbit = fbit;
        return rc2;
    };
    if (getenv("ALTO_DEBUG_PLAN"))
        fprintf(stderr, "[alto] mode %d R %d prec %d strategy %d L %d: atomic %d, staged %d/%d/%d (rows <= %d/%d/%d), fp64 %d, flags %d\n",
                mode, R, prec, plan.strategy, t->part->L, sl->n_atomic, sl->n_bucket[0], sl->n_bucket[1],
                sl->n_bucket[2], sl->w_bucket[0], sl->w_bucket[1], sl->w_bucket[2], (int)fp64, a.dec.fbit >= 0);
    const int32_t *p = sl->d;
    const int32_t *bucket_p = p + sl->n_atomic;
    CallTimer timer;
    rc = timer.begin(s);
    if (rc) return rc;
    for (int b = 0; b < SegLists::kBuckets; b++) {
        rc = run(bucket_p, sl->n_bucket[b], 1, sl->w_bucket[b]);
        if (rc) return rc;
        bucket_p += sl->n_bucket[b];
    }
    rc = run(p, sl->n_atomic, 0, 0);
    if (rc) return rc;
    if (fp64) {
        rc = launch_acc64_finish(out, t->acc64, outn, nacc, outn, s);
        if (rc) return rc;
    }
    return timer.end(s);
}

}  // namespace alto

using namespace alto;

extern "C" {

const char *alto_last_error(void) { return alto::g_err.c_str(); }

int alto_timing_enable(int enable) {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm_on = enable != 0;
    return ALTO_OK;
}

int alto_timing_read(double *ms_total, int64_t *calls) {
    if (!ms_total || !calls) return set_error(ALTO_E_INVAL, "null output pointer");
    std::vector<EventPair> pend;
    {
        std::lock_guard<std::mutex> lk(g_tm_mu);
        pend.swap(g_tm_pending);
    }
    double tot = 0.0;
    int rc = ALTO_OK;
    for (const EventPair &p : pend) {
        if (rc) break;
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
        if (e != hipSuccess) rc = hip_error(e, "alto_timing_read");
        tot += ms;
    }
    {
        std::lock_guard<std::mutex> lk(g_tm_mu);
        g_tm_free.insert(g_tm_free.end(), pend.begin(), pend.end());
    }
    *ms_total = tot;
    *calls = (int64_t)pend.size();
    return rc;
}

int alto_device_compute_units(void) { return cu_count(); }

int alto_build(const uint32_t *const *coords, const float *vals, int64_t nnz, const uint64_t *dims, int N,
               const alto_opts *opts, alto_tensor **out, hipStream_t s) {
    g_err.clear();
    if (!out || !dims) return set_error(ALTO_E_INVAL, "null dims or output handle pointer");
    *out = nullptr;
    if (N < 2 || N > kMaxModes) return set_error(ALTO_E_INVAL, "N must be in 2..8");
    if (nnz < 0) return set_error(ALTO_E_INVAL, "nnz must be >= 0");
    if (nnz > 0 && (!coords || !vals)) return set_error(ALTO_E_INVAL, "null coords or vals");
    for (int n = 0; n < N; n++) {
        if (dims[n] == 0 || dims[n] > (1ull << 32)) return set_error(ALTO_E_INVAL, "dims must be in 1..2^32");
        if (nnz > 0 && !coords[n]) return set_error(ALTO_E_INVAL, "null coordinate pointer");
    }
    alto_opts o{};
    if (opts) o = *opts;
    if (o.num_segments < 0) return set_error(ALTO_E_INVAL, "num_segments must be >= 0");
    alto_tensor *t = new alto_tensor();
    (void)hipGetDevice(&t->device);
    t->N = N;
    for (int n = 0; n < N; n++) t->dims[n] = dims[n];
    int rc = make_layout(t, o.key_bits);
    if (rc) {
        delete t;
        return rc;
    }
    t->nnz_in = nnz;
    t->nnz = nnz;
    const size_t kb = (size_t)t->key_bits / 8;
    void *keys_alt = nullptr, *dims_d = nullptr;
    float *vals_alt = nullptr;
    int *flag = nullptr;
    double *sums = nullptr;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(keys_alt);
        (void)hipFree(vals_alt);
        (void)hipFree(dims_d);
        (void)hipFree(flag);
        (void)hipFree(sums);
        alto_free(t);
        return code;
    };
#define ALTO_TRY(call)                                        \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return fail(hip_error(e_, #call)); \
    } while (0)
    if (nnz > 0) {
        ALTO_TRY(hipMalloc(&t->keys, kb * nnz));
        if (!t->h_ctab.empty()) {
            ALTO_TRY(hipMalloc(&t->ctab, t->h_ctab.size()));
            ALTO_TRY(hipMemcpyAsync(t->ctab, t->h_ctab.data(), t->h_ctab.size(), hipMemcpyHostToDevice, s));
        }
        if (!t->h_etab.empty()) {
            ALTO_TRY(hipMalloc(&t->etab, t->h_etab.size()));
            ALTO_TRY(hipMemcpyAsync(t->etab, t->h_etab.data(), t->h_etab.size(), hipMemcpyHostToDevice, s));
        }
        ALTO_TRY(hipMalloc(&t->vals, sizeof(float) * nnz));
        ALTO_TRY(hipMalloc(&keys_alt, kb * nnz));
        ALTO_TRY(hipMalloc(&vals_alt, sizeof(float) * nnz));
        ALTO_TRY(hipMalloc(&dims_d, sizeof(uint64_t) * kMaxModes));
        ALTO_TRY(hipMalloc(&flag, sizeof(int)));
        ALTO_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
        ALTO_TRY(hipMemcpyAsync(dims_d, t->dims, sizeof(uint64_t) * kMaxModes, hipMemcpyHostToDevice, s));
        ALTO_TRY(hipMemcpyAsync(t->vals, vals, sizeof(float) * nnz, hipMemcpyDeviceToDevice, s));
        CoordPtrs cp{};
        for (int n = 0; n < N; n++) cp.p[n] = coords[n];
        rc = launch_encode(t->key_bits, cp, (const uint64_t *)dims_d, nnz, t->tab, t->etab, t->keys, flag, s);
        if (rc) return fail(rc);
        int hflag = 0;
        ALTO_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        ALTO_TRY(hipStreamSynchronize(s));
        if (hflag) return fail(set_error(ALTO_E_RANGE, "a coordinate is not below its dimension"));
        rc = ensure_workspace(t, std::max(radix_sort_scratch(t->key_bits, nnz), coalesce_scratch(nnz)));
        if (rc) return fail(rc);
        bool in_alt = false;
        rc = radix_sort(t->key_bits, t->B, nnz, t->keys, t->vals, keys_alt, vals_alt, t->ws, t->ws_bytes, &in_alt, s);
        if (rc) return fail(rc);
        if (in_alt) {
            std::swap(t->keys, keys_alt);
            std::swap(t->vals, vals_alt);
        }
        int64_t nu = nnz;
        rc = coalesce(t->key_bits, nnz, t->keys, t->vals, keys_alt, vals_alt, t->ws, t->ws_bytes, &nu, s);
        if (rc) return fail(rc);
        if (nu != nnz) {
            std::swap(t->keys, keys_alt);
            std::swap(t->vals, vals_alt);
        }
        t->nnz = nu;
        ALTO_TRY(hipMalloc(&sums, sizeof(double) * 1025));
        rc = launch_sumsq(t->vals, t->nnz, sums, s);
        if (rc) return fail(rc);
        ALTO_TRY(hipMemcpyAsync(&t->norm2, sums + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
        ALTO_TRY(hipStreamSynchronize(s));
        (void)hipFree(keys_alt);
        (void)hipFree(vals_alt);
        (void)hipFree(dims_d);
        (void)hipFree(flag);
        (void)hipFree(sums);
        keys_alt = nullptr;
        vals_alt = nullptr;
        dims_d = nullptr;
        flag = nullptr;
        sums = nullptr;
    }
#undef ALTO_TRY
    rc = select_partition(t, o.num_segments, s);
    if (rc) return fail(rc);
    rc = compute_row_features(t, s);
    if (rc) return fail(rc);
    rc = noalloc_prepare_device();
    if (rc) return fail(rc);
    *out = t;
    return ALTO_OK;
}

int alto_layout(const uint64_t *dims, int N, int key_bits, alto_info_t *out) {
    g_err.clear();
    if (!dims || !out) return set_error(ALTO_E_INVAL, "null argument");
    if (N < 2 || N > kMaxModes) return set_error(ALTO_E_INVAL, "N must be in 2..8");
    for (int n = 0; n < N; n++)
        if (dims[n] == 0 || dims[n] > (1ull << 32)) return set_error(ALTO_E_INVAL, "dims must be in 1..2^32");
    alto_tensor t;
    t.N = N;
    for (int n = 0; n < N; n++) t.dims[n] = dims[n];
    const int rc = make_layout(&t, key_bits);
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    out->N = N;
    out->index_bits = t.B;
    out->key_bits = t.key_bits;
    for (int n = 0; n < N; n++) {
        out->dims[n] = dims[n];
        out->mode_bits[n] = t.nbits[n];
        out->mask_lo[n] = t.mask_lo[n];
        out->mask_hi[n] = t.mask_hi[n];
    }
    return ALTO_OK;
}

int alto_info(const alto_tensor *t, alto_info_t *out) {
    g_err.clear();
    if (!t || !out) return set_error(ALTO_E_INVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->N = t->N;
    out->index_bits = t->B;
    out->key_bits = t->key_bits;
    out->num_segments = t->part ? t->part->L : 0;
    out->nnz_in = t->nnz_in;
    out->nnz = t->nnz;
    for (int n = 0; n < t->N; n++) {
        out->dims[n] = t->dims[n];
        out->mode_bits[n] = t->nbits[n];
        out->mask_lo[n] = t->mask_lo[n];
        out->mask_hi[n] = t->mask_hi[n];
        out->fiber_reuse[n] = (double)t->nnz / (double)t->dims[n];
    }
    out->index_bytes = (double)t->nnz * t->key_bits / 8.0;
    out->coo_index_bytes = (double)t->nnz * t->N * 4.0;
    out->norm2 = t->norm2;
    const double kb = t->key_bits / 8.0;
    out->tensor_bytes = (double)t->nnz * (kb + 4.0) + (double)t->h_ctab.size() + (double)t->h_etab.size();
    auto part_bytes = [&](const Partition &p, double *orders) {
        double b = 8.0 * (p.L + 1) + 8.0 * p.L * t->N;
        for (int n = 0; n < t->N; n++) {
            if (p.d_cov[n]) b += 4.0 * (double)t->dims[n];
            if (p.okeys[n]) *orders += (double)t->nnz * (kb + 4.0);
        }
        for (const auto &kv : p.lists) {
            const SegLists &sl = kv.second;
            int n = sl.n_atomic;
            for (int q = 0; q < SegLists::kBuckets; q++) n += sl.n_bucket[q];
            b += 4.0 * std::max(1, n);
        }
        return b;
    };
    double orders = 0.0, parts = 0.0;
    if (t->part) parts += part_bytes(*t->part, &orders);
    for (const auto &p : t->spare) parts += part_bytes(*p, &orders);
    out->partition_bytes = parts;
    out->order_bytes = orders;
    out->scratch_bytes = (double)t->ws_bytes + (double)t->acc64_bytes;
    for (int n = 0; n < t->N; n++) out->flag_bit[n] = t->flag_bit[n];
    return ALTO_OK;
}

int alto_partition(alto_tensor *t, int num_segments, hipStream_t s) {
    g_err.clear();
    if (!t) return set_error(ALTO_E_INVAL, "null tensor handle");
    if (num_segments < 1) return set_error(ALTO_E_INVAL, "num_segments must be >= 1");
    return select_partition(t, num_segments, s);
}

int alto_mttkrp(alto_tensor *t, const void *const *factors, int R, int prec, int mode, float *out,
                const alto_exec *ex, hipStream_t s) {
    g_err.clear();
    return plan_and_run_mttkrp(t, factors, R, prec, mode, out, ex, s);
}

int alto_export_keys(const alto_tensor *t, void *keys_out, float *vals_out, hipStream_t s) {
    g_err.clear();
    if (!t) return set_error(ALTO_E_INVAL, "null tensor handle");
    if (t->nnz == 0) return ALTO_OK;
    if (keys_out) {
        // helper-flag bits are not part of the index
        if (t->flags_in_keys) {
            const int rc = launch_mask_keys(t->key_bits, t->keys, t->nnz, t->B, keys_out, s);
            if (rc) return rc;
        } else {
            ALTO_HIP(hipMemcpyAsync(keys_out, t->keys, (size_t)t->nnz * t->key_bits / 8, hipMemcpyDeviceToDevice, s));
        }
    }
    if (vals_out) ALTO_HIP(hipMemcpyAsync(vals_out, t->vals, sizeof(float) * t->nnz, hipMemcpyDeviceToDevice, s));
    return ALTO_OK;
}

int alto_export_flags(const alto_tensor *t, int mode, uint8_t *flags_out, int *lane_groups, hipStream_t s) {
    g_err.clear();
    if (!t) return set_error(ALTO_E_INVAL, "null tensor handle");
    if (mode < 0 || mode >= t->N) return set_error(ALTO_E_INVAL, "mode out of range");
    if (t->flag_bit[mode] < 0 || t->flag_L[mode] == 0 || !t->part || t->flag_L[mode] != t->part->L)
        return set_error(ALTO_E_STATE, "no helper flags of this mode for the current partition");
    if (lane_groups) *lane_groups = t->flag_NG[mode];
    if (t->nnz > 0 && flags_out) return launch_get_flags(t->key_bits, t->keys, t->nnz, t->flag_bit[mode], flags_out, s);
    return ALTO_OK;
}

int alto_export_mode_order(alto_tensor *t, int mode, void *keys_out, float *vals_out, hipStream_t s) {
    g_err.clear();
    int rc = check_tensor(t);
    if (rc) return rc;
    if (mode < 0 || mode >= t->N) return set_error(ALTO_E_INVAL, "mode out of range");
    if (t->nnz == 0) return ALTO_OK;
    rc = build_mode_order(t, mode, s);
    if (rc) return rc;
    const Partition &P = *t->part;
    if (keys_out) {
        if (t->key_bits <= 64) {
            rc = launch_expand_keys(t->key_bits, P.okeys[mode], t->nnz, t->tab, keys_out, s);
            if (rc) return rc;
        } else if (t->flags_in_keys) {
            rc = launch_mask_keys(t->key_bits, P.okeys[mode], t->nnz, t->B, keys_out, s);
            if (rc) return rc;
        } else {
            ALTO_HIP(hipMemcpyAsync(keys_out, P.okeys[mode], (size_t)t->nnz * t->key_bits / 8,
                                    hipMemcpyDeviceToDevice, s));
        }
    }
    if (vals_out) ALTO_HIP(hipMemcpyAsync(vals_out, P.ovals[mode], sizeof(float) * t->nnz, hipMemcpyDeviceToDevice, s));
    return ALTO_OK;
}

int alto_export_partition(const alto_tensor *t, int64_t *seg_out, uint32_t *ivl_out, hipStream_t s) {
    g_err.clear();
    if (!t) return set_error(ALTO_E_INVAL, "null tensor handle");
    const int L = t->part->L;
    if (seg_out)
        ALTO_HIP(hipMemcpyAsync(seg_out, t->part->d_seg, sizeof(int64_t) * (L + 1), hipMemcpyDeviceToDevice, s));
    if (ivl_out && L > 0)
        ALTO_HIP(hipMemcpyAsync(ivl_out, t->part->d_ivl, sizeof(uint32_t) * L * t->N * 2, hipMemcpyDeviceToDevice, s));
    return ALTO_OK;
}

int alto_export_coverage(const alto_tensor *t, int mode, uint32_t *cov_out, hipStream_t s) {
    g_err.clear();
    if (!t || !cov_out) return set_error(ALTO_E_INVAL, "null argument");
    if (mode < 0 || mode >= t->N) return set_error(ALTO_E_INVAL, "mode out of range");
    ALTO_HIP(hipMemcpyAsync(cov_out, t->part->d_cov[mode], sizeof(uint32_t) * t->dims[mode], hipMemcpyDeviceToDevice, s));
    return ALTO_OK;
}

int cp_als(alto_tensor *t, int R, int iters, int prec, void *const *factors, double *lambda, double *fit,
           const alto_exec *ex, hipStream_t s) {
    g_err.clear();
    return cp_als_impl(t, R, iters, prec, factors, lambda, fit, ex, s);
}

int alto_round_bf16(const double *in, uint16_t *out, int64_t n, hipStream_t s) {
    g_err.clear();
    if (n < 0 || (n > 0 && (!in || !out))) return set_error(ALTO_E_INVAL, "bad arguments");
    return launch_round_bf16(in, out, n, s);
}

void alto_free(alto_tensor *t) {
    if (!t) return;
    (void)hipDeviceSynchronize();
    t->part.reset();
    t->spare.clear();
    (void)hipFree(t->acc64);
    (void)hipFree(t->keys);
    (void)hipFree(t->ctab);
    (void)hipFree(t->etab);
    (void)hipFree(t->vals);
    (void)hipFree(t->ws);
    delete t;
}

int alto_mlp_forward(int B, int F, int H, int K, const float *params, const float *x, const float *t, const float *mask,
                     float *y, float *loss, hipStream_t s) {
    g_err.clear();
    return mlp_forward(B, F, H, K, params, x, t, mask, y, loss, s);
}

int alto_mlp_backward(int B, int F, int H, int K, const float *params, const float *x, const float *t,
                      const float *mask, float *grads, float *loss, hipStream_t s) {
    g_err.clear();
    return mlp_backward(B, F, H, K, params, x, t, mask, grads, loss, s);
}

int alto_mlp_adam(int64_t P, float *params, const float *grads, float *m, float *v, float lr, float beta1, float beta2,
                  float eps, int t, hipStream_t s) {
    g_err.clear();
    return mlp_adam(P, params, grads, m, v, lr, beta1, beta2, eps, t, s);
}

}  // extern "C"
