// Format generation on the device (Section 3.1 and 3.2 of the ALTO paper):
// linearization (bit-level gather), ordering by the linearized index (LSD
// radix sort over the B meaningful bits), coalescing of repeated positions,
// mode intervals of the equal-nonzero line segments and per-row coverage.
#include "common.h"

namespace alto {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a 256-thread block.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total, T *lds /* kWaves */) {
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    T x = wave_inclusive_scan(v);
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
        const T s = lds[w];
        if (w < wave) before += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

// ------------------------------------------------------------ generic scan
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kThreads) void scan_reduce_k(const TIn *in, int64_t n, TOut *bsum) {
    __shared__ TOut lds[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    TOut s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++)
        if (base + j < n) s += (TOut)in[base + j];
    TOut tot;
    block_exclusive_scan(s, &tot, lds);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// In-place exclusive scan of nb block sums by one block; writes the grand total.
template <typename TOut>
__global__ __launch_bounds__(kThreads) void scan_top_k(TOut *bsum, int64_t nb, TOut *total) {
    __shared__ TOut lds[kWaves];
    TOut carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
        const int64_t b = b0 + threadIdx.x;
        const TOut v = b < nb ? bsum[b] : (TOut)0;
        TOut tot;
        const TOut ex = block_exclusive_scan(v, &tot, lds);
        if (b < nb) bsum[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename TIn, typename TOut, bool kInclusive>
__global__ __launch_bounds__(kThreads) void scan_down_k(const TIn *in, int64_t n, const TOut *boff, TOut *out) {
    __shared__ TOut lds[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    TOut v[kScanItems];
    TOut s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        v[j] = base + j < n ? (TOut)in[base + j] : (TOut)0;
        s += v[j];
    }
    TOut tot;
    TOut run = block_exclusive_scan(s, &tot, lds) + boff[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        if (kInclusive) run += v[j];
        if (base + j < n) out[base + j] = run;
        if (!kInclusive) run += v[j];
    }
}

template <typename TIn, typename TOut, bool kInclusive>
size_t scan_bytes(int64_t n) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(TOut) + 256;
}

// scratch must hold scan_bytes(n); total (device, may be null) gets the sum.
template <typename TIn, typename TOut, bool kInclusive>
int device_scan(const TIn *in, TOut *out, int64_t n, TOut *total, void *scratch, hipStream_t s) {
    if (n <= 0) {
        if (total) ALTO_HIP(hipMemsetAsync(total, 0, sizeof(TOut), s));
        return ALTO_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    TOut *bsum = (TOut *)scratch;
    scan_reduce_k<TIn, TOut><<<(unsigned)nb, kThreads, 0, s>>>(in, n, bsum);
    scan_top_k<TOut><<<1, kThreads, 0, s>>>(bsum, nb, total);
    scan_down_k<TIn, TOut, kInclusive><<<(unsigned)nb, kThreads, 0, s>>>(in, n, bsum, out);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

// ------------------------------------------------------------ encode
template <typename K>
__global__ __launch_bounds__(kThreads) void encode_k(CoordPtrs c, const uint64_t *__restrict__ dims, int64_t n,
                                                     RunTable tab, K *__restrict__ keys, int *flag) {
    const int N = tab.N;
    uint64_t dm[kMaxModes];
#pragma unroll
    for (int m = 0; m < kMaxModes; m++) dm[m] = m < N ? dims[m] : 0;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        K key = KeyOps<K>::zero();
        bool bad = false;
#pragma unroll
        for (int m = 0; m < kMaxModes; m++) {
            if (m >= N) break;
            const uint32_t v = c.p[m][x];
            bad |= (uint64_t)v >= dm[m];
            const int nr = tab.nruns[m];
            for (int q = 0; q < nr; q++) {
                const uint32_t r = tab.run[m][q];
                const uint32_t bits = (uint32_t)(((uint64_t)v >> run_cpos(r)) & ((1ull << run_len(r)) - 1));
                KeyOps<K>::deposit(key, bits, run_kpos(r));
            }
        }
        if (bad) atomicOr(flag, 1);
        keys[x] = key;
    }
}

__device__ __forceinline__ void key_or(uint32_t &a, uint32_t b) { a |= b; }
__device__ __forceinline__ void key_or(uint64_t &a, uint64_t b) { a |= b; }
__device__ __forceinline__ void key_or(u128 &a, const u128 &b) {
    a.lo |= b.lo;
    a.hi |= b.hi;
}

// The same linearization through the deposit tables, staged in LDS once per
// block: one table entry per coordinate byte, OR-ed into the index.  The
// grid is capped so that every block streams many nonzeros.
template <typename K>
__global__ __launch_bounds__(kThreads) void encode_tab_k(CoordPtrs c, const uint64_t *__restrict__ dims, int64_t n,
                                                         RunTable tab, const K *__restrict__ etab,
                                                         K *__restrict__ keys, int *flag) {
    extern __shared__ __align__(16) char dyn[];
    K *const lt = reinterpret_cast<K *>(dyn);
    for (int q = threadIdx.x; q < tab.etab_entries; q += kThreads) lt[q] = etab[q];
    __syncthreads();
    const int N = tab.N;
    uint64_t dm[kMaxModes];
#pragma unroll
    for (int m = 0; m < kMaxModes; m++) dm[m] = m < N ? dims[m] : 0;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        K key = KeyOps<K>::zero();
        bool bad = false;
#pragma unroll
        for (int m = 0; m < kMaxModes; m++) {
            if (m >= N) break;
            const uint32_t v = c.p[m][x];
            bad |= (uint64_t)v >= dm[m];
            const K *tm = lt + tab.eoff[m];
            const int nb = tab.ebytes[m];
            for (int j = 0; j < nb; j++) key_or(key, tm[j * 256 + (int)((v >> (8 * j)) & 0xffu)]);
        }
        if (bad) atomicOr(flag, 1);
        keys[x] = key;
    }
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort, 8-bit digits.  Each block owns one tile of
// threads*ITEMS keys, split into one chunk of 64*ITEMS keys per wave;
// inside a wave, item j covers keys j*64 .. j*64+63 of the chunk.  A key's
// rank among equal digits comes from a ballot match over the 64 lanes plus a
// per-wave running counter, which keeps input order (stability) without
// atomics.

// Exclusive scan of 256 counters by one wave (4 per lane); returns the total.
__device__ __forceinline__ uint32_t wave_exclusive_scan256(const uint32_t *in, uint32_t *out, int lane) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        v[q] = in[lane * 4 + q];
        sum += v[q];
    }
    uint32_t inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off) inc += y;
    }
    uint32_t run = inc - sum;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        out[lane * 4 + q] = run;
        run += v[q];
    }
    return run;
}

// 512-thread blocks for keys of up to 64 bits, 256 for 128-bit keys (whose
// tile would otherwise not leave room for two blocks per CU)
template <typename K>
struct SortCfg {
    static constexpr int kThreads = sizeof(K) > 8 ? 256 : 512;
    static constexpr int kWaves = kThreads / 64;
    static constexpr int kItems = 8;
    static constexpr int kTile = kThreads * kItems;
};

__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

template <typename K>
__global__ __launch_bounds__(SortCfg<K>::kThreads) void rs_hist_k(const K *__restrict__ keys, int64_t n, int shift,
                                                                   uint32_t *__restrict__ hist, int64_t T) {
    constexpr int I = SortCfg<K>::kItems, NT = SortCfg<K>::kThreads, NW = SortCfg<K>::kWaves;
    __shared__ uint32_t cnt[NW][256];
    for (int q = threadIdx.x; q < NW * 256; q += NT) (&cnt[0][0])[q] = 0;
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const int64_t base = (int64_t)blockIdx.x * SortCfg<K>::kTile + (int64_t)wave * 64 * I;
    for (int j = 0; j < I; j++) {
        const int64_t x = base + (int64_t)j * 64 + lane;
        const bool valid = x < n;
        const uint32_t d = valid ? KeyOps<K>::digit(keys[x], shift) : 0u;
        const uint64_t m = match_digit(d, valid);
        if (valid && lane == (int)__builtin_ctzll(m)) cnt[wave][d] += (uint32_t)__builtin_popcountll(m);
    }
    __syncthreads();
    const int d = threadIdx.x;
    if (d < 256) {
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) tot += cnt[w][d];
        hist[(int64_t)d * T + blockIdx.x] = tot;
    }
}

template <typename K>
__global__ __launch_bounds__(SortCfg<K>::kThreads) void rs_scatter_k(const K *__restrict__ kin, const float *__restrict__ vin,
                                                         K *__restrict__ kout, float *__restrict__ vout, int64_t n,
                                                         int shift, const uint64_t *__restrict__ offs, int64_t T) {
    constexpr int I = SortCfg<K>::kItems;
    constexpr int TILE = SortCfg<K>::kTile, NT = SortCfg<K>::kThreads, NW = SortCfg<K>::kWaves;
    __shared__ uint32_t cnt[NW][256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t dtot[256];
    __shared__ uint64_t gbase[256];
    __shared__ K skeys[TILE];
    __shared__ float svals[TILE];

    for (int q = threadIdx.x; q < NW * 256; q += NT) (&cnt[0][0])[q] = 0;
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)wave * 64 * I;
    K k[I];
    float v[I];
    uint32_t dg[I], rk[I];
    const uint64_t lt = lanemask_lt();
    for (int j = 0; j < I; j++) {
        const int64_t x = base + (int64_t)j * 64 + lane;
        const bool valid = x < n;
        if (valid) {
            k[j] = kin[x];
            v[j] = vin[x];
        } else {
            k[j] = KeyOps<K>::zero();
            v[j] = 0.f;
        }
        const uint32_t d = valid ? KeyOps<K>::digit(k[j], shift) : 0u;
        const uint64_t m = match_digit(d, valid);
        const uint32_t before = cnt[wave][d];  // every lane reads before the leader writes
        rk[j] = before + (uint32_t)__builtin_popcountll(m & lt);
        dg[j] = valid ? d : 0xffffffffu;
        __builtin_amdgcn_wave_barrier();
        if (valid && lane == (int)__builtin_ctzll(m)) cnt[wave][d] = before + (uint32_t)__builtin_popcountll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint32_t c = cnt[w][d];
            cnt[w][d] = run;
            run += c;
        }
        dtot[d] = run;
        gbase[d] = offs[(int64_t)d * T + blockIdx.x];
    }
    __syncthreads();
    if (wave == 0) wave_exclusive_scan256(dtot, tstart, lane);
    __syncthreads();
    for (int j = 0; j < I; j++) {
        if (dg[j] == 0xffffffffu) continue;
        const uint32_t pos = tstart[dg[j]] + cnt[wave][dg[j]] + rk[j];
        skeys[pos] = k[j];
        svals[pos] = v[j];
    }
    __syncthreads();
    const int64_t nvalid = min((int64_t)TILE, n - (int64_t)blockIdx.x * TILE);
    for (int i = threadIdx.x; i < nvalid; i += NT) {
        const K key = skeys[i];
        const uint32_t d = KeyOps<K>::digit(key, shift);
        const uint64_t dst = gbase[d] + (uint64_t)(i - (int)tstart[d]);
        kout[dst] = key;
        vout[dst] = svals[i];
    }
}

template <typename K>
int radix_sort_t(int nbits, int64_t n, K *keys, float *vals, K *keys_alt, float *vals_alt, void *scratch,
                 bool *in_alt, hipStream_t s) {
    *in_alt = false;
    if (n <= 1 || nbits <= 0) return ALTO_OK;
    const int passes = (nbits + 7) / 8;
    const int64_t T = (n + SortCfg<K>::kTile - 1) / SortCfg<K>::kTile;
    uint32_t *hist = (uint32_t *)scratch;
    uint64_t *offs = (uint64_t *)((char *)scratch + ((256 * T * sizeof(uint32_t) + 255) & ~(size_t)255));
    void *scan_ws = (char *)offs + ((256 * T * sizeof(uint64_t) + 255) & ~(size_t)255);
    K *src_k = keys, *dst_k = keys_alt;
    float *src_v = vals, *dst_v = vals_alt;
    for (int p = 0; p < passes; p++) {
        const int shift = 8 * p;
        rs_hist_k<K><<<(unsigned)T, SortCfg<K>::kThreads, 0, s>>>(src_k, n, shift, hist, T);
        int rc = device_scan<uint32_t, uint64_t, false>(hist, offs, 256 * T, nullptr, scan_ws, s);
        if (rc) return rc;
        rs_scatter_k<K><<<(unsigned)T, SortCfg<K>::kThreads, 0, s>>>(src_k, src_v, dst_k, dst_v, n, shift, offs, T);
        ALTO_HIP(hipGetLastError());
        std::swap(src_k, dst_k);
        std::swap(src_v, dst_v);
    }
    *in_alt = (passes & 1) != 0;
    return ALTO_OK;
}

// ------------------------------------------------------------ coalesce
template <typename K>
__device__ __forceinline__ bool is_head(const K *keys, int64_t x) {
    return x == 0 || !KeyOps<K>::eq(keys[x], keys[x - 1]);
}

// Tiles of kScanTile positions; inside a tile, wave w owns positions
// w*1024 .. w*1024+1023 and item j of a wave covers j*64 .. j*64+63, so every
// load is a coalesced 64-wide read.
template <typename K>
__global__ __launch_bounds__(kThreads) void head_count_k(const K *__restrict__ keys, int64_t n, uint32_t *bcount) {
    __shared__ uint32_t lds[kWaves];
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)wave * 64 * kScanItems;
    uint32_t c = 0;
    for (int j = 0; j < kScanItems; j++) {
        const int64_t x = base + (int64_t)j * 64 + lane;
        if (x < n && is_head(keys, x)) c++;
    }
    uint32_t tot;
    block_exclusive_scan(c, &tot, lds);
    if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

template <typename K>
__global__ __launch_bounds__(kThreads) void compact_k(const K *__restrict__ keys, const float *__restrict__ vals,
                                                      int64_t n, const uint64_t *__restrict__ boff,
                                                      K *__restrict__ kout, float *__restrict__ vout) {
    __shared__ uint32_t wtot[kWaves];
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)wave * 64 * kScanItems;
    const uint64_t lt = lanemask_lt();
    uint32_t heads = 0;
    for (int j = 0; j < kScanItems; j++) {
        const int64_t x = base + (int64_t)j * 64 + lane;
        heads += (uint32_t)__builtin_popcountll(__ballot(x < n && is_head(keys, x)));
    }
    if (lane == 0) wtot[wave] = heads;
    __syncthreads();
    uint64_t pos = boff[blockIdx.x];
    for (int w = 0; w < wave; w++) pos += wtot[w];
    for (int j = 0; j < kScanItems; j++) {
        const int64_t x = base + (int64_t)j * 64 + lane;
        const bool h = x < n && is_head(keys, x);
        const uint64_t m = __ballot(h);
        if (h) {
            const uint64_t p = pos + (uint64_t)__builtin_popcountll(m & lt);
            const K key = keys[x];
            float sum = vals[x];
            for (int64_t y = x + 1; y < n && KeyOps<K>::eq(keys[y], key); y++) sum += vals[y];
            kout[p] = key;
            vout[p] = sum;
        }
        pos += (uint64_t)__builtin_popcountll(m);
    }
}

// ------------------------------------------------------------ intervals
template <typename K>
__global__ __launch_bounds__(kThreads) void intervals_k(const K *__restrict__ keys, const int64_t *__restrict__ seg,
                                                        RunTable tab, const K *__restrict__ ctab,
                                                        uint32_t *__restrict__ ivl) {
    constexpr int kTab = byte_table_entries(8 * (int)sizeof(K));
    __shared__ uint32_t smn[kWaves][kMaxModes], smx[kWaves][kMaxModes];
    __shared__ K ltab[kTab > 0 ? kTab : 1];
    const int l = blockIdx.x;
    const int N = tab.N;
    const int64_t b = seg[l], e = seg[l + 1];
    if constexpr (kTab > 0) {
        for (int q = threadIdx.x; q < kTab; q += kThreads) ltab[q] = ctab[q];
        __syncthreads();
    }
    uint32_t mn[kMaxModes], mx[kMaxModes];
#pragma unroll
    for (int m = 0; m < kMaxModes; m++) {
        mn[m] = 0xffffffffu;
        mx[m] = 0u;
    }
    for (int64_t x = b + threadIdx.x; x < e; x += kThreads) {
        const K key = keys[x];
        K cw{};
        if constexpr (kTab > 0) cw = compact_index(key, ltab);
#pragma unroll
        for (int m = 0; m < kMaxModes; m++) {
            if (m >= N) break;
            uint32_t c;
            if constexpr (kTab > 0) c = (uint32_t)(cw >> tab.coff[m]) & tab.cmask[m];
            else c = extract_mode(key, tab, m);
            mn[m] = min(mn[m], c);
            mx[m] = max(mx[m], c);
        }
    }
    const int lane = __lane_id(), wave = threadIdx.x / 64;
#pragma unroll
    for (int m = 0; m < kMaxModes; m++) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            mn[m] = min(mn[m], (uint32_t)__shfl_xor((int)mn[m], off));
            mx[m] = max(mx[m], (uint32_t)__shfl_xor((int)mx[m], off));
        }
        if (lane == 0) {
            smn[wave][m] = mn[m];
            smx[wave][m] = mx[m];
        }
    }
    __syncthreads();
    if (threadIdx.x < N) {
        const int m = threadIdx.x;
        uint32_t a = 0xffffffffu, z = 0u;
        for (int w = 0; w < kWaves; w++) {
            a = min(a, smn[w][m]);
            z = max(z, smx[w][m]);
        }
        ivl[((int64_t)l * N + m) * 2 + 0] = a;
        ivl[((int64_t)l * N + m) * 2 + 1] = z;
    }
}

// ------------------------------------------------------------ mode ordering
// Segment-local order by one mode: inside every line segment, a stable
// reordering of the nonzeros by their coordinate along `mode` (ties keep the
// linearized order).  One 1024-thread workgroup per segment runs an LSD radix
// sort on the coordinate's bits alone (the segments are already contiguous)
// with the index and value as payload: every pass reads its input in order
// and writes runs of one digit contiguously after reordering a tile in LDS,
// and the last pass lands in the output arrays.
constexpr int kSoThreads = 1024;
constexpr int kSoWaves = kSoThreads / 64;
constexpr int kSoItems = 4;
constexpr int kSoTile = kSoThreads * kSoItems;

template <typename K>
constexpr size_t seg_order_lds() {
    return (size_t)kSoTile * (sizeof(uint32_t) + sizeof(K) + sizeof(float));
}


// Buffers: rows R[2][n]; index and values alternate between the output
// (okeys, ovals) and one scratch pair (ks, vs), chosen so that the last pass
// writes the output.
template <typename K>
__global__ __launch_bounds__(kSoThreads) void seg_order_k(const K *__restrict__ keys, const float *__restrict__ vals,
                                                          const int64_t *__restrict__ seg, RunTable tab,
                                                          const K *__restrict__ ctab, int mode, int nbits,
                                                          uint32_t *__restrict__ R0, uint32_t *__restrict__ R1,
                                                          K *__restrict__ ks, float *__restrict__ vs,
                                                          K *__restrict__ okeys, float *__restrict__ ovals) {
    constexpr int kTab = byte_table_entries(8 * (int)sizeof(K));
    static_assert(kTab * sizeof(K) <= seg_order_lds<K>(), "byte tables fit the staging buffer");
    __shared__ uint32_t cnt[kSoWaves][256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t tot[256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t hist[256];
    // staging of one tile in digit order; the byte tables use the same memory
    // while the rows are decoded
    extern __shared__ __align__(16) char dyn[];
    K *const ltab = reinterpret_cast<K *>(dyn);
    K *const sk = reinterpret_cast<K *>(dyn);
    uint32_t *const sr = reinterpret_cast<uint32_t *>(dyn + (size_t)kSoTile * sizeof(K));
    float *const sv = reinterpret_cast<float *>(dyn + (size_t)kSoTile * (sizeof(K) + sizeof(uint32_t)));
    const int64_t sb = seg[blockIdx.x], n = seg[blockIdx.x + 1] - sb;
    const int passes = (nbits + 7) / 8;
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    if (passes == 0) {  // a one-row mode: the order is the linearized one
        for (int64_t i = threadIdx.x; i < n; i += kSoThreads) {
            okeys[sb + i] = keys[sb + i];
            ovals[sb + i] = vals[sb + i];
        }
        return;
    }
    // pass p reads (R[p&1], D_p) and writes (R[(p+1)&1], D_{p+1}); D_0 is the
    // tensor itself, D_passes the output, and D_p for 0 < p < passes the
    // output or the scratch pair, alternating
    K *Dk[2] = {okeys, ks};
    float *Dv[2] = {ovals, vs};
    auto dk = [&](int p) -> K * { return Dk[(passes - p) & 1]; };
    auto dv = [&](int p) -> float * { return Dv[(passes - p) & 1]; };
    uint32_t *Rr[2] = {R0, R1};
    // decode the rows into the pass-0 input; the histogram of the first digit on the way
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
    if constexpr (kTab > 0)
        for (int q = threadIdx.x; q < kTab; q += kSoThreads) ltab[q] = ctab[q];
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += kSoThreads) {
        const K key = keys[sb + i];
        uint32_t row;
        if constexpr (kTab > 0) row = (uint32_t)(compact_index(key, ltab) >> tab.coff[mode]) & tab.cmask[mode];
        else row = extract_mode(key, tab, mode);
        Rr[0][sb + i] = row;
        atomicAdd(&hist[row & 255u], 1u);
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    for (int p = 0; p < passes; p++) {
        const int shift = 8 * p;
        const bool last = p == passes - 1;
        const uint32_t *srow = Rr[p & 1];
        uint32_t *drow = Rr[(p + 1) & 1];
        const K *skey = p == 0 ? keys : dk(p);
        const float *sval = p == 0 ? vals : dv(p);
        K *dkey = dk(p + 1);
        float *dval = dv(p + 1);
        // exclusive scan of this digit's histogram; the next digit's is
        // counted while this pass writes
        if (wave == 0) {
            wave_exclusive_scan256(hist, base, lane);
#pragma unroll
            for (int q = 0; q < 4; q++) hist[lane * 4 + q] = 0;
        }
        __syncthreads();
        // stable scatter, one tile at a time in input order: within a tile,
        // wave w owns items [w*64*I, (w+1)*64*I), item j of a lane is
        // w*64*I + j*64 + lane
        for (int64_t t0 = 0; t0 < n; t0 += kSoTile) {
            uint32_t r[kSoItems], dg[kSoItems], rk[kSoItems];
            K kk[kSoItems];
            float vv[kSoItems];
#pragma unroll
            for (int j = 0; j < kSoItems; j++) {
                const int64_t x = t0 + (int64_t)wave * 64 * kSoItems + j * 64 + lane;
                const bool valid = x < n;
                r[j] = valid ? srow[sb + x] : 0u;
                kk[j] = valid ? skey[sb + x] : KeyOps<K>::zero();
                vv[j] = valid ? sval[sb + x] : 0.f;
            }
            for (int q = threadIdx.x; q < kSoWaves * 256; q += kSoThreads) (&cnt[0][0])[q] = 0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kSoItems; j++) {
                const int64_t x = t0 + (int64_t)wave * 64 * kSoItems + j * 64 + lane;
                const bool valid = x < n;
                const uint32_t d = (r[j] >> shift) & 255u;
                const uint64_t m = match_digit(d, valid);
                const uint32_t before = cnt[wave][d];  // every lane reads before the leader writes
                rk[j] = before + (uint32_t)__builtin_popcountll(m & lt);
                dg[j] = valid ? d : 0xffffffffu;
                __builtin_amdgcn_wave_barrier();
                if (valid && lane == (int)__builtin_ctzll(m)) cnt[wave][d] = before + (uint32_t)__builtin_popcountll(m);
                __builtin_amdgcn_wave_barrier();
            }
            __syncthreads();
            if (threadIdx.x < 256) {
                uint32_t run = 0;
#pragma unroll
                for (int w = 0; w < kSoWaves; w++) {
                    const uint32_t c = cnt[w][threadIdx.x];
                    cnt[w][threadIdx.x] = run;
                    run += c;
                }
                tot[threadIdx.x] = run;
            }
            __syncthreads();
            if (wave == 0) wave_exclusive_scan256(tot, tstart, lane);  // tile-local start of every digit
            __syncthreads();
            // the tile in digit order in LDS, then runs of one digit written out contiguously
#pragma unroll
            for (int j = 0; j < kSoItems; j++) {
                if (dg[j] == 0xffffffffu) continue;
                const uint32_t lp = tstart[dg[j]] + cnt[wave][dg[j]] + rk[j];
                sr[lp] = r[j];
                sk[lp] = kk[j];
                sv[lp] = vv[j];
            }
            __syncthreads();
            const int tn = (int)min((int64_t)kSoTile, n - t0);
            for (int i = threadIdx.x; i < tn; i += kSoThreads) {
                const uint32_t row = sr[i];
                const uint32_t d = (row >> shift) & 255u;
                const int64_t dst = sb + base[d] + (uint32_t)i - tstart[d];
                dkey[dst] = sk[i];
                dval[dst] = sv[i];
                if (!last) {
                    drow[dst] = row;
                    atomicAdd(&hist[(row >> (shift + 8)) & 255u], 1u);
                }
            }
            __syncthreads();
            if (threadIdx.x < 256) base[threadIdx.x] += tot[threadIdx.x];
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------ coverage
__global__ __launch_bounds__(kThreads) void coverage_marks_k(const uint32_t *__restrict__ ivl, int L, int N, int mode,
                                                             int32_t *__restrict__ diff) {
    const int l = blockIdx.x * kThreads + threadIdx.x;
    if (l >= L) return;
    const uint32_t s = ivl[((int64_t)l * N + mode) * 2 + 0];
    const uint32_t e = ivl[((int64_t)l * N + mode) * 2 + 1];
    if (s > e) return;  // an empty range of nonzeros has no interval (it reads as [2^32-1, 0])
    atomicAdd(&diff[s], 1);
    atomicAdd(&diff[(uint64_t)e + 1], -1);
}

// ------------------------------------------------------------ sum of squares
constexpr int kSumBlocks = 1024;

__global__ __launch_bounds__(kThreads) void sumsq_partial_k(const float *__restrict__ v, int64_t n, double *part) {
    __shared__ double lds[kWaves];
    double s = 0.0;
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        const double a = (double)v[x];
        s += a * a;
    }
    double tot;
    block_exclusive_scan(s, &tot, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void sum_partials_k(const double *part, int n, double *out) {
    __shared__ double lds[kWaves];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += kThreads) s += part[q];
    double tot;
    block_exclusive_scan(s, &tot, lds);
    if (threadIdx.x == 0) *out = tot;
}

unsigned grid_for(int64_t n, int per_block) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

}  // namespace

// ------------------------------------------------------------ helper flags
template <typename K>
__device__ __forceinline__ K with_bit(K k, int pos, bool v) {
    const K b = (K)1 << pos;
    return v ? (k | b) : (k & ~b);
}
template <>
__device__ __forceinline__ u128 with_bit<u128>(u128 k, int pos, bool v) {
    uint64_t &w = pos < 64 ? k.lo : k.hi;
    const uint64_t b = 1ull << (pos & 63);
    w = v ? (w | b) : (w & ~b);
    return k;
}

// Exact helper flags.  Segment l (one workgroup) of S nonzeros is cut
// into NG lane-group ranges as the MTTKRP kernel cuts it: offset o of the
// segment belongs to group floor(((o + 1) * NG - 1) / S).  Every nonzero
// claims its row for its range (l * NG + g); a row claimed by two ranges
// becomes kConflict.  A nonzero is then internal iff its row's owner is its
// own range.
constexpr uint32_t kOwnerEmpty = 0xffffffffu, kOwnerConflict = 0xfffffffeu;

template <typename K, bool kMark>
__global__ __launch_bounds__(kThreads) void owner_k(K *__restrict__ keys, const int64_t *__restrict__ seg, int NG,
                                                    RunTable tab, const K *__restrict__ ctab, int mode,
                                                    uint32_t *__restrict__ owner, int fbit) {
    constexpr int kTab = byte_table_entries(8 * (int)sizeof(K));
    __shared__ K lt[kTab > 0 ? kTab : 1];
    if constexpr (kTab > 0) {
        for (int q = threadIdx.x; q < kTab; q += kThreads) lt[q] = ctab[q];
        __syncthreads();
    }
    const int l = blockIdx.x;
    const int64_t sb = seg[l], S = seg[l + 1] - sb;
    for (int64_t o = threadIdx.x; o < S; o += kThreads) {
        const K key = keys[sb + o];
        uint32_t row;
        if constexpr (kTab > 0) row = (uint32_t)(compact_index(key, lt) >> tab.coff[mode]) & tab.cmask[mode];
        else row = extract_mode(key, tab, mode);
        const uint32_t chunk = (uint32_t)l * (uint32_t)NG + (uint32_t)(((o + 1) * NG - 1) / S);
        if constexpr (kMark) {
            keys[sb + o] = with_bit(key, fbit, owner[row] == chunk);
        } else {
            const uint32_t prev = atomicCAS(&owner[row], kOwnerEmpty, chunk);
            if (prev != kOwnerEmpty && prev != chunk) atomicExch(&owner[row], kOwnerConflict);
        }
    }
}

template <typename K>
__global__ __launch_bounds__(kThreads) void mask_keys_k(const K *__restrict__ keys, int64_t n, K keep,
                                                         K *__restrict__ out) {
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads)
        out[x] = keys[x] & keep;
}
template <>
__global__ __launch_bounds__(kThreads) void mask_keys_k<u128>(const u128 *__restrict__ keys, int64_t n, u128 keep,
                                                               u128 *__restrict__ out) {
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        const u128 k = keys[x];
        out[x] = u128{k.lo & keep.lo, k.hi & keep.hi};
    }
}

template <typename K>
__global__ __launch_bounds__(kThreads) void get_flags_k(const K *__restrict__ keys, int64_t n, int fbit,
                                                         uint8_t *__restrict__ out) {
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        const K k = keys[x];
        uint32_t b;
        if constexpr (sizeof(K) == 16) {
            const u128 &w = reinterpret_cast<const u128 &>(k);
            b = (uint32_t)((fbit < 64 ? w.lo : w.hi) >> (fbit & 63)) & 1u;
        } else {
            b = (uint32_t)(k >> fbit) & 1u;
        }
        out[x] = (uint8_t)b;
    }
}

// The segment-local mode orders keep their index words in compact form
// (each mode's coordinate in a contiguous bit field, as the byte tables
// assemble it), so the MTTKRP over them needs no table lookups.
template <typename K>
__global__ __launch_bounds__(kThreads) void compact_keys_k(K *__restrict__ keys, int64_t n, const K *__restrict__ ctab) {
    constexpr int kTab = byte_table_entries(8 * (int)sizeof(K));
    __shared__ K lt[kTab];
    for (int q = threadIdx.x; q < kTab; q += kThreads) lt[q] = ctab[q];
    __syncthreads();
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads)
        keys[x] = compact_index(keys[x], lt);
}

// compact form -> linearized index (the bit-level gather again, from the fields)
template <typename K>
__global__ __launch_bounds__(kThreads) void expand_keys_k(const K *__restrict__ cw, int64_t n, RunTable tab,
                                                           K *__restrict__ out) {
    for (int64_t x = (int64_t)blockIdx.x * kThreads + threadIdx.x; x < n; x += (int64_t)gridDim.x * kThreads) {
        const K c = cw[x];
        K k = 0;
        for (int m = 0; m < tab.N; m++) {
            const uint32_t v = (uint32_t)(c >> tab.coff[m]) & tab.cmask[m];
            for (int q = 0; q < tab.nruns[m]; q++) {
                const uint32_t r = tab.run[m][q];
                const int len = run_len(r);
                const uint32_t bits = (v >> run_cpos(r)) & (uint32_t)((1ull << len) - 1);
                KeyOps<K>::deposit(k, bits, run_kpos(r));
            }
        }
        out[x] = k;
    }
}

// ------------------------------------------------------------ row statistics
// Row counts of one mode over a strided sample of the nonzeros (selector
// features: how hot the hottest row is, how many rows the sample touches).
template <typename K>
__global__ __launch_bounds__(kThreads) void row_sample_k(const K *__restrict__ keys, int64_t S, int64_t M,
                                                         RunTable tab, const K *__restrict__ ctab, int mode,
                                                         uint32_t nb, bool hashed, uint32_t *__restrict__ cnt) {
    constexpr int kTab = byte_table_entries(8 * (int)sizeof(K));
    __shared__ K ltab[kTab > 0 ? kTab : 1];
    if constexpr (kTab > 0) {
        for (int q = threadIdx.x; q < kTab; q += kThreads) ltab[q] = ctab[q];
        __syncthreads();
    }
    const int lane = __lane_id();
    // every wave runs the same number of rounds (the ballots below need
    // the whole wave); lanes past S take no part
    const int64_t step = (int64_t)gridDim.x * kThreads;
    for (int64_t x0 = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); x0 < S; x0 += step) {
        const int64_t x = x0 + lane;
        bool todo = x < S;
        uint32_t b = 0;
        if (todo) {
            const K key = keys[x * M / S];  // S evenly spaced nonzeros
            uint32_t r;
            if constexpr (kTab > 0) r = (uint32_t)(compact_index(key, ltab) >> tab.coff[mode]) & tab.cmask[mode];
            else r = extract_mode(key, tab, mode);
            // Fibonacci hashing folds large modes onto nb buckets
            b = hashed ? (uint32_t)(((uint64_t)(r * 2654435769u) * nb) >> 32) : r;
        }
        // lanes with the same bucket add once: a hot row would otherwise
        // take one atomic per sampled nonzero on a single address
        uint64_t left = __ballot(todo);
        while (left) {
            const int leader = __builtin_ctzll(left);
            const uint32_t lb = (uint32_t)__shfl((int)b, leader);
            const uint64_t same = __ballot(todo && b == lb);
            if (lane == leader) atomicAdd(&cnt[lb], (uint32_t)__builtin_popcountll(same));
            if (todo && b == lb) todo = false;
            left &= ~same;
        }
    }
}

__global__ __launch_bounds__(kThreads) void count_stats_k(const uint32_t *__restrict__ cnt, uint32_t n,
                                                          uint32_t *__restrict__ res) {
    uint32_t mx = 0, nz = 0;
    for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < n; x += gridDim.x * kThreads) {
        const uint32_t c = cnt[x];
        mx = max(mx, c);
        nz += c != 0u;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
        nz += (uint32_t)__shfl_xor((int)nz, off);
    }
    if (__lane_id() == 0) {
        atomicMax(&res[0], mx);
        atomicAdd(&res[1], nz);
    }
}

// ------------------------------------------------------------ launchers
int launch_row_sample(int key_bits, const void *keys, int64_t S, int64_t M, const RunTable &tab,
                      const void *ctab, int mode, uint64_t dim, uint32_t nb, uint32_t *cnt, uint32_t *res,
                      hipStream_t s) {
    if (S <= 0 || nb == 0) return ALTO_OK;
    if (key_bits <= 64 && !ctab) return set_error(ALTO_E_INVAL, "internal: missing byte tables");
    const bool hashed = (uint64_t)nb < dim;
    const unsigned g = std::min<unsigned>(grid_for(S, kThreads * 4), 2048);
    if (key_bits == 32)
        row_sample_k<uint32_t><<<g, kThreads, 0, s>>>((const uint32_t *)keys, S, M, tab, (const uint32_t *)ctab,
                                                       mode, nb, hashed, cnt);
    else if (key_bits == 64)
        row_sample_k<uint64_t><<<g, kThreads, 0, s>>>((const uint64_t *)keys, S, M, tab, (const uint64_t *)ctab,
                                                       mode, nb, hashed, cnt);
    else
        row_sample_k<u128><<<g, kThreads, 0, s>>>((const u128 *)keys, S, M, tab, nullptr, mode, nb, hashed, cnt);
    ALTO_HIP(hipGetLastError());
    const unsigned g2 = std::min<unsigned>(grid_for(nb, kThreads * 4), 2048);
    count_stats_k<<<g2, kThreads, 0, s>>>(cnt, nb, res);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_compact_keys(int key_bits, void *keys, int64_t n, const void *ctab, hipStream_t s) {
    if (n <= 0) return ALTO_OK;
    if (key_bits > 64 || !ctab) return set_error(ALTO_E_INVAL, "internal: compact keys need byte tables");
    const unsigned g = std::min<unsigned>(grid_for(n, kThreads * 4), 4096);
    if (key_bits == 32) compact_keys_k<uint32_t><<<g, kThreads, 0, s>>>((uint32_t *)keys, n, (const uint32_t *)ctab);
    else compact_keys_k<uint64_t><<<g, kThreads, 0, s>>>((uint64_t *)keys, n, (const uint64_t *)ctab);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_expand_keys(int key_bits, const void *cw, int64_t n, const RunTable &tab, void *out, hipStream_t s) {
    if (n <= 0) return ALTO_OK;
    if (key_bits > 64) return set_error(ALTO_E_INVAL, "internal: no compact form for 128-bit keys");
    const unsigned g = std::min<unsigned>(grid_for(n, kThreads * 4), 4096);
    if (key_bits == 32) expand_keys_k<uint32_t><<<g, kThreads, 0, s>>>((const uint32_t *)cw, n, tab, (uint32_t *)out);
    else expand_keys_k<uint64_t><<<g, kThreads, 0, s>>>((const uint64_t *)cw, n, tab, (uint64_t *)out);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_get_flags(int key_bits, const void *keys, int64_t n, int fbit, uint8_t *out, hipStream_t s) {
    if (n <= 0) return ALTO_OK;
    const unsigned g = std::min<unsigned>(grid_for(n, kThreads * 4), 4096);
    if (key_bits == 32) get_flags_k<uint32_t><<<g, kThreads, 0, s>>>((const uint32_t *)keys, n, fbit, out);
    else if (key_bits == 64) get_flags_k<uint64_t><<<g, kThreads, 0, s>>>((const uint64_t *)keys, n, fbit, out);
    else get_flags_k<u128><<<g, kThreads, 0, s>>>((const u128 *)keys, n, fbit, out);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_owner_flags(int key_bits, void *keys, const int64_t *seg, int L, int NG, const RunTable &tab,
                       const void *ctab, int mode, uint32_t *owner, uint64_t dim, int fbit, hipStream_t s) {
    if (L <= 0) return ALTO_OK;
    if (key_bits <= 64 && !ctab) return set_error(ALTO_E_INVAL, "internal: missing byte tables");
    ALTO_HIP(hipMemsetAsync(owner, 0xff, sizeof(uint32_t) * dim, s));
    for (int pass = 0; pass < 2; pass++) {
#define ALTO_OWN(K, CT)                                                                                        \
    (pass == 0 ? owner_k<K, false><<<L, kThreads, 0, s>>>((K *)keys, seg, NG, tab, (const K *)(CT), mode, owner, fbit) \
               : owner_k<K, true><<<L, kThreads, 0, s>>>((K *)keys, seg, NG, tab, (const K *)(CT), mode, owner, fbit))
        if (key_bits == 32) ALTO_OWN(uint32_t, ctab);
        else if (key_bits == 64) ALTO_OWN(uint64_t, ctab);
        else ALTO_OWN(u128, nullptr);
#undef ALTO_OWN
        ALTO_HIP(hipGetLastError());
    }
    return ALTO_OK;
}

int launch_mask_keys(int key_bits, const void *keys, int64_t n, int B, void *out, hipStream_t s) {
    if (n <= 0) return ALTO_OK;
    const unsigned g = std::min<unsigned>(grid_for(n, kThreads * 4), 4096);
    if (key_bits == 32) {
        const uint32_t keep = B >= 32 ? 0xffffffffu : ((1u << B) - 1u);
        mask_keys_k<uint32_t><<<g, kThreads, 0, s>>>((const uint32_t *)keys, n, keep, (uint32_t *)out);
    } else if (key_bits == 64) {
        const uint64_t keep = B >= 64 ? ~0ull : ((1ull << B) - 1ull);
        mask_keys_k<uint64_t><<<g, kThreads, 0, s>>>((const uint64_t *)keys, n, keep, (uint64_t *)out);
    } else {
        const u128 keep{B >= 64 ? ~0ull : ((1ull << B) - 1ull), B >= 128 ? ~0ull : (B <= 64 ? 0ull : ((1ull << (B - 64)) - 1ull))};
        mask_keys_k<u128><<<g, kThreads, 0, s>>>((const u128 *)keys, n, keep, (u128 *)out);
    }
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_encode(int key_bits, const CoordPtrs &c, const uint64_t *dims, int64_t n, const RunTable &tab,
                  const void *etab, void *keys, int *d_flag, hipStream_t s) {
    if (n <= 0) return ALTO_OK;
    if (etab && tab.etab_entries > 0) {
        const unsigned g = std::min<unsigned>(grid_for(n, kThreads * 4), 2048);
        const size_t kb = key_bits / 8;
        const size_t lds = (size_t)tab.etab_entries * kb;
        if (lds > kEncodeTableMax) return set_error(ALTO_E_INVAL, "internal: deposit tables too large");
        if (key_bits == 32)
            encode_tab_k<uint32_t><<<g, kThreads, lds, s>>>(c, dims, n, tab, (const uint32_t *)etab, (uint32_t *)keys,
                                                            d_flag);
        else if (key_bits == 64)
            encode_tab_k<uint64_t><<<g, kThreads, lds, s>>>(c, dims, n, tab, (const uint64_t *)etab, (uint64_t *)keys,
                                                            d_flag);
        else
            encode_tab_k<u128><<<g, kThreads, lds, s>>>(c, dims, n, tab, (const u128 *)etab, (u128 *)keys, d_flag);
        ALTO_HIP(hipGetLastError());
        return ALTO_OK;
    }
    const unsigned g = grid_for(n, kThreads * 4);
    if (key_bits == 32) encode_k<uint32_t><<<g, kThreads, 0, s>>>(c, dims, n, tab, (uint32_t *)keys, d_flag);
    else if (key_bits == 64) encode_k<uint64_t><<<g, kThreads, 0, s>>>(c, dims, n, tab, (uint64_t *)keys, d_flag);
    else encode_k<u128><<<g, kThreads, 0, s>>>(c, dims, n, tab, (u128 *)keys, d_flag);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

size_t radix_sort_scratch(int key_bits, int64_t n) {
    const int tile = key_bits == 128 ? SortCfg<u128>::kTile : SortCfg<uint64_t>::kTile;
    const int64_t T = (n + tile - 1) / tile;
    const size_t a = (256 * T * sizeof(uint32_t) + 255) & ~(size_t)255;
    const size_t b = (256 * T * sizeof(uint64_t) + 255) & ~(size_t)255;
    return a + b + scan_bytes<uint32_t, uint64_t, false>(256 * T) + 256;
}

int radix_sort(int key_bits, int nbits, int64_t n, void *keys, float *vals, void *keys_alt, float *vals_alt,
               void *scratch, size_t scratch_bytes, bool *in_alt, hipStream_t s) {
    if (scratch_bytes < radix_sort_scratch(key_bits, n)) return set_error(ALTO_E_NOMEM, "radix sort scratch too small");
    if (key_bits == 32)
        return radix_sort_t<uint32_t>(nbits, n, (uint32_t *)keys, vals, (uint32_t *)keys_alt, vals_alt, scratch, in_alt, s);
    if (key_bits == 64)
        return radix_sort_t<uint64_t>(nbits, n, (uint64_t *)keys, vals, (uint64_t *)keys_alt, vals_alt, scratch, in_alt, s);
    return radix_sort_t<u128>(nbits, n, (u128 *)keys, vals, (u128 *)keys_alt, vals_alt, scratch, in_alt, s);
}

size_t coalesce_scratch(int64_t n) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile + 1;
    return (size_t)nb * (sizeof(uint32_t) + sizeof(uint64_t)) + scan_bytes<uint32_t, uint64_t, false>(nb) + 1024;
}

// Counts distinct keys (host value, synchronizes) and, if there are repeats,
// writes the coalesced tensor to keys_out/vals_out.
int coalesce(int key_bits, int64_t n, const void *keys, const float *vals, void *keys_out, float *vals_out,
             void *scratch, size_t scratch_bytes, int64_t *n_unique, hipStream_t s) {
    *n_unique = n;
    if (n <= 1) return ALTO_OK;
    if (scratch_bytes < coalesce_scratch(n)) return set_error(ALTO_E_NOMEM, "coalesce scratch too small");
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    uint32_t *bcount = (uint32_t *)scratch;
    uint64_t *boff = (uint64_t *)((char *)scratch + ((nb * sizeof(uint32_t) + 255) & ~(size_t)255));
    uint64_t *total = boff + nb;
    void *scan_ws = (char *)(total + 1) + 256;
#define ALTO_HC(K) head_count_k<K><<<(unsigned)nb, kThreads, 0, s>>>((const K *)keys, n, bcount)
    if (key_bits == 32) ALTO_HC(uint32_t);
    else if (key_bits == 64) ALTO_HC(uint64_t);
    else ALTO_HC(u128);
#undef ALTO_HC
    int rc = device_scan<uint32_t, uint64_t, false>(bcount, boff, nb, total, scan_ws, s);
    if (rc) return rc;
    uint64_t h = 0;
    ALTO_HIP(hipMemcpyAsync(&h, total, sizeof(h), hipMemcpyDeviceToHost, s));
    ALTO_HIP(hipStreamSynchronize(s));
    *n_unique = (int64_t)h;
    if ((int64_t)h == n) return ALTO_OK;
#define ALTO_CP(K) \
    compact_k<K><<<(unsigned)nb, kThreads, 0, s>>>((const K *)keys, vals, n, boff, (K *)keys_out, vals_out)
    if (key_bits == 32) ALTO_CP(uint32_t);
    else if (key_bits == 64) ALTO_CP(uint64_t);
    else ALTO_CP(u128);
#undef ALTO_CP
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_intervals(int key_bits, const void *keys, const int64_t *seg, int L, const RunTable &tab,
                     const void *ctab, uint32_t *ivl, hipStream_t s) {
    if (L <= 0) return ALTO_OK;
    if (key_bits <= 64 && !ctab) return set_error(ALTO_E_INVAL, "internal: missing byte tables");
    if (key_bits == 32)
        intervals_k<uint32_t><<<L, kThreads, 0, s>>>((const uint32_t *)keys, seg, tab, (const uint32_t *)ctab, ivl);
    else if (key_bits == 64)
        intervals_k<uint64_t><<<L, kThreads, 0, s>>>((const uint64_t *)keys, seg, tab, (const uint64_t *)ctab, ivl);
    else intervals_k<u128><<<L, kThreads, 0, s>>>((const u128 *)keys, seg, tab, nullptr, ivl);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

size_t coverage_scratch(uint64_t dim) {
    return ((dim + 1) * sizeof(int32_t) + 255 & ~(size_t)255) + scan_bytes<int32_t, int32_t, true>((int64_t)dim + 1);
}

int coverage(int N, int L, const uint32_t *d_ivl, int mode, uint64_t dim, uint32_t *cov, void *scratch,
             size_t scratch_bytes, hipStream_t s) {
    if (scratch_bytes < coverage_scratch(dim)) return set_error(ALTO_E_NOMEM, "coverage scratch too small");
    int32_t *diff = (int32_t *)scratch;
    void *scan_ws = (char *)scratch + (((dim + 1) * sizeof(int32_t) + 255) & ~(size_t)255);
    ALTO_HIP(hipMemsetAsync(diff, 0, (dim + 1) * sizeof(int32_t), s));
    if (L > 0) {
        coverage_marks_k<<<(L + kThreads - 1) / kThreads, kThreads, 0, s>>>(d_ivl, L, N, mode, diff);
        ALTO_HIP(hipGetLastError());
    }
    return device_scan<int32_t, int32_t, true>(diff, (int32_t *)cov, (int64_t)dim, nullptr, scan_ws, s);
}

size_t seg_order_scratch(int key_bits, int64_t n) {
    // two row arrays, one index array and one value array
    return (size_t)n * (2 * sizeof(uint32_t) + key_bits / 8 + sizeof(float)) + 1024;
}

int launch_seg_order(int key_bits, const void *keys, const float *vals, const int64_t *seg, int L,
                     const RunTable &tab, const void *ctab, int mode, int nbits, void *scratch, int64_t n,
                     void *okeys, float *ovals, hipStream_t s) {
    if (L <= 0 || n <= 0) return ALTO_OK;
    if (key_bits <= 64 && !ctab) return set_error(ALTO_E_INVAL, "internal: missing byte tables");
    auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = (char *)scratch;
    uint32_t *R0 = (uint32_t *)p;
    uint32_t *R1 = (uint32_t *)(p + align((size_t)n * 4));
    void *ks = p + 2 * align((size_t)n * 4);
    float *vs = (float *)(p + 2 * align((size_t)n * 4) + align((size_t)n * key_bits / 8));
#define ALTO_SO_(K)                                                                                              \
    do {                                                                                                         \
        const size_t lds = seg_order_lds<K>();                                                                   \
        if (lds > 64 * 1024) {                                                                                   \
            hipError_t e = hipFuncSetAttribute((const void *)seg_order_k<K>,                                     \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);            \
            if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute(MaxDynamicSharedMemorySize)");        \
        }                                                                                                        \
        seg_order_k<K><<<L, kSoThreads, lds, s>>>((const K *)keys, vals, seg, tab, (const K *)ctab, mode, nbits, \
                                                  R0, R1, (K *)ks, vs, (K *)okeys, ovals);                       \
    } while (0)
    if (key_bits == 32) ALTO_SO_(uint32_t);
    else if (key_bits == 64) ALTO_SO_(uint64_t);
    else ALTO_SO_(u128);
#undef ALTO_SO_
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_sumsq(const float *vals, int64_t n, double *out, hipStream_t s) {
    // out must have room for kSumBlocks + 1 doubles; the result lands in out[kSumBlocks]
    sumsq_partial_k<<<kSumBlocks, kThreads, 0, s>>>(vals, n, out);
    sum_partials_k<<<1, kThreads, 0, s>>>(out, kSumBlocks, out + kSumBlocks);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

}  // namespace alto
