// Mode-n MTTKRP on an ALTO tensor (Algorithms 1 and 2 of the ALTO paper),
// written for CDNA4 (64-lane waves, 160 KiB LDS per compute unit, one L2 per
// XCD).
//
// One workgroup processes one line segment.  The segment is cut into NG
// contiguous sub-ranges, one per lane group of G = R/VEC lanes; each lane
// owns VEC consecutive rank columns, so a factor row is gathered with one
// 16-byte load per lane.  Waves run independently (no workgroup barrier in
// the main loop).  Per tile of G nonzeros per group:
//   - every lane loads one nonzero of its own group (coalesced, prefetched one
//     tile ahead) and de-linearizes it (bit-level scatter of the index): one
//     LDS byte-table entry per index byte, OR-ed into a compact word holding
//     all coordinates (a {lo, hi} pair of words for 128-bit indices);
//   - the group then walks its G nonzeros in order: coordinates and value come
//     from the owning lane by ds_swizzle, the N-1 factor rows are gathered
//     (from LDS for small factor matrices staged there by the workgroup, else
//     from memory at a 32-bit offset off a scalar base) and multiplied, and
//     the product is added to a register accumulator while the output row
//     repeats; when the row changes the accumulator is flushed.
// A flush goes either to Temp (Algorithm 2, local staging: LDS rows
// [T^s, T^e] of the segment's mode interval, merged into the output when the
// segment is done: plain stores for rows no other segment covers, atomics
// otherwise) or out with atomics (Algorithm 2, atomic update).  Atomic
// flushes are queued in LDS and drained by the whole wave with R consecutive
// lanes per output row, so each atomic instruction covers whole lines (on
// this GPU global atomics cost per line touched); queue entries of one row
// at consecutive slots are summed first.  When the nonzeros come in
// linearized order the atomics are FP64, into an accumulator added into the
// output afterwards (precision: see gadd).  Rows that the helper flags
// (Section 3.3) mark as this lane group's alone skip the queue and are
// written with plain read-modify-writes.
#pragma once

#include <type_traits>
#include <utility>

#include "common.h"

namespace alto {

// Factor matrices of the modes other than the output mode, in the order of
// ModeDec (entry j is mode dec.om[j]).
struct FactorPtrs {
    const void *p[kMaxModes];
};

// Per-launch decode plan: om[j] (j < N-1) are the other modes, om[N-1] the
// output mode; coff/cmask locate each of them in the compact word.  Other
// modes with bit j of smask have their whole factor matrix (sbytes[j] bytes)
// copied to LDS at byte offset soff[j] and are gathered from there.
struct ModeDec {
    int fbit;     // index bit of the output mode's helper flag (-1: no flags)
    int compact;  // the index words are already compact words (keys of at most 64 bits)
    int om[kMaxModes];
    uint32_t coff[kMaxModes];
    uint32_t cmask[kMaxModes];
    uint32_t smask;
    uint32_t soff[kMaxModes];
    uint32_t sbytes[kMaxModes];
};

template <int... Is, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, Is...>, F &&f) {
    (f(std::integral_constant<int, Is>{}), ...);
}
// f(integral_constant<int, i>) for i = 0 .. n-1, unrolled at compile time
template <int n, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_impl(std::make_integer_sequence<int, n>{}, f);
}

// Value of lane k of this lane's group of G consecutive lanes.
template <int G, int k>
__device__ __forceinline__ uint32_t group_bcast(uint32_t x) {
    if constexpr (G == 1) {
        return x;
    } else if constexpr (G == 64) {
        return (uint32_t)__builtin_amdgcn_readlane((int)x, k);
    } else {
        static_assert(G <= 32 && (G & (G - 1)) == 0, "group size must be a power of two");
        // ds_swizzle bit mode inside each 32-lane half: lane = (lane & and) | or
        constexpr int pattern = ((32 - G) & 0x1f) | (k << 5);
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, pattern);
    }
}

constexpr uint32_t kNoRow = 0xffffffffu;

__device__ __forceinline__ uint32_t xcc_id() {
    // hwreg(HW_REG_XCC_ID, 0, 4): id 20, offset 0, 4 bits
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xfu;
}
// with helper flags the output row carries its flag in bit 31 (rows < 2^31 - 1)
constexpr uint32_t kOwnBit = 0x80000000u;

// FP32 add into LDS as a compare-and-swap loop.  Measured on gfx950, the LDS
// float atomic (ds_add_f32) sustains about 0.2 T lane-operations/s over the
// chip whatever the address pattern, while LDS compare-and-swap on 32-bit
// words runs several times faster; Temp flushes rarely collide, so the loop
// usually ends after one exchange.
__device__ __forceinline__ void lds_add(float *p, float v) {
    uint32_t *u = reinterpret_cast<uint32_t *>(p);
    uint32_t seen = *u, prev;
    do {
        prev = seen;
        seen = atomicCAS(u, prev, __float_as_uint(__uint_as_float(prev) + v));
    } while (seen != prev);
}

template <typename K>
__device__ __forceinline__ uint32_t key_bit(const K &k, int pos) {
    return (uint32_t)(k >> pos) & 1u;
}
template <>
__device__ __forceinline__ uint32_t key_bit<u128>(const u128 &k, int pos) {
    return (uint32_t)((pos < 64 ? k.lo : k.hi) >> (pos & 63)) & 1u;
}

template <typename FT>
struct FactorLoad;

// Loads at a byte offset from a factor matrix: 32-bit offsets let the
// gather use a scalar base plus one vector offset register.
template <>
struct FactorLoad<float> {
    static constexpr int kVec = 4;
    template <typename Off>
    __device__ __forceinline__ static void load(const void *base, Off off, float (&x)[4]) {
        const float4 q = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
        x[0] = q.x;
        x[1] = q.y;
        x[2] = q.z;
        x[3] = q.w;
    }
    template <typename Off>
    __device__ __forceinline__ static float load1(const void *base, Off off) {
        return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + off);
    }
};

__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

template <>
struct FactorLoad<uint16_t> {
    static constexpr int kVec = 8;
    template <typename Off>
    __device__ __forceinline__ static void load(const void *base, Off off, float (&x)[8]) {
        const uint4 q = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(base) + off);
        x[0] = bf16_to_f32(q.x & 0xffffu);
        x[1] = bf16_to_f32(q.x >> 16);
        x[2] = bf16_to_f32(q.y & 0xffffu);
        x[3] = bf16_to_f32(q.y >> 16);
        x[4] = bf16_to_f32(q.z & 0xffffu);
        x[5] = bf16_to_f32(q.z >> 16);
        x[6] = bf16_to_f32(q.w & 0xffffu);
        x[7] = bf16_to_f32(q.w >> 16);
    }
    template <typename Off>
    __device__ __forceinline__ static float load1(const void *base, Off off) {
        return bf16_to_f32(*reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(base) + off));
    }
};

// Compile-time shape of one instantiation.  RT = 0: any rank (one 64-lane
// wave per nonzero, up to four columns per lane).  NT = 0: any order <= 8.
template <int NT, int RT, typename FT>
struct MtCfg {
    static constexpr int kVec = RT ? FactorLoad<FT>::kVec : 1;
    static constexpr int kG = RT ? RT / kVec : 64;            // lanes per nonzero
    static constexpr int kGPW = 64 / kG;                      // lane groups per wave
    static constexpr int kCols = RT ? 1 : 4;                  // column chunks per lane (generic rank)
    static constexpr int kNMax = NT ? NT : kMaxModes;
    // nonzeros in flight per group: four for orders 3 and 4, two for order 5
    // (four gathered rows each; keeps the registers below the spill point),
    // one for the generic-order kernels (up to seven rows each)
    static constexpr int kUMax = NT == 0 ? 1 : (NT >= 5 ? 2 : 4);
    static constexpr int kU = kG >= kUMax ? kUMax : kG;
    // flush queue (rank-specialized atomic path): rows per wave
    static constexpr bool kQueue = RT != 0 && RT <= 64;
    static constexpr int kQRows = kQueue ? 2 * kGPW : 0;      // drained once it holds more than one row per group
};

// LDS row stride of Temp: one float of padding spreads rows over the banks.
__host__ __device__ inline int temp_stride(int R) { return R + 1; }

// LDS bytes of the per-wave flush queues of one workgroup.
template <int NT, int RT, typename FT>
__host__ __device__ constexpr int mt_queue_bytes(int threads) {
    using C = MtCfg<NT, RT, FT>;
    return C::kQueue ? (threads / 64) * C::kQRows * (RT + 1) * 4 : 0;
}


// kOrdered changes no code: launches over a segment-local mode order get a
// kernel symbol of their own, so that a kernel trace separates them from
// launches over the linearized order.
template <typename K, int NT, int RT, typename FT, bool kStaged, bool kWide, bool kOrdered = false>
__global__ __launch_bounds__(1024) void mttkrp_k(
    const K *__restrict__ keys, const float *__restrict__ vals, const int64_t *__restrict__ seg,
    const uint32_t *__restrict__ ivl, const uint32_t *__restrict__ cov, FactorPtrs fac, int R_rt, int N_rt, int mode,
    RunTable tab, ModeDec dec, const K *__restrict__ ctab, int ctab_off, float *__restrict__ out,
    double *__restrict__ acc64_base, uint64_t acc_stride, int nacc, const int32_t *__restrict__ seg_list, int n_list) {
    using C = MtCfg<NT, RT, FT>;
    constexpr int VEC = C::kVec, G = C::kG, GPW = C::kGPW, NM = C::kNMax, NCOL = C::kCols, U = C::kU;
    constexpr int NO = NM - 1;  // other modes
    using Off = std::conditional_t<kWide, uint64_t, uint32_t>;  // factor byte offsets
    constexpr bool QUEUE = C::kQueue && !kStaged;
    constexpr int QR = C::kQRows;
    constexpr int kTab = byte_table_entries(8 * (int)sizeof(K));  // byte tables in LDS (keys <= 64 bits)
    const int N = NT ? NT : N_rt;
    const int R = RT ? RT : R_rt;
    extern __shared__ float smem[];

    // XCD-aware order: consecutive list entries (neighbouring segments, which
    // touch neighbouring factor rows) go to the same L2.
    const int per = (n_list + 7) / 8;
    const int li = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (li >= n_list) return;
    const int l = seg_list ? seg_list[li] : li;  // no list: segments 0 .. n_list-1

    const int64_t sb = seg[l], S = seg[l + 1] - sb;
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const int NG = blockDim.x / G;
    const int gw = lane / G, c = lane % G;
    const int g = wave * GPW + gw;
    const int64_t gb = sb + (S * g) / NG;
    const int64_t ge = sb + (S * (g + 1)) / NG;
    const int64_t maxlen = (S + NG - 1) / NG;
    const int ntiles = (int)((maxlen + G - 1) / G);

    // Atomic updates of the output: FP32 atomics into out, or, with acc64,
    // FP64 atomics into an FP64 accumulator that is added into out after the
    // launch.  The strategies that visit the nonzeros in linearized order
    // send a hot row's contributions as up to millions of short runs; summed
    // by FP32 atomics in arbitrary order their rounding error grows like
    // sqrt(updates) and reaches 1e-4 relative on the skewed tensors, while
    // FP64 accumulation keeps it at the FP32 rounding of the runs.
    // with nacc > 1 each XCD adds into a copy of its own (chosen by the XCC
    // id register), which spreads the atomics on a small output's few lines
    double *const acc64 = acc64_base ? acc64_base + (uint64_t)(xcc_id() % (uint32_t)nacc) * acc_stride : nullptr;
    auto gadd = [&](uint64_t off, float v) {
        if (acc64) unsafeAtomicAdd(acc64 + off, (double)v);
        else unsafeAtomicAdd(out + off, v);
    };
    const int RP = temp_stride(R);
    float *const temp = smem;                                      // staged: Temp rows
    float *const qbuf = smem + (QUEUE ? wave * QR * (RT + 1) : 0);  // atomic: this wave's flush queue
    int qn = 0;                                                    // queued rows (wave-uniform)

    uint32_t lo = 0, width = 0;
    if constexpr (kStaged) {
        lo = ivl[((int64_t)l * N + mode) * 2 + 0];
        width = ivl[((int64_t)l * N + mode) * 2 + 1] - lo + 1;
        for (int q = threadIdx.x; q < (int)width * RP; q += blockDim.x) temp[q] = 0.f;
    }
    K *const ltab = reinterpret_cast<K *>(smem + ctab_off);
    if constexpr (kTab > 0) {
        if (!dec.compact) {
            constexpr int n16 = kTab * (int)sizeof(K) / 16;
            const uint4 *src = reinterpret_cast<const uint4 *>(ctab);
            uint4 *dst = reinterpret_cast<uint4 *>(ltab);
            for (int q = threadIdx.x; q < n16; q += blockDim.x) dst[q] = src[q];
        }
    } else {
        // 128-bit indices: tbytes128 tables of 256 {lo, hi} entries
        const int n16 = tab.tbytes128 * 256;
        const uint4 *src = reinterpret_cast<const uint4 *>(ctab);
        uint4 *dst = reinterpret_cast<uint4 *>(ltab);
        for (int q = threadIdx.x; q < n16; q += blockDim.x) dst[q] = src[q];
    }
    if constexpr (RT != 0 && !kStaged) {
        // small factor matrices of other modes, staged whole
        for (int j = 0; j < N - 1; j++) {
            if (!((dec.smask >> j) & 1u)) continue;
            const uint4 *src = reinterpret_cast<const uint4 *>(fac.p[j]);
            uint4 *dst = reinterpret_cast<uint4 *>(reinterpret_cast<char *>(smem) + dec.soff[j]);
            for (uint32_t q = threadIdx.x; q < dec.sbytes[j] / 16u; q += blockDim.x) dst[q] = src[q];
        }
    }
    __syncthreads();

    uint32_t cur = kNoRow;
    float acc[NCOL][VEC];
#pragma unroll
    for (int a = 0; a < NCOL; a++)
#pragma unroll
        for (int e = 0; e < VEC; e++) acc[a][e] = 0.f;

    // rows with a helper flag (bit 31) belong to this lane group alone:
    // plain read-modify-write of the output instead of atomics
    const uint32_t rmask = dec.fbit >= 0 ? ~kOwnBit : 0xffffffffu;

    // direct flush: LDS Temp (staged) or global atomics (generic rank)
    auto flush_direct = [&](uint32_t raw) {
        const uint32_t row = raw & rmask;
        const bool own = dec.fbit >= 0 && (raw & kOwnBit);
#pragma unroll
        for (int a = 0; a < NCOL; a++) {
            const int col0 = RT ? c * VEC : c + 64 * a;
            if (!RT && col0 >= R) continue;
            if constexpr (kStaged) {
                float *dst = temp + (uint64_t)(row - lo) * RP + col0;
#pragma unroll
                for (int e = 0; e < VEC; e++) lds_add(dst + e, acc[a][e]);
            } else if (own) {
                float *dst = out + (uint64_t)row * R + col0;
#pragma unroll
                for (int e = 0; e < VEC; e++) dst[e] += acc[a][e];
            } else {
                const uint64_t off = (uint64_t)row * R + col0;
#pragma unroll
                for (int e = 0; e < VEC; e++) gadd(off + e, acc[a][e]);
            }
        }
    };

    // The whole wave empties the queue: R consecutive lanes per queued row.
    // Entries of one output row at consecutive slots (neighbouring groups
    // that each ended a piece of the same run) are summed in slot order first,
    // so such a run costs one atomic per wave instead of one per group.
    auto drain = [&]() {
        if constexpr (QUEUE) {
            constexpr int PER = 64 / RT;  // rows per instruction
            auto row_at = [&](int q) { return __float_as_uint(qbuf[q * (RT + 1) + RT]); };
            bool dup = false;
            for (int q = lane + 1; q < qn; q += 64) dup |= row_at(q) == row_at(q - 1);
            if (__ballot(dup) == 0) {
                for (int q0 = 0; q0 < qn; q0 += PER) {
                    const int q = q0 + lane / RT, col = lane % RT;
                    if (q < qn)
                        gadd((uint64_t)(row_at(q) & rmask) * RT + col, qbuf[q * (RT + 1) + col]);
                }
            } else {
                for (int q0 = 0; q0 < qn; q0 += PER) {
                    const int q = q0 + lane / RT, col = lane % RT;
                    if (q < qn) {
                        const uint32_t row = row_at(q);
                        if (q == 0 || row_at(q - 1) != row) {
                            float sum = qbuf[q * (RT + 1) + col];
                            for (int q2 = q + 1; q2 < qn && row_at(q2) == row; q2++)
                                sum += qbuf[q2 * (RT + 1) + col];
                            gadd((uint64_t)(row & rmask) * RT + col, sum);
                        }
                    }
                }
            }
            qn = 0;
        }
    };

    // prefetch the first tile: lane c of group g owns items gb + t*G + c
    int64_t pos = gb + c;
    bool ok_n = pos < ge;
    K key_n = ok_n ? keys[pos] : KeyOps<K>::zero();
    float val_n = ok_n ? vals[pos] : 0.f;

    for (int t = 0; t < ntiles; t++) {
        const K key = key_n;
        const float v = val_n;
        const bool ok = ok_n;
        pos += G;
        ok_n = pos < ge;
        if (ok_n) {
            key_n = keys[pos];
            val_n = vals[pos];
        }
        // de-linearize this lane's nonzero: coordinates of the other modes
        // (in the order of fac) and the output row
        uint32_t idx[NO];
        uint32_t myrow;
        if constexpr (kTab > 0) {
            // key is 0 (all coordinates 0) past the end
            const K cw = dec.compact ? key : compact_index(key, ltab);
#pragma unroll
            for (int j = 0; j < NO; j++) idx[j] = j < N - 1 ? (uint32_t)(cw >> dec.coff[j]) & dec.cmask[j] : 0u;
            myrow = (uint32_t)(cw >> dec.coff[N - 1]) & dec.cmask[N - 1];
        } else {
            // 128-bit indices: OR of one {lo, hi} entry per index byte
            uint64_t clo = 0, chi = 0;
            const u128 *lt = reinterpret_cast<const u128 *>(ltab);
#pragma unroll
            for (int b = 0; b < 16; b++) {
                if (b >= tab.tbytes128) break;
                const uint64_t w = b < 8 ? KeyOps<K>::lo_word(key) : KeyOps<K>::hi_word(key);
                const u128 e = lt[b * 256 + (int)((w >> (8 * (b & 7))) & 0xffu)];
                clo |= e.lo;
                chi |= e.hi;
            }
            // bits [off, off + 32) of the 128-bit word (a field may straddle the halves)
            auto field = [&](uint32_t off, uint32_t mask) {
                uint64_t w;
                if (off >= 64) w = chi >> (off - 64);
                else if (off == 0) w = clo;
                else w = (clo >> off) | (chi << (64 - off));
                return (uint32_t)w & mask;
            };
#pragma unroll
            for (int j = 0; j < NO; j++) idx[j] = j < N - 1 ? field(dec.coff[j], dec.cmask[j]) : 0u;
            myrow = field(dec.coff[N - 1], dec.cmask[N - 1]);
        }
        if (!kStaged && dec.fbit >= 0 && key_bit(key, dec.fbit)) myrow |= kOwnBit;
        if (!ok) myrow = kNoRow;

        static_for<G / U>([&](auto kc) {
            constexpr int k0 = decltype(kc)::value * U;
            uint32_t rows[U];
            float p[U][NCOL][VEC];
            static_for<U>([&](auto uc) {
                constexpr int u = decltype(uc)::value;
                const uint32_t row = group_bcast<G, k0 + u>(myrow);
                const float vv = __uint_as_float(group_bcast<G, k0 + u>(__float_as_uint(v)));
                rows[u] = row;
#pragma unroll
                for (int a = 0; a < NCOL; a++)
#pragma unroll
                    for (int e = 0; e < VEC; e++) p[u][a][e] = vv;
#pragma unroll
                for (int j = 0; j < NO; j++) {
                    if (j >= N - 1) continue;
                    const uint32_t im = group_bcast<G, k0 + u>(idx[j]);
                    const Off rowoff = (Off)im * (Off)(R * (int)sizeof(FT));
                    if constexpr (RT != 0) {
                        float f[VEC];
                        if (!kStaged && ((dec.smask >> j) & 1u)) {
                            const uint32_t lo = dec.soff[j] + im * (uint32_t)(R * (int)sizeof(FT)) +
                                                (uint32_t)(c * VEC * (int)sizeof(FT));
                            FactorLoad<FT>::load(reinterpret_cast<const char *>(smem), lo, f);
                        } else {
                            FactorLoad<FT>::load(fac.p[j], rowoff + (Off)(c * VEC * (int)sizeof(FT)), f);
                        }
#pragma unroll
                        for (int e = 0; e < VEC; e++) p[u][0][e] *= f[e];
                    } else {
#pragma unroll
                        for (int a = 0; a < NCOL; a++) {
                            const int col = c + 64 * a;
                            const float f =
                                col < R ? FactorLoad<FT>::load1(fac.p[j], rowoff + (Off)(col * (int)sizeof(FT))) : 0.f;
                            p[u][a][0] *= f;
                        }
                    }
                }
            });
            // Register run-combining.  A new row ends the current run, which is
            // flushed; items past the end of the group's range carry row kNoRow,
            // so they flush the last run and accumulate into a run that never is.
#pragma unroll
            for (int u = 0; u < U; u++) {
                const bool nw = rows[u] != cur;
                const bool fls = nw && cur != kNoRow;
                if constexpr (QUEUE) {
                    // groups whose run ends append (row, accumulator) to the
                    // wave's queue, except for rows that are this group's
                    // alone (helper flag), which it adds to the output itself
                    const bool own = fls && (cur & ~rmask);
                    const uint64_t fl = __ballot(fls && !own && c == 0);
                    if (nw) {
                        if (own) {
                            float *dst = out + (uint64_t)(cur & rmask) * RT + c * VEC;
#pragma unroll
                            for (int q = 0; q < VEC; q++) dst[q] += acc[0][q];
                        } else if (fls) {
                            const int slot = qn + __builtin_popcountll(fl & ((1ull << (gw * G)) - 1ull));
                            float *e = qbuf + slot * (RT + 1);
#pragma unroll
                            for (int q = 0; q < VEC; q++) e[c * VEC + q] = acc[0][q];
                            if (c == 0) e[RT] = __uint_as_float(cur);
                        }
                        cur = rows[u];
#pragma unroll
                        for (int e = 0; e < VEC; e++) acc[0][e] = 0.f;
                    }
                    qn += __builtin_popcountll(fl);
                    if (qn > GPW) drain();  // room for the next item's flushes
                } else {
                    if (nw) {
                        if (fls) flush_direct(cur);
                        cur = rows[u];
#pragma unroll
                        for (int a = 0; a < NCOL; a++)
#pragma unroll
                            for (int e = 0; e < VEC; e++) acc[a][e] = 0.f;
                    }
                }
#pragma unroll
                for (int a = 0; a < NCOL; a++)
#pragma unroll
                    for (int e = 0; e < VEC; e++) acc[a][e] += p[u][a][e];
            }
        });
    }
    if constexpr (QUEUE) {
        const bool own = cur != kNoRow && (cur & ~rmask);
        const uint64_t fl = __ballot(cur != kNoRow && !own && c == 0);
        if (own) {
            float *dst = out + (uint64_t)(cur & rmask) * RT + c * VEC;
#pragma unroll
            for (int q = 0; q < VEC; q++) dst[q] += acc[0][q];
        } else if (cur != kNoRow) {
            const int slot = qn + __builtin_popcountll(fl & ((1ull << (gw * G)) - 1ull));
            float *e = qbuf + slot * (RT + 1);
#pragma unroll
            for (int q = 0; q < VEC; q++) e[c * VEC + q] = acc[0][q];
            if (c == 0) e[RT] = __uint_as_float(cur);
        }
        qn += __builtin_popcountll(fl);
        drain();
    } else {
        if (cur != kNoRow) flush_direct(cur);
    }
    if constexpr (kStaged) {
        // merge Temp into the output (the pull of Algorithm 2 for this segment)
        __syncthreads();
        const int total = (int)width * R;
        for (int q = threadIdx.x; q < total; q += blockDim.x) {
            const int r = q / R, col = q - r * R;
            const float v = temp[r * RP + col];
            if (v == 0.f) continue;
            const uint32_t row = lo + (uint32_t)r;
            if (cov[row] == 1u) out[(uint64_t)row * R + col] = v;
            else gadd((uint64_t)row * R + col, v);
        }
    }
}

struct MtLaunch {
    const void *keys;
    const float *vals;
    const int64_t *seg;
    const uint32_t *ivl;
    const uint32_t *cov;
    FactorPtrs fac;
    int R, N, mode;
    RunTable tab;
    ModeDec dec;
    const void *ctab;  // byte tables of the compact form (keys <= 64 bits)
    float *out;
    double *acc64;     // FP64 accumulator of the atomic updates (nullptr: FP32 atomics into out)
    uint64_t acc_stride;  // elements between its per-XCD copies
    int nacc;             // number of copies (>= 1)
    const int32_t *list;  // segments to process (nullptr: 0 .. n_list-1)
    int n_list;
    int staged;
    int temp_rows;     // LDS Temp rows to reserve (staged launches)
    int threads;       // workgroup size (multiple of 64, <= 1024)
    bool wide;         // some gathered factor matrix spans more than 4 GiB
    bool ordered;      // keys and values are a segment-local mode order
};

template <typename K, int NT, int RT, typename FT>
int launch_mt_cfg(const MtLaunch &a, hipStream_t s) {
    if (a.n_list <= 0) return ALTO_OK;
    const size_t main_lds = a.staged ? (size_t)a.temp_rows * temp_stride(a.R) * 4
                                     : (size_t)mt_queue_bytes<NT, RT, FT>(a.threads);
    const size_t tab_off = (main_lds + 15) / 16 * 16;
    const size_t tab_bytes = sizeof(K) <= 8 ? (a.dec.compact ? 0 : (size_t)byte_table_entries(8 * (int)sizeof(K)) * sizeof(K))
                                            : (size_t)a.tab.tbytes128 * 256 * 16;
    size_t lds = tab_off + tab_bytes;
    ModeDec dec = a.dec;
    if (RT == 0 || a.staged) dec.smask = 0;
    for (int j = 0; j < a.N - 1; j++)
        if ((dec.smask >> j) & 1u) {
            lds = (lds + 15) / 16 * 16;
            dec.soff[j] = (uint32_t)lds;
            lds += dec.sbytes[j];
        }
    if (lds > 160 * 1024) return set_error(ALTO_E_INVAL, "internal: MTTKRP launch exceeds the LDS size");
    if (tab_bytes && !a.ctab) return set_error(ALTO_E_INVAL, "internal: missing byte tables");
    const int per = (a.n_list + 7) / 8;
    const unsigned grid = (unsigned)per * 8;
    // generic-order and generic-rank kernels always use 64-bit factor offsets
    decltype(&mttkrp_k<K, NT, RT, FT, true, true>) kern;
    if constexpr (NT == 0 || RT == 0) {
        kern = a.staged ? mttkrp_k<K, NT, RT, FT, true, true> : mttkrp_k<K, NT, RT, FT, false, true>;
    } else {
        kern = a.staged ? (a.wide ? mttkrp_k<K, NT, RT, FT, true, true> : mttkrp_k<K, NT, RT, FT, true, false>)
                        : (a.wide ? mttkrp_k<K, NT, RT, FT, false, true>
                                  : (a.ordered ? mttkrp_k<K, NT, RT, FT, false, false, true>
                                               : mttkrp_k<K, NT, RT, FT, false, false>));
    }
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_error(e, "hipFuncSetAttribute(MaxDynamicSharedMemorySize)");
    }
    kern<<<grid, a.threads, lds, s>>>((const K *)a.keys, a.vals, a.seg, a.ivl, a.cov, a.fac, a.R, a.N, a.mode, a.tab,
                                      dec, (const K *)a.ctab, (int)(tab_off / 4), a.out, a.acc64, a.acc_stride,
                                      a.nacc < 1 ? 1 : a.nacc,
                                      a.list, a.n_list);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

template <typename K, int NT, typename FT>
int launch_mt_r(const MtLaunch &a, hipStream_t s) {
    switch (a.R) {
        case 8: return launch_mt_cfg<K, NT, 8, FT>(a, s);
        case 16: return launch_mt_cfg<K, NT, 16, FT>(a, s);
        case 32: return launch_mt_cfg<K, NT, 32, FT>(a, s);
        case 64: return launch_mt_cfg<K, NT, 64, FT>(a, s);
        default: return launch_mt_cfg<K, NT, 0, FT>(a, s);
    }
}

template <typename K, typename FT>
int launch_mt_n(const MtLaunch &a, hipStream_t s) {
    switch (a.N) {
        case 3: return launch_mt_r<K, 3, FT>(a, s);
        case 4: return launch_mt_r<K, 4, FT>(a, s);
        case 5: return launch_mt_r<K, 5, FT>(a, s);
        default: return launch_mt_r<K, 0, FT>(a, s);
    }
}

// One translation unit per (key width, precision) keeps compile times parallel.
int launch_mt_k32_f32(const MtLaunch &a, hipStream_t s);
int launch_mt_k64_f32(const MtLaunch &a, hipStream_t s);
int launch_mt_k128_f32(const MtLaunch &a, hipStream_t s);
int launch_mt_k32_bf16(const MtLaunch &a, hipStream_t s);
int launch_mt_k64_bf16(const MtLaunch &a, hipStream_t s);
int launch_mt_k128_bf16(const MtLaunch &a, hipStream_t s);

inline int launch_mt(const MtLaunch &a, int key_bits, int prec, hipStream_t s) {
    const bool bf = prec == ALTO_PREC_BF16;
    if (key_bits == 32) return bf ? launch_mt_k32_bf16(a, s) : launch_mt_k32_f32(a, s);
    if (key_bits == 64) return bf ? launch_mt_k64_bf16(a, s) : launch_mt_k64_f32(a, s);
    return bf ? launch_mt_k128_bf16(a, s) : launch_mt_k128_f32(a, s);
}

// Fill everything of *a that does not depend on the segment list: index and
// values (the segment-local order by `mode` when `sorted`), partition,
// factor pointers in decode order, LDS staging of small factor matrices, and
// the workgroup size of an atomic launch.  Allocates nothing.
int fill_mt_launch(const alto_tensor *t, const void *const *factors, int R, int prec, int mode, bool sorted,
                   MtLaunch *a);
// lanes that share one nonzero in the kernels of rank R (see MtCfg)
inline int mt_group_lanes(int R, int prec) {
    const bool spec = R == 8 || R == 16 || R == 32 || R == 64;
    return spec ? R / (prec == ALTO_PREC_BF16 ? 8 : 4) : 64;
}
// Checks of alto_mttkrp's arguments that do not depend on the plan.
int check_mttkrp_args(const alto_tensor *t, const void *const *factors, int R, int prec, int mode,
                      const float *out);

// out[e] += (float)(sum over the nacc copies of acc at e), for e < n
int launch_acc64_finish(float *out, const double *acc, uint64_t stride, int nacc, uint64_t n, hipStream_t s);
// number of distinct XCC ids the device reports (probed once per device)
int device_xcc_count();
// set-up of alto_mttkrp_noalloc on the current device
int noalloc_prepare_device();

}  // namespace alto
