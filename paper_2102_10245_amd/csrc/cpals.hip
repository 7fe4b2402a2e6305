// CP-ALS on the GPU (Section 2.2 of the ALTO paper; standard alternating
// least squares).  The MTTKRP of every mode runs on the ALTO tensor; the
// R x R normal equations (Hadamard product of Grams, inverted with a
// positive-pivot test and one ridge retry), the row solves, column norms,
// Grams and the fit are FP64.
// Factor storage is FP32 or BF16 (double -> binary32 -> bfloat16, both
// round-to-nearest-even).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "common.h"

namespace alto {
namespace {

constexpr int kT = 256;
constexpr int kGramTile = 32;
constexpr int kMaxParts = 256;

__device__ __forceinline__ double load_factor(const void *A, int prec, uint64_t q) {
    if (prec == ALTO_PREC_BF16)
        return (double)__uint_as_float((uint32_t)reinterpret_cast<const uint16_t *>(A)[q] << 16);
    return (double)reinterpret_cast<const float *>(A)[q];
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Partial Grams: block (x, y) adds rows of chunk x into the 32x32 tile y of
// A^T A.  partials[x][R][R].
__global__ __launch_bounds__(kT) void gram_partial_k(const void *__restrict__ A, int prec, uint64_t I, int R,
                                                     int nparts, double *__restrict__ partials) {
    __shared__ double sa[32][kGramTile + 1];
    __shared__ double sb[32][kGramTile + 1];
    const int tiles = (R + kGramTile - 1) / kGramTile;
    const int ta = blockIdx.y / tiles, tb = blockIdx.y % tiles;
    const int a0 = ta * kGramTile, b0 = tb * kGramTile;
    const uint64_t chunk = (I + nparts - 1) / nparts;
    const uint64_t r0 = (uint64_t)blockIdx.x * chunk, r1 = min(I, r0 + chunk);
    const int tx = threadIdx.x % kGramTile, ty = threadIdx.x / kGramTile;  // ty in 0..7
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint64_t i0 = r0; i0 < r1; i0 += 32) {
        for (int q = threadIdx.x; q < 32 * kGramTile; q += kT) {
            const int ri = q / kGramTile, cj = q % kGramTile;
            const uint64_t i = i0 + ri;
            const bool in = i < r1;
            sa[ri][cj] = (in && a0 + cj < R) ? load_factor(A, prec, i * R + a0 + cj) : 0.0;
            sb[ri][cj] = (in && b0 + cj < R) ? load_factor(A, prec, i * R + b0 + cj) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int ri = 0; ri < 32; ri++) {
            const double bv = sb[ri][tx];
#pragma unroll
            for (int k = 0; k < 4; k++) acc[k] += sa[ri][ty + 8 * k] * bv;
        }
        __syncthreads();
    }
    double *P = partials + (uint64_t)blockIdx.x * R * R;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int a = a0 + ty + 8 * k, b = b0 + tx;
        if (a < R && b < R) P[(uint64_t)a * R + b] = acc[k];
    }
}

// Fixed-order sum of partials: out[e] = sum_p partials[p][e].
__global__ __launch_bounds__(kT) void sum_parts_k(const double *__restrict__ partials, int nparts, int64_t n,
                                                  double *__restrict__ out, const int *status) {
    if (status && *status) return;
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int p = 0; p < nparts; p++) s += partials[(int64_t)p * n + e];
    out[e] = s;
}

// Row solves A(i, c) = sum_k Mn(i, k) Vinv(k, c) (FP64).  Thread (r, c) of a
// block handles column c of rows r, r + rows_per_pass, ...; Vinv is staged in
// LDS when R <= 64.  The solve is done twice (column norms first, then the
// normalized store) rather than keeping an FP64 copy of A_n.

__device__ __forceinline__ double solve_elem(const float *__restrict__ Mn, const double *__restrict__ vv, uint64_t i,
                                             int R, int c) {
    const float *m = Mn + i * R;
    double s = 0.0;
    for (int k = 0; k < R; k++) s += (double)m[k] * vv[k * R + c];
    return s;
}

// Per-block column sums of squares of the solved rows (no store).
__global__ __launch_bounds__(kT) void solve_norms_k(const float *__restrict__ Mn, const double *__restrict__ Vinv,
                                                    uint64_t I, int R, double *__restrict__ colsq_part,
                                                    const int *status) {
    extern __shared__ double sh[];
    if (*status) return;
    const bool vin_lds = R <= 64;
    double *sv = sh;
    double *red = sh + (vin_lds ? R * R : 0);  // kT partial sums
    if (vin_lds)
        for (int e = threadIdx.x; e < R * R; e += kT) sv[e] = Vinv[e];
    __syncthreads();
    const double *vv = vin_lds ? sv : Vinv;
    const int rows = R >= kT ? 1 : kT / R;
    const int r = threadIdx.x / R, c = threadIdx.x % R;
    double acc = 0.0;
    if (r < rows && threadIdx.x < rows * R) {
        for (uint64_t i = (uint64_t)blockIdx.x * rows + r; i < I; i += (uint64_t)gridDim.x * rows) {
            const double a = solve_elem(Mn, vv, i, R, c);
            acc += a * a;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    // R <= kT, so every column has a thread in row 0 of the block
    for (int cc = threadIdx.x; cc < R; cc += kT) {
        double s = 0.0;
        for (int q = 0; q < rows; q++) s += red[q * R + cc];
        colsq_part[(uint64_t)blockIdx.x * R + cc] = s;
    }
}

// lambda_c = sqrt(sum of the partial column sums of squares)
__global__ __launch_bounds__(kT) void lambda_k(const double *__restrict__ colsq_part, int nparts, int R,
                                               double *__restrict__ lambda, const int *status) {
    if (*status) return;
    for (int c = blockIdx.x * kT + threadIdx.x; c < R; c += gridDim.x * kT) {
        double s = 0.0;
        for (int p = 0; p < nparts; p++) s += colsq_part[(uint64_t)p * R + c];
        lambda[c] = sqrt(s);
    }
}

// A(i, c) = store(solve(i, c) / lambda_c) in the storage precision; for the
// last mode also the partial inner products sum_i lambda_c Mn(i,c) A(i,c).
__global__ __launch_bounds__(kT) void normalize_k(const float *__restrict__ Mn, const double *__restrict__ Vinv,
                                                  const double *__restrict__ lambda, uint64_t I, int R, int prec,
                                                  void *__restrict__ A, double *__restrict__ inner_part,
                                                  const int *status) {
    extern __shared__ double sh[];
    __shared__ double red[kT / 64];
    if (*status) return;
    const bool vin_lds = R <= 64;
    if (vin_lds)
        for (int e = threadIdx.x; e < R * R; e += kT) sh[e] = Vinv[e];
    __syncthreads();
    const double *vv = vin_lds ? sh : Vinv;
    const uint64_t n = I * (uint64_t)R;
    double inner = 0.0;
    for (uint64_t e = (uint64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (uint64_t)gridDim.x * kT) {
        const uint64_t i = e / R;
        const int c = (int)(e - i * R);
        const double lam = lambda[c];
        const double s = solve_elem(Mn, vv, i, R, c);
        const double a = lam > 0.0 ? s / lam : s;
        const float f = (float)a;
        double stored;
        if (prec == ALTO_PREC_BF16) {
            const uint16_t b = f32_to_bf16_rne(f);
            reinterpret_cast<uint16_t *>(A)[e] = b;
            stored = (double)__uint_as_float((uint32_t)b << 16);
        } else {
            reinterpret_cast<float *>(A)[e] = f;
            stored = (double)f;
        }
        if (inner_part) inner += lam * (double)Mn[e] * stored;
    }
    if (!inner_part) return;
    for (int off = 32; off >= 1; off >>= 1) inner += __shfl_xor(inner, off);
    if (__lane_id() == 0) red[threadIdx.x / 64] = inner;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kT / 64; w++) s += red[w];
        inner_part[blockIdx.x] = s;
    }
}

// fit = 1 - sqrt(max(0, |X|^2 + |Xhat|^2 - 2 <X,Xhat>)) / |X|
__global__ __launch_bounds__(kT) void fit_k(const double *__restrict__ G, int N, int R,
                                            const double *__restrict__ lambda, const double *__restrict__ inner_part,
                                            int nparts, double norm2, double *__restrict__ fit_out,
                                            const int *status) {
    __shared__ double red[kT / 64];
    __shared__ double red2[kT / 64];
    if (*status) return;
    const int RR = R * R;
    double xh = 0.0, in = 0.0;
    for (int e = threadIdx.x; e < RR; e += kT) {
        double h = lambda[e / R] * lambda[e % R];
        for (int m = 0; m < N; m++) h *= G[(int64_t)m * RR + e];
        xh += h;
    }
    for (int p = threadIdx.x; p < nparts; p += kT) in += inner_part[p];
    for (int off = 32; off >= 1; off >>= 1) {
        xh += __shfl_xor(xh, off);
        in += __shfl_xor(in, off);
    }
    if (__lane_id() == 0) {
        red[threadIdx.x / 64] = xh;
        red2[threadIdx.x / 64] = in;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kT / 64; w++) {
            a += red[w];
            b += red2[w];
        }
        double r2 = norm2 + a - 2.0 * b;
        if (r2 < 0.0) r2 = 0.0;
        *fit_out = norm2 > 0.0 ? 1.0 - sqrt(r2) / sqrt(norm2) : 0.0;
    }
}

// ---------------------------------------------------------------- rank-specialized update
// For R in {8, 16, 32, 64} one mode update after the MTTKRP is: the normal
// equations inverted in one block (Gauss-Jordan, below), a pass of row solves
// for the column norms, and a pass that solves again, scales by lambda,
// stores the factor and accumulates its Gram matrix (and, for the last mode,
// the inner product of the fit) from the stored values.  Rows are processed
// in tiles of 1024 / R rows staged in LDS, several tiles' loads in flight;
// thread (row group, column c) keeps column c of V^-1 in registers.

// V = Hadamard of the Grams of every mode except `skip` (+ ridge on the
// diagonal), inverted in place by Gauss-Jordan elimination without pivoting.
// For a symmetric positive definite V every pivot is positive (the pivots are
// the squared diagonal of its Cholesky factor), so a pivot <= 0 is the same
// failure test as a failed Cholesky factorization; the ridge retry follows.
// The matrix lives in LDS when R <= 128, else it is inverted in place in Vinv.
constexpr int kGjPer = 16;  // matrix elements per thread held as (row, column) pairs

__global__ __launch_bounds__(1024) void normal_eq_gj_k(const double *__restrict__ G, int N, int R, int skip,
                                                       double *__restrict__ Vinv, int *status) {
    extern __shared__ double shm[];
    __shared__ double ridge;
    if (*status) return;
    const int RR = R * R;
    const bool in_lds = R <= 128;
    double *A = in_lds ? shm : Vinv;
    double *colk = shm + (in_lds ? RR : 0);
    double *rowk = colk + R;
    const int nt = blockDim.x;
    // the (row, column) of the thread's elements, computed once when there
    // are at most kGjPer of them (row R marks none)
    const bool few = RR <= kGjPer * nt;
    int ei[kGjPer], ej[kGjPer];
#pragma unroll
    for (int q = 0; q < kGjPer; q++) {
        const int e = threadIdx.x + q * nt;
        ei[q] = e < RR ? e / R : R;
        ej[q] = e < RR ? e % R : 0;
    }
    bool bad = false;
    for (int attempt = 0; attempt < 2; attempt++) {
        if (threadIdx.x == 0) {
            double tr = 0.0;
            if (attempt > 0)  // the trace is only needed for the retry
                for (int r = 0; r < R; r++) {
                    double v = 1.0;
                    for (int m = 0; m < N; m++)
                        if (m != skip) v *= G[(int64_t)m * RR + r * R + r];
                    tr += v;
                }
            ridge = 1e-10 * tr / R;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < RR; e += nt) {
            double v = 1.0;
            for (int m = 0; m < N; m++)
                if (m != skip) v *= G[(int64_t)m * RR + e];
            A[e] = v + ((e / R == e % R) ? ridge : 0.0);
        }
        __syncthreads();
        bad = false;
        for (int k = 0; k < R; k++) {
            const double piv = A[k * R + k];
            if (!(piv > 0.0)) {  // same value in every thread: a uniform exit
                bad = true;
                break;
            }
            const double rp = 1.0 / piv;
            for (int i = threadIdx.x; i < R; i += nt) {
                colk[i] = A[i * R + k];
                rowk[i] = A[k * R + i] * rp;
            }
            __syncthreads();
            auto update = [&](int e, int i, int j) {
                double v;
                if (i == k) v = j == k ? rp : rowk[j];
                else if (j == k) v = -colk[i] * rp;
                else v = A[e] - colk[i] * rowk[j];
                A[e] = v;
            };
            if (few) {
#pragma unroll
                for (int q = 0; q < kGjPer; q++)
                    if (ei[q] < R) update(threadIdx.x + q * nt, ei[q], ej[q]);
            } else {
                for (int e = threadIdx.x; e < RR; e += nt) update(e, e / R, e % R);
            }
            __syncthreads();
        }
        if (!bad) break;
        __syncthreads();
    }
    if (bad) {
        if (threadIdx.x == 0) *status = 1;
        return;
    }
    if (in_lds)
        for (int e = threadIdx.x; e < RR; e += nt) Vinv[e] = A[e];
}

// The same elimination in one wave for R <= 32, with the matrix in
// registers: lane l holds column l % 32 of rows l / 32 + 2q (q < 16); only
// the pivot row and column go through LDS.  Each step reads all it needs
// first and then updates every element with selects, so the LDS round trips
// of a step overlap.  Per element the operations and their order are those
// of normal_eq_gj_k (only the retry's trace is summed in another order).
__global__ __launch_bounds__(64) void normal_eq_gj_wave_k(const double *__restrict__ G, int N, int R, int skip,
                                                          double *__restrict__ Vinv, int *status) {
    __shared__ double rowk[32], colk[32];
    if (*status) return;
    const int RR = R * R;
    const int lane = threadIdx.x, j = lane & 31, h = lane >> 5;
    double a[16];
    // V = Hadamard product of the Grams, multiplied in mode order; all of a
    // Gram's loads are issued together
    auto build = [&](double ridge) {
#pragma unroll
        for (int q = 0; q < 16; q++) a[q] = 1.0;
        for (int m = 0; m < N; m++) {
            if (m == skip) continue;
            double g[16];
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int i = h + 2 * q;
                g[q] = i < R && j < R ? G[(int64_t)m * RR + i * R + j] : 1.0;
            }
#pragma unroll
            for (int q = 0; q < 16; q++) a[q] *= g[q];
        }
#pragma unroll
        for (int q = 0; q < 16; q++) a[q] += h + 2 * q == j ? ridge : 0.0;
    };
    bool bad = false;
    for (int attempt = 0; attempt < 2; attempt++) {
        double ridge = 0.0;
        if (attempt > 0) {  // the trace is only needed for the retry
            double d = 0.0;
            if (lane < R) {
                d = 1.0;
                for (int m = 0; m < N; m++)
                    if (m != skip) d *= G[(int64_t)m * RR + lane * R + lane];
            }
            for (int off = 32; off >= 1; off >>= 1) d += __shfl_xor(d, off);
            ridge = 1e-10 * d / R;
        }
        build(ridge);
        bad = false;
        for (int k = 0; k < R; k++) {
            __syncthreads();  // the previous step's reads are done
            // row k lives in lanes with h == k % 2, register k / 2
            double rk = 0.0;
#pragma unroll
            for (int q = 0; q < 16; q++) {
                rk = q == (k >> 1) ? a[q] : rk;
            }
            if (h == (k & 1) && j < R) rowk[j] = rk;
            if (j == k) {
#pragma unroll
                for (int q = 0; q < 16; q++)
                    if (h + 2 * q < R) colk[h + 2 * q] = a[q];
            }
            __syncthreads();
            const double piv = rowk[k];
            if (!(piv > 0.0)) {  // the same value in every lane
                bad = true;
                break;
            }
            double ci[16];
#pragma unroll
            for (int q = 0; q < 16; q++) ci[q] = h + 2 * q < R ? colk[h + 2 * q] : 0.0;
            const double rp = 1.0 / piv;
            const double rj = (j < R ? rowk[j] : 0.0) * rp;
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int i = h + 2 * q;
                const double other = a[q] - ci[q] * rj;
                const double colv = -ci[q] * rp;
                const double rowv = j == k ? rp : rj;
                a[q] = i == k ? rowv : (j == k ? colv : other);
            }
        }
        if (!bad) break;
    }
    if (bad) {
        if (lane == 0) *status = 1;
        return;
    }
#pragma unroll
    for (int q = 0; q < 16; q++) {
        const int i = h + 2 * q;
        if (i < R && j < R) Vinv[i * R + j] = a[q];
    }
}

template <int R>
struct SolveShape {
    static constexpr int kRG = kT / R;       // row groups (threads per column)
    static constexpr int kRPT = 4;           // rows per thread per tile
    static constexpr int kTR = kRG * kRPT;   // rows per tile
    static constexpr int kDepth = 4;         // tiles in flight per block (loads issued ahead)
};

// Thread's float4 of tile `tile` of Mn (zeros past I, no load at all there).
template <int R>
__device__ __forceinline__ float4 load_tile(const float *__restrict__ Mn, uint64_t I, uint64_t tile) {
    constexpr int TR = SolveShape<R>::kTR;
    static_assert(TR * R == 4 * kT, "a tile is one float4 per thread");
    const uint64_t r0 = tile * TR;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r0 + (4u * threadIdx.x) / R < I) q = *reinterpret_cast<const float4 *>(Mn + r0 * R + 4u * threadIdx.x);
    return q;
}

// Runs body(tile) for the block's tiles (blockIdx.x, + gridDim.x, ...) with
// the tile staged in Ms.  The loads of the next kDepth tiles are in flight
// while a tile is processed, so a block keeps kDepth * 4 KiB of reads
// outstanding instead of stalling on one tile at a time.
template <int R, class Body>
__device__ __forceinline__ void for_each_tile(const float *__restrict__ Mn, uint64_t I, float *Ms, Body body) {
    using S = SolveShape<R>;
    constexpr int D = S::kDepth;
    const uint64_t ntiles = (I + S::kTR - 1) / S::kTR;
    const uint64_t stride = gridDim.x;
    float4 q[D];
#pragma unroll
    for (int j = 0; j < D; j++) q[j] = load_tile<R>(Mn, I, blockIdx.x + j * stride);
    for (uint64_t t0 = blockIdx.x; t0 < ntiles; t0 += D * stride) {
#pragma unroll
        for (int j = 0; j < D; j++) {
            const uint64_t tile = t0 + j * stride;
            if (tile >= ntiles) break;  // same for the whole block
            reinterpret_cast<float4 *>(Ms)[threadIdx.x] = q[j];
            q[j] = load_tile<R>(Mn, I, tile + D * stride);
            __syncthreads();
            body(tile);
            __syncthreads();
        }
    }
}

template <int R>
__device__ __forceinline__ double row_dot(const float *Ms, int r, const double (&vc)[R]) {
    const float4 *m = reinterpret_cast<const float4 *>(Ms + r * R);
    double s = 0.0;
#pragma unroll
    for (int k4 = 0; k4 < R / 4; k4++) {
        const float4 q = m[k4];
        s = fma((double)q.x, vc[4 * k4 + 0], s);
        s = fma((double)q.y, vc[4 * k4 + 1], s);
        s = fma((double)q.z, vc[4 * k4 + 2], s);
        s = fma((double)q.w, vc[4 * k4 + 3], s);
    }
    return s;
}

// Pass 1: per-block column sums of squares of A = Mn V^-1.
template <int R>
__global__ __launch_bounds__(kT) void solve_colsq_k(const float *__restrict__ Mn, const double *__restrict__ Vinv,
                                                    uint64_t I, double *__restrict__ colsq_part, const int *status) {
    using S = SolveShape<R>;
    __shared__ __align__(16) float Ms[S::kTR * R];
    __shared__ double red[kT];
    if (*status) return;
    const int c = threadIdx.x % R, rg = threadIdx.x / R;
    double vc[R];
#pragma unroll
    for (int k = 0; k < R; k++) vc[k] = Vinv[k * R + c];
    double acc = 0.0;
    for_each_tile<R>(Mn, I, Ms, [&](uint64_t) {
#pragma unroll
        for (int q = 0; q < S::kRPT; q++) {
            const double a = row_dot<R>(Ms, rg + S::kRG * q, vc);
            acc = fma(a, a, acc);
        }
    });
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < R) {
        double s = 0.0;
        for (int g = 0; g < S::kRG; g++) s += red[g * R + threadIdx.x];
        colsq_part[(uint64_t)blockIdx.x * R + threadIdx.x] = s;
    }
}

// Register blocking of the Gram accumulation: thread (slice s, sub-block b)
// sums the 4x4 sub-block b of A^T A over the tile rows s, s + kS, ...  Each
// row then costs four 16-byte LDS reads for 16 FMAs.
template <int R>
struct GramShape {
    static constexpr int kB = R / 4;                 // sub-blocks per side
    static constexpr int kNB = kB * kB;              // sub-blocks
    static_assert(kT % kNB == 0, "sub-blocks divide the block");
    static constexpr int kS = kT / kNB;              // row slices
    static constexpr int kEPT = (R * R + kT - 1) / kT;  // Gram entries per thread in the final fold
};

// Pass 2: A(i, c) = store(solve(i, c) / lambda_c); per-block partial Gram of
// the stored rows, and (inner_part != nullptr) the partial inner products
// sum_i lambda_c Mn(i, c) A(i, c).
template <int R>
__global__ __launch_bounds__(kT) void normalize_gram_k(const float *__restrict__ Mn, const double *__restrict__ Vinv,
                                                       const double *__restrict__ lambda, uint64_t I, int prec,
                                                       void *__restrict__ A, double *__restrict__ gram_part,
                                                       double *__restrict__ inner_part, const int *status) {
    using S = SolveShape<R>;
    using GS = GramShape<R>;
    constexpr int TR = S::kTR;
    __shared__ __align__(16) float Ms[TR * R];
    __shared__ __align__(16) double As[TR * R];
    __shared__ double red[kT / 64];
    if (*status) return;
    const int c = threadIdx.x % R, rg = threadIdx.x / R;
    const int blk = threadIdx.x % GS::kNB, slice = threadIdx.x / GS::kNB;
    const int bi = blk / GS::kB, bj = blk % GS::kB;
    double vc[R];
#pragma unroll
    for (int k = 0; k < R; k++) vc[k] = Vinv[k * R + c];
    const double lam = lambda[c];
    double g[16];
#pragma unroll
    for (int j = 0; j < 16; j++) g[j] = 0.0;
    double inner = 0.0;
    for_each_tile<R>(Mn, I, Ms, [&](uint64_t tile) {
        const uint64_t r0 = tile * TR;
#pragma unroll
        for (int q = 0; q < S::kRPT; q++) {
            const int r = rg + S::kRG * q;
            const double s = row_dot<R>(Ms, r, vc);
            const double a = lam > 0.0 ? s / lam : s;
            const float f = (float)a;
            double stored = 0.0;
            if (r0 + r < I) {
                const uint64_t e = (r0 + r) * R + c;
                if (prec == ALTO_PREC_BF16) {
                    const uint16_t b = f32_to_bf16_rne(f);
                    reinterpret_cast<uint16_t *>(A)[e] = b;
                    stored = (double)__uint_as_float((uint32_t)b << 16);
                } else {
                    reinterpret_cast<float *>(A)[e] = f;
                    stored = (double)f;
                }
                inner += lam * (double)Ms[r * R + c] * stored;
            }
            As[r * R + c] = stored;
        }
        __syncthreads();
        for (int r = slice; r < TR; r += GS::kS) {
            const double2 *row = reinterpret_cast<const double2 *>(As + r * R);
            const double2 x0 = row[2 * bi], x1 = row[2 * bi + 1];
            const double2 y0 = row[2 * bj], y1 = row[2 * bj + 1];
            const double x[4] = {x0.x, x0.y, x1.x, x1.y}, y[4] = {y0.x, y0.y, y1.x, y1.y};
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int v = 0; v < 4; v++) g[4 * u + v] = fma(x[u], y[v], g[4 * u + v]);
        }
    });
    // fold the slices' partial sums in slice order, a tile's worth of slices
    // at a time through As, into entries threadIdx.x + j * kT of the block's Gram
    double *P = gram_part + (uint64_t)blockIdx.x * R * R;
    if constexpr (GS::kS == 1) {
#pragma unroll
        for (int u = 0; u < 4; u++)
#pragma unroll
            for (int v = 0; v < 4; v++) P[(4 * bi + u) * R + 4 * bj + v] = g[4 * u + v];
    } else {
        constexpr int kPer = (TR * R) / (R * R);  // slices per round
        static_assert(GS::kS % kPer == 0, "whole rounds");
        double tot[GS::kEPT];
#pragma unroll
        for (int j = 0; j < GS::kEPT; j++) tot[j] = 0.0;
        for (int s0 = 0; s0 < GS::kS; s0 += kPer) {
            if (slice >= s0 && slice < s0 + kPer) {
                double *dst = As + (slice - s0) * R * R;
#pragma unroll
                for (int u = 0; u < 4; u++)
#pragma unroll
                    for (int v = 0; v < 4; v++) dst[(4 * bi + u) * R + 4 * bj + v] = g[4 * u + v];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < GS::kEPT; j++) {
                const int e = threadIdx.x + j * kT;
                if (e < R * R)
                    for (int k = 0; k < kPer; k++) tot[j] += As[k * R * R + e];
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < GS::kEPT; j++) {
            const int e = threadIdx.x + j * kT;
            if (e < R * R) P[e] = tot[j];
        }
    }
    if (!inner_part) return;
    for (int off = 32; off >= 1; off >>= 1) inner += __shfl_xor(inner, off);
    if (__lane_id() == 0) red[threadIdx.x / 64] = inner;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < kT / 64; w++) sum += red[w];
        inner_part[blockIdx.x] = sum;
    }
}

// ---------------------------------------------------------------- FP64 matrix cores (R = 16, 32)
// The row solves as 16-row tile products on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): S = Mn_tile V^-1, then the Gram of the stored
// tile, S_st^T S_st, from the same registers.  Every wave streams its own
// tiles (no LDS, no barriers in the loop).  Operand layout of the
// instruction (16x4 A, 4x16 B, 16x16 D): lane l holds A(l%16, l/16) and
// B(l/16, l%16); register q of D holds D(4q + l/16, l%16).  A lane loads
// the float4s at columns 4(l/16 + 4t) .. +3 of tile row l%16; the solve's
// contraction index runs over them in that order, and the matching rows
// of V^-1 sit in registers.  Register q of the solve's output block then
// holds rows 4q + l/16 of the tile: exactly the A and B operands of the
// Gram product over those four rows.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int R>
struct MfShape {
    static_assert(R == 16 || R == 32, "matrix-core row solves for R = 16, 32");
    static constexpr int kB = R / 16;          // 16-column blocks; also float4 loads per lane per tile
    static constexpr int kWaves = kT / 64;
};

template <int R>
__device__ __forceinline__ void mf_load(const float *__restrict__ Mn, uint64_t I, uint64_t tile, int lane,
                                        float4 (&q)[MfShape<R>::kB]) {
    const uint64_t row = tile * 16 + (lane & 15);
#pragma unroll
    for (int t = 0; t < MfShape<R>::kB; t++)
        q[t] = row < I ? *reinterpret_cast<const float4 *>(Mn + row * R + 4 * ((lane >> 4) + 4 * t))
                       : make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int R>
__device__ __forceinline__ void mf_vinv(const double *__restrict__ Vinv, int lane,
                                        double (&vb)[MfShape<R>::kB][4][MfShape<R>::kB]) {
#pragma unroll
    for (int t = 0; t < MfShape<R>::kB; t++)
#pragma unroll
        for (int e = 0; e < 4; e++)
#pragma unroll
            for (int cb = 0; cb < MfShape<R>::kB; cb++)
                vb[t][e][cb] = Vinv[(4 * ((lane >> 4) + 4 * t) + e) * R + 16 * cb + (lane & 15)];
}

// s[cb][q] = S(4q + l/16, 16 cb + l%16) of the tile
template <int R>
__device__ __forceinline__ void mf_solve(const float4 (&q)[MfShape<R>::kB],
                                         const double (&vb)[MfShape<R>::kB][4][MfShape<R>::kB],
                                         dbl4 (&s)[MfShape<R>::kB]) {
    constexpr int B = MfShape<R>::kB;
#pragma unroll
    for (int cb = 0; cb < B; cb++) s[cb] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < B; t++) {
        const double a[4] = {(double)q[t].x, (double)q[t].y, (double)q[t].z, (double)q[t].w};
#pragma unroll
        for (int e = 0; e < 4; e++)
#pragma unroll
            for (int cb = 0; cb < B; cb++) s[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], vb[t][e][cb], s[cb], 0, 0, 0);
    }
}

// Runs body(tile, q) over the wave's tiles (global wave w: tiles w, w + W,
// ...), with the next tile's loads in flight.
template <int R, class Body>
__device__ __forceinline__ void mf_for_each_tile(const float *__restrict__ Mn, uint64_t I, int lane, Body body) {
    constexpr int B = MfShape<R>::kB;
    const uint64_t nw = (uint64_t)gridDim.x * MfShape<R>::kWaves;
    const uint64_t w = (uint64_t)blockIdx.x * MfShape<R>::kWaves + threadIdx.x / 64;
    const uint64_t ntiles = (I + 15) / 16;
    float4 q[B];
    mf_load<R>(Mn, I, w, lane, q);
    for (uint64_t tile = w; tile < ntiles; tile += nw) {
        float4 cur[B];
#pragma unroll
        for (int t = 0; t < B; t++) cur[t] = q[t];
        mf_load<R>(Mn, I, tile + nw, lane, q);
        body(tile, cur);
    }
}

// Pass 1 on the matrix cores: per-block column sums of squares of S.
template <int R>
__global__ __launch_bounds__(kT) void solve_colsq_mf_k(const float *__restrict__ Mn, const double *__restrict__ Vinv,
                                                       uint64_t I, double *__restrict__ colsq_part,
                                                       const int *status) {
    constexpr int B = MfShape<R>::kB;
    __shared__ double red[MfShape<R>::kWaves][R];
    if (*status) return;
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    double vb[B][4][B];
    mf_vinv<R>(Vinv, lane, vb);
    double cs[B];
#pragma unroll
    for (int cb = 0; cb < B; cb++) cs[cb] = 0.0;
    mf_for_each_tile<R>(Mn, I, lane, [&](uint64_t, const float4 (&q)[B]) {
        dbl4 s[B];
        mf_solve<R>(q, vb, s);
#pragma unroll
        for (int cb = 0; cb < B; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++) cs[cb] = fma(s[cb][r], s[cb][r], cs[cb]);
    });
#pragma unroll
    for (int cb = 0; cb < B; cb++) {
        cs[cb] += __shfl_xor(cs[cb], 16);
        cs[cb] += __shfl_xor(cs[cb], 32);
        if (lane < 16) red[wave][16 * cb + lane] = cs[cb];
    }
    __syncthreads();
    if (threadIdx.x < R) {
        double sum = 0.0;
        for (int w = 0; w < MfShape<R>::kWaves; w++) sum += red[w][threadIdx.x];
        colsq_part[(uint64_t)blockIdx.x * R + threadIdx.x] = sum;
    }
}

// Pass 2 on the matrix cores: A = store(S / lambda), per-block partial Gram
// of the stored rows, and (inner_part != nullptr) the partial inner products
// sum_i lambda_c Mn(i, c) A(i, c).
template <int R>
__global__ __launch_bounds__(kT) void normalize_gram_mf_k(const float *__restrict__ Mn,
                                                          const double *__restrict__ Vinv,
                                                          const double *__restrict__ lambda, uint64_t I, int prec,
                                                          void *__restrict__ A, double *__restrict__ gram_part,
                                                          double *__restrict__ inner_part, const int *status) {
    constexpr int B = MfShape<R>::kB;
    constexpr int W = MfShape<R>::kWaves;
    __shared__ double red[W][R * R];
    __shared__ double ired[W];
    if (*status) return;
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    double vb[B][4][B];
    mf_vinv<R>(Vinv, lane, vb);
    double lam[B];
#pragma unroll
    for (int cb = 0; cb < B; cb++) lam[cb] = lambda[16 * cb + (lane & 15)];
    dbl4 g[B][B];
#pragma unroll
    for (int a = 0; a < B; a++)
#pragma unroll
        for (int b = 0; b < B; b++) g[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    double inner = 0.0;
    const bool with_inner = inner_part != nullptr;
    mf_for_each_tile<R>(Mn, I, lane, [&](uint64_t tile, const float4 (&q)[B]) {
        dbl4 s[B];
        mf_solve<R>(q, vb, s);
        dbl4 st[B];
#pragma unroll
        for (int cb = 0; cb < B; cb++) {
            const int c = 16 * cb + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const uint64_t row = tile * 16 + 4 * r + (lane >> 4);
                const double a = lam[cb] > 0.0 ? s[cb][r] / lam[cb] : s[cb][r];
                const float f = (float)a;
                double stored = 0.0;
                if (row < I) {
                    const uint64_t e = row * R + c;
                    if (prec == ALTO_PREC_BF16) {
                        const uint16_t b = f32_to_bf16_rne(f);
                        reinterpret_cast<uint16_t *>(A)[e] = b;
                        stored = (double)__uint_as_float((uint32_t)b << 16);
                    } else {
                        reinterpret_cast<float *>(A)[e] = f;
                        stored = (double)f;
                    }
                    if (with_inner) inner += lam[cb] * (double)Mn[e] * stored;
                }
                st[cb][r] = stored;
            }
        }
#pragma unroll
        for (int a = 0; a < B; a++)
#pragma unroll
            for (int b = 0; b < B; b++)
#pragma unroll
                for (int r = 0; r < 4; r++) g[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(st[a][r], st[b][r], g[a][b], 0, 0, 0);
    });
    // block (a, b), register q of lane l: Gram(16a + 4q + l/16, 16b + l%16)
#pragma unroll
    for (int a = 0; a < B; a++)
#pragma unroll
        for (int b = 0; b < B; b++)
#pragma unroll
            for (int qq = 0; qq < 4; qq++)
                red[wave][(16 * a + 4 * qq + (lane >> 4)) * R + 16 * b + (lane & 15)] = g[a][b][qq];
    if (with_inner) {
        for (int off = 32; off >= 1; off >>= 1) inner += __shfl_xor(inner, off);
        if (lane == 0) ired[wave] = inner;
    }
    __syncthreads();
    double *P = gram_part + (uint64_t)blockIdx.x * R * R;
    for (int e = threadIdx.x; e < R * R; e += kT) {
        double sum = 0.0;
        for (int w = 0; w < W; w++) sum += red[w][e];
        P[e] = sum;
    }
    if (with_inner && threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < W; w++) sum += ired[w];
        inner_part[blockIdx.x] = sum;
    }
}

// Fixed-order reduction of partials in two levels: slice y of the grid sums
// partials [y*P/S, (y+1)*P/S) into tmp[y], then sum_slices_k adds the S
// slices.  out[e] = sum_p partials[p][e] for every launch size.
constexpr int kSlices = 16;

__global__ __launch_bounds__(kT) void sum_slices_partial_k(const double *__restrict__ partials, int nparts,
                                                           int64_t n, double *__restrict__ tmp, const int *status) {
    if (status && *status) return;
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n) return;
    const int y = blockIdx.y;
    const int p0 = (int)((int64_t)nparts * y / kSlices), p1 = (int)((int64_t)nparts * (y + 1) / kSlices);
    double s = 0.0;
#pragma unroll 8
    for (int p = p0; p < p1; p++) s += partials[(int64_t)p * n + e];  // loads overlap, adds in order
    tmp[(int64_t)y * n + e] = s;
}

// out[e] = sum of the slices (sqrt_out: lambda = sqrt of the column sums)
__global__ __launch_bounds__(kT) void sum_slices_k(const double *__restrict__ tmp, int64_t n,
                                                   double *__restrict__ out, int sqrt_out, const int *status) {
    if (status && *status) return;
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n) return;
    double s = 0.0;
    for (int y = 0; y < kSlices; y++) s += tmp[(int64_t)y * n + e];
    out[e] = sqrt_out ? sqrt(s) : s;
}

__global__ __launch_bounds__(kT) void round_bf16_k(const double *__restrict__ in, uint16_t *__restrict__ out,
                                                   int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
        out[e] = f32_to_bf16_rne((float)in[e]);
}

int parts_for(uint64_t I) {
    const uint64_t p = (I + 255) / 256;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(kMaxParts, p));
}

struct AlsWs {
    float *Mn;
    double *G, *Vinv, *parts, *colsq, *inner, *fit, *tmp;
    int *status;
};

// Blocks of the rank-specialized passes: as many as are resident at once
// (occupancy x compute units, at most kMaxSolveBlocks), so that each block
// streams many tiles with several of them in flight.
constexpr int kMaxSolveBlocks = 2048;

struct SolveGrid {
    int solve = 1, norm = 1;
};

// R = 16 and 32 run the row solves on the FP64 matrix cores unless
// ALTO_CPALS_MFMA=0 asks for the vector kernels.
template <int R>
constexpr bool has_mf() { return R == 16 || R == 32; }

bool use_mf() {
    static const bool on = [] {
        const char *e = getenv("ALTO_CPALS_MFMA");
        return !(e && *e && atol(e) == 0);
    }();
    return on;
}

template <int R>
int solve_grid(SolveGrid *g) {
    int dev = 0, cus = 0, a = 0, b = 0;
    ALTO_HIP(hipGetDevice(&dev));
    ALTO_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if constexpr (has_mf<R>()) {
        if (use_mf()) {
            ALTO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void *)solve_colsq_mf_k<R>, kT, 0));
            ALTO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void *)normalize_gram_mf_k<R>, kT, 0));
        }
    }
    if (a == 0) {
        ALTO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void *)solve_colsq_k<R>, kT, 0));
        ALTO_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void *)normalize_gram_k<R>, kT, 0));
    }
    g->solve = std::clamp(a * cus, 1, kMaxSolveBlocks);
    g->norm = std::clamp(b * cus, 1, kMaxSolveBlocks);
    return ALTO_OK;
}

// One mode update after its MTTKRP (Mn), rank-specialized; see above.
template <int R>
int update_mode_r(AlsWs &w, const SolveGrid &grid, uint64_t I, int prec, void *factor, double *lambda, bool last,
                  int *nparts_inner, hipStream_t s) {
    bool mf = false;
    if constexpr (has_mf<R>()) mf = use_mf();
    // work units: 16-row tiles per wave of 4 (matrix cores), or tiles of 1024 / R rows
    const uint64_t units = mf ? ((I + 15) / 16 + kT / 64 - 1) / (kT / 64) : (I + SolveShape<R>::kTR - 1) / SolveShape<R>::kTR;
    const int nbs = (int)std::max<uint64_t>(1, std::min<uint64_t>(grid.solve, units));
    const int nbn = (int)std::max<uint64_t>(1, std::min<uint64_t>(grid.norm, units));
    double *inner = last ? w.inner : nullptr;
    if constexpr (has_mf<R>()) {
        if (mf) solve_colsq_mf_k<R><<<nbs, kT, 0, s>>>(w.Mn, w.Vinv, I, w.colsq, w.status);
    }
    if (!mf) solve_colsq_k<R><<<nbs, kT, 0, s>>>(w.Mn, w.Vinv, I, w.colsq, w.status);
    sum_slices_partial_k<<<dim3((R + kT - 1) / kT, kSlices), kT, 0, s>>>(w.colsq, nbs, R, w.tmp, w.status);
    sum_slices_k<<<(R + kT - 1) / kT, kT, 0, s>>>(w.tmp, R, lambda, 1, w.status);
    if constexpr (has_mf<R>()) {
        if (mf) normalize_gram_mf_k<R><<<nbn, kT, 0, s>>>(w.Mn, w.Vinv, lambda, I, prec, factor, w.parts, inner, w.status);
    }
    if (!mf) normalize_gram_k<R><<<nbn, kT, 0, s>>>(w.Mn, w.Vinv, lambda, I, prec, factor, w.parts, inner, w.status);
    const int64_t RR = (int64_t)R * R;
    sum_slices_partial_k<<<dim3((unsigned)((RR + kT - 1) / kT), kSlices), kT, 0, s>>>(w.parts, nbn, RR, w.tmp,
                                                                                  w.status);
    *nparts_inner = nbn;
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

int launch_gram(const void *A, int prec, uint64_t I, int R, double *G, double *partials, int nparts,
                hipStream_t s) {
    const int tiles = (R + kGramTile - 1) / kGramTile;
    gram_partial_k<<<dim3(nparts, tiles * tiles), kT, 0, s>>>(A, prec, I, R, nparts, partials);
    const int64_t n = (int64_t)R * R;
    sum_parts_k<<<(unsigned)((n + kT - 1) / kT), kT, 0, s>>>(partials, nparts, n, G, nullptr);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int launch_round_bf16(const double *in, uint16_t *out, int64_t n, hipStream_t s) {
    if (n == 0) return ALTO_OK;
    const int64_t g = std::min<int64_t>(65536, (n + kT - 1) / kT);
    round_bf16_k<<<(unsigned)g, kT, 0, s>>>(in, out, n);
    ALTO_HIP(hipGetLastError());
    return ALTO_OK;
}

int cp_als_impl(alto_tensor *t, int R, int iters, int prec, void *const *factors, double *lambda, double *fit,
                const alto_exec *ex, hipStream_t s) {
    if (!t) return set_error(ALTO_E_INVAL, "null tensor handle");
    if (R < 1 || R > ALTO_MAX_RANK) return set_error(ALTO_E_INVAL, "R must be in 1..256");
    if (iters < 0) return set_error(ALTO_E_INVAL, "iters must be >= 0");
    if (prec != ALTO_PREC_F32 && prec != ALTO_PREC_BF16) return set_error(ALTO_E_INVAL, "unknown precision");
    if (!factors || !lambda || (iters > 0 && !fit)) return set_error(ALTO_E_INVAL, "null argument");
    for (int n = 0; n < t->N; n++)
        if (!factors[n]) return set_error(ALTO_E_INVAL, "null factor pointer");
    if (t->nnz == 0) return set_error(ALTO_E_INVAL, "CP-ALS of an empty tensor");
    for (int n = 0; n < t->N; n++)
        if (t->dims[n] > 0xffffffffull)
            return set_error(ALTO_E_INVAL, "CP-ALS needs every mode to have fewer than 2^32 rows");
    const int N = t->N;
    uint64_t maxI = 0;
    for (int n = 0; n < N; n++) maxI = std::max(maxI, t->dims[n]);
    const int RR = R * R;
    const int P = parts_for(maxI);
    int rc0 = ALTO_OK;
    // the MTTKRP output and the FP64 work arrays live in their own allocation
    // (the tensor workspace may be regrown by a re-partition)
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const bool special = R == 8 || R == 16 || R == 32 || R == 64;
    SolveGrid grid;
    if (special) {
        switch (R) {
            case 8: rc0 = solve_grid<8>(&grid); break;
            case 16: rc0 = solve_grid<16>(&grid); break;
            case 32: rc0 = solve_grid<32>(&grid); break;
            default: rc0 = solve_grid<64>(&grid); break;
        }
        if (rc0) return rc0;
    }
    const size_t oMn = take(sizeof(float) * maxI * R),
                 oG = take(sizeof(double) * N * RR),
                 oVi = take(sizeof(double) * RR), oP = take(sizeof(double) * (size_t)std::max(P, grid.norm) * RR),
                 oC = take(sizeof(double) * (size_t)std::max(kMaxParts, grid.solve) * R),
                 oT = take(sizeof(double) * (size_t)kSlices * RR), oI = take(sizeof(double) * std::max(2048, kMaxSolveBlocks)),
                 oF = take(sizeof(double) * std::max(1, iters)), oS = take(sizeof(int));
    char *base = nullptr;
    ALTO_HIP(hipMalloc(&base, off));
    AlsWs w;
    w.Mn = (float *)(base + oMn);
    w.G = (double *)(base + oG);
    w.Vinv = (double *)(base + oVi);
    w.parts = (double *)(base + oP);
    w.colsq = (double *)(base + oC);
    w.inner = (double *)(base + oI);
    w.tmp = (double *)(base + oT);
    w.fit = (double *)(base + oF);
    w.status = (int *)(base + oS);
    int rc = ALTO_OK;
    auto done = [&](int code) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(base);
        return code;
    };
#define ALS_HIP(call)                                            \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return done(hip_error(e_, #call)); \
    } while (0)
    ALS_HIP(hipMemsetAsync(w.status, 0, sizeof(int), s));
    for (int n = 0; n < N; n++) {
        rc = launch_gram(factors[n], prec, t->dims[n], R, w.G + (size_t)n * RR, w.parts, parts_for(t->dims[n]), s);
        if (rc) return done(rc);
    }
    const size_t vin_lds = sizeof(double) * (R <= 64 ? RR : 0);
    const size_t neq_lds = sizeof(double) * ((R <= 128 ? RR : 0) + 2 * R);
    const int neq_threads = RR <= 1024 ? 256 : 1024;
    if (neq_lds > 64 * 1024)
        ALS_HIP(hipFuncSetAttribute((const void *)normal_eq_gj_k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)neq_lds));
    for (int it = 0; it < iters; it++) {
        for (int n = 0; n < N; n++) {
            const uint64_t I = t->dims[n];
            rc = plan_and_run_mttkrp(t, (const void *const *)factors, R, prec, n, w.Mn, ex, s);
            if (rc) return done(rc);
            if (R <= 32) normal_eq_gj_wave_k<<<1, 64, 0, s>>>(w.G, N, R, n, w.Vinv, w.status);
            else normal_eq_gj_k<<<1, neq_threads, neq_lds, s>>>(w.G, N, R, n, w.Vinv, w.status);
            const bool last = n == N - 1;
            if (special) {
                int nin = 0;
                switch (R) {
                    case 8: rc = update_mode_r<8>(w, grid, I, prec, factors[n], lambda, last, &nin, s); break;
                    case 16: rc = update_mode_r<16>(w, grid, I, prec, factors[n], lambda, last, &nin, s); break;
                    case 32: rc = update_mode_r<32>(w, grid, I, prec, factors[n], lambda, last, &nin, s); break;
                    default: rc = update_mode_r<64>(w, grid, I, prec, factors[n], lambda, last, &nin, s); break;
                }
                if (rc) return done(rc);
                sum_slices_k<<<(unsigned)((RR + kT - 1) / kT), kT, 0, s>>>(w.tmp, RR, w.G + (size_t)n * RR, 0,
                                                                           w.status);
                if (last) fit_k<<<1, kT, 0, s>>>(w.G, N, R, lambda, w.inner, nin, t->norm2, w.fit + it, w.status);
                ALS_HIP(hipGetLastError());
                continue;
            }
            const int rows = R >= kT ? 1 : kT / R;
            const int gsolve = (int)std::max<uint64_t>(1, std::min<uint64_t>(kMaxParts, (I + rows - 1) / rows));
            solve_norms_k<<<gsolve, kT, vin_lds + sizeof(double) * kT, s>>>(w.Mn, w.Vinv, I, R, w.colsq, w.status);
            lambda_k<<<(R + kT - 1) / kT, kT, 0, s>>>(w.colsq, gsolve, R, lambda, w.status);
            const uint64_t elems = I * (uint64_t)R;
            const int gnorm = (int)std::min<uint64_t>(2048, (elems + kT - 1) / kT);
            normalize_k<<<gnorm, kT, vin_lds, s>>>(w.Mn, w.Vinv, lambda, I, R, prec, factors[n],
                                                   last ? w.inner : nullptr, w.status);
            const int Pn = parts_for(I);
            const int tiles = (R + kGramTile - 1) / kGramTile;
            gram_partial_k<<<dim3(Pn, tiles * tiles), kT, 0, s>>>(factors[n], prec, I, R, Pn, w.parts);
            sum_parts_k<<<(unsigned)((RR + kT - 1) / kT), kT, 0, s>>>(w.parts, Pn, RR, w.G + (size_t)n * RR,
                                                                     w.status);
            if (last) fit_k<<<1, kT, 0, s>>>(w.G, N, R, lambda, w.inner, gnorm, t->norm2, w.fit + it, w.status);
            ALS_HIP(hipGetLastError());
        }
    }
    int st = 0;
    ALS_HIP(hipMemcpyAsync(&st, w.status, sizeof(int), hipMemcpyDeviceToHost, s));
    if (iters > 0) ALS_HIP(hipMemcpyAsync(fit, w.fit, sizeof(double) * iters, hipMemcpyDeviceToHost, s));
    ALS_HIP(hipStreamSynchronize(s));
#undef ALS_HIP
    if (st) return done(set_error(ALTO_E_NOTSPD, "normal-equation matrix is not positive definite"));
    return done(ALTO_OK);
}

}  // namespace alto
