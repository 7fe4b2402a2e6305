/*
 * FP64 CPU oracle for ALTO-based sparse MTTKRP and CP-ALS.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no source with the HIP
 * library (no headers, helpers or tables in common).
 *
 * Every routine here is the plain definition of what the method computes,
 * written to be checked by eye against the paper
 *   "ALTO: Adaptive Linearized Storage of Sparse Tensors" (Helal et al.,
 *   ICS 2021, arXiv 2102.10245),
 * with no blocking, fusion or reordering beyond what the definition states.
 * Floating point is IEEE double throughout, except the BF16 rounding rule,
 * which is defined on the binary32 bit pattern.
 *
 * Conventions: coordinates are 0-based uint32; `coords` is an array of N
 * pointers, each to M coordinates (structure of arrays); factor matrices
 * are row-major I_n x R; a linearized index of up to 128 bits is held as
 * two uint64 words (lo, hi).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXN 16

/* ------------------------------------------------------------------ */
/* Bit layout (Section 3.1, the encoding of the 4x8x2 example and      */
/* Eq. 1).  b_n = ceil(log2 I_n) bits per mode, 0 for a mode of length */
/* 1.  The bits are handed out one "level" at a time starting from the */
/* least significant end: level l holds bit l of every mode that has   */
/* more than l bits, and inside a level the shorter mode takes the     */
/* lower position (ties: lower mode number first).  Hence the most     */
/* significant bits belong to the longest mode, i.e. the space is      */
/* split along the longest mode first.                                 */
/* ------------------------------------------------------------------ */

static int or_ceil_log2(uint64_t x)
{
    int b = 0;
    while (b < 64 && ((uint64_t)1 << b) < x) b++;
    return b;
}

/* Returns B (total bits) on success, -1 if a dim is 0 or above 2^32,
 * -2 if B exceeds 128.  nbits[n], mask_lo[n], mask_hi[n] are outputs. */
int oracle_layout(int N, const uint64_t *dims, int *nbits, uint64_t *mask_lo,
                  uint64_t *mask_hi)
{
    int order[OR_MAXN];
    int maxb = 0, pos = 0;
    if (N < 1 || N > OR_MAXN) return -1;
    for (int n = 0; n < N; n++) {
        if (dims[n] == 0 || dims[n] > ((uint64_t)1 << 32)) return -1;
        nbits[n] = or_ceil_log2(dims[n]);
        if (nbits[n] > maxb) maxb = nbits[n];
        mask_lo[n] = mask_hi[n] = 0;
        order[n] = n;
    }
    /* modes by increasing length; equal lengths keep mode order */
    for (int a = 1; a < N; a++) {
        int v = order[a], b = a - 1;
        while (b >= 0 && dims[order[b]] > dims[v]) { order[b + 1] = order[b]; b--; }
        order[b + 1] = v;
    }
    for (int lvl = 0; lvl < maxb; lvl++) {
        for (int q = 0; q < N; q++) {
            int n = order[q];
            if (nbits[n] <= lvl) continue;
            if (pos >= 128) return -2;
            if (pos < 64) mask_lo[n] |= (uint64_t)1 << pos;
            else          mask_hi[n] |= (uint64_t)1 << (pos - 64);
            pos++;
        }
    }
    return pos;
}

/* Linearization = bit-level gather (Section 3.1, Fig. 4a): the k-th
 * lowest set bit of MASK(n) receives bit k of i_n. */
static void or_encode_one(int N, const uint32_t *idx, const uint64_t *mask_lo,
                          const uint64_t *mask_hi, uint64_t *lo, uint64_t *hi)
{
    uint64_t l = 0, h = 0;
    for (int n = 0; n < N; n++) {
        int k = 0;
        for (int p = 0; p < 128; p++) {
            uint64_t m = p < 64 ? (mask_lo[n] >> p) & 1 : (mask_hi[n] >> (p - 64)) & 1;
            if (!m) continue;
            if (k < 32 && ((idx[n] >> k) & 1u)) {
                if (p < 64) l |= (uint64_t)1 << p;
                else        h |= (uint64_t)1 << (p - 64);
            }
            k++;
        }
    }
    *lo = l;
    *hi = h;
}

void oracle_encode(int N, int64_t M, const uint32_t *const *coords,
                   const uint64_t *mask_lo, const uint64_t *mask_hi,
                   uint64_t *key_lo, uint64_t *key_hi)
{
    uint32_t idx[OR_MAXN];
    for (int64_t x = 0; x < M; x++) {
        for (int n = 0; n < N; n++) idx[n] = coords[n][x];
        or_encode_one(N, idx, mask_lo, mask_hi, &key_lo[x], &key_hi[x]);
    }
}

/* De-linearization = bit-level scatter, EXTRACT(pos, MASK(n)) of
 * Algorithm 1: bit k of i_n is the k-th lowest set bit of MASK(n). */
static uint32_t or_extract(uint64_t lo, uint64_t hi, uint64_t mlo, uint64_t mhi)
{
    uint64_t v = 0;
    int k = 0;
    for (int p = 0; p < 128; p++) {
        uint64_t m = p < 64 ? (mlo >> p) & 1 : (mhi >> (p - 64)) & 1;
        if (!m) continue;
        uint64_t bit = p < 64 ? (lo >> p) & 1 : (hi >> (p - 64)) & 1;
        v |= bit << k;
        k++;
    }
    return (uint32_t)v;
}

void oracle_decode(int N, int64_t M, const uint64_t *key_lo, const uint64_t *key_hi,
                   const uint64_t *mask_lo, const uint64_t *mask_hi,
                   uint32_t *const *coords)
{
    for (int64_t x = 0; x < M; x++)
        for (int n = 0; n < N; n++)
            coords[n][x] = or_extract(key_lo[x], key_hi ? key_hi[x] : 0,
                                      mask_lo[n], mask_hi[n]);
}

/* ------------------------------------------------------------------ */
/* Ordering (Section 3.1, second stage of generation): nonzeros are    */
/* arranged by the value of their linearized index.  Ties are kept in  */
/* input order (a stable sort).                                        */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t hi, lo; int64_t at; } or_kv;

static int or_cmp_kv(const void *a, const void *b)
{
    const or_kv *x = (const or_kv *)a, *y = (const or_kv *)b;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    return x->at < y->at ? -1 : (x->at > y->at);
}

/* perm[j] = input position of the j-th element in sorted order. */
int oracle_sort_perm(int64_t M, const uint64_t *key_lo, const uint64_t *key_hi, int64_t *perm)
{
    or_kv *a = (or_kv *)malloc((size_t)(M > 0 ? M : 1) * sizeof(or_kv));
    if (!a) return -1;
    for (int64_t x = 0; x < M; x++) {
        a[x].lo = key_lo[x];
        a[x].hi = key_hi ? key_hi[x] : 0;
        a[x].at = x;
    }
    qsort(a, (size_t)M, sizeof(or_kv), or_cmp_kv);
    for (int64_t x = 0; x < M; x++) perm[x] = a[x].at;
    free(a);
    return 0;
}

/* Coalescing of repeated positions (the paper does not discuss them;
 * a repeated coordinate is read as the sum of its values).  Input is
 * sorted; output keeps the first key of each run and the FP64 sum of the
 * run's values, taken in sorted (stable) order.  Returns M_unique. */
int64_t oracle_coalesce(int64_t M, const uint64_t *key_lo, const uint64_t *key_hi,
                        const double *vals, uint64_t *out_lo, uint64_t *out_hi,
                        double *out_vals)
{
    int64_t u = -1;
    for (int64_t x = 0; x < M; x++) {
        uint64_t h = key_hi ? key_hi[x] : 0;
        if (u < 0 || key_lo[x] != out_lo[u] || (out_hi ? out_hi[u] : 0) != h) {
            u++;
            out_lo[u] = key_lo[x];
            if (out_hi) out_hi[u] = h;
            out_vals[u] = 0.0;
        }
        out_vals[u] += vals[x];
    }
    return u + 1;
}

/* ------------------------------------------------------------------ */
/* Workload partitioning (Section 3.2): L line segments with the same  */
/* number of nonzeros.  When M is not a multiple of L, segment l is    */
/* [floor(l*M/L), floor((l+1)*M/L)).  L is capped at M.                */
/* ------------------------------------------------------------------ */

int oracle_partition(int64_t M, int L, int64_t *seg /* L_eff + 1 */)
{
    int Le = (int64_t)L < M ? L : (int)M;
    if (L < 1) return -1;
    for (int l = 0; l <= Le; l++)
        seg[l] = (int64_t)(((unsigned __int128)l * (unsigned __int128)M) / (unsigned __int128)Le);
    return Le;
}

/* Mode intervals T_{l,n} = [T^s, T^e] (Section 3.2): the smallest closed
 * coordinate range along mode n holding every nonzero of segment l.
 * ivl layout: ivl[(l*N + n)*2 + {0,1}] = {start, end}. */
void oracle_intervals(int N, int Le, const int64_t *seg, const uint64_t *key_lo,
                      const uint64_t *key_hi, const uint64_t *mask_lo,
                      const uint64_t *mask_hi, uint32_t *ivl)
{
    for (int l = 0; l < Le; l++) {
        for (int n = 0; n < N; n++) {
            uint32_t s = UINT32_MAX, e = 0;
            for (int64_t x = seg[l]; x < seg[l + 1]; x++) {
                uint32_t i = or_extract(key_lo[x], key_hi ? key_hi[x] : 0, mask_lo[n], mask_hi[n]);
                if (i < s) s = i;
                if (i > e) e = i;
            }
            ivl[((int64_t)l * N + n) * 2 + 0] = s;
            ivl[((int64_t)l * N + n) * 2 + 1] = e;
        }
    }
}

/* Coverage of output row b along mode n: the number of segments whose
 * mode-n interval holds b, i.e. the segments that pull into row b in the
 * accumulation of Algorithm 2.  A count of 1 marks an exclusive row. */
void oracle_coverage(int N, int Le, const uint32_t *ivl, int mode, uint64_t dim,
                     uint32_t *cov)
{
    for (uint64_t b = 0; b < dim; b++) {
        uint32_t c = 0;
        for (int l = 0; l < Le; l++) {
            uint32_t s = ivl[((int64_t)l * N + mode) * 2 + 0];
            uint32_t e = ivl[((int64_t)l * N + mode) * 2 + 1];
            if (s <= b && b <= e) c++;
        }
        cov[b] = c;
    }
}

/* ------------------------------------------------------------------ */
/* MTTKRP (Section 2.2; Algorithm 1, elementwise):                     */
/*   out(i, r) = sum over nonzeros x with i_mode(x) = i of             */
/*               v_x * prod_{m != mode} A_m(i_m(x), r).                */
/* Plain COO loop over the original coordinates; the ALTO ordering,    */
/* partitioning and conflict resolution only change summation order.   */
/* ------------------------------------------------------------------ */

void oracle_mttkrp(int N, int64_t M, const uint32_t *const *coords, const double *vals,
                   const uint64_t *dims, const double *const *factors, int R, int mode,
                   double *out)
{
    memset(out, 0, (size_t)dims[mode] * (size_t)R * sizeof(double));
    for (int64_t x = 0; x < M; x++) {
        double *o = out + (size_t)coords[mode][x] * (size_t)R;
        for (int r = 0; r < R; r++) {
            double p = vals[x];
            for (int m = 0; m < N; m++) {
                if (m == mode) continue;
                p *= factors[m][(size_t)coords[m][x] * (size_t)R + (size_t)r];
            }
            o[r] += p;
        }
    }
}

/* The same definition spread over the host's cores with OpenMP: thread t
 * sums a contiguous share of the nonzeros into an output of its own, and
 * those outputs are added in thread order at the end, so only the order of
 * the floating-point sums differs from oracle_mttkrp.  It exists to time
 * the oracle on every core.  Returns the number of threads used, or -1 if
 * the private outputs cannot be allocated. */
int oracle_mttkrp_par(int N, int64_t M, const uint32_t *const *coords, const double *vals,
                      const uint64_t *dims, const double *const *factors, int R, int mode,
                      double *out)
{
    const size_t n_out = (size_t)dims[mode] * (size_t)R;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nt * n_out, sizeof(double));
    if (!priv) return -1;
    int used = 1;
#pragma omp parallel num_threads(nt)
    {
        int t = 0, T = 1;
#ifdef _OPENMP
        t = omp_get_thread_num();
        T = omp_get_num_threads();
#endif
        if (t == 0) used = T;
        double *mine = priv + (size_t)t * n_out;
        const int64_t x0 = M * t / T, x1 = M * (t + 1) / T;
        for (int64_t x = x0; x < x1; x++) {
            double *o = mine + (size_t)coords[mode][x] * (size_t)R;
            for (int r = 0; r < R; r++) {
                double p = vals[x];
                for (int m = 0; m < N; m++) {
                    if (m == mode) continue;
                    p *= factors[m][(size_t)coords[m][x] * (size_t)R + (size_t)r];
                }
                o[r] += p;
            }
        }
    }
    memset(out, 0, n_out * sizeof(double));
    for (int t = 0; t < used; t++)
        for (size_t q = 0; q < n_out; q++) out[q] += priv[(size_t)t * n_out + q];
    free(priv);
    return used;
}

/* Same definition restricted to a list of output rows (for checks at
 * sizes where the full dense output is not needed).  rows[] are distinct.
 * out is nrows x R. */
int oracle_mttkrp_rows(int N, int64_t M, const uint32_t *const *coords, const double *vals,
                       const uint64_t *dims, const double *const *factors, int R, int mode,
                       int64_t nrows, const uint32_t *rows, double *out)
{
    int64_t *slot = (int64_t *)malloc((size_t)dims[mode] * sizeof(int64_t));
    if (!slot) return -1;
    for (uint64_t b = 0; b < dims[mode]; b++) slot[b] = -1;
    for (int64_t q = 0; q < nrows; q++) slot[rows[q]] = q;
    memset(out, 0, (size_t)nrows * (size_t)R * sizeof(double));
    for (int64_t x = 0; x < M; x++) {
        int64_t q = slot[coords[mode][x]];
        if (q < 0) continue;
        for (int r = 0; r < R; r++) {
            double p = vals[x];
            for (int m = 0; m < N; m++) {
                if (m == mode) continue;
                p *= factors[m][(size_t)coords[m][x] * (size_t)R + (size_t)r];
            }
            out[q * R + r] += p;
        }
    }
    free(slot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* CP-ALS (Section 2.2).  The paper gives no formulas and defers to    */
/* SPLATT / Tensor Toolbox; this is the standard Kolda-Bader ALS:      */
/*   for each mode n:  M_n = MTTKRP_n;  V = Hadamard of G_m, m != n;   */
/*   A_n = M_n V^{-1} (Cholesky; one ridge retry);  lambda = column    */
/*   2-norms of A_n;  A_n /= lambda;  G_n = A_n^T A_n.                 */
/*   fit = 1 - ||X - Xhat|| / ||X||, after the last mode.              */
/* ------------------------------------------------------------------ */

/* In-place lower Cholesky of the R x R row-major matrix a.  0 on success. */
static int or_cholesky(int R, double *a)
{
    for (int j = 0; j < R; j++) {
        double d = a[j * R + j];
        for (int k = 0; k < j; k++) d -= a[j * R + k] * a[j * R + k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        a[j * R + j] = d;
        for (int i = j + 1; i < R; i++) {
            double s = a[i * R + j];
            for (int k = 0; k < j; k++) s -= a[i * R + k] * a[j * R + k];
            a[i * R + j] = s / d;
        }
        for (int i = 0; i < j; i++) a[i * R + j] = 0.0;
    }
    return 0;
}

typedef struct { const uint32_t *const *c; int N; } or_tuple_ctx;
static or_tuple_ctx or_tctx;

static int or_cmp_tuple(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    for (int n = 0; n < or_tctx.N; n++) {
        uint32_t u = or_tctx.c[n][x], v = or_tctx.c[n][y];
        if (u != v) return u < v ? -1 : 1;
    }
    return x < y ? -1 : (x > y);
}

/* ||X||^2 of the tensor a COO list describes (repeated coordinates summed). */
double oracle_norm2(int N, int64_t M, const uint32_t *const *coords, const double *vals)
{
    int64_t *ord = (int64_t *)malloc((size_t)(M > 0 ? M : 1) * sizeof(int64_t));
    double s = 0.0, run = 0.0;
    if (!ord) return -1.0;
    for (int64_t x = 0; x < M; x++) ord[x] = x;
    or_tctx.c = coords;
    or_tctx.N = N;
    qsort(ord, (size_t)M, sizeof(int64_t), or_cmp_tuple);
    for (int64_t j = 0; j < M; j++) {
        int same = j > 0;
        for (int n = 0; same && n < N; n++)
            if (coords[n][ord[j]] != coords[n][ord[j - 1]]) same = 0;
        if (!same && j > 0) { s += run * run; run = 0.0; }
        run += vals[ord[j]];
    }
    if (M > 0) s += run * run;
    free(ord);
    return s;
}

/* Gram G = A^T A (R x R) of an I x R matrix.  Every entry is the sum over
 * rows i = 0, 1, ..., I-1 in that order (rows in the outer loop only so the
 * matrix is read row by row). */
static void or_gram(uint64_t I, int R, const double *A, double *G)
{
    for (int q = 0; q < R * R; q++) G[q] = 0.0;
    for (uint64_t i = 0; i < I; i++)
        for (int a = 0; a < R; a++)
            for (int b = 0; b < R; b++) G[a * R + b] += A[i * R + a] * A[i * R + b];
}

/* factors: N pointers to I_n x R FP64 matrices (in: initial guess; out:
 * the normalized result).  lambda: R.  fit: iters entries.  Returns 0, or
 * -1 if a normal-equation matrix stays non-positive-definite after the
 * ridge, -2 on allocation failure. */
int oracle_cp_als(int N, int64_t M, const uint32_t *const *coords, const double *vals,
                  const uint64_t *dims, int R, int iters, double *const *factors,
                  double *lambda, double *fit)
{
    double *G = (double *)malloc((size_t)N * R * R * sizeof(double));
    double *V = (double *)malloc((size_t)R * R * sizeof(double));
    uint64_t maxI = 0;
    for (int n = 0; n < N; n++) if (dims[n] > maxI) maxI = dims[n];
    double *Mn = (double *)malloc((size_t)maxI * R * sizeof(double));
    double *y = (double *)malloc((size_t)R * sizeof(double));
    int rc = 0;
    if (!G || !V || !Mn || !y) { rc = -2; goto done; }

    double normX2 = oracle_norm2(N, M, coords, vals);
    for (int n = 0; n < N; n++) or_gram(dims[n], R, factors[n], G + (size_t)n * R * R);
    for (int r = 0; r < R; r++) lambda[r] = 1.0;

    for (int it = 0; it < iters; it++) {
        for (int n = 0; n < N; n++) {
            const uint64_t I = dims[n];
            double *A = factors[n];
            oracle_mttkrp(N, M, coords, vals, dims, (const double *const *)factors, R, n, Mn);

            /* V = Hadamard product of the other modes' Grams */
            for (int q = 0; q < R * R; q++) V[q] = 1.0;
            for (int m = 0; m < N; m++)
                if (m != n)
                    for (int q = 0; q < R * R; q++) V[q] *= G[(size_t)m * R * R + q];
            double *Vc = (double *)malloc((size_t)R * R * sizeof(double));
            if (!Vc) { rc = -2; goto done; }
            memcpy(Vc, V, (size_t)R * R * sizeof(double));
            if (or_cholesky(R, Vc) != 0) {
                double tr = 0.0;
                for (int r = 0; r < R; r++) tr += V[r * R + r];
                memcpy(Vc, V, (size_t)R * R * sizeof(double));
                for (int r = 0; r < R; r++) Vc[r * R + r] += 1e-10 * tr / R;
                if (or_cholesky(R, Vc) != 0) { free(Vc); rc = -1; goto done; }
            }
            /* A_n(i,:) = M_n(i,:) V^{-1}: solve L y = m, then L^T a = y */
            for (uint64_t i = 0; i < I; i++) {
                const double *m = Mn + i * R;
                for (int a = 0; a < R; a++) {
                    double s = m[a];
                    for (int k = 0; k < a; k++) s -= Vc[a * R + k] * y[k];
                    y[a] = s / Vc[a * R + a];
                }
                for (int a = R - 1; a >= 0; a--) {
                    double s = y[a];
                    for (int k = a + 1; k < R; k++) s -= Vc[k * R + a] * A[i * R + k];
                    A[i * R + a] = s / Vc[a * R + a];
                }
            }
            free(Vc);
            /* lambda = column 2-norms; normalize the columns */
            /* (column sums over i = 0..I-1 in order, rows in the outer loop) */
            for (int r = 0; r < R; r++) y[r] = 0.0;
            for (uint64_t i = 0; i < I; i++)
                for (int r = 0; r < R; r++) y[r] += A[i * R + r] * A[i * R + r];
            for (int r = 0; r < R; r++) lambda[r] = sqrt(y[r]);
            for (uint64_t i = 0; i < I; i++)
                for (int r = 0; r < R; r++)
                    if (lambda[r] > 0.0) A[i * R + r] /= lambda[r];
            or_gram(I, R, A, G + (size_t)n * R * R);
        }
        /* fit after the last mode:  ||X - Xhat||^2 = ||X||^2 + ||Xhat||^2 - 2<X,Xhat> */
        {
            double xhat2 = 0.0, inner = 0.0;
            for (int a = 0; a < R; a++)
                for (int b = 0; b < R; b++) {
                    double h = lambda[a] * lambda[b];
                    for (int m = 0; m < N; m++) h *= G[(size_t)m * R * R + a * R + b];
                    xhat2 += h;
                }
            const int last = N - 1;
            const double *A = factors[last];
            for (uint64_t i = 0; i < dims[last]; i++)
                for (int r = 0; r < R; r++) inner += lambda[r] * Mn[i * R + r] * A[i * R + r];
            double res2 = normX2 + xhat2 - 2.0 * inner;
            if (res2 < 0.0) res2 = 0.0;
            fit[it] = normX2 > 0.0 ? 1.0 - sqrt(res2) / sqrt(normX2) : 0.0;
        }
    }
done:
    free(G);
    free(V);
    free(Mn);
    free(y);
    return rc;
}

/* ------------------------------------------------------------------ */
/* BF16 storage rule: a double is first rounded to binary32 (round to  */
/* nearest even, the C conversion), then to bfloat16 by round to       */
/* nearest even on the upper 16 bits.  NaN stays a quiet NaN.          */
/* ------------------------------------------------------------------ */

uint16_t oracle_bf16_bits(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

void oracle_bf16_round(int64_t n, const double *in, uint16_t *bits, double *out)
{
    for (int64_t q = 0; q < n; q++) {
        uint16_t b = oracle_bf16_bits(in[q]);
        uint32_t u = (uint32_t)b << 16;
        float f;
        memcpy(&f, &u, 4);
        if (bits) bits[q] = b;
        if (out) out[q] = (double)f;
    }
}

/* ------------------------------------------------------------------ */
/* Conflict-resolution rule of Section 3.3: fiber reuse along mode n   */
/* is M / I_n; local staging is used when it is more than the four     */
/* memory operations of buffered accumulation, atomics otherwise.      */
/* Returns 1 for staging, 0 for atomics.                               */
/* ------------------------------------------------------------------ */

int oracle_heuristic_staging(int64_t M, uint64_t dim)
{
    return (double)M / (double)dim > 4.0;
}

/* ------------------------------------------------------------------ */
/* Selector network: a multilayer perceptron with two hidden layers of */
/* H units and ReLU,  y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,       */
/* loss = sum(mask * (y - t)^2) / sum(mask).  Forward and backward by  */
/* the chain rule.  Row-major weights: W1 H x F, W2 H x H, W3 K x H.   */
/* x: B x F, t and mask: B x K, y: B x K.                              */
/* ------------------------------------------------------------------ */

double oracle_mlp_forward(int B, int F, int H, int K, const double *W1, const double *b1,
                          const double *W2, const double *b2, const double *W3,
                          const double *b3, const double *x, const double *t,
                          const double *mask, double *y)
{
    double *h1 = (double *)malloc((size_t)H * sizeof(double));
    double *h2 = (double *)malloc((size_t)H * sizeof(double));
    double loss = 0.0, cnt = 0.0;
    for (int s = 0; s < B; s++) {
        for (int j = 0; j < H; j++) {
            double a = b1[j];
            for (int f = 0; f < F; f++) a += W1[j * F + f] * x[s * F + f];
            h1[j] = a > 0.0 ? a : 0.0;
        }
        for (int j = 0; j < H; j++) {
            double a = b2[j];
            for (int q = 0; q < H; q++) a += W2[j * H + q] * h1[q];
            h2[j] = a > 0.0 ? a : 0.0;
        }
        for (int k = 0; k < K; k++) {
            double a = b3[k];
            for (int q = 0; q < H; q++) a += W3[k * H + q] * h2[q];
            y[s * K + k] = a;
            if (t && mask) {
                double d = a - t[s * K + k];
                loss += mask[s * K + k] * d * d;
                cnt += mask[s * K + k];
            }
        }
    }
    free(h1);
    free(h2);
    return cnt > 0.0 ? loss / cnt : 0.0;
}

/* Gradients of the masked mean-squared loss with respect to every
 * weight and bias (accumulated over the batch, overwritten). */
double oracle_mlp_backward(int B, int F, int H, int K, const double *W1, const double *b1,
                           const double *W2, const double *b2, const double *W3,
                           const double *b3, const double *x, const double *t,
                           const double *mask, double *gW1, double *gb1, double *gW2,
                           double *gb2, double *gW3, double *gb3)
{
    double *z1 = (double *)malloc((size_t)H * sizeof(double));
    double *h1 = (double *)malloc((size_t)H * sizeof(double));
    double *z2 = (double *)malloc((size_t)H * sizeof(double));
    double *h2 = (double *)malloc((size_t)H * sizeof(double));
    double *d2 = (double *)malloc((size_t)H * sizeof(double));
    double *d1 = (double *)malloc((size_t)H * sizeof(double));
    double *dy = (double *)malloc((size_t)K * sizeof(double));
    double cnt = 0.0, loss = 0.0;
    for (int q = 0; q < B * K; q++) cnt += mask[q];
    memset(gW1, 0, (size_t)H * F * sizeof(double));
    memset(gb1, 0, (size_t)H * sizeof(double));
    memset(gW2, 0, (size_t)H * H * sizeof(double));
    memset(gb2, 0, (size_t)H * sizeof(double));
    memset(gW3, 0, (size_t)K * H * sizeof(double));
    memset(gb3, 0, (size_t)K * sizeof(double));
    for (int s = 0; s < B && cnt > 0.0; s++) {
        for (int j = 0; j < H; j++) {
            double a = b1[j];
            for (int f = 0; f < F; f++) a += W1[j * F + f] * x[s * F + f];
            z1[j] = a;
            h1[j] = a > 0.0 ? a : 0.0;
        }
        for (int j = 0; j < H; j++) {
            double a = b2[j];
            for (int q = 0; q < H; q++) a += W2[j * H + q] * h1[q];
            z2[j] = a;
            h2[j] = a > 0.0 ? a : 0.0;
        }
        for (int k = 0; k < K; k++) {
            double a = b3[k];
            for (int q = 0; q < H; q++) a += W3[k * H + q] * h2[q];
            double d = a - t[s * K + k];
            loss += mask[s * K + k] * d * d;
            dy[k] = 2.0 * mask[s * K + k] * d / cnt;
        }
        for (int k = 0; k < K; k++) {
            gb3[k] += dy[k];
            for (int q = 0; q < H; q++) gW3[k * H + q] += dy[k] * h2[q];
        }
        for (int q = 0; q < H; q++) {
            double g = 0.0;
            for (int k = 0; k < K; k++) g += W3[k * H + q] * dy[k];
            d2[q] = z2[q] > 0.0 ? g : 0.0;
        }
        for (int j = 0; j < H; j++) {
            gb2[j] += d2[j];
            for (int q = 0; q < H; q++) gW2[j * H + q] += d2[j] * h1[q];
        }
        for (int q = 0; q < H; q++) {
            double g = 0.0;
            for (int j = 0; j < H; j++) g += W2[j * H + q] * d2[j];
            d1[q] = z1[q] > 0.0 ? g : 0.0;
        }
        for (int j = 0; j < H; j++) {
            gb1[j] += d1[j];
            for (int f = 0; f < F; f++) gW1[j * F + f] += d1[j] * x[s * F + f];
        }
    }
    free(z1); free(h1); free(z2); free(h2); free(d2); free(d1); free(dy);
    return cnt > 0.0 ? loss / cnt : 0.0;
}
