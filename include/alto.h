/*
 * alto.h — C ABI of libalto, an MI355X (gfx950) library for sparse tensors
 * stored in the ALTO format and for the MTTKRP / CP-ALS computations on them.
 *
 * Paper: "ALTO: Adaptive Linearized Storage of Sparse Tensors",
 * Helal et al., ICS 2021 (arXiv 2102.10245).
 *
 * General rules for every entry point
 *   - Return value: ALTO_OK (0) or one of the ALTO_E_* codes below; on error
 *     alto_last_error() returns a message for the calling thread, and no
 *     output argument has been written unless stated otherwise.
 *   - Pointers marked "device" point to memory of the current HIP device,
 *     owned by the caller; pointers marked "host" point to host memory.
 *     The library never frees caller memory.
 *   - Streams: every call that launches device work takes a hipStream_t and
 *     enqueues its work on it, in order.  Unless a call says that it
 *     synchronizes, it returns before the work completes.
 *   - Indices are 0-based.  Dense matrices (factors, MTTKRP outputs) are
 *     row-major I x R with no padding (row r starts at element r*R).
 *   - A tensor handle may be used by one thread at a time.
 */
#ifndef ALTO_H
#define ALTO_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ALTO_MAX_MODES 8
#define ALTO_MAX_RANK 256

/* Error codes. */
#define ALTO_OK 0
#define ALTO_E_INVAL 1       /* bad argument: null pointer, N outside 2..8, a dim of 0 or above 2^32,
                                mode >= N, R outside 1..256, unknown enum value */
#define ALTO_E_TOO_WIDE 2    /* the linearized index needs more than 128 bits, or more bits than
                                a requested key width */
#define ALTO_E_RANGE 3       /* a coordinate is >= its dimension (checked when validation is on) */
#define ALTO_E_NOMEM 4       /* device allocation failed */
#define ALTO_E_HIP 5         /* a HIP runtime call failed */
#define ALTO_E_NOTSPD 6      /* CP-ALS: normal-equation matrix not positive definite after a ridge */
#define ALTO_E_STATE 7       /* call not valid for this handle (e.g. no selector weights loaded) */

/* Factor-matrix storage precision.  Accumulation is always FP32 in the
 * MTTKRP and FP64 in the CP-ALS normal equations. */
typedef enum {
    ALTO_PREC_F32 = 0,  /* factors are float (binary32) */
    ALTO_PREC_BF16 = 1  /* factors are bfloat16 bit patterns (uint16_t) */
} alto_prec;

/* Conflict resolution for the MTTKRP output (Section 3.3, Algorithm 2). */
typedef enum {
    ALTO_STRATEGY_AUTO = 0,    /* the plan alto_select describes (network, timing fallback, reuse rule) */
    ALTO_STRATEGY_ATOMIC = 1,  /* every partial result goes to the output by atomics, summed in an
                                  FP64 accumulator that is added into the output after the launch */
    ALTO_STRATEGY_STAGED = 2,  /* per-segment partials in on-chip local memory over the segment's
                                  mode interval, then merged into the output; segments whose
                                  interval does not fit fall back to atomics */
    ALTO_STRATEGY_SORTED = 3   /* inside every line segment the nonzeros are taken in order of
                                  their mode-n coordinate (a stable reordering built on first
                                  use and kept per mode: one extra copy of index and values), so
                                  each (segment, row) run is summed in registers and written
                                  with one FP32 atomic per column */
} alto_strategy;

typedef struct alto_tensor alto_tensor;  /* opaque */

/* Options of alto_build.  A NULL pointer means all defaults. */
typedef struct alto_opts {
    int key_bits;      /* 0: smallest of 32, 64, 128 that holds the index; else 32, 64 or 128 */
    int num_segments;  /* L, the number of line segments; 0: 8 per compute unit */
    int validate;      /* nonzero: check every coordinate against its dim (one extra pass) */
} alto_opts;

/* Execution choice of alto_mttkrp / cp_als.  A NULL pointer means AUTO
 * with the tensor's current partition. */
typedef struct alto_exec {
    int strategy;      /* alto_strategy */
    int num_segments;  /* 0: keep the current partition; else re-partition into this many */
} alto_exec;

/* Description of a built tensor (host struct filled by alto_info). */
typedef struct alto_info_t {
    int N;                                 /* number of modes */
    int index_bits;                        /* B = sum of per-mode bits (Eq. 1 per nonzero) */
    int key_bits;                          /* storage width of one index: 32, 64 or 128 */
    int num_segments;                      /* current L (at most nnz) */
    int64_t nnz_in;                        /* COO entries given to alto_build */
    int64_t nnz;                           /* distinct coordinates after coalescing repeats */
    uint64_t dims[ALTO_MAX_MODES];
    int mode_bits[ALTO_MAX_MODES];         /* b_n = ceil(log2 I_n), 0 when I_n = 1 */
    uint64_t mask_lo[ALTO_MAX_MODES];      /* MASK(n), bits 0..63 */
    uint64_t mask_hi[ALTO_MAX_MODES];      /* MASK(n), bits 64..127 */
    double fiber_reuse[ALTO_MAX_MODES];    /* nnz / I_n (Section 3.3) */
    double index_bytes;                    /* nnz * key_bits / 8 as stored */
    double coo_index_bytes;                /* nnz * N * 4 (uint32 COO coordinates) */
    double norm2;                          /* ||X||^2 in FP64 (sum of squared coalesced values) */
    /* device memory the handle holds now, in bytes (it grows as MTTKRP
     * plans are first used): */
    double tensor_bytes;                   /* the ALTO tensor: index, values, byte tables */
    double partition_bytes;                /* kept partitions: segment bounds, intervals,
                                              coverage, segment lists */
    double order_bytes;                    /* segment-local mode orders (`sorted`): per mode and
                                              kept partition, a reordered copy of index and values */
    double scratch_bytes;                  /* reusable workspace and per-XCD output replicas */
    int flag_bit[ALTO_MAX_MODES];          /* index bit of the mode's helper flag (Section 3.3),
                                              one of the spare bits at or above index_bits;
                                              -1: the mode has none */
} alto_info_t;

/*
 * alto_build — linearize a COO tensor and order it (Section 3.1), then cut
 * it into L equal-nonzero line segments with their mode intervals
 * (Section 3.2).
 *   coords  host array of N device pointers; coords[n] holds nnz uint32
 *           coordinates of mode n (structure of arrays).
 *   vals    device, nnz floats.
 *   nnz     number of COO entries, >= 0.  Repeated coordinates are summed
 *           into one nonzero (FP32, in input order).
 *   dims    host, N mode lengths, each in 1..2^32.
 *   N       2..8.
 *   opts    may be NULL.
 *   out     receives the new handle; free it with alto_free.
 * The handle owns device copies of the index and values; the caller's
 * buffers may be reused once the stream has passed this call.  This call
 * synchronizes the stream once (the count of distinct nonzeros and the
 * segment intervals come back to the host).
 */
int alto_build(const uint32_t *const *coords, const float *vals, int64_t nnz,
               const uint64_t *dims, int N, const alto_opts *opts, alto_tensor **out,
               hipStream_t stream);

/* alto_layout — the bit layout alto_build uses for these mode lengths
 * (Section 3.1), without building anything: fills N, index_bits, key_bits,
 * dims, mode_bits, mask_lo and mask_hi of *out (other fields zero).
 * key_bits as in alto_opts.  Host only; needs no GPU. */
int alto_layout(const uint64_t *dims, int N, int key_bits, alto_info_t *out);

/*
 * alto_append — add a batch of COO nonzeros to a built tensor (incremental
 * format generation, for streaming decomposition, where a tensor grows batch
 * by batch and the factors are refitted after each): the batch alone is
 * linearized and radix-sorted (Section 3.1), merged with the tensor's
 * ordered index in one pass, repeated coordinates are summed (the tensor's
 * value first, then the batch's in input order, FP32), and the partition is
 * rebuilt with the same requested segment count.  The result is bit for bit
 * the tensor alto_build makes from the earlier COO input followed by the
 * batch.  Arguments as for alto_build; the dims are the tensor's (every
 * coordinate must be below them: ALTO_E_RANGE otherwise, with the tensor
 * unchanged).  Segment-local orders and timed plans of the old tensor are
 * dropped.  Synchronizes the stream.
 */
int alto_append(alto_tensor *t, const uint32_t *const *coords, const float *vals, int64_t nnz,
                hipStream_t stream);

/* alto_info — fill *out (host) with the tensor's description.  No device work. */
int alto_info(const alto_tensor *t, alto_info_t *out);

/*
 * alto_partition — make the cut of the ordered tensor into L equal-nonzero
 * segments (Section 3.2) current: segment l holds positions
 * [floor(l*nnz/L), floor((l+1)*nnz/L)), L capped at nnz, with its mode
 * intervals and per-row coverage.  A partition built earlier (the last four
 * are kept) is reused; building one synchronizes the stream once.
 */
int alto_partition(alto_tensor *t, int num_segments, hipStream_t stream);

/*
 * alto_mttkrp — mode-`mode` MTTKRP (Section 2.2, Algorithms 1 and 2):
 *   out(i, r) = sum over nonzeros x with i_mode(x) = i of
 *               v_x * prod_{m != mode} A_m(i_m(x), r).
 *   factors  host array of N device pointers to I_m x R matrices in the
 *            precision `prec` (entry `mode` is not read and may be NULL);
 *            each pointer, and out, 16-byte aligned.
 *   R        1..256.
 *   out      device, I_mode x R floats; overwritten (rows with no nonzero
 *            become 0).
 *   ex       may be NULL (AUTO, current partition).  If ex->num_segments
 *            (or the selector's choice) differs from the current L, the
 *            partition into that many segments becomes the current one; it
 *            is built on first use (which synchronizes the stream) and kept,
 *            with up to three other recent partitions, for later calls.
 * Asynchronous otherwise.  Products and run sums in FP32; the strategies
 * that take the nonzeros in linearized order (atomic, staged) add them
 * into an FP64 accumulator that is rounded into out at the end, the
 * segment-local order (sorted) adds one FP32 atomic per (segment, row) run.
 * Atomics make the summation order, hence the last bits, run-dependent.
 */
int alto_mttkrp(alto_tensor *t, const void *const *factors, int R, int prec, int mode,
                float *out, const alto_exec *ex, hipStream_t stream);

/*
 * alto_mttkrp_noalloc — for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result as alto_mttkrp with
 * ex = {ALTO_STRATEGY_ATOMIC, 0}, on the tensor's current partition, with
 * no device allocation and no memset.  Its only scratch memory, the FP64
 * accumulator of the atomic updates (I_mode x R doubles), is a static
 * device array of 32 MiB that each GPU the library runs on holds until the
 * process ends.
 *   Arguments as for alto_mttkrp.  out is overwritten.
 *   Errors: ALTO_E_INVAL as alto_mttkrp, and when I_mode * R * 8 bytes
 *           exceed 32 MiB (I_mode * R <= 4 Mi); ALTO_E_STATE if the tensor
 *           has no partition.
 * Every call on one GPU shares that GPU's array and leaves the last call's
 * partial sums in it: calls that overlap in time on one GPU (on different
 * streams, or from several threads) race and give wrong results.  Calls
 * ordered on one stream are safe.  Asynchronous.
 */
int alto_mttkrp_noalloc(const alto_tensor *t, const void *const *factors, int R, int prec, int mode,
                        float *out, hipStream_t stream);

/*
 * cp_als — `iters` iterations of CP-ALS (Section 2.2): for each mode n in
 * turn, M_n = MTTKRP_n; V = Hadamard product of the Grams A_m^T A_m, m != n
 * (FP64); A_n = M_n V^{-1}, V inverted by Gauss-Jordan elimination whose
 * pivots must stay positive (the Cholesky criterion; one retry with a ridge
 * of 1e-10*trace(V)/R); lambda = column 2-norms; A_n /= lambda;
 * then the Gram of the stored A_n.  After the last mode of each iteration:
 * fit = 1 - ||X - [[lambda; A_1..A_N]]|| / ||X||.
 *   factors  host array of N device pointers, I_n x R in precision `prec`:
 *            the initial guess on entry, the normalized result on return.
 *   lambda   device, R doubles (output).
 *   fit      host, iters doubles (output).
 *   ex       strategy/partition for the MTTKRPs (NULL: AUTO per mode).
 * Synchronizes the stream once, at the end.  Returns ALTO_E_NOTSPD if a
 * normal-equation matrix stays indefinite (factors then hold the last
 * completed update).
 */
int cp_als(alto_tensor *t, int R, int iters, int prec, void *const *factors, double *lambda,
           double *fit, const alto_exec *ex, hipStream_t stream);

/*
 * alto_select — the execution the library would pick for an MTTKRP of this
 * mode and rank (ALTO_STRATEGY_AUTO):
 *   - no selector weights loaded: the reuse rule of Section 3.3 (staged if
 *     nnz / I_mode > 4, atomic otherwise) with the current L;
 *   - weights loaded, tensor inside the range the network was trained on:
 *     the network's choice; with the environment variable
 *     ALTO_SELECT_MARGIN = m > 0 (log2 time, default 0), when other
 *     candidates are predicted within m of that choice, the fastest of the
 *     (at most three) closest ones found by timing them, on the same terms
 *     as below;
 *   - weights loaded, tensor outside that range: the fastest candidate found
 *     by timing every (strategy, L) the network chooses among.  An AUTO
 *     alto_mttkrp or cp_als does that timing on first use of (mode, R, prec)
 *     and the tensor keeps the result; until then this call reports the reuse
 *     rule.
 * Host only.
 */
int alto_select(const alto_tensor *t, int mode, int R, int prec, alto_exec *out);

/*
 * alto_selector_load — install selector weights (host floats, layout:
 * header {F = 15, H, K, nL} then feature mean[F], feature scale[F], the
 * training range fmin[F], fmax[F], the nL candidate segment counts,
 * W1[H*F], b1[H], W2[H*H], b2[H], W3[K*H], b3[K], with K = S*nL outputs
 * (S = 2 or 3 strategies) = predicted log2 times of (atomic, L_0) ..
 * (atomic, L_{nL-1}), (staged, L_0) .. (staged, L_{nL-1}), then (sorted,
 * L_0) .. when S = 3.  The network sees (feature - mean) / scale.
 * n is the total float count; n == 0 unloads.
 */
int alto_selector_load(const float *weights, size_t n);

/* alto_selector_features — the F = 15 selector features of (tensor, mode,
 * R, prec), written to host `out`: log2 I_mode, log2 nnz, log2 nnz/I_mode,
 * N, log2 R, prec, B/32, key bits/64, log2 of the sum and of the largest of
 * the other dims, log2 bytes of the smallest other factor matrix,
 * log2 I_mode*R, and two measures of the mode's skew taken by alto_build
 * (and alto_append) from the row counts of S = min(nnz, 2^20) evenly spaced
 * nonzeros: log2(largest row count * I_mode / S) and log2(distinct rows in
 * the sample / min(S, I_mode)) (modes over 2^24 rows are counted in 2^24
 * hashed buckets); last, log2(max(1, nnz / 65536)) when R is 8, 16, 32 or 64
 * and the smallest other factor matrix takes at most 64 KB (the MTTKRP then
 * gathers it from LDS while segments hold at least 65 536 nonzeros), else -1.
 * Host only. */
int alto_selector_features(const alto_tensor *t, int mode, int R, int prec, float *out);

/*
 * Selector network kernels (two hidden layers of H ReLU units, K outputs):
 *   y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,  loss = sum(mask*(y-t)^2)/sum(mask).
 * All arrays are device float32, row-major; params = {W1[H*F], b1[H],
 * W2[H*H], b2[H], W3[K*H], b3[K]} packed in that order.
 * alto_mlp_forward writes y[B*K] and, if loss != NULL, the loss (device, 1 float).
 * alto_mlp_backward writes the gradient of the loss w.r.t. params (same
 * packing) into grads and the loss into loss (device, may be NULL).
 * alto_mlp_adam applies one Adam step (lr, beta1, beta2, eps, step count t>=1)
 * to params using the moment buffers m and v (device, same packing).
 */
int alto_mlp_forward(int B, int F, int H, int K, const float *params, const float *x,
                     const float *t, const float *mask, float *y, float *loss, hipStream_t stream);
int alto_mlp_backward(int B, int F, int H, int K, const float *params, const float *x,
                      const float *t, const float *mask, float *grads, float *loss,
                      hipStream_t stream);
int alto_mlp_adam(int64_t P, float *params, const float *grads, float *m, float *v, float lr,
                  float beta1, float beta2, float eps, int t, hipStream_t stream);

/*
 * Inspection of a built tensor (device-to-device copies into caller buffers):
 *   alto_export_keys:      keys_out (device) nnz indices of key_bits/8 bytes each
 *                          (128-bit indices as {lo, hi} uint64 pairs), vals_out
 *                          (device) nnz floats, in the tensor's order.  Either may be NULL.
 *   alto_export_partition: seg_out (device, L+1 int64 segment starts) and ivl_out
 *                          (device, L*N*2 uint32: [l][n] = {T^s, T^e}).  Either may be NULL.
 *   alto_export_coverage:  cov_out (device, I_mode uint32): number of segments
 *                          whose mode interval holds each row.
 *   alto_export_mode_order: the segment-local order by `mode` on the current
 *                          partition (the order the `sorted` strategy reads;
 *                          built now if it does not exist yet): keys_out and
 *                          vals_out as for alto_export_keys.  Inside every
 *                          segment the nonzeros are in increasing coordinate
 *                          along `mode`, ties in the tensor's order.
 */
int alto_export_keys(const alto_tensor *t, void *keys_out, float *vals_out, hipStream_t stream);
int alto_export_mode_order(alto_tensor *t, int mode, void *keys_out, float *vals_out, hipStream_t stream);
int alto_export_partition(const alto_tensor *t, int64_t *seg_out, uint32_t *ivl_out,
                          hipStream_t stream);
int alto_export_coverage(const alto_tensor *t, int mode, uint32_t *cov_out, hipStream_t stream);

/*
 * alto_transpose — sparse tensor transposition, one of the operations the
 * paper's related work (sparse tensor operations) names for the format:
 * the tensor's nonzeros in lexicographic order of their coordinates taken
 * in the mode order perm[0], perm[1], .., perm[N-1] (perm[0] most
 * significant), as COO.  Each linearized index is rewritten as the
 * lexicographic index of the permuted coordinates (the same B bits, grouped
 * by mode), then one stable LSD radix sort over those B bits orders them.
 *   perm        host, N distinct mode numbers.
 *   coords_out  host array of N device pointers; coords_out[j] receives nnz
 *               uint32 coordinates along mode perm[j].
 *   vals_out    device, nnz floats.
 * Allocates its own scratch (about 2 * (key_bits/8 + 4) bytes per nonzero)
 * and synchronizes the stream before returning.
 */
int alto_transpose(const alto_tensor *t, const int *perm, uint32_t *const *coords_out, float *vals_out,
                   hipStream_t stream);

/*
 * alto_export_flags — the helper flags of `mode` (Section 3.3: spare index
 * bits marking a nonzero as internal, i.e. its mode-`mode` row is updated by
 * no other unit of work, so the atomic strategy writes it without atomics).
 * Here the unit is a lane group: the current partition's segment l of S
 * nonzeros is cut into G groups, group g taking positions
 * [floor(l*nnz/L) + floor(S*g/G), floor(l*nnz/L) + floor(S*(g+1)/G)), and a
 * nonzero is flagged iff its row lies in the mode interval (min..max row,
 * Section 3.2) of no other group.  Flags are computed by the first
 * atomic-strategy MTTKRP of the mode on the partition (for the lane groups
 * of that launch).
 *   flags_out    device, nnz bytes (0/1) in the tensor's order; may be NULL.
 *   lane_groups  host, receives G; may be NULL.
 * ALTO_E_STATE if the mode has no flags for the current partition.
 */
int alto_export_flags(const alto_tensor *t, int mode, uint8_t *flags_out, int *lane_groups,
                      hipStream_t stream);

/*
 * alto_round_bf16 — storage rule for bfloat16 factors: each double is
 * rounded to binary32 (nearest even), then to bfloat16 (nearest even);
 * NaN stays a quiet NaN.  in: device n doubles; out: device n uint16.
 */
int alto_round_bf16(const double *in, uint16_t *out, int64_t n, hipStream_t stream);

/* alto_free — release the handle and its device memory (synchronizes the
 * device memory of the handle only; safe on NULL). */
void alto_free(alto_tensor *t);

/* alto_last_error — message of the calling thread's last failed call
 * ("" if none).  The pointer stays valid until the thread's next call. */
const char *alto_last_error(void);

/* alto_device_compute_units — compute units of the current device (host query). */
int alto_device_compute_units(void);

/*
 * Kernel timing, for measurement.  While enabled, every MTTKRP the library
 * runs (alto_mttkrp, and those inside alto_cp_als and the selector's timing
 * of candidates) records a pair of HIP events on its stream: the first just
 * before its first MTTKRP kernel, the second after its last one (the FP64
 * accumulator finish included).  The output clear and the plan set-up before
 * the kernels lie outside the pair, so the pair measures what a kernel trace
 * reports for the MTTKRP kernels of the call.
 *
 * alto_timing_enable — enable != 0 starts recording, 0 stops it (pairs
 *   already recorded stay until read).  Always ALTO_OK.
 * alto_timing_read — waits for every recorded pair and writes the sum of
 *   their elapsed times (milliseconds) to *ms_total and their number to
 *   *calls (host pointers), then clears the record.  ALTO_E_INVAL for a null
 *   pointer; a HIP error if an event cannot be read.
 * The record is per process, shared by all threads and streams.
 */
int alto_timing_enable(int enable);
int alto_timing_read(double *ms_total, int64_t *calls);

#ifdef __cplusplus
}
#endif

#endif /* ALTO_H */
