/*
 * Seeded synthetic sparse-tensor generator.
 *
 * Produces COO coordinates, values and dense factor matrices from a seed.
 * It holds none of the tensor method's arithmetic (no linearization,
 * ordering, partitioning or products); both the HIP library's tests and
 * the CPU oracle take their inputs from here.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a
 * counter-based generator: stream k of seed s draws its i-th word as
 * mix(state_k + (i + 1) * gamma) with state_k = mix(s + (k + 1) * gamma),
 * so results do not depend on the number of threads.
 *
 * Index distributions per mode: uniform, or finite Zipf(s) over ranks
 * 1..I (P(r) proportional to r^-s) sampled by inversion of its table of
 * cumulative weights with a guide table (Chen & Asau 1974); ranks map to
 * indices through a seeded Fisher-Yates permutation so that hot indices
 * are spread over the mode rather than clustered at 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t stream_state(uint64_t seed, uint64_t k) { return mix64(seed + (k + 1) * GAMMA); }
static inline uint64_t draw(uint64_t st, uint64_t i) { return mix64(st + (i + 1) * GAMMA); }
static inline double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }         /* [0,1) */
static inline double u01_open(uint64_t w) { return ((double)(w >> 11) + 1.0) * 0x1.0p-53; } /* (0,1] */

/* Raw words of one stream (exposed for the generator's own tests). */
void synth_words(uint64_t seed, uint64_t stream, int64_t n, uint64_t *out)
{
    uint64_t st = stream_state(seed, stream);
    for (int64_t i = 0; i < n; i++) out[i] = draw(st, (uint64_t)i);
}

/* perm[r] = index of rank r (0-based), seeded Fisher-Yates. */
static void make_perm(uint64_t seed, uint64_t stream, uint32_t I, uint32_t *perm)
{
    uint64_t st = stream_state(seed, stream);
    for (uint32_t r = 0; r < I; r++) perm[r] = r;
    for (uint32_t r = I; r > 1; r--) {
        uint64_t w = draw(st, (uint64_t)(I - r));
        uint32_t j = (uint32_t)(((unsigned __int128)w * r) >> 64);
        uint32_t t = perm[r - 1];
        perm[r - 1] = perm[j];
        perm[j] = t;
    }
}

/*
 * Coordinates of one mode: M draws, indices in [0, I).
 * s <= 0: uniform; s > 0: Zipf(s) over ranks mapped through a permutation.
 * Stream numbers used: 2*mode+1 for the draws, 2*mode+2 for the permutation.
 * Returns 0, or -1 on allocation failure.
 */
int synth_mode_coords(uint64_t seed, int mode, uint32_t I, double s, int64_t M, uint32_t *out)
{
    uint64_t st = stream_state(seed, (uint64_t)(2 * mode + 1));
    if (s <= 0.0) {
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < M; x++)
            out[x] = (uint32_t)(((unsigned __int128)draw(st, (uint64_t)x) * I) >> 64);
        return 0;
    }
    double *cdf = (double *)malloc((size_t)I * sizeof(double));
    uint32_t *perm = (uint32_t *)malloc((size_t)I * sizeof(uint32_t));
    const uint32_t G = I < (1u << 20) ? I : (1u << 20);
    uint32_t *guide = (uint32_t *)malloc(((size_t)G + 1) * sizeof(uint32_t));
    if (!cdf || !perm || !guide) { free(cdf); free(perm); free(guide); return -1; }
    double acc = 0.0;
    for (uint32_t r = 0; r < I; r++) { acc += pow((double)r + 1.0, -s); cdf[r] = acc; }
    for (uint32_t r = 0; r < I; r++) cdf[r] /= acc;
    cdf[I - 1] = 1.0;
    /* guide[j] = first rank whose cumulative weight exceeds j/G */
    {
        uint32_t r = 0;
        for (uint32_t j = 0; j <= G; j++) {
            double th = (double)j / (double)G;
            while (r < I - 1 && cdf[r] <= th) r++;
            guide[j] = r;
        }
    }
    make_perm(seed, (uint64_t)(2 * mode + 2), I, perm);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < M; x++) {
        double u = u01(draw(st, (uint64_t)x));
        uint32_t j = (uint32_t)(u * G);
        uint32_t lo = guide[j], hi = guide[j + 1 <= G ? j + 1 : G];
        /* smallest r in [lo, hi] with cdf[r] > u */
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > u) hi = mid; else lo = mid + 1;
        }
        out[x] = perm[lo];
    }
    free(cdf);
    free(perm);
    free(guide);
    return 0;
}

/* Values: dist 0 = U(0,1) on a 2^-24 grid, dist 1 = lognormal(0,1) (Box-Muller),
 * both rounded to binary32.  Stream 1000. */
void synth_values(uint64_t seed, int dist, int64_t M, float *out)
{
    uint64_t st = stream_state(seed, 1000);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < M; x++) {
        if (dist == 0) {
            out[x] = (float)((double)(draw(st, (uint64_t)x) >> 40) * 0x1.0p-24);
        } else {
            double u1 = u01_open(draw(st, 2 * (uint64_t)x));
            double u2 = u01(draw(st, 2 * (uint64_t)x + 1));
            double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            out[x] = (float)exp(z);
        }
    }
}

/* Dense factor matrix I x R (row-major) with entries k/256, k uniform in
 * 1..255, so every entry is exactly representable in bfloat16 and binary32.
 * Stream 2000 + mode. */
void synth_factor(uint64_t seed, int mode, int64_t I, int R, float *out)
{
    uint64_t st = stream_state(seed, 2000 + (uint64_t)mode);
    int64_t n = I * (int64_t)R;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; q++) {
        uint64_t k = 1 + (((draw(st, (uint64_t)q) >> 32) * 255ull) >> 32);
        out[q] = (float)k * (1.0f / 256.0f);
    }
}
