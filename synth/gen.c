/*
 * gen.c -- seeded synthetic sparse-matrix inputs (shared by tests, the oracle
 * checks and the benchmark).  Holds none of the product arithmetic: it only
 * draws row indices and values for a column-major pattern whose column
 * lengths were already chosen by the caller.
 *
 * Random numbers come from SplitMix64 used as a counter-based generator
 * (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): draw c of stream s under seed k is mix64(key(k,s) + (c+1)*G)
 * with G = 0x9E3779B97F4A7C15.  Every column / position has its own counter,
 * so the output does not depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix64(seed ^ mix64(stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL));
}
static inline uint64_t draw(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * GOLDEN); }
/* uniform in [0, 1) with 53 random bits */
static inline double unif(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }
/* uniform in (0, 1] */
static inline double unif_pos(uint64_t r) { return ((double)(r >> 11) + 1.0) * (1.0 / 9007199254740992.0); }

enum { STREAM_ROWS = 1, STREAM_VALS = 2, STREAM_DENSE = 3 };

/* Smallest index r with cdf[r] > u (cdf nondecreasing, cdf[len-1] == 1). */
static inline int64_t sample_cdf(const double *cdf, int64_t len, double u)
{
    int64_t lo = 0, hi = len - 1;
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct { double key; int32_t row; } keyed_t;
static int cmp_key_desc(const void *a, const void *b)
{
    double x = ((const keyed_t *)a)->key, y = ((const keyed_t *)b)->key;
    if (x > y) return -1;
    if (x < y) return 1;
    int32_t r = ((const keyed_t *)a)->row, s = ((const keyed_t *)b)->row;
    return (r > s) - (r < s);
}

/*
 * Fill row indices (strictly increasing within each column) and values.
 *   m, n, ptr       : the pattern's shape; column j gets ptr[j+1]-ptr[j] rows.
 *   rank_cdf, perm  : optional row-popularity law.  If rank_cdf is NULL rows are
 *                     uniform; otherwise a row rank r is drawn from the cumulative
 *                     table rank_cdf[0..m-1] and mapped to row perm[r].
 *   value_kind      : 0 uniform [-1,1); 1 random sign times exp(N(0,1));
 *                     2 integers in {-8..-1, 1..8}; 3 all ones.
 * Sampling is without replacement inside a column: rejection with a per-thread
 * bitmap when the column holds at most half the rows, weighted reservoir keys
 * u^(1/w) (Efraimidis & Spirakis, 2006) otherwise.  Returns 0 on success.
 */
int syn_fill(int64_t m, int64_t n, uint64_t seed, const int64_t *ptr,
             const double *rank_cdf, const int32_t *perm, int value_kind,
             int32_t *idx, double *val)
{
    const uint64_t krow = stream_key(seed, STREAM_ROWS);
    const uint64_t kval = stream_key(seed, STREAM_VALS);
    const uint64_t kden = stream_key(seed, STREAM_DENSE);
    int failed = 0;
#pragma omp parallel
    {
        uint8_t *seen = (uint8_t *)calloc((size_t)m + 1, 1);
        keyed_t *keys = NULL;
        if (!seen) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 4096)
        for (int64_t j = 0; j < n; ++j) {
            if (failed) continue;
            int64_t p0 = ptr[j], L = ptr[j + 1] - ptr[j];
            int32_t *rows = idx + p0;
            if (L <= 0) continue;
            if (L == m) {
                for (int64_t r = 0; r < m; ++r) rows[r] = (int32_t)r;
            } else if (2 * L <= m) {
                uint64_t ctr = (uint64_t)j << 20;  /* private counter range per column */
                int64_t got = 0;
                while (got < L) {
                    double u = unif(draw(krow, ctr++));
                    int64_t r = rank_cdf ? perm[sample_cdf(rank_cdf, m, u)] : (int64_t)(u * (double)m);
                    if (r >= m) r = m - 1;
                    if (seen[r]) continue;
                    seen[r] = 1;
                    rows[got++] = (int32_t)r;
                }
                for (int64_t t = 0; t < L; ++t) seen[rows[t]] = 0;
                if (L > 1) qsort(rows, (size_t)L, sizeof(int32_t), cmp_i32);
            } else {
                if (!keys) keys = (keyed_t *)malloc(sizeof(keyed_t) * (size_t)m);
                if (!keys) {
#pragma omp atomic write
                    failed = 1;
                    continue;
                }
                for (int64_t r = 0; r < m; ++r) { keys[r].row = (int32_t)r; keys[r].key = 1.0; }
                if (rank_cdf) {
                    for (int64_t rk = 0; rk < m; ++rk) {
                        double w = rank_cdf[rk] - (rk ? rank_cdf[rk - 1] : 0.0);
                        keys[perm[rk]].key = w > 0 ? w : 1e-300;   /* weight of that row */
                    }
                }
                for (int64_t r = 0; r < m; ++r) {
                    double u = unif_pos(draw(kden, ((uint64_t)j << 24) + (uint64_t)r));
                    keys[r].key = log(u) / keys[r].key;   /* = log(u^(1/w)) */
                }
                qsort(keys, (size_t)m, sizeof(keyed_t), cmp_key_desc);
                for (int64_t t = 0; t < L; ++t) rows[t] = keys[t].row;
                qsort(rows, (size_t)L, sizeof(int32_t), cmp_i32);
            }
            for (int64_t t = 0; t < L; ++t) {
                uint64_t pos = (uint64_t)(p0 + t);
                double *o = val + p0 + t;
                switch (value_kind) {
                case 0: *o = 2.0 * unif(draw(kval, pos)) - 1.0; break;
                case 1: {
                    uint64_t r1 = draw(kval, 2 * pos), r2 = draw(kval, 2 * pos + 1);
                    double g = sqrt(-2.0 * log(unif_pos(r1))) * cos(6.283185307179586 * unif(r2));
                    double mag = exp(g);
                    *o = (r2 & 1) ? -mag : mag;
                    break;
                }
                case 2: {
                    int64_t k = (int64_t)(draw(kval, pos) % 16);   /* 0..15 */
                    *o = (double)(k < 8 ? k - 8 : k - 7);           /* -8..-1, 1..8 */
                    break;
                }
                default: *o = 1.0; break;
                }
            }
        }
        free(seen);
        free(keys);
    }
    return failed ? -1 : 0;
}

/* Uniform vector in [-1,1) (kind 0) or integers in [-8,8] (kind 2). */
void syn_vector(int64_t len, uint64_t seed, uint64_t stream, int kind, double *out)
{
    const uint64_t k = stream_key(seed, 100 + stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < len; ++i) {
        uint64_t r = draw(k, (uint64_t)i);
        out[i] = (kind == 2) ? (double)((int64_t)(r % 17) - 8) : 2.0 * unif(r) - 1.0;
    }
}
