/*
 * Seeded synthetic graph generators: Graph500-style Kronecker (R-MAT with
 * the four initiator probabilities), Erdos-Renyi G(n,p) by geometric edge
 * skipping (Batagelj and Brandes, Phys. Rev. E 71, 2005), and a Chung-Lu
 * power-law graph.  They emit raw (src, dst) tuples: self-loops and duplicate
 * edges are left in, because removing them is the CSR builder's job.
 *
 * These generators feed both the triangle-counting library and its CPU
 * oracle.  They contain none of the triangle-counting arithmetic.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea and Flood, OOPSLA 2014) applied to key + counter *
 * golden-ratio increment.  A draw therefore depends only on (seed, stream,
 * counter), so the tuples are the same for any thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* key for (seed, stream): two rounds of mixing so nearby seeds decorrelate */
static inline uint64_t gg_key(uint64_t seed, uint64_t stream)
{
    return sm64_mix(sm64_mix(seed + GOLDEN) ^ (stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL));
}

static inline uint64_t gg_draw(uint64_t key, uint64_t ctr)
{
    return sm64_mix(key + (ctr + 1) * GOLDEN);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double gg_unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, bound) by Lemire's multiply-high (bias < bound/2^64) */
static inline uint64_t gg_below(uint64_t r, uint64_t bound)
{
    return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

/* ---------------------------------------------------------------- permute */

/* Fisher-Yates shuffle of the identity on [0, n), serial stream `stream`. */
void gg_permutation(int64_t n, uint64_t seed, uint64_t stream, int32_t *perm)
{
    uint64_t key = gg_key(seed, stream);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)gg_below(gg_draw(key, (uint64_t)i), (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

void gg_relabel(int64_t m, int32_t *src, int32_t *dst, const int32_t *perm)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        src[e] = perm[src[e]];
        dst[e] = perm[dst[e]];
    }
}

/* --------------------------------------------------------------- Kronecker */

/*
 * m = edgefactor * 2^scale tuples.  For each tuple and each of the `scale`
 * bit positions one uniform draw picks a quadrant of the 2x2 initiator:
 * [0,A) top-left, [A,A+B) top-right (dst bit set), [A+B,A+B+C) bottom-left
 * (src bit set), else bottom-right (both set).  Vertex ids are then permuted
 * by a seeded Fisher-Yates shuffle.  Caller owns src/dst (m entries each).
 */
int gg_kronecker(int scale, int64_t edgefactor, double A, double B, double C,
                 uint64_t seed, int32_t *src, int32_t *dst)
{
    if (scale < 1 || scale > 30 || edgefactor < 1) return -1;
    const int64_t n = (int64_t)1 << scale;
    const int64_t m = edgefactor * n;
    const uint64_t key = gg_key(seed, 1);
    const double ab = A + B, abc = A + B + C;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint32_t s = 0, d = 0;
        for (int b = 0; b < scale; ++b) {
            double r = gg_unit(gg_draw(key, (uint64_t)e * (uint64_t)scale + (uint64_t)b));
            uint32_t sb = 0, db = 0;
            if (r < A) { }
            else if (r < ab) { db = 1; }
            else if (r < abc) { sb = 1; }
            else { sb = 1; db = 1; }
            s |= sb << b;
            d |= db << b;
        }
        src[e] = (int32_t)s;
        dst[e] = (int32_t)d;
    }
    int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!perm) return -2;
    gg_permutation(n, seed, 2, perm);
    gg_relabel(m, src, dst, perm);
    free(perm);
    return 0;
}

/* ------------------------------------------------------------ Erdos-Renyi */

/*
 * G(n,p) on pairs (v, w) with w < v, by geometric skipping over the
 * lexicographic list of pairs.  Pass src == NULL to only count the edges;
 * the same (seed) produces the same edges on the counting and filling passes.
 * Returns the edge count, or -1 on bad arguments / -2 if cap is exceeded.
 */
int64_t gg_erdos_renyi(int64_t n, double p, uint64_t seed, int32_t *src, int32_t *dst, int64_t cap)
{
    if (n < 1 || !(p >= 0.0) || p > 1.0) return -1;
    if (p == 0.0 || n < 2) return 0;
    const uint64_t key = gg_key(seed, 3);
    const double lq = log1p(-p);
    int64_t v = 1, w = -1, cnt = 0;
    uint64_t ctr = 0;
    while (v < n) {
        double r = gg_unit(gg_draw(key, ctr++));
        int64_t skip = (p >= 1.0) ? 0 : (int64_t)floor(log1p(-r) / lq);
        w += 1 + skip;
        while (w >= v && v < n) { w -= v; ++v; }
        if (v < n) {
            if (src) {
                if (cnt >= cap) return -2;
                src[cnt] = (int32_t)v;
                dst[cnt] = (int32_t)w;
            }
            ++cnt;
        }
    }
    return cnt;
}

/* ---------------------------------------------------------------- Chung-Lu */

/*
 * Expected-degree weights w_i = wmax * (i0 / (i + i0))^(1/(gamma-1)),
 * i = 0..n-1, with i0 found by bisection so that the mean weight is
 * `mean_deg`.  Writes the weights (n doubles) and returns i0 (or -1).
 */
double gg_chung_lu_weights(int64_t n, double gamma, double mean_deg, double wmax, double *w)
{
    if (n < 2 || gamma <= 1.0 || mean_deg <= 0.0 || wmax < mean_deg) return -1.0;
    const double ex = 1.0 / (gamma - 1.0);
    double lo = 1e-9, hi = (double)n * 1e3;
    for (int it = 0; it < 200; ++it) {
        double mid = sqrt(lo * hi);
        /* fixed 256-way blocking: the sum does not depend on the thread count */
        double part[256];
#pragma omp parallel for schedule(static)
        for (int blk = 0; blk < 256; ++blk) {
            double acc = 0.0;
            for (int64_t i = n * blk / 256; i < n * (blk + 1) / 256; ++i)
                acc += wmax * pow(mid / ((double)i + mid), ex);
            part[blk] = acc;
        }
        double s = 0.0;
        for (int blk = 0; blk < 256; ++blk) s += part[blk];
        if (s / (double)n < mean_deg) lo = mid; else hi = mid;
        if (hi / lo < 1.0 + 1e-12) break;
    }
    const double i0 = sqrt(lo * hi);
    for (int64_t i = 0; i < n; ++i) w[i] = wmax * pow(i0 / ((double)i + i0), ex);
    return i0;
}

/*
 * m = round(sum(w)/2) tuples; each endpoint is drawn with probability
 * proportional to its weight (inverse CDF by binary search).  Vertex ids are
 * then permuted so that hubs are spread over the id range.
 */
int gg_chung_lu(int64_t n, const double *w, int64_t m, uint64_t seed, int32_t *src, int32_t *dst)
{
    if (n < 2 || m < 0) return -1;
    double *cdf = (double *)malloc((size_t)n * sizeof(double));
    if (!cdf) return -2;
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) { acc += w[i]; cdf[i] = acc; }
    const double total = acc;
    const uint64_t key = gg_key(seed, 4);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        for (int side = 0; side < 2; ++side) {
            double t = gg_unit(gg_draw(key, 2 * (uint64_t)e + (uint64_t)side)) * total;
            int64_t lo = 0, hi = n - 1;           /* first i with cdf[i] > t */
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (cdf[mid] > t) hi = mid; else lo = mid + 1;
            }
            if (side == 0) src[e] = (int32_t)lo; else dst[e] = (int32_t)lo;
        }
    }
    free(cdf);
    int32_t *perm = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!perm) return -2;
    gg_permutation(n, seed, 5, perm);
    gg_relabel(m, src, dst, perm);
    free(perm);
    return 0;
}

/* raw 64-bit draws, exposed for the generator's own statistical tests */
void gg_draws(uint64_t seed, uint64_t stream, int64_t count, uint64_t *out)
{
    const uint64_t key = gg_key(seed, stream);
    for (int64_t i = 0; i < count; ++i) out[i] = gg_draw(key, (uint64_t)i);
}
