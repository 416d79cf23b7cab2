/*
 * Seeded synthetic texts for wavelet tree / wavelet matrix construction.
 *
 * Random numbers only: this file holds none of the index construction.  It is
 * shared by the tests (to feed the oracle and the GPU library the same input)
 * and by the benchmark.
 *
 * Generators: splitmix64 (Steele, Lea, Flood 2014) to derive seeds and
 * xoshiro256** (Blackman, Vigna 2018) for the streams.  Every text is cut into
 * fixed-size chunks; chunk c draws from its own stream, seeded from
 * (seed, stream tag, c), so the output does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CHUNK ((uint64_t)1 << 16)

static uint64_t splitmix64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t s[4];
} xo_t;

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t xo_next(xo_t *x)
{
    uint64_t *s = x->s;
    uint64_t r = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return r;
}

static void xo_seed(xo_t *x, uint64_t seed, uint64_t tag, uint64_t idx)
{
    uint64_t sm = seed * 0xD1B54A32D192ED03ull ^ tag * 0x8CB92BA72F3D8DD7ull ^ idx;
    for (int i = 0; i < 4; i++) x->s[i] = splitmix64(&sm);
}

/* uniform integer in [0, m), m >= 1, by the high word of a 64x64 product */
static uint64_t xo_below(xo_t *x, uint64_t m)
{
    return (uint64_t)(((unsigned __int128)xo_next(x) * m) >> 64);
}

/* uniform double in [0, 1) with 53 random bits */
static double xo_unit(xo_t *x) { return (double)(xo_next(x) >> 11) * 0x1.0p-53; }

static void store(void *out, uint32_t sym_bytes, uint64_t i, uint64_t v)
{
    if (sym_bytes == 1) ((uint8_t *)out)[i] = (uint8_t)v;
    else if (sym_bytes == 2) ((uint16_t *)out)[i] = (uint16_t)v;
    else ((uint32_t *)out)[i] = (uint32_t)v;
}

/* i.i.d. uniform symbols over [0, sigma) */
void gen_uniform(void *out, uint64_t n, uint32_t sym_bytes, uint64_t sigma, uint64_t seed)
{
    int64_t nchunks = (int64_t)((n + CHUNK - 1) / CHUNK);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; c++) {
        xo_t x;
        xo_seed(&x, seed, 1, (uint64_t)c);
        uint64_t a = (uint64_t)c * CHUNK, b = a + CHUNK < n ? a + CHUNK : n;
        for (uint64_t i = a; i < b; i++) store(out, sym_bytes, i, xo_below(&x, sigma));
    }
}

/* ---- Gamma / Dirichlet for the Markov transition rows ------------------- */

static double std_normal(xo_t *x)
{
    /* Marsaglia polar method */
    for (;;) {
        double u = 2.0 * xo_unit(x) - 1.0, v = 2.0 * xo_unit(x) - 1.0;
        double s = u * u + v * v;
        if (s > 0.0 && s < 1.0) return u * sqrt(-2.0 * log(s) / s);
    }
}

/* Gamma(shape a, scale 1): Marsaglia-Tsang for a >= 1; a < 1 by the
 * U^(1/a) boost */
static double gamma_draw(xo_t *x, double a)
{
    if (a < 1.0) {
        double u = xo_unit(x);
        while (u <= 0.0) u = xo_unit(x);
        return gamma_draw(x, a + 1.0) * pow(u, 1.0 / a);
    }
    double d = a - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
    for (;;) {
        double z = std_normal(x), v = 1.0 + c * z;
        if (v <= 0.0) continue;
        v = v * v * v;
        double u = xo_unit(x);
        if (u < 1.0 - 0.0331 * z * z * z * z) return d * v;
        if (u > 0.0 && log(u) < 0.5 * z * z + d * (1.0 - v + log(v))) return d * v;
    }
}

/*
 * Order-2 Markov text over [0, sigma): one transition row per state
 * (previous two symbols), each row drawn from Dirichlet(alpha, ..., alpha);
 * sampling by the inverse of the row's cumulative distribution.  The text is
 * made of independent chains of chain_len symbols; each chain starts from two
 * uniform symbols.  sigma <= 256 (uint8 output).
 */
int gen_markov2(uint8_t *out, uint64_t n, uint32_t sigma, double alpha, uint64_t seed,
                uint64_t chain_len)
{
    if (sigma < 1 || sigma > 256 || chain_len < 2) return -1;
    uint64_t states = (uint64_t)sigma * sigma;
    uint64_t *cdf = (uint64_t *)malloc(states * sigma * sizeof(uint64_t));
    double *w = (double *)malloc(sigma * sizeof(double));
    if (!cdf || !w) {
        free(cdf);
        free(w);
        return -2;
    }
    xo_t x;
    xo_seed(&x, seed, 2, 0);
    for (uint64_t s = 0; s < states; s++) {
        double tot = 0.0;
        for (uint32_t k = 0; k < sigma; k++) {
            w[k] = gamma_draw(&x, alpha);
            tot += w[k];
        }
        if (!(tot > 0.0)) { /* all draws underflowed: fall back to uniform */
            for (uint32_t k = 0; k < sigma; k++) w[k] = 1.0;
            tot = sigma;
        }
        /* cumulative thresholds scaled to 2^64 (last entry saturates) */
        double run = 0.0;
        for (uint32_t k = 0; k < sigma; k++) {
            run += w[k] / tot;
            double t = run * 18446744073709551616.0;
            cdf[s * sigma + k] = (k + 1 == sigma || t >= 18446744073709551615.0)
                                     ? UINT64_MAX
                                     : (uint64_t)t;
        }
    }
    free(w);
    int64_t nchains = (int64_t)((n + chain_len - 1) / chain_len);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nchains; c++) {
        xo_t r;
        xo_seed(&r, seed, 3, (uint64_t)c);
        uint64_t a = (uint64_t)c * chain_len, b = a + chain_len < n ? a + chain_len : n;
        uint32_t p2 = (uint32_t)xo_below(&r, sigma), p1 = (uint32_t)xo_below(&r, sigma);
        for (uint64_t i = a; i < b; i++) {
            uint32_t sym;
            if (i == a) sym = p2;
            else if (i == a + 1) sym = p1;
            else {
                const uint64_t *row = cdf + ((uint64_t)p2 * sigma + p1) * sigma;
                uint64_t u = xo_next(&r);
                /* first k with u < row[k] */
                uint32_t lo = 0, hi = sigma - 1;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) / 2;
                    if (u < row[mid]) hi = mid;
                    else lo = mid + 1;
                }
                sym = lo;
                p2 = p1;
                p1 = sym;
            }
            out[i] = (uint8_t)sym;
        }
    }
    free(cdf);
    return 0;
}

/*
 * Zipf(s) over ranks 1..sigma (weights r^-s, finite support), drawn by the
 * inverse of the cumulative distribution; rank r is written as symbol id
 * perm[r-1], where perm is a seeded uniform permutation of [0, sigma)
 * (Fisher-Yates), or the identity when permute == 0.
 */
int gen_zipf(void *out, uint64_t n, uint32_t sym_bytes, uint64_t sigma, double s, uint64_t seed,
             int permute)
{
    if (sigma < 1) return -1;
    double *cdf = (double *)malloc(sigma * sizeof(double));
    uint32_t *perm = (uint32_t *)malloc(sigma * sizeof(uint32_t));
    if (!cdf || !perm) {
        free(cdf);
        free(perm);
        return -2;
    }
    double tot = 0.0;
    for (uint64_t r = 0; r < sigma; r++) tot += pow((double)(r + 1), -s);
    double run = 0.0;
    for (uint64_t r = 0; r < sigma; r++) {
        run += pow((double)(r + 1), -s) / tot;
        cdf[r] = run;
    }
    cdf[sigma - 1] = 2.0; /* every u < 1 lands inside */
    for (uint64_t r = 0; r < sigma; r++) perm[r] = (uint32_t)r;
    if (permute) {
        xo_t x;
        xo_seed(&x, seed, 4, 0);
        for (uint64_t i = sigma - 1; i > 0; i--) {
            uint64_t j = xo_below(&x, i + 1);
            uint32_t t = perm[i];
            perm[i] = perm[j];
            perm[j] = t;
        }
    }
    int64_t nchunks = (int64_t)((n + CHUNK - 1) / CHUNK);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; c++) {
        xo_t x;
        xo_seed(&x, seed, 5, (uint64_t)c);
        uint64_t a = (uint64_t)c * CHUNK, b = a + CHUNK < n ? a + CHUNK : n;
        for (uint64_t i = a; i < b; i++) {
            double u = xo_unit(&x);
            uint64_t lo = 0, hi = sigma - 1;
            while (lo < hi) {
                uint64_t mid = (lo + hi) / 2;
                if (u < cdf[mid]) hi = mid;
                else lo = mid + 1;
            }
            store(out, sym_bytes, i, perm[lo]);
        }
    }
    free(cdf);
    free(perm);
    return 0;
}

/* uniform 64-bit words from stream (seed, tag): positions, query mixes, ... */
void gen_u64(uint64_t *out, uint64_t m, uint64_t bound, uint64_t seed, uint64_t tag)
{
    int64_t nchunks = (int64_t)((m + CHUNK - 1) / CHUNK);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; c++) {
        xo_t x;
        xo_seed(&x, seed, 100 + tag, (uint64_t)c);
        uint64_t a = (uint64_t)c * CHUNK, b = a + CHUNK < m ? a + CHUNK : m;
        for (uint64_t i = a; i < b; i++) out[i] = bound ? xo_below(&x, bound) : xo_next(&x);
    }
}

/* uniform doubles in [0,1) from stream (seed, tag) */
void gen_unit(double *out, uint64_t m, uint64_t seed, uint64_t tag)
{
    int64_t nchunks = (int64_t)((m + CHUNK - 1) / CHUNK);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; c++) {
        xo_t x;
        xo_seed(&x, seed, 200 + tag, (uint64_t)c);
        uint64_t a = (uint64_t)c * CHUNK, b = a + CHUNK < m ? a + CHUNK : m;
        for (uint64_t i = a; i < b; i++) out[i] = xo_unit(&x);
    }
}
