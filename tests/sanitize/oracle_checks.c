/*
 * Host sanitizer run of the oracle (tests/test_sanitizers_host.py builds it
 * with -fsanitize=address,undefined): every oracle routine on many small
 * random texts and the edge sizes, with cross-checks that keep the run
 * meaningful (the two query formulations agree, the all-cores builder equals
 * the one-thread builder, Z equals the level's zero count, sampled level bits
 * equal the level words).  Exits nonzero on a failed check; the sanitizers
 * abort on a memory or undefined-behaviour error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "wt_oracle.h"

int orc_par_build(int kind, const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint64_t *bits,
                  uint64_t W, uint64_t *zeros, int threads);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(c, ...)                                  \
    do {                                               \
        if (!(c)) {                                    \
            fprintf(stderr, "check failed: " __VA_ARGS__); \
            fprintf(stderr, "\n");                     \
            failures++;                                \
        }                                              \
    } while (0)

static void put(void *t, uint32_t b, uint64_t i, uint32_t v)
{
    if (b == 1) ((uint8_t *)t)[i] = (uint8_t)v;
    else if (b == 2) ((uint16_t *)t)[i] = (uint16_t)v;
    else ((uint32_t *)t)[i] = v;
}

static void one_case(uint64_t n, uint32_t L, uint32_t b)
{
    void *text = malloc(n ? n * b : 1);
    for (uint64_t i = 0; i < n; i++) put(text, b, i, L ? (uint32_t)(next_u64() & ((1ull << L) - 1)) : 0u);
    const uint64_t W = orc_words_per_level(n);
    const uint64_t LW = (uint64_t)(L ? L : 1) * (W ? W : 1);
    for (int kind = 0; kind < 2; kind++) {
        uint64_t *bits = calloc(LW, 8), *bits2 = calloc(LW, 8);
        uint64_t *zeros = calloc(L ? L : 1, 8), *zeros2 = calloc(L ? L : 1, 8);
        CHECK(orc_build(kind, text, n, b, L, bits, W, zeros) == ORC_OK, "build n=%llu L=%u", (unsigned long long)n, L);
        if (L <= 20) {
            CHECK(orc_par_build(kind, text, n, b, L, bits2, W, zeros2, 3) == ORC_OK, "par_build");
            CHECK(memcmp(bits, bits2, LW * 8) == 0 && memcmp(zeros, zeros2, (L ? L : 1) * 8) == 0,
                  "par_build differs n=%llu L=%u kind=%d", (unsigned long long)n, L, kind);
        }
        for (uint32_t l = 0; l < L; l++) {
            uint64_t ones = 0;
            for (uint64_t w = 0; w < W; w++) ones += (uint64_t)__builtin_popcountll(bits[l * W + w]);
            CHECK(zeros[l] + ones == n, "Z level %u", l);
            uint32_t *rd = calloc(W / 8 + 1, 4);
            const uint64_t cap = orc_sel_capacity(n);
            uint32_t *s0 = calloc(cap ? cap : 1, 4), *s1 = calloc(cap ? cap : 1, 4);
            CHECK(orc_directory(bits + l * W, n, W, rd, s0, s1) == ORC_OK, "directory");
            free(rd);
            free(s0);
            free(s1);
            if (n) {
                uint64_t pos[8];
                uint8_t got[8];
                for (int q = 0; q < 8; q++) pos[q] = next_u64() % n;
                CHECK(orc_sample_level(kind, text, n, b, L, l, pos, 8, got) == ORC_OK, "sample");
                for (int q = 0; q < 8; q++)
                    CHECK(got[q] == ((bits[l * W + pos[q] / 64] >> (pos[q] % 64)) & 1), "sampled bit");
            }
        }
        /* queries: plain definitions and the walks on the levels agree */
        const uint64_t m = 64;
        uint32_t syms[64];
        uint64_t args[64], a1[64], a2[64];
        for (int op = 0; op < 3; op++) {
            for (uint64_t q = 0; q < m; q++) {
                syms[q] = L ? (uint32_t)(next_u64() & ((1ull << L) - 1)) : 0u;
                args[q] = op == 2 ? next_u64() % (n + 2) : next_u64() % (n + 2);
            }
            CHECK(orc_queries_def(text, n, b, L, op, syms, args, m, a1) == ORC_OK, "queries_def");
            CHECK(orc_queries_walk(kind, bits, W, zeros, n, L, op, syms, args, m, a2) == ORC_OK, "queries_walk");
            CHECK(memcmp(a1, a2, sizeof a1) == 0, "queries differ op=%d n=%llu L=%u kind=%d", op,
                  (unsigned long long)n, L, kind);
        }
        free(bits);
        free(bits2);
        free(zeros);
        free(zeros2);
    }
    if (L >= 2 && L <= 12 && n) {
        uint64_t pos[16], out[16];
        for (int q = 0; q < 16; q++) pos[q] = next_u64() % n;
        for (uint32_t l = 0; l < L; l++) CHECK(orc_map_wt_to_wm(text, n, b, L, l, pos, 16, out) == ORC_OK, "map");
        const uint64_t pool_words = L * ((n + 63) / 64) + (1ull << L);
        uint64_t *nodes = calloc(2 * (1ull << L), 8), *pool = calloc(pool_words, 8);
        CHECK(orc_pointer_tree(text, n, b, L, nodes, pool, pool_words) == ORC_OK, "pointer tree");
        free(nodes);
        free(pool);
    }
    if (L && L < 8 * b && n) {  /* a symbol out of range is an error */
        put(text, b, n / 2, 1u << L);
        uint64_t *bits = calloc(LW, 8), *zeros = calloc(L, 8);
        CHECK(orc_build(0, text, n, b, L, bits, W, zeros) == ORC_ERANGE, "range error");
        free(bits);
        free(zeros);
    }
    free(text);
}

int main(void)
{
    const uint64_t sizes[] = {0, 1, 2, 63, 64, 65, 511, 512, 513, 1000, 4097, 9000};
    const uint32_t widths[] = {1, 2, 4};
    for (unsigned si = 0; si < sizeof sizes / sizeof sizes[0]; si++)
        for (unsigned wi = 0; wi < 3; wi++)
            for (uint32_t L = 0; L <= (widths[wi] == 1 ? 8u : (widths[wi] == 2 ? 16u : 22u)); L += (L < 9 ? 1 : 3))
                one_case(sizes[si], L, widths[wi]);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer checks ok\n");
    return 0;
}
