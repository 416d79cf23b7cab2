/*
 * The oracle's top-down construction, run on every host core (OpenMP).
 *
 * TEST AND BASELINE INFRASTRUCTURE ONLY, like wt_oracle.c: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code with the GPU library.
 *
 * Same algorithm as orc_build (Fischer, Kurpicz, Loebel, arXiv 1702.07578):
 *   - level l holds bit l (MSB first) of every symbol of the current sequence
 *     (Section 2);
 *   - WM (Section 5): the next sequence is the stable partition of the whole
 *     sequence by bit l, zeros first;
 *   - WT (Section 2, Observation 1): the next sequence is, inside every run of
 *     equal l-bit prefix (one tree node), the stable partition by bit l.
 * Parallel form of one level (the per-core counting and interleaved prefix
 * sum of Section 3.2, applied to the top-down split): the sequence is cut
 * into one slice per thread (slice borders on multiples of 64, so each
 * thread writes whole words of the level); every thread counts, per node, the
 * zeros and ones of its slice; one prefix sum over (node, thread) gives
 * every thread's first destination of each node's zeros and ones; every
 * thread then moves its slice, in order, to those destinations.  Node t of
 * the WT is the prefix t (the sequence is sorted by the l-bit prefix, so the
 * nodes follow in increasing prefix order); the WM has one node.
 *
 * Limits: lg_sigma <= ORC_PAR_MAX_LEVELS (per-thread counters of 2^(L-1)
 * nodes).  The result equals orc_build's bit for bit (pinned in the tests).
 */
#include "wt_oracle.h"

#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PAR_MAX_LEVELS 20

static uint32_t par_sym(const void *text, uint32_t b, uint64_t i)
{
    if (b == 1) return ((const uint8_t *)text)[i];
    if (b == 2) return ((const uint16_t *)text)[i];
    return ((const uint32_t *)text)[i];
}

int orc_par_max_threads(void) { return omp_get_max_threads(); }

/* ceil(n / 64) rounded up to a multiple of 8 (the level layout) */
static uint64_t par_words(uint64_t n) { return ((n + 63) / 64 + 7) / 8 * 8; }

/* threads <= 0: every thread OpenMP offers */
int orc_par_build(int kind, const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint64_t *bits,
                  uint64_t W, uint64_t *zeros, int threads)
{
    if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4) return ORC_EINVAL;
    if (kind != ORC_WT && kind != ORC_WM) return ORC_EINVAL;
    if (L > ORC_PAR_MAX_LEVELS) return ORC_EINVAL;
    if (W < par_words(n)) return ORC_EINVAL;
    const int T = threads > 0 ? threads : omp_get_max_threads();

    int bad = 0;
#pragma omp parallel for num_threads(T) reduction(| : bad) schedule(static)
    for (uint64_t i = 0; i < n; i++) bad |= (par_sym(text, sym_bytes, i) >> L) != 0;
    if (bad) return ORC_ERANGE;
    if (L == 0) return ORC_OK;

    uint32_t *seq = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint32_t *tmp = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    const uint64_t max_nodes = (kind == ORC_WT) ? ((uint64_t)1 << (L - 1)) : 1;
    /* cnt[(t * nodes + node) * 2 + bit]; afterwards the destination cursors */
    uint64_t *cnt = (uint64_t *)malloc((size_t)T * max_nodes * 2 * sizeof(uint64_t));
    uint64_t *lo = (uint64_t *)malloc((size_t)(T + 1) * sizeof(uint64_t));
    if (!seq || !tmp || !cnt || !lo) {
        free(seq);
        free(tmp);
        free(cnt);
        free(lo);
        return ORC_ENOMEM;
    }
    /* slice t is [lo[t], lo[t+1]): borders on multiples of 64 */
    for (int t = 0; t <= T; t++) {
        uint64_t x = (uint64_t)((unsigned __int128)n * (uint64_t)t / (uint64_t)T);
        lo[t] = (t == T) ? n : (x + 63) / 64 * 64;
        if (lo[t] > n) lo[t] = n;
    }
    for (int t = 1; t <= T; t++)
        if (lo[t] < lo[t - 1]) lo[t] = lo[t - 1];

#pragma omp parallel for num_threads(T) schedule(static)
    for (uint64_t i = 0; i < n; i++) seq[i] = par_sym(text, sym_bytes, i);

    memset(bits, 0, (size_t)L * W * sizeof(uint64_t));
    for (uint32_t l = 0; l < L; l++) {
        uint64_t *lv = bits + (uint64_t)l * W;
        const uint64_t nodes = (kind == ORC_WT) ? ((uint64_t)1 << l) : 1;
        const uint32_t sh = L - 1 - l;
        /* bits of the level, and the per-thread counts per node */
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            uint64_t *c = cnt + (uint64_t)t * nodes * 2;
            memset(c, 0, (size_t)nodes * 2 * sizeof(uint64_t));
            for (uint64_t i = lo[t]; i < lo[t + 1]; i++) {
                const uint32_t a = seq[i];
                const uint32_t bt = (a >> sh) & 1u;
                const uint64_t node = (kind == ORC_WT && l > 0) ? (a >> (L - l)) : 0;
                c[node * 2 + bt]++;
                if (bt) lv[i / 64] |= (uint64_t)1 << (i % 64);
            }
        }
        uint64_t nz = 0;
        for (int t = 0; t < T; t++)
            for (uint64_t k = 0; k < nodes; k++) nz += cnt[((uint64_t)t * nodes + k) * 2];
        zeros[l] = nz;
        if (l + 1 == L) break;
        /* one prefix sum over (node, thread): node k starts where node k-1
         * ends; inside it the zeros of every thread in thread order, then the
         * ones of every thread in thread order */
        uint64_t run = 0;
        for (uint64_t k = 0; k < nodes; k++) {
            uint64_t z = 0;
            for (int t = 0; t < T; t++) z += cnt[((uint64_t)t * nodes + k) * 2];
            uint64_t zc = run, oc = run + z;
            for (int t = 0; t < T; t++) {
                uint64_t *c = cnt + ((uint64_t)t * nodes + k) * 2;
                const uint64_t cz = c[0], co = c[1];
                c[0] = zc;
                c[1] = oc;
                zc += cz;
                oc += co;
            }
            run = oc;
        }
#pragma omp parallel num_threads(T)
        {
            const int t = omp_get_thread_num();
            uint64_t *c = cnt + (uint64_t)t * nodes * 2;
            for (uint64_t i = lo[t]; i < lo[t + 1]; i++) {
                const uint32_t a = seq[i];
                const uint32_t bt = (a >> sh) & 1u;
                const uint64_t node = (kind == ORC_WT && l > 0) ? (a >> (L - l)) : 0;
                tmp[c[node * 2 + bt]++] = a;
            }
        }
        uint32_t *sw = seq;
        seq = tmp;
        tmp = sw;
    }
    free(seq);
    free(tmp);
    free(cnt);
    free(lo);
    return ORC_OK;
}
