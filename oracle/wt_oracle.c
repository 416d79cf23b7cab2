/*
 * Reference oracle for wavelet tree (WT) and wavelet matrix (WM) construction.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, single-threaded, deliberately slow C that
 * computes what the paper (Fischer, Kurpicz, Loebel, "Simple, Fast and
 * Lightweight Parallel Wavelet Tree Construction", arXiv 1702.07578) defines,
 * straight from the definitions, so that the GPU library can be checked bit for
 * bit against it.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library; the product path never does.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What is computed, and where it is defined:
 *   - bit(k,a), prefix(k,a): Section 2 (Preliminaries), MSB-first bit k and the
 *     k most significant bits read as an integer.
 *   - WT levels: Section 2, "Wavelet Trees", level-wise tree and Observation 1:
 *     level l holds bit l of every symbol, the symbols grouped into intervals by
 *     their l-bit prefix (in increasing prefix order), text order inside each
 *     interval.  Computed top-down: the level-l sequence is split, inside every
 *     run of equal l-bit prefix, into the symbols with bit l = 0 followed by
 *     those with bit l = 1.
 *   - WM levels and Z: Section 5, definition of the wavelet matrix: level 0 is
 *     the MSBs in text order; a symbol at position i of level l-1 moves to
 *     rank_0(BV_{l-1}, i) if its bit is 0, else to Z[l-1] + rank_1(BV_{l-1}, i).
 *     That is a stable partition of the whole level by the bit, zeros first.
 *     Z[l] is the number of zeros of level l.
 *   - Hist / SPos: Section 3.1 (Algorithm 1) and Section 5.1: the number of
 *     symbols per l-bit prefix, and the start of each prefix's interval, with
 *     intervals ordered by prefix (WT) or by the bit reversal of the prefix (WM,
 *     Observation 2 and the bit-reversal permutation of Section 5).
 *     Computed here by direct counting, not by the bottom-up merge.
 *   - rank/select: Section 2, rank_b(BV,i) = number of b in BV[0,i),
 *     select_b(BV,i) = position of the i-th b (1-based i, 0-based position).
 *   - Directories: the paper only says the level bit vectors are augmented with
 *     binary rank and select structures (Section 2, Section 5).  The layout here
 *     is the library's own: a cumulative count of ones before every 512-bit
 *     block, plus the block that holds every 4096-th one (and zero).
 *     Parity unpinned by the paper: pinned only by its own definition.
 *   - Queries access/rank/select on the sequence (Section 1/2: the indexes
 *     answer them in O(lg sigma)); computed here from their plain definitions on
 *     the text, and separately by walks over the oracle's own levels.
 *
 * Bit layout of every level: LSB-first inside little-endian 64-bit words
 * (position p is bit p%64 of word p/64); W words per level, W = ceil(n/64)
 * rounded up to a multiple of 8; every bit at or past n is zero.
 */
#include "wt_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---- symbols and bit primitives (Section 2) ----------------------------- */

static uint32_t sym_at(const void *text, uint32_t sym_bytes, uint64_t i)
{
    if (sym_bytes == 1) return ((const uint8_t *)text)[i];
    if (sym_bytes == 2) return ((const uint16_t *)text)[i];
    return ((const uint32_t *)text)[i];
}

/* bit(k, a): the k-th most significant of the L bits of a */
static uint32_t bit_of(uint32_t L, uint32_t k, uint32_t a)
{
    return (uint32_t)(((uint64_t)a >> (L - 1 - k)) & 1u);
}

/* prefix(k, a): the k most significant of the L bits of a; prefix(0,a) = 0 */
static uint64_t prefix_of(uint32_t L, uint32_t k, uint32_t a)
{
    if (k == 0) return 0;
    return (uint64_t)a >> (L - k);
}

/* reverse the k low bits of x (the bit-reversal permutation pi_k of Section 5) */
uint64_t orc_reverse_bits(uint64_t x, uint32_t k)
{
    uint64_t r = 0;
    for (uint32_t i = 0; i < k; i++) {
        r = (r << 1) | (x & 1u);
        x >>= 1;
    }
    return r;
}

uint64_t orc_words_per_level(uint64_t n)
{
    uint64_t w = (n + 63) / 64;
    return (w + 7) / 8 * 8;
}

static void set_bit(uint64_t *words, uint64_t pos)
{
    words[pos / 64] |= (uint64_t)1 << (pos % 64);
}

static uint32_t get_bit(const uint64_t *words, uint64_t pos)
{
    return (uint32_t)((words[pos / 64] >> (pos % 64)) & 1u);
}

int orc_check_symbols(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L)
{
    if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4) return ORC_EINVAL;
    if (L > 32) return ORC_EINVAL;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t a = sym_at(text, sym_bytes, i);
        if (L < 32 && (a >> L) != 0) return ORC_ERANGE;
    }
    return ORC_OK;
}

/* ---- construction, top-down from the definitions ----------------------- */

int orc_build(int kind, const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L,
              uint64_t *bits, uint64_t W, uint64_t *zeros)
{
    int rc = orc_check_symbols(text, n, sym_bytes, L);
    if (rc != ORC_OK) return rc;
    if (kind != ORC_WT && kind != ORC_WM) return ORC_EINVAL;
    if (W < orc_words_per_level(n)) return ORC_EINVAL;
    if (L == 0) return ORC_OK;

    memset(bits, 0, (size_t)(L * W * sizeof(uint64_t)));
    uint32_t *seq = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint32_t *tmp = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!seq || !tmp) {
        free(seq);
        free(tmp);
        return ORC_ENOMEM;
    }
    for (uint64_t i = 0; i < n; i++) seq[i] = sym_at(text, sym_bytes, i);

    for (uint32_t l = 0; l < L; l++) {
        uint64_t *lv = bits + (uint64_t)l * W;
        uint64_t nz = 0;
        /* level l: bit l of every symbol of the current sequence, in order */
        for (uint64_t i = 0; i < n; i++) {
            if (bit_of(L, l, seq[i])) set_bit(lv, i);
            else nz++;
        }
        zeros[l] = nz;
        if (l + 1 == L) break;

        if (kind == ORC_WM) {
            /* WM: stable partition of the whole level by bit l, zeros first */
            uint64_t z = 0, o = nz;
            for (uint64_t i = 0; i < n; i++) {
                if (bit_of(L, l, seq[i])) tmp[o++] = seq[i];
                else tmp[z++] = seq[i];
            }
        } else {
            /* WT: inside every maximal run of equal l-bit prefix (one tree
             * node), stable partition by bit l, zeros first */
            uint64_t a = 0;
            while (a < n) {
                uint64_t p = prefix_of(L, l, seq[a]);
                uint64_t b = a;
                uint64_t cz = 0;
                while (b < n && prefix_of(L, l, seq[b]) == p) {
                    if (!bit_of(L, l, seq[b])) cz++;
                    b++;
                }
                uint64_t z = a, o = a + cz;
                for (uint64_t i = a; i < b; i++) {
                    if (bit_of(L, l, seq[i])) tmp[o++] = seq[i];
                    else tmp[z++] = seq[i];
                }
                a = b;
            }
        }
        uint32_t *sw = seq;
        seq = tmp;
        tmp = sw;
    }
    free(seq);
    free(tmp);
    return ORC_OK;
}

/* ---- histograms and interval starts, by direct counting ----------------- */

int orc_hist(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint32_t level,
             uint64_t *hist)
{
    if (level > L || level > 26) return ORC_EINVAL;
    int rc = orc_check_symbols(text, n, sym_bytes, L);
    if (rc != ORC_OK) return rc;
    uint64_t keys = (uint64_t)1 << level;
    memset(hist, 0, (size_t)(keys * sizeof(uint64_t)));
    for (uint64_t i = 0; i < n; i++) hist[prefix_of(L, level, sym_at(text, sym_bytes, i))]++;
    return ORC_OK;
}

/* SPos[p] = number of symbols whose level-bit prefix q comes before p:
 * q < p for the WT, reverse(q) < reverse(p) for the WM. */
int orc_spos(int kind, const uint64_t *hist, uint32_t level, uint64_t *spos)
{
    if (level > 26) return ORC_EINVAL;
    uint64_t keys = (uint64_t)1 << level;
    /* visit the prefixes in interval order (i for the WT, pi_level(i) for the
     * WM) and hand out consecutive starts */
    uint64_t run = 0;
    for (uint64_t i = 0; i < keys; i++) {
        uint64_t p = (kind == ORC_WT) ? i : orc_reverse_bits(i, level);
        spos[p] = run;
        run += hist[p];
    }
    return ORC_OK;
}

/* ---- binary rank / select by counting (Section 2) ----------------------- */

uint64_t orc_rank_bv(const uint64_t *words, uint64_t i, uint32_t b)
{
    uint64_t c = 0;
    for (uint64_t p = 0; p < i; p++)
        if (get_bit(words, p) == b) c++;
    return c;
}

/* position of the k-th (1-based) b in words[0,n); n if there is none */
uint64_t orc_select_bv(const uint64_t *words, uint64_t n, uint64_t k, uint32_t b)
{
    uint64_t c = 0;
    for (uint64_t p = 0; p < n; p++) {
        if (get_bit(words, p) == b) {
            c++;
            if (c == k) return p;
        }
    }
    return n;
}

/* ---- directories (library-defined layout) ------------------------------- */

uint64_t orc_sel_capacity(uint64_t n)
{
    return (n + ORC_SEL_SPACING - 1) / ORC_SEL_SPACING + 1;
}

int orc_directory(const uint64_t *words, uint64_t n, uint64_t W, uint32_t *rank_dir,
                  uint32_t *sel0, uint32_t *sel1)
{
    uint64_t nb = W / 8;
    uint64_t cap = orc_sel_capacity(n);
    /* rank_dir[j] = ones in [0, 512 j), j = 0..nb, counted bit by bit */
    uint64_t ones = 0;
    for (uint64_t j = 0; j <= nb; j++) {
        rank_dir[j] = (uint32_t)ones;
        if (j == nb) break;
        for (uint64_t p = 512 * j; p < 512 * (j + 1) && p < n; p++) ones += get_bit(words, p);
    }
    for (uint64_t q = 0; q < cap; q++) {
        sel0[q] = 0xFFFFFFFFu;
        sel1[q] = 0xFFFFFFFFu;
    }
    /* sel_b[q] = block holding the (q*SPACING + 1)-th b of [0, n) */
    uint64_t c0 = 0, c1 = 0;
    for (uint64_t p = 0; p < n; p++) {
        if (get_bit(words, p)) {
            if (c1 % ORC_SEL_SPACING == 0) sel1[c1 / ORC_SEL_SPACING] = (uint32_t)(p / 512);
            c1++;
        } else {
            if (c0 % ORC_SEL_SPACING == 0) sel0[c0 / ORC_SEL_SPACING] = (uint32_t)(p / 512);
            c0++;
        }
    }
    return ORC_OK;
}

/* ---- queries from their plain definitions on the text ------------------- */

typedef struct {
    uint32_t sym;
    uint64_t pos;
} occ_t;

static int occ_cmp(const void *x, const void *y)
{
    const occ_t *a = (const occ_t *)x, *b = (const occ_t *)y;
    if (a->sym != b->sym) return a->sym < b->sym ? -1 : 1;
    if (a->pos != b->pos) return a->pos < b->pos ? -1 : 1;
    return 0;
}

/* occurrence list: every (symbol, position) pair, sorted by symbol then
 * position; the occurrences of c are a contiguous, position-ordered range */
static occ_t *make_occ(const void *text, uint64_t n, uint32_t sym_bytes)
{
    occ_t *o = (occ_t *)malloc((size_t)(n ? n : 1) * sizeof(occ_t));
    if (!o) return NULL;
    for (uint64_t i = 0; i < n; i++) {
        o[i].sym = sym_at(text, sym_bytes, i);
        o[i].pos = i;
    }
    qsort(o, (size_t)n, sizeof(occ_t), occ_cmp);
    return o;
}

/* first index in o[0,n) whose (sym,pos) is >= (c,p) */
static uint64_t occ_lower(const occ_t *o, uint64_t n, uint64_t c, uint64_t p)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        int less = (o[mid].sym < c) || (o[mid].sym == c && o[mid].pos < p);
        if (less) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

int orc_queries_def(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, int op,
                    const uint32_t *syms, const uint64_t *args, uint64_t m, uint64_t *out)
{
    uint64_t sigma_end = (L >= 32) ? ((uint64_t)1 << 32) : ((uint64_t)1 << L);
    occ_t *o = NULL;
    if (op != ORC_Q_ACCESS) {
        o = make_occ(text, n, sym_bytes);
        if (!o) return ORC_ENOMEM;
    }
    for (uint64_t q = 0; q < m; q++) {
        if (op == ORC_Q_ACCESS) {
            /* access(i) = T[i] */
            uint64_t i = args[q];
            out[q] = (i < n) ? sym_at(text, sym_bytes, i) : 0xFFFFFFFFull;
        } else if (op == ORC_Q_RANK) {
            /* rank_c(i) = #{ j < i : T[j] = c } */
            uint64_t c = syms[q], i = args[q];
            if (i > n) out[q] = UINT64_MAX;
            else if (c >= sigma_end) out[q] = 0;
            else out[q] = occ_lower(o, n, c, i) - occ_lower(o, n, c, 0);
        } else {
            /* select_c(k) = the j with T[j] = c and rank_c(j) = k - 1 */
            uint64_t c = syms[q], k = args[q];
            uint64_t a = (c < sigma_end) ? occ_lower(o, n, c, 0) : 0;
            uint64_t b = (c < sigma_end) ? occ_lower(o, n, c + 1, 0) : 0;
            if (c >= sigma_end || k == 0 || k > b - a) out[q] = UINT64_MAX;
            else out[q] = o[a + k - 1].pos;
        }
    }
    free(o);
    return ORC_OK;
}

/* rank_c(i) = #{ j < i : T[j] = c } (Section 2) for many (c, i) pairs on a
 * long text, without the occurrence lists: the queries are visited in
 * increasing i while one left-to-right scan of the text keeps, for every
 * symbol, how often it has occurred so far.  The same sentinels as above
 * (UINT64_MAX for i > n, 0 for c >= 2^L).  Needs 2^L counters: L <= 26. */
typedef struct {
    uint64_t pos;
    uint64_t q;
} rq_t;

static int rq_cmp(const void *x, const void *y)
{
    const rq_t *a = (const rq_t *)x, *b = (const rq_t *)y;
    if (a->pos != b->pos) return a->pos < b->pos ? -1 : 1;
    return a->q < b->q ? -1 : (a->q > b->q);
}

int orc_rank_scan(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, const uint32_t *syms,
                  const uint64_t *pos, uint64_t m, uint64_t *out)
{
    if (L > 26) return ORC_EINVAL;
    int rc = orc_check_symbols(text, n, sym_bytes, L);
    if (rc != ORC_OK) return rc;
    uint64_t sigma_end = (uint64_t)1 << L;
    uint64_t *count = (uint64_t *)calloc((size_t)sigma_end, sizeof(uint64_t));
    rq_t *order = (rq_t *)malloc((size_t)(m ? m : 1) * sizeof(rq_t));
    if (!count || !order) {
        free(count);
        free(order);
        return ORC_ENOMEM;
    }
    for (uint64_t q = 0; q < m; q++) {
        order[q].pos = pos[q];
        order[q].q = q;
    }
    qsort(order, (size_t)m, sizeof(rq_t), rq_cmp);
    uint64_t i = 0; /* count[] covers T[0, i) */
    for (uint64_t r = 0; r < m; r++) {
        uint64_t p = order[r].pos, q = order[r].q;
        if (p > n) {
            out[q] = UINT64_MAX;
            continue;
        }
        while (i < p) count[sym_at(text, sym_bytes, i++)]++;
        out[q] = (syms[q] < sigma_end) ? count[syms[q]] : 0;
    }
    free(count);
    free(order);
    return ORC_OK;
}

/* ---- queries by walking the oracle's own levels (textbook walks) -------- */

int orc_queries_walk(int kind, const uint64_t *bits, uint64_t W, const uint64_t *zeros,
                     uint64_t n, uint32_t L, int op, const uint32_t *syms, const uint64_t *args,
                     uint64_t m, uint64_t *out)
{
    uint64_t sigma_end = (L >= 32) ? ((uint64_t)1 << 32) : ((uint64_t)1 << L);
    uint64_t s_stack[33];
    for (uint64_t q = 0; q < m; q++) {
        if (op == ORC_Q_ACCESS) {
            uint64_t i = args[q];
            if (i >= n) {
                out[q] = 0xFFFFFFFFull;
                continue;
            }
            uint64_t c = 0, s = 0, e = n;
            for (uint32_t l = 0; l < L; l++) {
                const uint64_t *lv = bits + (uint64_t)l * W;
                uint32_t b = get_bit(lv, i);
                c = 2 * c + b;
                if (kind == ORC_WM) {
                    i = b ? zeros[l] + orc_rank_bv(lv, i, 1) : orc_rank_bv(lv, i, 0);
                } else {
                    uint64_t r0s = orc_rank_bv(lv, s, 0), r0e = orc_rank_bv(lv, e, 0);
                    uint64_t z = r0e - r0s;
                    if (b == 0) {
                        i = s + orc_rank_bv(lv, i, 0) - r0s;
                        e = s + z;
                    } else {
                        i = s + z + orc_rank_bv(lv, i, 1) - orc_rank_bv(lv, s, 1);
                        s = s + z;
                    }
                }
            }
            out[q] = c;
        } else if (op == ORC_Q_RANK) {
            uint64_t c = syms[q], i = args[q];
            if (i > n) {
                out[q] = UINT64_MAX;
                continue;
            }
            if (c >= sigma_end) {
                out[q] = 0;
                continue;
            }
            uint64_t s = 0, e = n, p = i;
            for (uint32_t l = 0; l < L; l++) {
                const uint64_t *lv = bits + (uint64_t)l * W;
                uint32_t b = bit_of(L, l, (uint32_t)c);
                if (kind == ORC_WM) {
                    if (b) {
                        p = zeros[l] + orc_rank_bv(lv, p, 1);
                        s = zeros[l] + orc_rank_bv(lv, s, 1);
                    } else {
                        p = orc_rank_bv(lv, p, 0);
                        s = orc_rank_bv(lv, s, 0);
                    }
                } else {
                    uint64_t r0s = orc_rank_bv(lv, s, 0), r0e = orc_rank_bv(lv, e, 0);
                    uint64_t z = r0e - r0s;
                    if (b == 0) {
                        p = s + orc_rank_bv(lv, p, 0) - r0s;
                        e = s + z;
                    } else {
                        p = s + z + orc_rank_bv(lv, p, 1) - orc_rank_bv(lv, s, 1);
                        s = s + z;
                    }
                }
            }
            out[q] = p - s;
        } else {
            uint64_t c = syms[q], k = args[q];
            if (c >= sigma_end || k == 0) {
                out[q] = UINT64_MAX;
                continue;
            }
            /* top-down: interval [s,e) of c on every level */
            uint64_t s = 0, e = n;
            for (uint32_t l = 0; l < L; l++) {
                const uint64_t *lv = bits + (uint64_t)l * W;
                uint32_t b = bit_of(L, l, (uint32_t)c);
                s_stack[l] = s;
                if (kind == ORC_WM) {
                    if (b) {
                        s = zeros[l] + orc_rank_bv(lv, s, 1);
                        e = zeros[l] + orc_rank_bv(lv, e, 1);
                    } else {
                        s = orc_rank_bv(lv, s, 0);
                        e = orc_rank_bv(lv, e, 0);
                    }
                } else {
                    uint64_t r0s = orc_rank_bv(lv, s, 0), r0e = orc_rank_bv(lv, e, 0);
                    uint64_t z = r0e - r0s;
                    if (b == 0) e = s + z;
                    else s = s + z;
                }
            }
            if (k > e - s) {
                out[q] = UINT64_MAX;
                continue;
            }
            /* bottom-up: map the k-th occurrence back to level 0 */
            uint64_t p = (kind == ORC_WM) ? s + k - 1 : k - 1;
            for (uint32_t l = L; l-- > 0;) {
                const uint64_t *lv = bits + (uint64_t)l * W;
                uint32_t b = bit_of(L, l, (uint32_t)c);
                if (kind == ORC_WM) {
                    p = b ? orc_select_bv(lv, n, p - zeros[l] + 1, 1) : orc_select_bv(lv, n, p + 1, 0);
                } else {
                    uint64_t sl = s_stack[l];
                    uint64_t pos = orc_select_bv(lv, n, orc_rank_bv(lv, sl, b) + p + 1, b);
                    p = pos - sl;
                }
            }
            out[q] = p;
        }
    }
    return ORC_OK;
}

/* ---- single level bits at sampled positions ----------------------------- */

typedef struct {
    uint64_t key;  /* level-bit prefix of the interval */
    uint64_t rank; /* 0-based occurrence index inside the interval */
    uint64_t slot; /* index into the caller's arrays */
} samp_t;

static int samp_cmp(const void *x, const void *y)
{
    const samp_t *a = (const samp_t *)x, *b = (const samp_t *)y;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->rank != b->rank) return a->rank < b->rank ? -1 : 1;
    return 0;
}

/*
 * Bit `level` of the WT or WM at the given positions, computed without the
 * other levels: position p of the level belongs to the interval of the prefix
 * key whose start SPos[key] <= p < SPos[key] + Hist[key]; it holds bit `level`
 * of the (p - SPos[key])-th symbol of the text with that prefix (text order).
 * The level must be at most 26 so that the prefix histogram stays small.
 */
int orc_sample_level(int kind, const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L,
                     uint32_t level, const uint64_t *positions, uint64_t m, uint8_t *out)
{
    if (level >= L || level > 26) return ORC_EINVAL;
    uint64_t keys = (uint64_t)1 << level;
    uint64_t *hist = (uint64_t *)malloc(keys * sizeof(uint64_t));
    uint64_t *spos = (uint64_t *)malloc(keys * sizeof(uint64_t));
    uint64_t *order = (uint64_t *)malloc(keys * sizeof(uint64_t));
    uint64_t *seen = (uint64_t *)calloc(keys, sizeof(uint64_t));
    samp_t *req = (samp_t *)malloc((size_t)(m ? m : 1) * sizeof(samp_t));
    int rc = ORC_OK;
    if (!hist || !spos || !order || !seen || !req) {
        rc = ORC_ENOMEM;
        goto done;
    }
    rc = orc_hist(text, n, sym_bytes, L, level, hist);
    if (rc != ORC_OK) goto done;
    /* interval starts: keys visited in interval order, summing sizes */
    for (uint64_t i = 0; i < keys; i++) order[i] = (kind == ORC_WT) ? i : orc_reverse_bits(i, level);
    {
        uint64_t run = 0;
        for (uint64_t i = 0; i < keys; i++) {
            spos[order[i]] = run;
            run += hist[order[i]];
        }
    }
    for (uint64_t q = 0; q < m; q++) {
        uint64_t p = positions[q];
        if (p >= n) {
            rc = ORC_EINVAL;
            goto done;
        }
        /* the interval holding p: the last interval (in order) starting at <= p
         * that is non-empty */
        uint64_t lo = 0, hi = keys; /* search over interval order */
        while (hi - lo > 1) {
            uint64_t mid = (lo + hi) / 2;
            if (spos[order[mid]] <= p) lo = mid;
            else hi = mid;
        }
        while (hist[order[lo]] == 0 || spos[order[lo]] + hist[order[lo]] <= p) lo++;
        req[q].key = order[lo];
        req[q].rank = p - spos[order[lo]];
        req[q].slot = q;
    }
    qsort(req, (size_t)m, sizeof(samp_t), samp_cmp);
    /* one pass over the text; per key, count occurrences and answer the
     * requests in (key, rank) order */
    {
        /* first request index per key */
        uint64_t *first = order; /* reuse: first[key] = index into req, or m */
        for (uint64_t k = 0; k < keys; k++) first[k] = m;
        for (uint64_t q = m; q-- > 0;) first[req[q].key] = q;
        for (uint64_t i = 0; i < n; i++) {
            uint32_t a = sym_at(text, sym_bytes, i);
            uint64_t k = prefix_of(L, level, a);
            uint64_t r = seen[k]++;
            uint64_t q = first[k];
            while (q < m && req[q].key == k && req[q].rank == r) {
                out[req[q].slot] = (uint8_t)bit_of(L, level, a);
                q++;
            }
            first[k] = q;
        }
    }
done:
    free(hist);
    free(spos);
    free(order);
    free(seen);
    free(req);
    return rc;
}

/* ---- position of a WT bit in the WM (Section 5.1; Lemma 5) -------------- */

/* Level `level` of the WT and of the WM hold the same intervals (one per
 * level-bit prefix, same size, same content in the same order), the WT's in
 * prefix order and the WM's in bit-reversed prefix order.  Position i of WT
 * level `level` lies in the interval of prefix bp (the prefix whose WT
 * interval contains i), at offset i - SPos_WT[bp]; the same bit sits at
 * SPos_WM[bp] + that offset in the WM.  Computed here from the direct counts. */
int orc_map_wt_to_wm(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint32_t level,
                     const uint64_t *positions, uint64_t m, uint64_t *out)
{
    if (level >= L || level > 26) return ORC_EINVAL;
    uint64_t keys = (uint64_t)1 << level;
    uint64_t *hist = (uint64_t *)malloc(keys * sizeof(uint64_t));
    uint64_t *swt = (uint64_t *)malloc(keys * sizeof(uint64_t));
    uint64_t *swm = (uint64_t *)malloc(keys * sizeof(uint64_t));
    int rc = ORC_OK;
    if (!hist || !swt || !swm) {
        rc = ORC_ENOMEM;
        goto done;
    }
    if ((rc = orc_hist(text, n, sym_bytes, L, level, hist)) != ORC_OK) goto done;
    orc_spos(ORC_WT, hist, level, swt);
    orc_spos(ORC_WM, hist, level, swm);
    for (uint64_t q = 0; q < m; q++) {
        uint64_t i = positions[q];
        if (i >= n) {
            rc = ORC_EINVAL;
            goto done;
        }
        /* bp: the last prefix whose interval starts at or before i (WT
         * starts do not decrease with the prefix; an empty interval shares
         * its start with the next one, so the last such prefix is never
         * empty) */
        uint64_t lo = 0, hi = keys;
        while (hi - lo > 1) {
            uint64_t mid = (lo + hi) / 2;
            if (swt[mid] <= i) lo = mid;
            else hi = mid;
        }
        out[q] = swm[lo] + (i - swt[lo]);
    }
done:
    free(hist);
    free(swt);
    free(swm);
    return rc;
}


/* ---- pointer-based wavelet tree (Section 2) ------------------------------ */

/* Node (l, p) of the pointer-based tree is the node reached from the root by
 * the l-bit prefix p; its bit vector holds bit(l, a) of every symbol a of T
 * with prefix(l, a) = p, in text order.  Entry e = 2^l - 1 + p of `nodes`
 * receives {first pool word, number of bits}; each node's bits start at bit
 * 0 of a fresh pool word (LSB-first) and take ceil(bits / 64) words, the
 * nodes one after the other in entry order.  Pool words not covered by a node
 * are zero. */
int orc_pointer_tree(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint64_t *nodes,
                     uint64_t *pool, uint64_t pool_words)
{
    int rc = orc_check_symbols(text, n, sym_bytes, L);
    if (rc != ORC_OK) return rc;
    if (L > 26) return ORC_EINVAL;
    if (L == 0) return ORC_OK;
    uint64_t entries = ((uint64_t)1 << L) - 1;
    uint64_t *fill = (uint64_t *)calloc((size_t)entries, sizeof(uint64_t));
    if (!fill) return ORC_ENOMEM;
    /* node sizes: how many symbols carry each prefix */
    for (uint64_t e = 0; e < entries; e++) nodes[2 * e + 1] = 0;
    for (uint32_t l = 0; l < L; l++) {
        uint64_t first = ((uint64_t)1 << l) - 1;
        for (uint64_t i = 0; i < n; i++) nodes[2 * (first + prefix_of(L, l, sym_at(text, sym_bytes, i))) + 1]++;
    }
    /* runs of whole words, in entry order */
    uint64_t w = 0;
    for (uint64_t e = 0; e < entries; e++) {
        nodes[2 * e] = w;
        w += (nodes[2 * e + 1] + 63) / 64;
    }
    if (w > pool_words) {
        free(fill);
        return ORC_EINVAL;
    }
    memset(pool, 0, (size_t)(pool_words * sizeof(uint64_t)));
    /* append each symbol's bit to its node on every level, in text order */
    for (uint64_t i = 0; i < n; i++) {
        uint32_t a = sym_at(text, sym_bytes, i);
        for (uint32_t l = 0; l < L; l++) {
            uint64_t e = ((uint64_t)1 << l) - 1 + prefix_of(L, l, a);
            uint64_t q = fill[e]++;
            if (bit_of(L, l, a)) pool[nodes[2 * e] + q / 64] |= (uint64_t)1 << (q % 64);
        }
    }
    free(fill);
    return ORC_OK;
}
