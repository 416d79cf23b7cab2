/*
 * Oracle for wavelet tree / wavelet matrix construction: TEST INFRASTRUCTURE.
 * Declarations for wt_oracle.c.  Host pointers only.  Not used by, and sharing
 * nothing with, the GPU library.
 */
#ifndef WT_ORACLE_H
#define WT_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-3)
#define ORC_ENOMEM (-6)

#define ORC_WT 0
#define ORC_WM 1

#define ORC_Q_ACCESS 0
#define ORC_Q_RANK 1
#define ORC_Q_SELECT 2

/* one select sample every ORC_SEL_SPACING ones (zeros) */
#define ORC_SEL_SPACING 4096u

uint64_t orc_reverse_bits(uint64_t x, uint32_t k);
uint64_t orc_words_per_level(uint64_t n);
uint64_t orc_sel_capacity(uint64_t n);
int orc_check_symbols(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L);

/* levels [L][W] (LSB-first words) and Z[L] of the WT (kind 0) or WM (kind 1) */
int orc_build(int kind, const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L,
              uint64_t *bits, uint64_t W, uint64_t *zeros);
/* Hist[p] for every level-bit prefix p, p < 2^level */
int orc_hist(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint32_t level,
             uint64_t *hist);
/* interval starts from Hist: prefix order (WT) or bit-reversed order (WM) */
int orc_spos(int kind, const uint64_t *hist, uint32_t level, uint64_t *spos);

uint64_t orc_rank_bv(const uint64_t *words, uint64_t i, uint32_t b);
uint64_t orc_select_bv(const uint64_t *words, uint64_t n, uint64_t k, uint32_t b);

/* rank_dir[W/8 + 1], sel0/sel1[orc_sel_capacity(n)] of one level */
int orc_directory(const uint64_t *words, uint64_t n, uint64_t W, uint32_t *rank_dir,
                  uint32_t *sel0, uint32_t *sel1);

/* queries: op 0 access(args=i), 1 rank(syms=c, args=i), 2 select(syms=c, args=k) */
int orc_queries_def(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, int op,
                    const uint32_t *syms, const uint64_t *args, uint64_t m, uint64_t *out);
/* rank only, for long texts: one scan of the text, queries in position order (L <= 26) */
int orc_rank_scan(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, const uint32_t *syms,
                  const uint64_t *pos, uint64_t m, uint64_t *out);
int orc_queries_walk(int kind, const uint64_t *bits, uint64_t W, const uint64_t *zeros,
                     uint64_t n, uint32_t L, int op, const uint32_t *syms, const uint64_t *args,
                     uint64_t m, uint64_t *out);

/* position in WM level `level` of the bit at WT position positions[q] */
int orc_map_wt_to_wm(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint32_t level,
                     const uint64_t *positions, uint64_t m, uint64_t *out);

/* pointer-based WT: nodes[2e] = first pool word, nodes[2e+1] = bits of node
 * e = 2^l - 1 + p (prefix p of length l); bits LSB-first from a fresh word */
int orc_pointer_tree(const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L, uint64_t *nodes,
                     uint64_t *pool, uint64_t pool_words);

/* bit `level` of the WT/WM at the given positions (0/1 per position) */
int orc_sample_level(int kind, const void *text, uint64_t n, uint32_t sym_bytes, uint32_t L,
                     uint32_t level, const uint64_t *positions, uint64_t m, uint8_t *out);
#endif
