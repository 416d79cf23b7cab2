/*
 * wt.h -- C ABI of the MI355X (gfx950) wavelet tree / wavelet matrix library.
 *
 * Builds, on the GPU, the level-wise wavelet tree (WT) and the wavelet matrix
 * (WM) of an integer text T[0,n) over [0, 2^lg_sigma), bottom-up as in
 * Fischer, Kurpicz, Loebel, "Simple, Fast and Lightweight Parallel Wavelet Tree
 * Construction" (arXiv 1702.07578): prefix histograms per tile of the text
 * (Section 3.2, per-core histograms of Algorithm 2), merged upward level by
 * level (Algorithm 1, histogram update), interval starts by a zero-based prefix
 * sum over (key, tile) in prefix order for the WT and bit-reversed order for
 * the WM (Section 3.2 and Section 5.1), and a stable scatter of every level's
 * bits into place (Algorithm 1, bit placement).  It also builds binary
 * rank/select directories over every level and answers batched access, rank
 * and select queries (Section 2 and Section 5: O(lg sigma) walks).
 *
 * Conventions (every call):
 *   - Pointers named d_* and all pointers inside wt_levels are DEVICE pointers;
 *     everything else is host memory.
 *   - The caller owns all memory.  The library never allocates or frees device
 *     memory: outputs live in one caller buffer carved by wt_levels_bind, and
 *     temporaries in a caller workspace sized by wt_workspace_bytes.
 *   - Every device call is asynchronous on the given stream; buffers must stay
 *     alive until the stream has passed the call.  Calls on different streams
 *     must use different workspaces.
 *   - Host-detected errors return immediately with a negative code and enqueue
 *     nothing.  A symbol >= 2^lg_sigma is detected on the device: the build
 *     completes (with unspecified level contents) and sets the status word,
 *     read by wt_get_status.
 *   - Limits: n < 2^32 (positions fit 32 bits), lg_sigma <= 32, sym_bytes in
 *     {1, 2, 4}.  The WT with lg_sigma > WT_MAX_TREE_LEVELS returns
 *     WT_ENOTSUP (its deep levels use dense per-prefix interval tables).
 *
 * Bit layout of a level: position p is bit p%64 of 64-bit word p/64 (LSB
 * first); words_per_level = ceil(n/64) rounded up to a multiple of 8; all bits
 * at positions >= n are zero.  Level l holds bit l (MSB first) of the symbols:
 * bit(l, a) = (a >> (lg_sigma - 1 - l)) & 1 (Section 2).
 */
#ifndef WT_H
#define WT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status / error codes */
#define WT_OK 0
#define WT_EINVAL (-1)   /* bad argument: null pointer, sym_bytes, lg_sigma, n, kind */
#define WT_ENOSPACE (-2) /* output or workspace buffer too small */
#define WT_ERANGE (-3)   /* a symbol is >= 2^lg_sigma (device-detected) */
#define WT_EHIP (-4)     /* a HIP runtime call failed */
#define WT_ENOTSUP (-5)  /* valid but unsupported configuration */

#define WT_MAX_TREE_LEVELS 26
/* one select sample per WT_SEL_SPACING ones (zeros) of a level */
#define WT_SEL_SPACING 4096u

typedef enum { WT_TREE = 0, WT_MATRIX = 1 } wt_kind;

/*
 * Non-owning view of a built (or to-be-built) structure, filled by
 * wt_levels_bind.  All arrays are in device memory inside the bound buffer.
 *   bits      [lg_sigma][words_per_level] level bit vectors (layout above).
 *   zeros     [lg_sigma] number of zeros of each level (Z of Section 5; also
 *             filled for the WT, where it is the same count).
 *   rank_dir  [lg_sigma][rank_stride]: entry j (0 <= j <= words_per_level/8)
 *             is the number of ones in bits [0, 512 j) of the level.
 *   sel0/sel1 [lg_sigma][sel_stride]: entry q is the index of the 512-bit
 *             block holding the (q*WT_SEL_SPACING + 1)-th zero / one of the
 *             level (positions < n only); 0xFFFFFFFF past the last sample.
 *   status    one int32: WT_OK or WT_ERANGE after a build.
 */
typedef struct wt_levels {
    uint64_t n;
    uint32_t lg_sigma;
    uint32_t kind; /* wt_kind */
    uint64_t words_per_level;
    uint64_t rank_stride; /* uint32 entries per level in rank_dir */
    uint64_t sel_stride;  /* uint32 entries per level in sel0 / sel1 */
    uint64_t *bits;
    uint64_t *zeros;
    uint32_t *rank_dir;
    uint32_t *sel0;
    uint32_t *sel1;
    int32_t *status;
} wt_levels;

/* Optional tuning knobs; zero fields mean "choose automatically". */
typedef struct wt_tune {
    uint32_t tile_log2;  /* accepted and ignored: a tile is always 2048 symbols (one wave's registers) */
    uint32_t group_bits; /* levels handled per pass over the text, 1..8 */
    uint32_t grid;       /* ranges of consecutive tiles per text, one wave each (0: 12288) */
    uint32_t persist;    /* workgroups per launch, looping over all work items (0: one per item); the
                            scatter counts them as groups of 4 waves (persist * 4 waves) */
} wt_tune;

/* Bytes of the output buffer for a text of length n over lg_sigma levels
 * (same for the WT and the WM).  Host only. */
size_t wt_output_bytes(uint64_t n, uint32_t lg_sigma);

/* Bytes of device workspace a build needs.  Host only.  0 with tune NULL is
 * never returned for a valid configuration; returns 0 for an invalid one. */
size_t wt_workspace_bytes(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_kind kind);
size_t wt_workspace_bytes_tuned(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_kind kind,
                                const wt_tune *tune);

/* Carve a caller device buffer of `bytes` bytes at d_mem (256-byte aligned)
 * into a wt_levels view.  Host only; touches no device memory.
 * WT_EINVAL / WT_ENOSPACE on bad arguments. */
int wt_levels_bind(wt_levels *out, void *d_mem, size_t bytes, uint64_t n, uint32_t lg_sigma,
                   wt_kind kind);

/*
 * Build the wavelet tree (wt_build) or the wavelet matrix (wm_build) of the
 * device text d_text[0,n) of sym_bytes-byte unsigned symbols, plus Z and the
 * rank/select directories, into *out (bound with the same n, lg_sigma and the
 * matching kind).  d_ws/ws_bytes: device workspace of at least
 * wt_workspace_bytes(...).  Asynchronous on `stream`.
 */
int wt_build(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
             wt_levels *out, void *d_ws, size_t ws_bytes, hipStream_t stream);
int wm_build(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
             wt_levels *out, void *d_ws, size_t ws_bytes, hipStream_t stream);
/* Same, with tuning knobs (tune may be NULL). */
int wt_build_tuned(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes,
                   uint32_t lg_sigma, wt_levels *out, void *d_ws, size_t ws_bytes,
                   const wt_tune *tune, hipStream_t stream);

/*
 * Batched queries over a built structure s (WT or WM, by s->kind), m queries,
 * one result each, asynchronous on `stream`.
 *   access(i) = T[i]; 0xFFFFFFFF if i >= n.
 *   rank(c, i) = number of c in T[0,i) (Section 2); UINT64_MAX if i > n;
 *                0 if c >= 2^lg_sigma.
 *   select(c, k) = position of the k-th c (k >= 1, 0-based result);
 *                UINT64_MAX if k = 0, c >= 2^lg_sigma or k > rank(c, n).
 */
int wt_access(const wt_levels *s, const uint64_t *d_pos, uint64_t m, uint32_t *d_out,
              hipStream_t stream);
int wt_rank(const wt_levels *s, const uint32_t *d_sym, const uint64_t *d_pos, uint64_t m,
            uint64_t *d_out, hipStream_t stream);
int wt_select(const wt_levels *s, const uint32_t *d_sym, const uint64_t *d_k, uint64_t m,
              uint64_t *d_out, hipStream_t stream);

/* Synchronise `stream` and return the status word of s: WT_OK or WT_ERANGE
 * (or WT_EHIP if the synchronisation failed). */
int wt_get_status(const wt_levels *s, hipStream_t stream);

/* Static message for a code. */
const char *wt_strerror(int code);

/*
 * Batched build: `count` independent texts, each with its own length, symbol
 * width, lg_sigma, kind and output view, built by one sequence of launches
 * whose kernels loop over the work items of every text (with tune->persist
 * set, a fixed number of workgroups loops over all items: a persistent grid).
 * d_ws: workspace of wt_batch_workspace_bytes(items, count, tune) bytes.
 *   wt_batch_prepare  copies the per-text descriptors and work-item tables
 *                     into the workspace on `stream` and waits for `stream`
 *                     (host call; the copy is done when it returns).
 *   wt_batch_launch   enqueues the kernels only (no host copies, no memset):
 *                     capturable in a HIP graph and replayable, provided the
 *                     items and workspace are those of the last prepare.
 *   wt_batch_build    prepare followed by launch.
 */
typedef struct wt_batch_item {
    const void *d_text;
    uint64_t n;
    uint32_t sym_bytes;
    uint32_t lg_sigma;
    uint32_t kind;  /* wt_kind */
    uint32_t reserved;
    wt_levels *out; /* host pointer to a bound view */
} wt_batch_item;

size_t wt_batch_workspace_bytes(const wt_batch_item *items, uint32_t count, const wt_tune *tune);
int wt_batch_prepare(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                     const wt_tune *tune, hipStream_t stream);
int wt_batch_launch(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                    const wt_tune *tune, hipStream_t stream);
int wt_batch_build(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                   const wt_tune *tune, hipStream_t stream);

/*
 * Conversion between the two structures of one text (Section 5.1: on every
 * level the WT and the WM hold the same intervals, the WT's in prefix order,
 * the WM's in bit-reversed prefix order).  wt_convert reads a built WT or WM
 * (*src) and writes the other one (*dst, bound with the same n and lg_sigma
 * and the other kind): levels, Z and directories.  The interval tables are
 * walked down from level 0 with the source's rank directory; every word of
 * the destination is then gathered from the source interval by interval.
 * d_ws: workspace of wt_convert_workspace_bytes(n, lg_sigma) bytes (the walk
 * holds 3 * 2^(lg_sigma+1) words).  Asynchronous on `stream`; src must not
 * change until the stream has passed the call.
 * WT_ENOTSUP for lg_sigma > WT_MAX_TREE_LEVELS; WT_EINVAL for mismatched views.
 */
size_t wt_convert_workspace_bytes(uint64_t n, uint32_t lg_sigma);
int wt_convert(const wt_levels *src, wt_levels *dst, void *d_ws, size_t ws_bytes, hipStream_t stream);

/*
 * Merge of partial structures (Section 3.2, domain decomposition; Lemma 4): parts[c]
 * (host array of bound views, same kind and lg_sigma, built on this device)
 * hold the structures of consecutive pieces of a text; *dst (same kind and
 * lg_sigma, n = the pieces' total) receives the structure of the whole text:
 * levels, Z (the pieces' sum) and directories.  On every level the whole
 * text's interval of a prefix is the pieces' intervals of that prefix in
 * piece order, the intervals in the kind's prefix order; one prefix sum over
 * (prefix, piece) places them.  d_ws: wt_merge_workspace_bytes(n, lg_sigma,
 * count) bytes.  Copies the views to the device on `stream` and waits for
 * that copy (host call); the rest is asynchronous.  WT_ENOTSUP for lg_sigma >
 * WT_MAX_TREE_LEVELS or count * 2^(lg_sigma+1) > 2^30.
 */
size_t wt_merge_workspace_bytes(uint64_t n, uint32_t lg_sigma, uint32_t count);
int wt_merge(const wt_levels *parts, uint32_t count, wt_levels *dst, void *d_ws, size_t ws_bytes,
             hipStream_t stream);

/*
 * Both structures of one text (Section 5.1: the WT and the WM hold the same
 * intervals of every level, in prefix order and in bit-reversed prefix
 * order).  With lg_sigma <= 8 (one group of levels) the WT's build writes the
 * WM as well: the tiles are split once, and every run of a level is copied
 * to its WT interval and to its WM interval; the histogram and border passes
 * are shared.  With more levels the WM is built and the WT is gathered from
 * its intervals as wt_convert does.  wt (kind WT_TREE) and wm (kind WT_MATRIX) are bound for (n,
 * lg_sigma); both receive exactly what wt_build and wm_build write (levels,
 * Z, directories, status).  Workspace: wt_pair_workspace_bytes(n, sym_bytes,
 * lg_sigma).  Asynchronous on `stream`; argument errors as for wt_build_tuned.
 */
size_t wt_pair_workspace_bytes(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma);
int wt_pair_build(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_levels *wt,
                  wt_levels *wm, void *d_ws, size_t ws_bytes, hipStream_t stream);
/* Same, with tuning knobs (tune may be NULL: then identical to the calls
 * above).  tune->grid sets the ranges of consecutive tiles per text, so a
 * short text can be cut into ranges of several tiles each; tune->group_bits
 * below lg_sigma takes the several-group path (WM build, then the WT gathered
 * from it); tune->persist caps the workgroups of every launch. */
size_t wt_pair_workspace_bytes_tuned(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, const wt_tune *tune);
int wt_pair_build_tuned(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_levels *wt,
                        wt_levels *wm, void *d_ws, size_t ws_bytes, const wt_tune *tune, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * wt_pair_build with its workspace taken from a scratch array that the
 * library keeps on every GPU it runs on (WT_NOALLOC_SCRATCH_BYTES, held from
 * the library's code object load until the process ends; its device address
 * is looked up once per device, on the first call made with that device
 * current).  The caller still passes the text and the two bound output views;
 * outputs, status and argument errors are those of wt_pair_build.  Allocates
 * nothing and copies nothing from the host: every step is a kernel launch on
 * `stream`.
 * WT_ENOSPACE, before any device work, when the text needs more workspace than
 * the scratch holds (wt_pair_workspace_bytes(n, sym_bytes, lg_sigma) >
 * WT_NOALLOC_SCRATCH_BYTES; for example byte texts of 2^30 symbols with up to
 * 8 levels fit, 2^26 symbols of 16 levels do not).  WT_EHIP if the scratch's
 * device address cannot be obtained.
 * All calls on one GPU share that GPU's scratch, which keeps the last call's
 * contents (no kernel reads a workspace entry it has not written in the same
 * call): calls that overlap on one GPU, from any stream or thread, race and
 * must be serialised by the caller.
 */
#define WT_NOALLOC_SCRATCH_BYTES (64u << 20)
int wt_pair_build_noalloc(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_levels *wt,
                          wt_levels *wm, hipStream_t stream);

/*
 * Construction by sorting (Section 3.2, construction using sorting,
 * Algorithm 2; the WM version of Section 5.1): the second build strategy,
 * with the same result as wt_build_tuned (levels, Z, directories, status).
 * The text is cut into chunks; the chunks' histograms of the full symbols are
 * counted once; then, from the last level up, the histograms of the level's
 * prefixes are merged from the next level's, one zero-based prefix sum over
 * (prefix, chunk) in prefix order (WT) or bit-reversed prefix order (WM)
 * gives each chunk's start per prefix, a stable counting sort by the level's
 * prefix writes a sorted copy of the text, and the level's bits are bit l of
 * that copy.  Level 0 is read from the text.
 * wt_ps_workspace_bytes: workspace bytes (about n * sym_bytes for the sorted
 * copy plus the chunk tables), 0 when unsupported.  lg_sigma is at most 12
 * (WT_ENOTSUP above); other argument rules, outputs and error reporting as for
 * wt_build_tuned.  d_text must be aligned to sym_bytes.  Asynchronous.
 */
size_t wt_ps_workspace_bytes(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma);
int wt_ps_build(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
                wt_levels *out, void *d_ws, size_t ws_bytes, hipStream_t stream);

/*
 * Export of a built WT to node-local bit vectors (Section 2: the
 * pointer-based tree keeps one bit vector per node).  Node (l, p), the prefix
 * p of length l, is entry e = 2^l - 1 + p of d_nodes (2^lg_sigma - 1 entries
 * of two uint64: the first pool word of the node, and its number of bits);
 * its children are entries 2e + 1 and 2e + 2.  The node's bits are the
 * interval of p on WT level l, stored from bit 0 of its first pool word
 * (LSB-first), the nodes' runs one after the other in entry order.
 * wt_export_pool_words(n, lg_sigma) bounds the pool; the words past the last
 * node's run within that bound receive zeros or nothing.  d_ws: workspace of
 * wt_convert_workspace_bytes(n, lg_sigma).  Asynchronous on `stream`.
 * WT_EINVAL if *wt is not a WT; WT_ENOTSUP for lg_sigma > WT_MAX_TREE_LEVELS.
 */
uint64_t wt_export_pool_words(uint64_t n, uint32_t lg_sigma);
int wt_export_nodes(const wt_levels *wt, uint64_t *d_nodes, uint64_t *d_pool, uint64_t pool_words,
                    void *d_ws, size_t ws_bytes, hipStream_t stream);

/*
 * Position map of Lemma 5: the position j in WM level l of the bit at
 * position i of WT level l, in O(1) per query from
 *   U  the unary histogram 1^{c_0} 0 1^{c_1} 0 ... of the symbol counts
 *      (n + 2^lg_sigma bits, LSB-first words, with the library's rank and
 *      select directories: rank_dir per 512-bit block, select samples every
 *      WT_SEL_SPACING zeros / ones),
 *  X  the WM interval starts of every level: level l's 2^l prefixes at
 *      X + 2^l - 1.
 *   j = i for l <= 1; otherwise, with c = rank_0(U, select_1(U, i + 1)) (the
 *   symbol of the (i+1)-th smallest text symbol), bp = prefix(l, c) and
 *   off = i - rank_1(U, select_0(U, bp << (lg_sigma - l))) (0 when that
 *   shifted prefix is 0), j = X[2^l - 1 + bp] + off.
 * wt_posmap_bytes: size of the caller buffer; wt_posmap_bind carves it
 * (host only).  wt_posmap_build fills it from a built WT or WM *s (same
 * workspace as wt_convert).  wt_posmap_query answers m positions of one
 * level: UINT64_MAX for i >= n or level >= lg_sigma.  Requires lg_sigma <=
 * WT_MAX_TREE_LEVELS and n + 2^lg_sigma < 2^32 (else WT_ENOTSUP).
 */
typedef struct wt_posmap {
    uint64_t n;
    uint32_t lg_sigma;
    uint32_t reserved;
    uint64_t u_len;   /* n + 2^lg_sigma bits of U */
    uint64_t u_words; /* words of U, a multiple of 8 */
    uint64_t rank_stride, sel_stride;
    uint64_t *U;
    uint32_t *rank_dir;
    uint32_t *sel0;
    uint32_t *sel1;
    uint32_t *X;
} wt_posmap;

size_t wt_posmap_bytes(uint64_t n, uint32_t lg_sigma);
int wt_posmap_bind(wt_posmap *m, void *d_mem, size_t bytes, uint64_t n, uint32_t lg_sigma);
int wt_posmap_build(const wt_levels *s, wt_posmap *m, void *d_ws, size_t ws_bytes, hipStream_t stream);
int wt_posmap_query(const wt_posmap *m, uint32_t level, const uint64_t *d_pos, uint64_t count,
                    uint64_t *d_out, hipStream_t stream);

/*
 * Timing aid: enqueue one build exactly like wt_build_tuned and, after every
 * kernel launch i (i < capacity), record the caller's event events[i] on
 * `stream` and store the launch's kernel id (see wt_kernel_name) in
 * kernel_ids[i].  *recorded receives the number of launches (which may exceed
 * capacity; launches past capacity are not recorded).  Asynchronous: the
 * caller records a start event before the call and synchronises before
 * reading elapsed times.  The events must be created by the caller
 * (hipEventCreate, timing enabled).
 */
int wt_build_recorded(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes,
                      uint32_t lg_sigma, wt_levels *out, void *d_ws, size_t ws_bytes,
                      const wt_tune *tune, hipStream_t stream, hipEvent_t *events,
                      uint32_t *kernel_ids, uint32_t capacity, uint32_t *recorded);
/* wt_pair_build with the same event recording as wt_build_recorded */
int wt_pair_build_recorded(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
                           wt_levels *wt, wt_levels *wm, void *d_ws, size_t ws_bytes, hipStream_t stream,
                           hipEvent_t *events, uint32_t *kernel_ids, uint32_t capacity, uint32_t *recorded);

/*
 * Profiling aid: run one build like wt_build_tuned, recording a HIP event
 * after every kernel, wait for it, and add each kernel's duration to
 * ms_by_kernel[id] (ids: see wt_kernel_name; n_ids entries, >= WT_NUM_KERNEL_IDS)
 * and its launch count to launches_by_kernel[id].  Synchronous.
 */
#define WT_NUM_KERNEL_IDS 16
int wt_build_profiled(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes,
                      uint32_t lg_sigma, wt_levels *out, void *d_ws, size_t ws_bytes,
                      const wt_tune *tune, hipStream_t stream, double *ms_by_kernel,
                      uint32_t *launches_by_kernel, uint32_t n_ids);
const char *wt_kernel_name(uint32_t id);

#ifdef __cplusplus
}
#endif
#endif /* WT_H */
