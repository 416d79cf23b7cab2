// Conversion between the level-wise wavelet tree and the wavelet matrix of
// the same text, and the tables of the WT-to-WM position map.
//
// Section 5.1: on every level the WT and the WM hold the same intervals (one
// per bit prefix of the level's length, the same bits in the same order),
// the WT's in prefix order and the WM's in bit-reversed prefix order.  So
// either structure yields, level by level, every prefix's interval length and
// its start in both orders, and the other structure is gathered interval by
// interval.  The walk goes down from level 0: a prefix's interval splits into
// its two children by the zeros and ones it holds on the current level,
// counted with the source's rank directory (WM: a zero child continues at
// rank_0 of the interval start, a one child at Z + rank_1; WT: the children
// are adjacent).  From a WT the WM starts are the zero-based prefix sums of
// the lengths in bit-reversed order.
//
// Lemma 5: the position map needs the unary histogram U = 1^{c_0} 0 1^{c_1} 0
// ... of the symbol counts c_s (the leaf level of the walk) with its rank and
// select directories, and X, the WM interval starts of every level.
#include "wt_device.h"

namespace wtg {

// walk tables of level l: WM start, length, WT start, 2^l u32 each
__host__ __device__ inline uint64_t ctab_off(uint32_t l) { return 3ull * ((1ull << l) - 1ull); }

__global__ void k_cwalk_init(uint32_t *tab, uint64_t n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        tab[0] = 0;
        tab[1] = (uint32_t)n;
        tab[2] = 0;
    }
}

// level l -> level l + 1 of the walk, one thread per l-bit prefix
__global__ __launch_bounds__(256) void k_cwalk_step(wt_levels src, uint32_t *tab, uint32_t l)
{
    const uint64_t np = 1ull << l;
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const uint32_t *cur = tab + ctab_off(l);
    uint32_t *nxt = tab + ctab_off(l + 1);
    const uint32_t ms = cur[p], h = cur[np + p], ws = cur[2 * np + p];
    const uint64_t *bits = src.bits + (uint64_t)l * src.words_per_level;
    const uint32_t *rd = src.rank_dir + (uint64_t)l * src.rank_stride;
    // the interval on this level of the source: WM start or WT start
    const uint32_t s = (src.kind == WT_MATRIX) ? ms : ws;
    uint32_t r1s = 0, ones = 0;
    if (h) {
        r1s = (uint32_t)rank1_dir(bits, rd, s);
        ones = (uint32_t)rank1_dir(bits, rd, (uint64_t)s + h) - r1s;
    }
    const uint64_t nn = 2 * np;
    uint32_t m0 = 0, m1 = 0;  // WM starts of the children (from a WT: by a later scan)
    if (src.kind == WT_MATRIX) {
        m0 = ms - r1s;
        m1 = (uint32_t)src.zeros[l] + r1s;
    }
    nxt[2 * p] = m0;
    nxt[nn + 2 * p] = h - ones;
    nxt[2 * nn + 2 * p] = ws;
    nxt[2 * p + 1] = m1;
    nxt[nn + 2 * p + 1] = ones;
    nxt[2 * nn + 2 * p + 1] = ws + (h - ones);
}

// WM starts of every level from the lengths: zero-based prefix sums with
// the prefixes visited in bit-reversed order (one block per level)
__global__ __launch_bounds__(1024) void k_cwm_starts(uint32_t *tab, uint32_t L)
{
    __shared__ uint32_t part[1024];
    const uint32_t l = blockIdx.x;
    if (l >= L) return;
    const uint64_t np = 1ull << l;
    uint32_t *ms = tab + ctab_off(l);
    const uint32_t *len = ms + np;
    const uint32_t t = threadIdx.x;
    const uint64_t per = (np + 1023) / 1024;
    const uint64_t i0 = t * per, i1 = min(np, i0 + per);
    uint32_t s = 0;
    for (uint64_t i = i0; i < i1; i++) s += len[rev_bits((uint32_t)i, l)];
    part[t] = s;
    __syncthreads();
    // exclusive scan of the 1024 partial sums (Hillis-Steele in LDS)
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t x = (t >= off) ? part[t - off] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (uint64_t i = i0; i < i1; i++) {
        const uint32_t p = rev_bits((uint32_t)i, l);
        ms[p] = run;
        run += len[p];
    }
}

// Word w of level l of dst, gathered from level l of src interval by interval
// (the intervals sorted by their start in dst's order).
__global__ __launch_bounds__(256) void k_cgather(wt_levels src, wt_levels dst, const uint32_t *tab,
                                                 uint32_t l)
{
    __shared__ uint32_t bnd[2];
    const uint64_t W = dst.words_per_level;
    const uint64_t n = dst.n;
    const uint32_t np = 1u << l;
    const uint32_t *ms = tab + ctab_off(l), *len = ms + np, *ws = len + np;
    const bool to_wt = (dst.kind == WT_TREE);
    // start of the interval of rank r in dst order
    auto start = [&](uint32_t r) -> uint64_t { return to_wt ? ws[r] : ms[rev_bits(r, l)]; };
    // the last interval (in dst order) in [a, b) starting at or before pos
    // (start(a) <= pos); an empty interval shares its start with the next
    // one, so it is never the last such interval
    auto search = [&](uint64_t pos, uint32_t a, uint32_t b) -> uint32_t {
        while (b - a > 1) {
            const uint32_t mid = (a + b) >> 1;
            if (start(mid) <= pos) a = mid;
            else b = mid;
        }
        return a;
    };
    // the block's words lie between the intervals of its first and last
    // positions: one full search each (wave 0 and wave 1), then every thread
    // searches between
    const uint64_t w0 = (uint64_t)blockIdx.x * blockDim.x;
    const uint64_t p_first = w0 << 6;
    const uint64_t p_last = min(min(w0 + blockDim.x, W) << 6, n) - 1;  // used only when p_first < n
    if (p_first < n && threadIdx.x < 128) {
        const uint32_t slot = threadIdx.x >> 6;
        const uint64_t r = wave_search_last_le(np, slot ? p_last : p_first,
                                               [&](uint64_t q) { return start((uint32_t)q); });
        if ((threadIdx.x & 63) == 0) bnd[slot] = (uint32_t)r;
    }
    __syncthreads();
    const uint64_t w = w0 + threadIdx.x;
    if (w >= W) return;
    const uint64_t *sb = src.bits + (uint64_t)l * src.words_per_level;
    const uint64_t ws0 = w << 6;
    const uint64_t we = min(ws0 + 64, n);
    uint64_t val = 0;
    uint64_t pos = ws0;
    uint32_t lo = np;  // rank (in dst order) of the previous piece's interval
    while (pos < we) {
        // the next interval in dst order when it starts at pos and is not
        // empty, else a search between the block's bounds
        const uint32_t pn = to_wt ? lo + 1 : rev_bits(lo + 1, l);
        if (lo + 1 < np && (to_wt ? ws[pn] : ms[pn]) == pos && len[pn] != 0) {
            lo = lo + 1;
        } else if (lo < np) {
            // empty intervals follow the previous one: a bracket that
            // doubles from it until an interval starts past pos, then a
            // search inside it
            const uint32_t hi = bnd[1] + 1;
            uint32_t a = lo, b = lo + 1, step = 1;
            while (b < hi && start(b) <= pos) {
                a = b;
                step <<= 1;
                b = a + step;
            }
            lo = search(pos, a, max(min(b, hi), a + 1));  // never empty
        } else {
            lo = search(pos, bnd[0], bnd[1] + 1);
        }
        const uint32_t p = to_wt ? lo : rev_bits(lo, l);
        const uint64_t ds = to_wt ? ws[p] : ms[p];
        const uint64_t ss = to_wt ? ms[p] : ws[p];
        uint64_t end = ds + len[p];
        if (end > we) end = we;
        if (end <= pos) break;  // never for consistent tables
        const uint32_t cnt = (uint32_t)(end - pos);
        const uint64_t s = ss + (pos - ds);
        const uint32_t sh = (uint32_t)(s & 63);
        uint64_t x = sb[s >> 6] >> sh;
        if (sh && sh + cnt > 64) x |= sb[(s >> 6) + 1] << (64 - sh);
        if (cnt < 64) x &= (1ull << cnt) - 1;
        val |= x << (pos - ws0);
        pos = end;
    }
    dst.bits[(uint64_t)l * W + w] = val;
}

// Z of the source, and its status (a source built from symbols out of range
// makes the destination just as unspecified)
__global__ void k_ccopy_zeros(wt_levels src, wt_levels dst)
{
    for (uint32_t l = threadIdx.x; l < dst.lg_sigma; l += blockDim.x) dst.zeros[l] = src.zeros[l];
    if (threadIdx.x == 0) *dst.status = *src.status;
}

// U: 1^{c_0} 0 1^{c_1} 0 ... 1^{c_{s-1}} 0 over positions [0, n + s), zero
// past it; the zero after symbol c's ones sits at (count of symbols <= c) + c
// = WT start + length + c of the leaf-level walk entry of c.
__global__ __launch_bounds__(256) void k_cunary(wt_posmap m, const uint32_t *tab)
{
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= m.u_words) return;
    const uint32_t L = m.lg_sigma;
    const uint64_t sig = 1ull << L;
    const uint32_t *len = tab + ctab_off(L) + sig, *ws = len + sig;
    auto zero_at = [&](uint64_t c) -> uint64_t { return (uint64_t)ws[c] + len[c] + c; };
    const uint64_t b0 = w << 6;
    const uint64_t valid = (m.u_len > b0) ? min<uint64_t>(64, m.u_len - b0) : 0;
    uint64_t val = (valid == 64) ? ~0ull : ((1ull << valid) - 1);
    // first symbol whose zero is at or past b0
    uint64_t lo = 0, hi = sig;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (zero_at(mid) < b0) lo = mid + 1;
        else hi = mid;
    }
    for (uint64_t c = lo; c < sig; c++) {
        const uint64_t z = zero_at(c);
        if (z >= b0 + 64) break;
        val &= ~(1ull << (z - b0));
    }
    m.U[w] = val;
}

// X: WM start of every prefix of levels 0 .. L-1
__global__ __launch_bounds__(256) void k_cstarts(wt_posmap m, const uint32_t *tab)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t tot = (1ull << m.lg_sigma) - 1;
    if (e >= tot) return;
    const uint32_t l = 63 - __clzll(e + 1);
    const uint64_t p = e - ((1ull << l) - 1);
    m.X[e] = tab[ctab_off(l) + p];
}

// ---------------------------------------------------------------------------
// Merging partial structures (Section 3.2, domain decomposition; Lemma 4): `count`
// structures of the same kind built from consecutive pieces of a text.  On
// level l the whole text's interval of prefix k is the concatenation, piece
// by piece, of the pieces' intervals of k (text order is piece order), and
// the intervals follow each other in the kind's prefix order.  So each
// piece is walked like a conversion source (its intervals' starts in its own
// order and their lengths), one zero-based prefix sum over (prefix in order,
// piece) gives every piece interval's start in the whole, and every word of
// the whole is gathered from the pieces.

// walk of every piece; piece c's tables at tabs + c * stride
__global__ __launch_bounds__(256) void k_mwalk(const wt_levels *__restrict__ parts, uint32_t count,
                                               uint32_t *tabs, uint64_t stride, uint32_t l)
{
    const uint64_t np = 1ull << l;
    const uint64_t item = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= np * count) return;
    const uint32_t c = (uint32_t)(item >> l);
    const uint64_t p = item & (np - 1);
    const wt_levels &src = parts[c];
    uint32_t *tab = tabs + c * stride;
    if (l == 0 && p == 0) {
        // level 0 is written by the first step itself
        tab[0] = 0;
        tab[1] = (uint32_t)src.n;
        tab[2] = 0;
    }
    const uint32_t *cur = tab + ctab_off(l);
    uint32_t *nxt = tab + ctab_off(l + 1);
    const uint32_t ms = (l == 0) ? 0u : cur[p];
    const uint32_t h = (l == 0) ? (uint32_t)src.n : cur[np + p];
    const uint32_t ws = (l == 0) ? 0u : cur[2 * np + p];
    const uint64_t *bits = src.bits + (uint64_t)l * src.words_per_level;
    const uint32_t *rd = src.rank_dir + (uint64_t)l * src.rank_stride;
    const uint32_t s = (src.kind == WT_MATRIX) ? ms : ws;
    uint32_t r1s = 0, ones = 0;
    if (h) {
        r1s = (uint32_t)rank1_dir(bits, rd, s);
        ones = (uint32_t)rank1_dir(bits, rd, (uint64_t)s + h) - r1s;
    }
    const uint64_t nn = 2 * np;
    nxt[2 * p] = ms - r1s;
    nxt[nn + 2 * p] = h - ones;
    nxt[2 * nn + 2 * p] = ws;
    nxt[2 * p + 1] = (uint32_t)src.zeros[l] + r1s;
    nxt[nn + 2 * p + 1] = ones;
    nxt[2 * nn + 2 * p + 1] = ws + (h - ones);
}

// starts in the whole of every (prefix, piece) interval of level l: a
// zero-based prefix sum over the prefixes in the kind's order, pieces in
// order inside a prefix (one block per level); mtab + count * (2^l - 1) holds
// level l, entry p * count + c
__global__ __launch_bounds__(1024) void k_mstarts(const uint32_t *tabs, uint64_t stride, uint32_t count,
                                                  uint32_t kind, uint32_t *mtab)
{
    __shared__ uint32_t part[1024];
    const uint32_t l = blockIdx.x;
    const uint64_t np = 1ull << l;
    const uint64_t ne = np * count;
    uint32_t *out = mtab + (uint64_t)count * (np - 1);
    const uint32_t t = threadIdx.x;
    const uint64_t per = (ne + 1023) / 1024;
    const uint64_t i0 = t * per, i1 = min(ne, i0 + per);
    auto entry = [&](uint64_t i, uint32_t &p, uint32_t &c) {
        const uint32_t k = (uint32_t)(i / count);
        c = (uint32_t)(i % count);
        p = (kind == WT_TREE) ? k : rev_bits(k, l);
    };
    uint32_t s = 0;
    for (uint64_t i = i0; i < i1; i++) {
        uint32_t p, c;
        entry(i, p, c);
        s += tabs[c * stride + ctab_off(l) + np + p];
    }
    part[t] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t x = (t >= off) ? part[t - off] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (uint64_t i = i0; i < i1; i++) {
        uint32_t p, c;
        entry(i, p, c);
        out[(uint64_t)p * count + c] = run;
        run += tabs[c * stride + ctab_off(l) + np + p];
    }
}

// word w of level l of the whole, gathered from the pieces
__global__ __launch_bounds__(256) void k_mgather(const wt_levels *__restrict__ parts, uint32_t count,
                                                 const uint32_t *tabs, uint64_t stride,
                                                 const uint32_t *mtab, wt_levels dst, uint32_t l)
{
    __shared__ uint64_t mb[2];
    const uint64_t W = dst.words_per_level;
    const uint64_t np = 1ull << l;
    const uint64_t ne = np * count;
    const uint32_t *ds = mtab + (uint64_t)count * (np - 1);
    const bool wt = (dst.kind == WT_TREE);
    // start (in the whole) of the (prefix, piece) interval at position m of the
    // whole's order
    auto start_at = [&](uint64_t m) -> uint64_t {
        const uint32_t k = (uint32_t)(m / count), c = (uint32_t)(m % count);
        const uint32_t p = wt ? k : rev_bits(k, l);
        return ds[(uint64_t)p * count + c];
    };
    // the block's words lie between the intervals of its first and last
    // positions: one full search each (wave 0 and wave 1)
    const uint64_t wb0 = (uint64_t)blockIdx.x * blockDim.x;
    const uint64_t p_first = wb0 << 6;
    if (p_first < dst.n && threadIdx.x < 128) {
        const uint64_t p_last = min(min(wb0 + blockDim.x, W) << 6, dst.n) - 1;
        const uint32_t slot = threadIdx.x >> 6;
        const uint64_t r = wave_search_last_le(ne, slot ? p_last : p_first, start_at);
        if ((threadIdx.x & 63) == 0) mb[slot] = r;
    }
    __syncthreads();
    const uint64_t w = wb0 + threadIdx.x;
    if (w >= W) return;
    const uint64_t b0 = w << 6;
    const uint64_t we = min(b0 + 64, dst.n);
    const uint64_t mlo = mb[0], mhi = mb[1] + 1;  // set whenever b0 < n
    uint64_t val = 0;
    uint64_t pos = b0;
    uint64_t lo = ne;  // position (in the whole's order) of the previous piece's interval
    while (pos < we) {
        // the last (prefix, piece) interval, in the whole's order, starting
        // at or before pos (never an empty one: it shares the next start);
        // the next one in order is taken directly when it starts at pos and
        // is not empty
        bool next = false;
        if (lo + 1 < ne) {
            const uint32_t k = (uint32_t)((lo + 1) / count), c = (uint32_t)((lo + 1) % count);
            const uint32_t p = wt ? k : rev_bits(k, l);
            next = ds[(uint64_t)p * count + c] == pos &&
                   tabs[c * stride + ctab_off(l) + np + p] != 0;
        }
        if (next) {
            lo = lo + 1;
        } else {
            uint64_t a = mlo, hi = mhi;
            if (lo < ne) {
                // after a piece: a bracket that doubles from its interval
                // until an interval starts past pos (empty intervals between)
                uint64_t step = 1;
                a = lo;
                hi = lo + 1;
                while (hi < mhi && start_at(hi) <= pos) {
                    a = hi;
                    step <<= 1;
                    hi = a + step;
                }
                if (hi > mhi) hi = mhi;
                if (hi <= a) hi = a + 1;  // never empty
            }
            while (hi - a > 1) {
                const uint64_t mid = (a + hi) >> 1;
                if (start_at(mid) <= pos) a = mid;
                else hi = mid;
            }
            lo = a;
        }
        const uint32_t k = (uint32_t)(lo / count), c = (uint32_t)(lo % count);
        const uint32_t p = wt ? k : rev_bits(k, l);
        const uint32_t *tab = tabs + c * stride + ctab_off(l);
        const uint64_t start = ds[(uint64_t)p * count + c];
        const uint64_t src0 = wt ? tab[2 * np + p] : tab[p];  // start in the piece's own order
        uint64_t end = start + tab[np + p];
        if (end > we) end = we;
        if (end <= pos) break;  // never for consistent tables
        const uint32_t cnt = (uint32_t)(end - pos);
        const uint64_t s = src0 + (pos - start);
        const uint64_t *sb = parts[c].bits + (uint64_t)l * parts[c].words_per_level;
        const uint32_t sh = (uint32_t)(s & 63);
        uint64_t x = sb[s >> 6] >> sh;
        if (sh && sh + cnt > 64) x |= sb[(s >> 6) + 1] << (64 - sh);
        if (cnt < 64) x &= (1ull << cnt) - 1;
        val |= x << (pos - b0);
        pos = end;
    }
    dst.bits[(uint64_t)l * W + w] = val;
}

__global__ void k_mzeros(const wt_levels *__restrict__ parts, uint32_t count, wt_levels dst)
{
    for (uint32_t l = threadIdx.x; l < dst.lg_sigma; l += blockDim.x) {
        uint64_t z = 0;
        for (uint32_t c = 0; c < count; c++) z += parts[c].zeros[l];
        dst.zeros[l] = z;
    }
}

// ---------------------------------------------------------------------------
// Export to node-local bit vectors (Section 2: the pointer-based WT keeps one
// bit vector per node; the level-wise WT concatenates a level's nodes).  Node
// (l, p) is entry 2^l - 1 + p of the node table (children of entry e at 2e+1
// and 2e+2); its bits are the interval of prefix p on WT level l, copied to a
// word-aligned run of the pool so that every node's bit vector starts at
// bit 0 of a word.

// pool words of every node, then their zero-based prefix sum (one block):
// nodes[e] = {first pool word, bits}
__global__ __launch_bounds__(1024) void k_xoffsets(const uint32_t *tab, uint32_t L, uint64_t *nodes)
{
    __shared__ uint64_t part[1024];
    const uint64_t ne = (1ull << L) - 1;
    const uint32_t t = threadIdx.x;
    const uint64_t per = (ne + 1023) / 1024;
    const uint64_t e0 = t * per, e1 = min(ne, e0 + per);
    auto len_of = [&](uint64_t e) -> uint64_t {
        const uint32_t l = 63 - __clzll(e + 1);
        const uint64_t p = e - ((1ull << l) - 1);
        return tab[ctab_off(l) + (1ull << l) + p];
    };
    uint64_t s = 0;
    for (uint64_t e = e0; e < e1; e++) s += (len_of(e) + 63) >> 6;
    part[t] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint64_t x = (t >= off) ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint64_t run = part[t] - s;
    for (uint64_t e = e0; e < e1; e++) {
        const uint64_t h = len_of(e);
        nodes[2 * e] = run;
        nodes[2 * e + 1] = h;
        run += (h + 63) >> 6;
    }
}

// pool word q: the node whose run holds it (binary search over the node
// table), and the 64 bits of its interval at that offset
__global__ __launch_bounds__(256) void k_xgather(wt_levels wt, const uint32_t *tab, const uint64_t *nodes,
                                                 uint64_t *pool, uint64_t pool_words)
{
    __shared__ uint64_t xb[2];
    const uint64_t ne = (1ull << wt.lg_sigma) - 1;
    // the nodes of the block's first and last words, by two whole waves (the
    // grid has no block past the pool)
    const uint64_t q0 = (uint64_t)blockIdx.x * blockDim.x;
    if (threadIdx.x < 128) {
        const uint32_t slot = threadIdx.x >> 6;
        const uint64_t qe = min(q0 + blockDim.x, pool_words) - 1;
        const uint64_t r = wave_search_last_le(ne, slot ? qe : q0, [&](uint64_t m) { return nodes[2 * m]; });
        if ((threadIdx.x & 63) == 0) xb[slot] = r;
    }
    __syncthreads();
    const uint64_t q = q0 + threadIdx.x;
    if (q >= pool_words) return;
    // last node whose run starts at or before q (empty nodes share the next
    // node's start, so the last one is not empty), between the block's nodes
    uint64_t lo = xb[0], hi = xb[1] + 1;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (nodes[2 * mid] <= q) lo = mid;
        else hi = mid;
    }
    const uint64_t h = nodes[2 * lo + 1];
    const uint64_t k = q - nodes[2 * lo];  // word of the node
    if (k * 64 >= h) {                      // never for a consistent table
        pool[q] = 0;
        return;
    }
    const uint32_t l = 63 - __clzll(lo + 1);
    const uint64_t p = lo - ((1ull << l) - 1);
    const uint64_t s = (uint64_t)tab[ctab_off(l) + 2 * (1ull << l) + p] + k * 64;  // WT position
    const uint32_t cnt = (uint32_t)min<uint64_t>(64, h - k * 64);
    const uint64_t *sb = wt.bits + (uint64_t)l * wt.words_per_level;
    const uint32_t sh = (uint32_t)(s & 63);
    uint64_t x = sb[s >> 6] >> sh;
    if (sh && sh + cnt > 64) x |= sb[(s >> 6) + 1] << (64 - sh);
    if (cnt < 64) x &= (1ull << cnt) - 1;
    pool[q] = x;
}

static inline uint32_t blocks_for(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

hipError_t launch_export_nodes(const wt_levels &wt, const uint32_t *d_tab, uint64_t *d_nodes,
                               uint64_t *d_pool, uint64_t pool_words, const LaunchCtx &ctx)
{
    hipLaunchKernelGGL(k_xoffsets, dim3(1), dim3(1024), 0, ctx.stream, d_tab, wt.lg_sigma, d_nodes);
    if (pool_words)
        hipLaunchKernelGGL(k_xgather, dim3(blocks_for(pool_words, 256)), dim3(256), 0, ctx.stream, wt, d_tab,
                           d_nodes, d_pool, pool_words);
    if (ctx.after) ctx.after(ctx.user, KID_GATHER);
    return hipGetLastError();
}

hipError_t launch_merge(const wt_levels *d_parts, uint32_t count, uint32_t *d_tabs, uint64_t stride,
                        uint32_t *d_mtab, const wt_levels &dst, const LaunchCtx &ctx)
{
    const uint32_t L = dst.lg_sigma;
    for (uint32_t l = 0; l < L; l++)
        hipLaunchKernelGGL(k_mwalk, dim3(blocks_for((1ull << l) * count, 256)), dim3(256), 0, ctx.stream,
                           d_parts, count, d_tabs, stride, l);
    hipLaunchKernelGGL(k_mstarts, dim3(L), dim3(1024), 0, ctx.stream, d_tabs, stride, count, dst.kind,
                       d_mtab);
    if (ctx.after) ctx.after(ctx.user, KID_WALK);
    if (dst.words_per_level > 0)
        for (uint32_t l = 0; l < L; l++)
            hipLaunchKernelGGL(k_mgather, dim3(blocks_for(dst.words_per_level, 256)), dim3(256), 0,
                               ctx.stream, d_parts, count, d_tabs, stride, d_mtab, dst, l);
    hipLaunchKernelGGL(k_mzeros, dim3(1), dim3(64), 0, ctx.stream, d_parts, count, dst);
    if (ctx.after) ctx.after(ctx.user, KID_GATHER);
    return hipGetLastError();
}

hipError_t launch_convert_walk(const wt_levels &src, uint32_t *d_tab, uint32_t levels,
                               bool need_wm_starts, const LaunchCtx &ctx)
{
    hipLaunchKernelGGL(k_cwalk_init, dim3(1), dim3(64), 0, ctx.stream, d_tab, src.n);
    for (uint32_t l = 0; l < levels; l++)
        hipLaunchKernelGGL(k_cwalk_step, dim3(blocks_for(1ull << l, 256)), dim3(256), 0, ctx.stream,
                           src, d_tab, l);
    if (need_wm_starts && src.kind == WT_TREE && src.lg_sigma > 0)
        hipLaunchKernelGGL(k_cwm_starts, dim3(src.lg_sigma), dim3(1024), 0, ctx.stream, d_tab,
                           src.lg_sigma);
    if (ctx.after) ctx.after(ctx.user, KID_WALK);
    return hipGetLastError();
}

hipError_t launch_convert_gather(const wt_levels &src, const wt_levels &dst, const uint32_t *d_tab,
                                 const LaunchCtx &ctx)
{
    for (uint32_t l = 0; l < dst.lg_sigma; l++)
        hipLaunchKernelGGL(k_cgather, dim3(blocks_for(dst.words_per_level, 256)), dim3(256), 0,
                           ctx.stream, src, dst, d_tab, l);
    hipLaunchKernelGGL(k_ccopy_zeros, dim3(1), dim3(64), 0, ctx.stream, src, dst);
    if (ctx.after) ctx.after(ctx.user, KID_GATHER);
    return hipGetLastError();
}

hipError_t launch_posmap_fill(const wt_posmap &m, const uint32_t *d_tab, const LaunchCtx &ctx)
{
    hipLaunchKernelGGL(k_cunary, dim3(blocks_for(m.u_words, 256)), dim3(256), 0, ctx.stream, m, d_tab);
    const uint64_t tot = (1ull << m.lg_sigma) - 1;
    if (tot)
        hipLaunchKernelGGL(k_cstarts, dim3(blocks_for(tot, 256)), dim3(256), 0, ctx.stream, m, d_tab);
    if (ctx.after) ctx.after(ctx.user, KID_GATHER);
    return hipGetLastError();
}

}  // namespace wtg
