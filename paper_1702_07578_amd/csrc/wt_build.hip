// Construction kernels: per-tile prefix histograms, column scans over tiles,
// interval starts, border-word zeroing, the stable level scatter, and (for a
// wavelet tree with more levels than one pass handles) the interval walk and
// gather of the deep levels from wavelet-matrix levels.
//
// Method (Fischer, Kurpicz, Loebel, arXiv 1702.07578):
//   * every tile of the text is one "core" of Algorithm 2: its histogram of
//     the group key (the next K bits of every symbol) is built once and merged
//     upward to every shorter prefix (Algorithm 1, Hist[i] = Hist[2i] +
//     Hist[2i+1]), instead of re-scanning the text per level;
//   * interval starts are a zero-based prefix sum over (key, tile), keys in
//     prefix order for the WT and bit-reversed order for the WM (Section 3.2,
//     "w.r.t. id"; Section 5.1, id replaced by the bit-reversal permutation);
//   * every level's bits are placed stably (text order inside an interval,
//     Algorithm 1 bit placement), here by splitting the tile in LDS one bit at
//     a time: after the split by bit a, the tile is ordered by its reversed
//     (a+1)-bit key (Observation 2), so each key's bits form one contiguous run
//     that is copied to its interval start, for the WT and WM alike (Section
//     5.1: both have the same intervals, in a different order).
#include "wt_tiles.h"

namespace wtg {

// ---------------------------------------------------------------------------
// init: copy one descriptor into the workspace and clear the status word

__global__ void k_init(TextDesc d, TextDesc *dst)
{
    if (threadIdx.x == 0) {
        *dst = d;
        *d.status = WT_OK;
    }
    for (uint32_t l = threadIdx.x; l < d.L; l += blockDim.x) d.zeros[l] = 0;
}

// batch: clear the status word and Z of every text
__global__ void k_init_batch(const TextDesc *__restrict__ descs, uint32_t nd)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const TextDesc &d = descs[i];
    *d.status = WT_OK;
    for (uint32_t l = 0; l < d.L; l++) d.zeros[l] = 0;
}

// ---------------------------------------------------------------------------
// K0: per-range histogram of the group key (and the symbol range check).
// Each lane reads 16-byte units of the range; units past the range end are
// read symbol by symbol.

template <typename E>
__device__ inline void count_unit(const uint4 &u, uint32_t shift, uint32_t mask, uint32_t L,
                                  bool check, bool &bad, uint32_t *hist)
{
    const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) {
#pragma unroll
        for (uint32_t s = 0; s < 4 / sizeof(E); s++) {
            const uint32_t e = (sizeof(E) == 4) ? w4[q] : ((w4[q] >> (s * 8 * sizeof(E))) & ((1u << (8 * sizeof(E))) - 1u));
            if (check && (e >> L) != 0) bad = true;
            atomicAdd(&hist[(e >> shift) & mask], 1u);
        }
    }
}

template <typename E>
__device__ void hist_range(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r, uint32_t *sh)
{
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    const uint32_t nk = 1u << Kg, mask = nk - 1u;
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint64_t span = (uint64_t)d.R << d.log2S;
    const uint64_t start = (uint64_t)r * span;
    const uint64_t len = min(span, d.n - start);
    const E *src = (const E *)seq_in(d, g) + start;
    uint32_t *hist = sh + w * nk;

    for (uint32_t i = tid; i < kTileWaves * nk; i += kTileThreads) sh[i] = 0;
    __syncthreads();
    bool bad = false;
    const bool check = (g == 0) && (d.L < 32);
    const uint32_t per_unit = 16 / sizeof(E);
    uint64_t done = 0;
    if (((uintptr_t)src & 15) == 0) {
        const uint4 *u = (const uint4 *)src;
        const uint64_t nu = len / per_unit;
        uint64_t i = tid;
        for (; i + 3 * kTileThreads < nu; i += 4 * kTileThreads) {
            const uint4 a0 = u[i], a1 = u[i + kTileThreads], a2 = u[i + 2 * kTileThreads],
                        a3 = u[i + 3 * kTileThreads];
            count_unit<E>(a0, shift, mask, d.L, check, bad, hist);
            count_unit<E>(a1, shift, mask, d.L, check, bad, hist);
            count_unit<E>(a2, shift, mask, d.L, check, bad, hist);
            count_unit<E>(a3, shift, mask, d.L, check, bad, hist);
        }
        for (; i < nu; i += kTileThreads) count_unit<E>(u[i], shift, mask, d.L, check, bad, hist);
        done = nu * per_unit;
    }
    for (uint64_t i = done + tid; i < len; i += kTileThreads) {
        const uint32_t e = src[i];
        if (check && (e >> d.L) != 0) bad = true;
        atomicAdd(&hist[(e >> shift) & mask], 1u);
    }
    if (bad) atomicExch(d.status, (int32_t)WT_ERANGE);
    __syncthreads();
    uint32_t *H = d.H + (uint64_t)r * nk;
    for (uint32_t k = tid; k < nk; k += kTileThreads) {
        uint32_t s = 0;
#pragma unroll
        for (uint32_t ww = 0; ww < kTileWaves; ww++) s += sh[ww * nk + k];
        H[k] = s;
    }
}

__global__ __launch_bounds__(kTileThreads) void k_hist(const TextDesc *__restrict__ descs,
                                                       const uint32_t *__restrict__ bases,
                                                       uint32_t nd, uint32_t nitems, uint32_t g)
{
    __shared__ uint32_t sh[kTileWaves * (1u << kMaxGroupBits)];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t r = item - item_base(bases, nd, ti);
        if (g >= d.G || r >= d.nranges) continue;
        const uint32_t Kg = group_bits(d, g);
        if (d.b == 1) hist_range<uint8_t>(d, g, Kg, r, sh);
        else if (d.b == 2) hist_range<uint16_t>(d, g, Kg, r, sh);
        else hist_range<uint32_t>(d, g, Kg, r, sh);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K1a: per chunk of ranges, column sums of the range histograms

__global__ __launch_bounds__(256) void k_chunk_sum(const TextDesc *__restrict__ descs,
                                                   const uint32_t *__restrict__ bases, uint32_t nd,
                                                   uint32_t nitems, uint32_t g)
{
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t c = item - item_base(bases, nd, ti);
        if (g >= d.G || c >= d.nchunks) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        const uint32_t nk = 1u << Kg;
        const uint32_t t0 = c * d.CH, t1 = min(d.nranges, t0 + d.CH);
        for (uint32_t k = threadIdx.x; k < nk; k += blockDim.x) {
            uint32_t s = 0;
            for (uint32_t t = t0; t < t1; t++) s += d.H[(uint64_t)t * nk + k];
            d.CS[(uint64_t)c * nk + k] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// K1b: per text, chunk prefixes, key totals of every group level (merged
// upward), key bases in prefix and reversed order, Z, and for a deep WT the
// first row of the interval walk.

__global__ __launch_bounds__(256) void k_key_scan(const TextDesc *__restrict__ descs, uint32_t nd,
                                                  uint32_t g)
{
    const TextDesc &d = descs[blockIdx.x];
    if (g >= d.G) return;
    const uint32_t Kg = group_bits(d, g);
    if (Kg == 0) return;
    const uint32_t nk = 1u << Kg;
    const uint32_t tid = threadIdx.x;
    // chunk prefixes and totals of the deepest group level
    for (uint32_t k = tid; k < nk; k += blockDim.x) {
        uint32_t run = 0;
        for (uint32_t c = 0; c < d.nchunks; c++) {
            uint32_t x = d.CS[(uint64_t)c * nk + k];
            d.CS[(uint64_t)c * nk + k] = run;
            run += x;
        }
        d.HT[lvl_off(Kg) + k] = run;
    }
    __syncthreads();
    // merge upward: totals of every shorter key
    for (uint32_t a = Kg; a-- > 0;) {
        for (uint32_t k = tid; k < (1u << a); k += blockDim.x)
            d.HT[lvl_off(a) + k] = d.HT[lvl_off(a + 1) + 2 * k] + d.HT[lvl_off(a + 1) + 2 * k + 1];
        __syncthreads();
    }
    // key bases per level, one thread per (level, order)
    if (tid < 2 * (Kg + 1)) {
        const uint32_t a = tid >> 1;
        const bool rev = tid & 1;
        const uint32_t *ht = d.HT + lvl_off(a);
        uint32_t *kb = (rev ? d.KBpi : d.KBid) + lvl_off(a);
        uint32_t run = 0;
        for (uint32_t i = 0; i < (1u << a); i++) {
            uint32_t k = rev ? rev_bits(i, a) : i;
            kb[k] = run;
            run += ht[k];
        }
    }
    // Z of the group's levels: zeros of level a = symbols whose next bit is 0,
    // i.e. the even keys one level deeper (Section 5.1)
    if (tid < Kg) {
        const uint32_t a = tid;
        const uint32_t *ht = d.HT + lvl_off(a + 1);
        uint64_t z = 0;
        for (uint32_t k = 0; k < (2u << a); k += 2) z += ht[k];
        d.zeros[g * d.K + a] = z;
    }
    __syncthreads();
    // deep WT: intervals of the K-bit prefixes (level K) seed the walk
    if (d.kind == WT_TREE && d.G > 1 && g == 0) {
        const uint32_t np = 1u << d.K;
        uint32_t *tab = d.walk;  // walk_off(K, K) == 0
        for (uint32_t p = tid; p < np; p += blockDim.x) {
            tab[p] = d.KBpi[lvl_off(Kg) + p];
            tab[np + p] = d.HT[lvl_off(Kg) + p];
            tab[2 * np + p] = d.KBid[lvl_off(Kg) + p];
        }
    }
}

// ---------------------------------------------------------------------------
// K1c: per chunk, range-exclusive prefix of every column

__global__ __launch_bounds__(256) void k_tile_prefix(const TextDesc *__restrict__ descs,
                                                     const uint32_t *__restrict__ bases,
                                                     uint32_t nd, uint32_t nitems, uint32_t g)
{
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t c = item - item_base(bases, nd, ti);
        if (g >= d.G || c >= d.nchunks) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        const uint32_t nk = 1u << Kg;
        const uint32_t t0 = c * d.CH, t1 = min(d.nranges, t0 + d.CH);
        for (uint32_t k = threadIdx.x; k < nk; k += blockDim.x) {
            uint32_t run = d.CS[(uint64_t)c * nk + k];
            for (uint32_t t = t0; t < t1; t++) {
                uint32_t x = d.H[(uint64_t)t * nk + k];
                d.TP[(uint64_t)t * nk + k] = run;
                run += x;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K1d: clear the output words shared between ranges: a range's runs of key k
// start at G (its first tile's interval start); when G is not word-aligned
// the word holding G also holds bits of the previous range (or the previous
// key) and both sides fill it by atomic OR.  Also clears the padding words.

__global__ __launch_bounds__(kTileThreads) void k_zero_borders(const TextDesc *__restrict__ descs,
                                                               const uint32_t *__restrict__ bases,
                                                               uint32_t nd, uint32_t nitems,
                                                               uint32_t g)
{
    __shared__ uint32_t G[kTab];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t r = item - item_base(bases, nd, ti);
        if (g >= d.G || r >= d.nranges) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        range_start_G(d, g, Kg, r, G);
        for (uint32_t e = threadIdx.x; e < lvl_off(Kg); e += kTileThreads) {
            const uint32_t a = 31 - __clz(e + 1);  // level of table entry e
            const uint32_t gs = G[e];
            if ((gs & 63) != 0) level_ptr(d, g, a)[gs >> 6] = 0;
        }
        if (r == 0) {
            // padding words, and the word holding position n (its bits past n
            // must stay zero; the run ending there fills it by atomic OR)
            const uint64_t first = d.n >> 6;
            for (uint32_t a = 0; a < Kg; a++) {
                uint64_t *out = level_ptr(d, g, a);
                for (uint64_t wd = first + threadIdx.x; wd < d.W; wd += kTileThreads) out[wd] = 0;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Deep WT levels (levels >= K when the WT has more than one group).  The WT
// and WM levels hold the same intervals in a different order (Section 5.1).
// Walk: the WM interval of prefix p on level l splits into prefix 2p at
// rank_0 of its ends and 2p+1 at Z + rank_1 (the WM definition, Section 5);
// in the WT both children stay inside the parent's range, 2p first.

__global__ __launch_bounds__(256) void k_walk(const TextDesc *__restrict__ descs,
                                              const uint32_t *__restrict__ bases, uint32_t nd,
                                              uint32_t nitems, uint32_t step)
{
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= nitems) return;
    const uint32_t ti = find_text(bases, nd, item);
    const TextDesc &d = descs[ti];
    const uint32_t p = item - item_base(bases, nd, ti);
    const uint32_t l = d.K + step;
    if (d.kind != WT_TREE || d.G <= 1 || l + 1 >= d.L || p >= (1u << l)) return;
    const uint32_t np = 1u << l;
    const uint32_t *cur = d.walk + walk_off(d.K, l);
    uint32_t *nxt = d.walk + walk_off(d.K, l + 1);
    const uint64_t *bits = d.tmp_bits + (uint64_t)(l - d.K) * d.W;
    const uint32_t *rd = d.tmp_rank + (uint64_t)(l - d.K) * d.rank_stride;
    const uint32_t ms = cur[p], h = cur[np + p], wts = cur[2 * np + p];
    uint32_t r1s = 0, ones = 0;
    if (h) {
        r1s = (uint32_t)rank1_dir(bits, rd, ms);
        ones = (uint32_t)rank1_dir(bits, rd, (uint64_t)ms + h) - r1s;
    }
    const uint32_t z = (uint32_t)d.zeros[l];
    const uint32_t nn = 2 * np;
    nxt[2 * p] = ms - r1s;
    nxt[nn + 2 * p] = h - ones;
    nxt[2 * nn + 2 * p] = wts;
    nxt[2 * p + 1] = z + r1s;
    nxt[nn + 2 * p + 1] = ones;
    nxt[2 * nn + 2 * p + 1] = wts + (h - ones);
}

// Gather: every word of WT level l >= K from the WM level's intervals.
__global__ __launch_bounds__(256) void k_gather(const TextDesc *__restrict__ descs,
                                                const uint32_t *__restrict__ bases, uint32_t nd,
                                                uint32_t nitems)
{
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= nitems) return;
    const uint32_t ti = find_text(bases, nd, item);
    const TextDesc &d = descs[ti];
    const uint64_t idx = item - item_base(bases, nd, ti);
    if (d.kind != WT_TREE || d.G <= 1) return;
    const uint32_t l = d.K + (uint32_t)(idx / d.W);
    const uint64_t w = idx % d.W;
    if (l >= d.L) return;
    uint64_t *out = d.bits + (uint64_t)l * d.W;
    const uint64_t *wm = d.tmp_bits + (uint64_t)(l - d.K) * d.W;
    const uint32_t np = 1u << l;
    const uint32_t *tab = d.walk + walk_off(d.K, l);
    const uint64_t ws = w << 6;
    const uint64_t we = min(ws + 64, d.n);
    uint64_t val = 0;
    uint64_t pos = ws;
    while (pos < we) {
        // largest p with wt_start[p] <= pos: the non-empty interval holding pos
        uint32_t lo = 0, hi = np;
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (tab[2 * np + mid] <= pos) lo = mid;
            else hi = mid;
        }
        const uint64_t ts = tab[2 * np + lo], hh = tab[np + lo], ms = tab[lo];
        uint64_t end = ts + hh;
        if (end > we) end = we;
        if (end <= pos) break;  // cannot happen for consistent tables
        const uint32_t cnt = (uint32_t)(end - pos);
        const uint64_t s = ms + (pos - ts);
        const uint32_t sh = (uint32_t)(s & 63);
        uint64_t x = wm[s >> 6] >> sh;
        if (sh && sh + cnt > 64) x |= wm[(s >> 6) + 1] << (64 - sh);
        if (cnt < 64) x &= (1ull << cnt) - 1;
        val |= x << (pos - ws);
        pos = end;
    }
    out[w] = val;
}

// ---------------------------------------------------------------------------
// host-side launchers

static inline void after(const LaunchCtx &ctx, uint32_t kid)
{
    if (ctx.after) ctx.after(ctx.user, kid);
}

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

static inline uint32_t grid_for(uint32_t nitems, uint32_t cap)
{
    return (cap && nitems > cap) ? cap : nitems;
}

hipError_t launch_init(const TextDesc &d, TextDesc *d_dst, const LaunchCtx &ctx)
{
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, ctx.stream, d, d_dst);
    after(ctx, KID_INIT);
    return hipGetLastError();
}

hipError_t launch_init_batch(const TextDesc *d_descs, uint32_t nd, const LaunchCtx &ctx)
{
    hipLaunchKernelGGL(k_init_batch, dim3(cdiv(nd, 256)), dim3(256), 0, ctx.stream, d_descs, nd);
    after(ctx, KID_INIT);
    return hipGetLastError();
}

hipError_t launch_group(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx)
{
    const uint32_t g = gl.g, nd = gl.nd;
    if (gl.nranges == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist, dim3(grid_for(gl.nranges, gl.grid_cap)), dim3(kTileThreads), 0,
                       ctx.stream, d_descs, gl.range_bases, nd, gl.nranges, g);
    after(ctx, KID_HIST);
    if (!gl.any_levels) return hipGetLastError();
    hipLaunchKernelGGL(k_chunk_sum, dim3(grid_for(gl.nchunks, gl.grid_cap)), dim3(256), 0,
                       ctx.stream, d_descs, gl.chunk_bases, nd, gl.nchunks, g);
    after(ctx, KID_CHUNK_SUM);
    hipLaunchKernelGGL(k_key_scan, dim3(nd), dim3(256), 0, ctx.stream, d_descs, nd, g);
    after(ctx, KID_KEY_SCAN);
    hipLaunchKernelGGL(k_tile_prefix, dim3(grid_for(gl.nchunks, gl.grid_cap)), dim3(256), 0,
                       ctx.stream, d_descs, gl.chunk_bases, nd, gl.nchunks, g);
    after(ctx, KID_TILE_PREFIX);
    hipLaunchKernelGGL(k_zero_borders, dim3(grid_for(gl.nranges, gl.grid_cap)), dim3(kTileThreads),
                       0, ctx.stream, d_descs, gl.range_bases, nd, gl.nranges, g);
    after(ctx, KID_ZERO_BORDERS);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_scatter(d_descs, gl, ctx);
}

hipError_t launch_walk(const TextDesc *d_descs, const uint32_t *bases, uint32_t nd,
                       uint32_t nitems, uint32_t step, const LaunchCtx &ctx)
{
    if (nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk, dim3(cdiv(nitems, 256)), dim3(256), 0, ctx.stream, d_descs, bases,
                       nd, nitems, step);
    after(ctx, KID_WALK);
    return hipGetLastError();
}

hipError_t launch_gather(const TextDesc *d_descs, const uint32_t *bases, uint32_t nd,
                         uint32_t nitems, const LaunchCtx &ctx)
{
    if (nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(cdiv(nitems, 256)), dim3(256), 0, ctx.stream, d_descs,
                       bases, nd, nitems);
    after(ctx, KID_GATHER);
    return hipGetLastError();
}

}  // namespace wtg
