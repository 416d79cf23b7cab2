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
#include "wt_device.h"

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
// K0: per-tile histogram of the group key (and the symbol range check)

template <typename E>
__device__ void hist_tile(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t t, uint32_t *sh)
{
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    const uint32_t nk = 1u << Kg, mask = nk - 1u;
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint64_t S = 1ull << d.log2S;
    const uint64_t start = (uint64_t)t << d.log2S;
    const uint32_t len = (uint32_t)min(S, d.n - start);
    const E *src = (const E *)seq_in(d, g) + start;

    for (uint32_t i = tid; i < kTileWaves * nk; i += kTileThreads) sh[i] = 0;
    __syncthreads();
    bool bad = false;
    const bool check = (g == 0) && (d.L < 32);
    for (uint32_t i = tid; i < len; i += kTileThreads) {
        uint32_t e = src[i];
        if (check && (e >> d.L) != 0) bad = true;
        atomicAdd(&sh[w * nk + ((e >> shift) & mask)], 1u);
    }
    if (bad) atomicExch(d.status, (int32_t)WT_ERANGE);
    __syncthreads();
    uint32_t *H = d.H + (uint64_t)t * nk;
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
        const uint32_t t = item - item_base(bases, nd, ti);
        if (g >= d.G || t >= d.ntiles) continue;
        const uint32_t Kg = group_bits(d, g);
        if (d.b == 1) hist_tile<uint8_t>(d, g, Kg, t, sh);
        else if (d.b == 2) hist_tile<uint16_t>(d, g, Kg, t, sh);
        else hist_tile<uint32_t>(d, g, Kg, t, sh);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K1a: per chunk of tiles, column sums of the tile histograms

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
        const uint32_t t0 = c * d.CH, t1 = min(d.ntiles, t0 + d.CH);
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
// K1c: per chunk, tile-exclusive prefix of every column

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
        const uint32_t t0 = c * d.CH, t1 = min(d.ntiles, t0 + d.CH);
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
// Per-tile tables, shared by border zeroing and the scatter.
//   h[a][k]  symbols of the tile with a-bit group key k (merged upward)
//   G[a][k]  interval start of (key k, this tile) on level a of the group:
//            key base (prefix or reversed order) + tile prefix (merged upward)
//   lo[a][k] start of key k inside the tile's own order after a splits,
//            i.e. keys in reversed order (Observation 2)
//   wb[a][k] first output word of key k's run, counting the words of every
//            run of the tile on level a in key order; words[a] the total

constexpr uint32_t kTab = (2u << kMaxGroupBits);  // >= 2^(K+1) - 1 entries

struct TileTabs {
    uint32_t h[kTab];
    uint32_t G[kTab];
    uint32_t lo[kTab];
    uint32_t wb[kTab];
    uint32_t words[kMaxGroupBits + 1];
};

__device__ inline bool use_prefix_order(const TextDesc &d, uint32_t g, uint32_t a, uint32_t Kg)
{
    // WT output levels of the first group use prefix order; everything else
    // (WM levels, the WT's temporary WM levels, the re-ordering target of the
    // next group) uses reversed order.
    return d.kind == WT_TREE && g == 0 && a < Kg;
}

// exclusive scan of n <= 256 values (4 per lane) by one wave; get(i) / put(i, x)
template <typename Get, typename Put>
__device__ inline uint32_t wave_exscan_256(uint32_t n, Get get, Put put)
{
    const uint32_t lane = lane_id();
    uint32_t v[4];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t r = 0; r < 4; r++) {
        uint32_t i = lane * 4 + r;
        v[r] = (i < n) ? get(i) : 0u;
        s += v[r];
    }
    uint32_t incl = wave_incl_scan(s);
    uint32_t ex = incl - s;
#pragma unroll
    for (uint32_t r = 0; r < 4; r++) {
        uint32_t i = lane * 4 + r;
        if (i < n) put(i, ex);
        ex += v[r];
    }
    return __shfl(incl, 63, 64);
}

__device__ void tile_tables(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t t, TileTabs &tb)
{
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    const uint32_t nk = 1u << Kg;
    const uint32_t *H = d.H + (uint64_t)t * nk;
    const uint32_t *TP = d.TP + (uint64_t)t * nk;
    for (uint32_t k = tid; k < nk; k += kTileThreads) {
        tb.h[lvl_off(Kg) + k] = H[k];
        tb.G[lvl_off(Kg) + k] = TP[k];
    }
    __syncthreads();
    for (uint32_t a = Kg; a-- > 0;) {
        for (uint32_t k = tid; k < (1u << a); k += kTileThreads) {
            tb.h[lvl_off(a) + k] = tb.h[lvl_off(a + 1) + 2 * k] + tb.h[lvl_off(a + 1) + 2 * k + 1];
            tb.G[lvl_off(a) + k] = tb.G[lvl_off(a + 1) + 2 * k] + tb.G[lvl_off(a + 1) + 2 * k + 1];
        }
        __syncthreads();
    }
    for (uint32_t a = 0; a <= Kg; a++) {
        const uint32_t *kb = (use_prefix_order(d, g, a, Kg) ? d.KBid : d.KBpi) + lvl_off(a);
        for (uint32_t k = tid; k < (1u << a); k += kTileThreads) tb.G[lvl_off(a) + k] += kb[k];
    }
    __syncthreads();
    for (uint32_t a = w; a <= Kg; a += kTileWaves) {
        const uint32_t o = lvl_off(a);
        // local starts in reversed key order
        wave_exscan_256(
            1u << a, [&](uint32_t i) { return tb.h[o + rev_bits(i, a)]; },
            [&](uint32_t i, uint32_t x) { tb.lo[o + rev_bits(i, a)] = x; });
        if (a < Kg) {
            uint32_t tot = wave_exscan_256(
                1u << a,
                [&](uint32_t k) {
                    uint32_t hh = tb.h[o + k];
                    if (hh == 0) return 0u;
                    uint64_t gs = tb.G[o + k];
                    return (uint32_t)(((gs + hh - 1) >> 6) - (gs >> 6) + 1);
                },
                [&](uint32_t k, uint32_t x) { tb.wb[o + k] = x; });
            if (lane_id() == 0) tb.words[a] = tot;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// K1d: clear every output word that some run of this tile covers only in
// part (it is shared with other runs and is filled by atomic OR), and the
// padding words of every level of the group.

__global__ __launch_bounds__(kTileThreads) void k_zero_borders(const TextDesc *__restrict__ descs,
                                                               const uint32_t *__restrict__ bases,
                                                               uint32_t nd, uint32_t nitems,
                                                               uint32_t g)
{
    __shared__ TileTabs tb;
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t t = item - item_base(bases, nd, ti);
        if (g >= d.G || t >= d.ntiles) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        tile_tables(d, g, Kg, t, tb);
        for (uint32_t a = 0; a < Kg; a++) {
            uint64_t *out = level_ptr(d, g, a);
            const uint32_t o = lvl_off(a);
            for (uint32_t k = threadIdx.x; k < (1u << a); k += kTileThreads) {
                const uint64_t hh = tb.h[o + k];
                if (hh == 0) continue;
                const uint64_t gs = tb.G[o + k], ge = gs + hh;
                const uint64_t fw = gs >> 6, lw = (ge - 1) >> 6;
                const bool first_full = ((gs & 63) == 0) && (hh >= 64);
                if (!first_full) out[fw] = 0;
                if ((ge & 63) != 0) out[lw] = 0;
            }
            if (t == 0) {
                const uint64_t used = (d.n + 63) >> 6;
                for (uint64_t wd = used + threadIdx.x; wd < d.W; wd += kTileThreads) out[wd] = 0;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K2: the stable scatter of a tile into every level of the group

struct ScatterSmem {
    uint8_t buf[2][kTileBufBytes];
    uint64_t bitbuf[kTileBufBytes / 64 + 1];
    TileTabs tb;
    uint32_t wz[kTileWaves], wv[kTileWaves];
};

// copy the tile's level-a runs from bitbuf to their interval starts
__device__ inline void copy_runs(const TextDesc &d, uint32_t g, uint32_t a, ScatterSmem &sm)
{
    const uint32_t o = lvl_off(a), nk = 1u << a;
    const uint32_t words = sm.tb.words[a];
    uint64_t *out = level_ptr(d, g, a);
    for (uint32_t q = threadIdx.x; q < words; q += kTileThreads) {
        uint32_t lo = 0, hi = nk;  // largest key whose first word index <= q
        while (hi - lo > 1) {
            uint32_t mid = (lo + hi) >> 1;
            if (sm.tb.wb[o + mid] <= q) lo = mid;
            else hi = mid;
        }
        const uint32_t k = lo;
        const uint64_t gs = sm.tb.G[o + k], hh = sm.tb.h[o + k];
        const uint64_t gw = (gs >> 6) + (q - sm.tb.wb[o + k]);
        const uint64_t ws = gw << 6;
        const uint64_t b0 = gs > ws ? gs : ws;
        const uint64_t b1 = (gs + hh) < ws + 64 ? (gs + hh) : ws + 64;
        const uint32_t cnt = (uint32_t)(b1 - b0);
        const uint32_t src = sm.tb.lo[o + k] + (uint32_t)(b0 - gs);
        const uint32_t sh = src & 63;
        uint64_t val = sm.bitbuf[src >> 6] >> sh;
        if (sh) val |= sm.bitbuf[(src >> 6) + 1] << (64 - sh);
        if (cnt < 64) val &= (1ull << cnt) - 1;
        val <<= (b0 & 63);
        if (cnt == 64) out[gw] = val;
        else atomicOr((unsigned long long *)&out[gw], (unsigned long long)val);
    }
}

template <typename E>
__device__ void scatter_tile(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t t, ScatterSmem &sm)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t S = 1ull << d.log2S;
    const uint64_t start = (uint64_t)t << d.log2S;
    const uint32_t len = (uint32_t)min(S, d.n - start);
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint32_t kmask = (1u << Kg) - 1u;
    const bool reorder = (g + 1 < d.G);
    const E *src = (const E *)seq_in(d, g) + start;
    E *cur = (E *)sm.buf[0];
    E *nxt = (E *)sm.buf[1];

    for (uint32_t i = tid; i < len; i += kTileThreads) cur[i] = src[i];
    if (tid == 0) sm.bitbuf[S >> 6] = 0;
    tile_tables(d, g, Kg, t, sm.tb);  // ends with a barrier

    const uint32_t nch = (len + 63) >> 6;
    const uint32_t cpw = (nch + kTileWaves - 1) / kTileWaves;
    const uint32_t c0 = min(w * cpw, nch), c1 = min(c0 + cpw, nch);

    for (uint32_t a = 0; a < Kg; a++) {
        const uint32_t bsh = shift + Kg - 1 - a;  // bit (g*K + a) of the symbol
        // pass A: this level's bits in the current order, and zero counts
        uint32_t zc = 0, vc = 0;
        for (uint32_t c = c0; c < c1; c++) {
            const uint32_t i = c * 64 + lane;
            const bool valid = i < len;
            const uint32_t e = valid ? (uint32_t)cur[i] : 0u;
            const uint64_t B = __ballot(valid && ((e >> bsh) & 1u));
            const uint64_t V = __ballot(valid);
            if (lane == 0) sm.bitbuf[c] = B;
            zc += __popcll(V & ~B);
            vc += __popcll(V);
        }
        if (lane == 0) {
            sm.wz[w] = zc;
            sm.wv[w] = vc;
        }
        __syncthreads();
        uint32_t base0 = 0, base1 = 0;
        for (uint32_t ww = 0; ww < kTileWaves; ww++) {
            base1 += sm.wz[ww];
            if (ww < w) {
                base0 += sm.wz[ww];
                base1 += sm.wv[ww] - sm.wz[ww];
            }
        }
        // level a runs -> global
        copy_runs(d, g, a, sm);
        // pass B: stable split by bit a (zeros first) into the next order, or,
        // after the group's last bit, straight into the next group's sequence
        const bool last = (a + 1 == Kg);
        if (!last || reorder) {
            E *gout = (E *)seq_out(d, g);
            const uint32_t ok = lvl_off(Kg);
            for (uint32_t c = c0; c < c1; c++) {
                const uint32_t i = c * 64 + lane;
                const bool valid = i < len;
                const uint32_t e = valid ? (uint32_t)cur[i] : 0u;
                const uint32_t bv = (e >> bsh) & 1u;
                const uint64_t B = __ballot(valid && bv);
                const uint64_t V = __ballot(valid);
                const uint32_t r1 = mbcnt64(B);
                const uint32_t dst = bv ? base1 + r1 : base0 + (lane - r1);
                if (valid) {
                    if (!last) {
                        nxt[dst] = (E)e;
                    } else {
                        const uint32_t v = (e >> shift) & kmask;
                        gout[sm.tb.G[ok + v] + (dst - sm.tb.lo[ok + v])] = (E)e;
                    }
                }
                base0 += __popcll(V & ~B);
                base1 += __popcll(B);
            }
        }
        __syncthreads();
        E *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
}

__global__ __launch_bounds__(kTileThreads) void k_scatter(const TextDesc *__restrict__ descs,
                                                          const uint32_t *__restrict__ bases,
                                                          uint32_t nd, uint32_t nitems, uint32_t g)
{
    __shared__ ScatterSmem sm;
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t t = item - item_base(bases, nd, ti);
        if (g >= d.G || t >= d.ntiles) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        if (d.b == 1) scatter_tile<uint8_t>(d, g, Kg, t, sm);
        else if (d.b == 2) scatter_tile<uint16_t>(d, g, Kg, t, sm);
        else scatter_tile<uint32_t>(d, g, Kg, t, sm);
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
    if (gl.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist, dim3(grid_for(gl.ntiles, gl.grid_cap)), dim3(kTileThreads), 0,
                       ctx.stream, d_descs, gl.tile_bases, nd, gl.ntiles, g);
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
    hipLaunchKernelGGL(k_zero_borders, dim3(grid_for(gl.ntiles, gl.grid_cap)), dim3(kTileThreads),
                       0, ctx.stream, d_descs, gl.tile_bases, nd, gl.ntiles, g);
    after(ctx, KID_ZERO_BORDERS);
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(gl.ntiles, gl.grid_cap)), dim3(kTileThreads), 0,
                       ctx.stream, d_descs, gl.tile_bases, nd, gl.ntiles, g);
    after(ctx, KID_SCATTER);
    return hipGetLastError();
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
