// K2: the stable scatter of a range of tiles into every level of a group.
//
// Algorithm 1 places bit l of every symbol at the next free slot of its
// interval, scanning the text in order, so inside an interval the bits are in
// text order.  Here every wave owns one range of consecutive tiles and walks
// it tile by tile, with no barrier shared with other waves.  A tile (at most
// kWaveTile symbols) sits in the wave's registers, 64 symbols per chunk; it is
// ordered one bit at a time: after splitting by bits 0..a-1 of the group key
// (zeros first, stably) the tile is ordered by its reversed a-bit key
// (Observation 2), so level a's bits of every key form one contiguous run.
// The ballot of bit a that drives the split of order a is, chunk by chunk,
// level a of the tile in that order.  The split offsets come from the tile's
// key counts (one LDS histogram, merged upward), not from a counting pass.
// Each run is then copied to its interval start on the level (prefix order
// for the WT, bit-reversed order for the WM; Section 5.1).  Consecutive tiles
// put a key's runs next to each other, so the word a run ends in is kept in
// LDS and completed by the next tile's run of that key; only words shared
// with another range are filled by atomic OR.  With more than one group, the
// split by the group's last bit writes every symbol straight to its position
// in the next group's sequence.
#include "wt_tiles.h"

namespace wtg {

constexpr uint32_t kChunks = kWaveTile / 64;              // chunks of 64 symbols per tile
constexpr uint32_t kRuns = (1u << kMaxGroupBits) - 1;      // (level, key) pairs of levels 0..K-1
constexpr uint32_t kKeyTab = (2u << kMaxGroupBits) - 1;    // (level, key) pairs of levels 0..K
// full output words of one tile over all levels (<= kChunks per level), and
// the finest key prefix sums (2^K + 1 entries) that share their array
constexpr uint32_t kMaxWords = (kMaxGroupBits * kChunks > (1u << kMaxGroupBits) + 1)
                                   ? kMaxGroupBits * kChunks : (1u << kMaxGroupBits) + 1;
constexpr uint32_t kNoPend = 0xFFFFFFFFu;
constexpr uint32_t kForeignLow = 0x80000000u;  // pending word's low bits belong to another range

// One wave's LDS.  Tables are indexed lvl_off(a) + key for level a.
template <typename E>
struct WaveSmem {
    uint64_t bits[kMaxGroupBits][kChunks];  // level a of the tile, in order a
    uint64_t pend_v[kRuns];                 // bits so far of the word a key's run ends in
    uint32_t h[kKeyTab];                    // the tile's count of every key
    uint32_t G[kKeyTab];                    // global start of the key's bits for this tile
    uint32_t pend_w[kRuns];                 // that word's index (kNoPend: none)
    uint16_t lo[kKeyTab];                   // start of the key in the tile order of its level
    uint16_t wb[kRuns];                     // first full word of every run, all levels
    uint16_t kw[kMaxWords];                 // run of every full word (also a scratch scan)
    E elem[kWaveTile];                      // the tile, in its next order
};

// orders the wave's LDS accesses (the wave runs in lockstep; no s_barrier)
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive prefix maximum over the 64 lanes of a wave
__device__ inline uint32_t wave_incl_max(uint32_t x)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x = max(x, y);
    }
    return x;
}

// exclusive scan of n <= 64 PER values by one wave, PER consecutive values
// per lane; get(i) / put(i, x); returns the total
template <uint32_t PER, typename Get, typename Put>
__device__ inline uint32_t wave_exscan_n(uint32_t n, Get get, Put put)
{
    const uint32_t lane = lane_id();
    uint32_t v[PER];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t r = 0; r < PER; r++) {
        const uint32_t i = lane * PER + r;
        v[r] = (i < n) ? get(i) : 0u;
        s += v[r];
    }
    const uint32_t incl = wave_incl_scan(s);
    uint32_t ex = incl - s;
#pragma unroll
    for (uint32_t r = 0; r < PER; r++) {
        const uint32_t i = lane * PER + r;
        if (i < n) put(i, ex);
        ex += v[r];
    }
    return __shfl(incl, 63, 64);
}

// level of table entry e (entries lvl_off(a) .. lvl_off(a+1)-1 are level a)
__device__ inline uint32_t level_of(uint32_t e) { return 31 - __clz(e + 1); }

// cnt (<= 64) bits of level a starting at tile-order bit s
__device__ inline uint64_t stream_bits(const uint64_t *src, uint32_t s, uint32_t cnt)
{
    const uint32_t sh = s & 63;
    uint64_t x = src[s >> 6] >> sh;
    if (sh + cnt > 64) x |= src[(s >> 6) + 1] << (64 - sh);
    if (cnt < 64) x &= (1ull << cnt) - 1;
    return x;
}

// acc_lo/acc_hi of lane c := the 64-bit wave-uniform value B
__device__ inline void put_lane(uint32_t &acc_lo, uint32_t &acc_hi, uint64_t B, uint32_t c)
{
    asm volatile("s_mov_b32 m0, %2\n\tv_writelane_b32 %0, %1, m0"
                 : "+v"(acc_lo)
                 : "s"((uint32_t)B), "s"(c)
                 : "m0");
    asm volatile("s_mov_b32 m0, %2\n\tv_writelane_b32 %0, %1, m0"
                 : "+v"(acc_hi)
                 : "s"((uint32_t)(B >> 32)), "s"(c)
                 : "m0");
}

// G at the first tile of range r: the range prefix of every finest key merged
// upward, plus the key bases of each level.
__device__ inline void wave_range_start(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r,
                                        uint32_t *G)
{
    const uint32_t lane = lane_id();
    const uint32_t nk = 1u << Kg;
    const uint32_t *TP = d.TP + (uint64_t)r * nk;
    for (uint32_t k = lane; k < nk; k += 64) G[lvl_off(Kg) + k] = TP[k];
    wave_sync();
    for (uint32_t a = Kg; a-- > 0;) {
        for (uint32_t k = lane; k < (1u << a); k += 64)
            G[lvl_off(a) + k] = G[lvl_off(a + 1) + 2 * k] + G[lvl_off(a + 1) + 2 * k + 1];
        wave_sync();
    }
    for (uint32_t a = 0; a <= Kg; a++) {
        const uint32_t *kb = (use_prefix_order(d, g, a, Kg) ? d.KBid : d.KBpi) + lvl_off(a);
        for (uint32_t k = lane; k < (1u << a); k += 64) G[lvl_off(a) + k] += kb[k];
    }
    wave_sync();
}

// full words of run e: [ceil(G/64), floor((G+h)/64))
__device__ inline uint32_t full_words(uint32_t gs, uint32_t hh)
{
    const uint32_t f = (gs + 63) >> 6, l = (uint32_t)(((uint64_t)gs + hh) >> 6);
    return l > f ? l - f : 0u;
}

// Words that a run of this tile covers completely, all levels at once, by
// plain stores: the full words of all runs are numbered run by run, and the
// lanes take consecutive words.
template <typename E>
__device__ void copy_full_words(const TextDesc &d, uint32_t g, uint32_t Kg, WaveSmem<E> &sm)
{
    const uint32_t lane = lane_id();
    const uint32_t nr = lvl_off(Kg);
    const uint32_t total = wave_exscan_n<4>(
        nr, [&](uint32_t e) { return full_words(sm.G[e], sm.h[e]); },
        [&](uint32_t e, uint32_t x) { sm.wb[e] = (uint16_t)x; });
    // run of every word: the run whose first word it is, carried forward
    for (uint32_t q = lane; q < total; q += 64) sm.kw[q] = 0;
    wave_sync();
    for (uint32_t e = lane; e < nr; e += 64)
        if (full_words(sm.G[e], sm.h[e]) != 0) sm.kw[sm.wb[e]] = (uint16_t)e;
    wave_sync();
    constexpr uint32_t PER = (kMaxGroupBits * kChunks + 63) / 64;
    uint32_t m = 0;
#pragma unroll
    for (uint32_t i = 0; i < PER; i++) {
        const uint32_t q = lane * PER + i;
        if (q < total) m = max(m, (uint32_t)sm.kw[q]);
    }
    uint32_t run = __shfl_up(wave_incl_max(m), 1, 64);
    if (lane == 0) run = 0;
#pragma unroll
    for (uint32_t i = 0; i < PER; i++) {
        const uint32_t q = lane * PER + i;
        if (q < total) {
            run = max(run, (uint32_t)sm.kw[q]);
            sm.kw[q] = (uint16_t)run;
        }
    }
    wave_sync();
    for (uint32_t q = lane; q < total; q += 64) {
        const uint32_t e = sm.kw[q], a = level_of(e);
        const uint32_t gs = sm.G[e];
        const uint64_t gw = ((gs + 63) >> 6) + (q - sm.wb[e]);
        if (gw < d.W)
            level_ptr(d, g, a)[gw] =
                stream_bits(sm.bits[a], sm.lo[e] + (uint32_t)((gw << 6) - gs), 64);
    }
    wave_sync();
}

// First and last word of every run (one lane per run, all levels): merged
// with the word kept from earlier tiles of the range, stored when complete,
// kept otherwise.
template <typename E>
__device__ void run_end_words(const TextDesc &d, uint32_t g, uint32_t Kg, WaveSmem<E> &sm)
{
    for (uint32_t e = lane_id(); e < lvl_off(Kg); e += 64) {
        const uint32_t hh = sm.h[e];
        if (hh == 0) continue;
        const uint32_t a = 31 - __clz(e + 1);
        uint64_t *out = level_ptr(d, g, a);
        const uint64_t *src = sm.bits[a];
        const uint32_t ls = sm.lo[e];
        const uint64_t gs = sm.G[e], ge = gs + hh;
        const uint64_t fw = gs >> 6, lw = (ge - 1) >> 6;
        uint32_t newp = kNoPend;
        uint64_t newv = 0;
        if ((gs & 63) != 0 || hh < 64) {
            const uint64_t b1 = ge < ((fw + 1) << 6) ? ge : ((fw + 1) << 6);
            uint64_t val = stream_bits(src, ls, (uint32_t)(b1 - gs)) << (gs & 63);
            bool lowok = (gs & 63) == 0;
            const uint32_t pw = sm.pend_w[e];
            if (!lowok && pw != kNoPend && (pw & ~kForeignLow) == fw) {
                val |= sm.pend_v[e];
                lowok = (pw & kForeignLow) == 0;
            }
            if (b1 == ((fw + 1) << 6)) {
                if (fw >= d.W) continue;  // never for consistent tables
                if (lowok) out[fw] = val;
                else atomicOr((unsigned long long *)&out[fw], (unsigned long long)val);
            } else {
                newp = (uint32_t)fw | (lowok ? 0u : kForeignLow);
                newv = val;
            }
        }
        if (lw != fw && (ge & 63) != 0 && lw < d.W) {
            newp = (uint32_t)lw;
            newv = stream_bits(src, ls + (uint32_t)((lw << 6) - gs), (uint32_t)(ge - (lw << 6)));
        }
        sm.pend_w[e] = newp;
        sm.pend_v[e] = newv;
    }
}

// One split (or, MODE 2, only the ballots) of the tile by bit `bit`: the
// ballots are level a in the current order; MODE 0 writes every symbol to
// its place in the next order in LDS, MODE 1 to its place in the next
// group's sequence (global).
template <typename E, uint32_t NCH, bool FULL, int MODE>
__device__ inline void split_pass(const TextDesc &d, uint32_t (&v)[NCH], uint32_t len, uint32_t a,
                                  uint32_t bit, uint32_t shift, uint32_t Kg, E *gout,
                                  WaveSmem<E> &sm)
{
    const uint32_t lane = lane_id();
    const uint32_t nch = FULL ? NCH : (len + 63) >> 6;
    const uint32_t kmask = (1u << Kg) - 1u;
    uint32_t acc_lo = 0, acc_hi = 0;
    // the zeros of level a in the tile: the start of the first key whose bit
    // a is one, in the order of level a + 1
    uint32_t base0 = 0;
    uint32_t base1 = MODE == 2 ? 0u : __builtin_amdgcn_readfirstlane((uint32_t)sm.lo[lvl_off(a + 1) + 1]);
#pragma unroll
    for (uint32_t c = 0; c < NCH; c++) {
        if (FULL || c < nch) {
            const bool ok = FULL || c * 64 + lane < len;
            const uint32_t x = v[c];
            const bool one = ok && (x & bit) != 0;
            const uint64_t B = __ballot(one);
            put_lane(acc_lo, acc_hi, B, c);
            if (MODE != 2) {
                const uint32_t d1 = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, base1));
                const uint32_t d0 = (base0 + base1) + lane - d1;
                const uint32_t dst = one ? d1 : d0;
                if (ok) {
                    if (MODE == 0) {
                        sm.elem[dst] = (E)x;
                    } else {
                        const uint32_t key = (x >> shift) & kmask;
                        const uint32_t gi = sm.G[lvl_off(Kg) + key] + (dst - sm.lo[lvl_off(Kg) + key]);
                        if (gi < d.n) gout[gi] = (E)x;
                    }
                }
                const uint32_t ones = __popcll(B);
                base0 += (FULL ? 64u : min(64u, len - c * 64)) - ones;
                base1 += ones;
            }
        }
    }
    if (lane < nch) sm.bits[a][lane] = ((uint64_t)acc_hi << 32) | acc_lo;
}

// One tile of NCH chunks.  FULL: the tile holds exactly 64 NCH symbols
// (every tile but possibly the text's last one); otherwise the chunks past
// the text's end are masked lane by lane.
template <typename E, uint32_t NCH, bool FULL>
__device__ void wave_tile(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t t, WaveSmem<E> &sm)
{
    const uint32_t lane = lane_id();
    const uint64_t start = (uint64_t)t << d.log2S;
    const uint32_t len = FULL ? NCH * 64 : (uint32_t)(d.n - start);
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint32_t nk = 1u << Kg, kmask = nk - 1u;
    const bool reorder = (g + 1 < d.G);
    const E *src = (const E *)seq_in(d, g) + start + lane;
    uint32_t *h = sm.h;
    // lane holds a symbol of chunk c
    auto valid = [&](uint32_t c) { return FULL || c * 64 + lane < len; };

    // 1. the tile into registers: chunk c, lane l holds symbol 64 c + l
    uint32_t v[NCH];
#pragma unroll
    for (uint32_t c = 0; c < NCH; c++) v[c] = valid(c) ? (uint32_t)src[c * 64] : 0u;

    // 2. the tile's count of every key: the finest level by LDS atomics, the
    //    others as differences of the finest prefix sums P
    for (uint32_t k = lane; k < nk; k += 64) h[lvl_off(Kg) + k] = 0;
    wave_sync();
#pragma unroll
    for (uint32_t c = 0; c < NCH; c++)
        if (valid(c)) atomicAdd(&h[lvl_off(Kg) + ((v[c] >> shift) & kmask)], 1u);
    wave_sync();
    uint16_t *P = sm.kw;
    wave_exscan_n<4>(
        nk, [&](uint32_t k) { return h[lvl_off(Kg) + k]; },
        [&](uint32_t k, uint32_t x) { P[k] = (uint16_t)x; });
    if (lane == 0) P[nk] = (uint16_t)len;
    wave_sync();
    for (uint32_t e = lane; e < lvl_off(Kg); e += 64) {
        const uint32_t a = level_of(e), k = e - lvl_off(a), sh = Kg - a;
        h[e] = (uint32_t)P[(k + 1) << sh] - (uint32_t)P[k << sh];
    }
    wave_sync();
    // 3. start of every key in the tile order of its level (keys in reversed
    //    order): one scan over the levels one after the other, each of which
    //    adds len; level Kg only when the symbols move on to the next group
    const uint32_t lmax = reorder ? Kg : Kg - 1;
    wave_exscan_n<8>(
        lvl_off(lmax + 1),
        [&](uint32_t i) {
            const uint32_t a = level_of(i);
            return h[lvl_off(a) + rev_bits(i - lvl_off(a), a)];
        },
        [&](uint32_t i, uint32_t x) {
            const uint32_t a = level_of(i);
            sm.lo[lvl_off(a) + rev_bits(i - lvl_off(a), a)] = (uint16_t)(x - a * len);
        });
    wave_sync();

    // 4. split by one bit at a time; the ballots are the levels
    E *gout = (E *)seq_out(d, g);
    for (uint32_t a = 0; a + 1 < Kg; a++) {
        split_pass<E, NCH, FULL, 0>(d, v, len, a, 1u << (shift + Kg - 1 - a), shift, Kg, gout, sm);
        wave_sync();
#pragma unroll
        for (uint32_t c = 0; c < NCH; c++)
            if (valid(c)) v[c] = sm.elem[c * 64 + lane];
        wave_sync();
    }
    if (reorder) split_pass<E, NCH, FULL, 1>(d, v, len, Kg - 1, 1u << shift, shift, Kg, gout, sm);
    else split_pass<E, NCH, FULL, 2>(d, v, len, Kg - 1, 1u << shift, shift, Kg, gout, sm);
    wave_sync();

    // 5. every level's runs to their interval starts
    copy_full_words(d, g, Kg, sm);
    run_end_words(d, g, Kg, sm);
    wave_sync();
    // the next tile's runs start where this tile's end
    for (uint32_t e = lane; e < lvl_off(Kg + 1); e += 64) sm.G[e] += h[e];
    wave_sync();
}

template <typename E>
__device__ void wave_range(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r, WaveSmem<E> &sm)
{
    const uint32_t lane = lane_id();
    wave_range_start(d, g, Kg, r, sm.G);
    for (uint32_t e = lane; e < kRuns; e += 64) sm.pend_w[e] = kNoPend;
    wave_sync();
    const uint32_t t0 = r * d.R, t1 = min(d.ntiles, t0 + d.R);
    for (uint32_t t = t0; t < t1; t++) {
        if (((uint64_t)(t + 1) << d.log2S) > d.n) wave_tile<E, kChunks, false>(d, g, Kg, t, sm);
        else if (d.log2S == 11) wave_tile<E, 32, true>(d, g, Kg, t, sm);
        else wave_tile<E, 16, true>(d, g, Kg, t, sm);
    }
    // words still open at the end of the range are shared with the next one
    for (uint32_t e = lane; e < lvl_off(Kg); e += 64) {
        const uint32_t pw = sm.pend_w[e];
        if (pw == kNoPend) continue;
        const uint32_t a = 31 - __clz(e + 1);
        if ((pw & ~kForeignLow) < d.W)
            atomicOr((unsigned long long *)&level_ptr(d, g, a)[pw & ~kForeignLow],
                     (unsigned long long)sm.pend_v[e]);
    }
    wave_sync();
}

// Work item = (text, range); wave w of workgroup b takes items
// b * kScatWaves + w, then strides by the whole grid.
template <typename E>
__global__ __launch_bounds__(kScatWaves * 64) void k_scatter(const TextDesc *__restrict__ descs,
                                                             const uint32_t *__restrict__ bases,
                                                             uint32_t nd, uint32_t nitems, uint32_t g)
{
    __shared__ WaveSmem<E> sm[kScatWaves];
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t item = blockIdx.x * kScatWaves + w; item < nitems;
         item += gridDim.x * kScatWaves) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t r = item - item_base(bases, nd, ti);
        if (d.b != sizeof(E) || g >= d.G || r >= d.nranges) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        wave_range<E>(d, g, Kg, r, sm[w]);
    }
}

hipError_t launch_scatter(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx)
{
    uint32_t grid = (gl.nranges + kScatWaves - 1) / kScatWaves;
    if (gl.grid_cap && grid > gl.grid_cap) grid = gl.grid_cap;
    const dim3 block(kScatWaves * 64);
    if (gl.bmask & 1u)
        hipLaunchKernelGGL(k_scatter<uint8_t>, dim3(grid), block, 0, ctx.stream, d_descs,
                           gl.range_bases, gl.nd, gl.nranges, gl.g);
    if (gl.bmask & 2u)
        hipLaunchKernelGGL(k_scatter<uint16_t>, dim3(grid), block, 0, ctx.stream, d_descs,
                           gl.range_bases, gl.nd, gl.nranges, gl.g);
    if (gl.bmask & 4u)
        hipLaunchKernelGGL(k_scatter<uint32_t>, dim3(grid), block, 0, ctx.stream, d_descs,
                           gl.range_bases, gl.nd, gl.nranges, gl.g);
    if (ctx.after) ctx.after(ctx.user, KID_SCATTER);
    return hipGetLastError();
}

}  // namespace wtg
