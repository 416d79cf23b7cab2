// K2: the stable scatter of a range of tiles into every level of a group.
//
// Algorithm 1 places bit l of every symbol at the next free slot of its
// interval, scanning the text in order, so inside an interval the bits are in
// text order.  Here one workgroup walks a range of consecutive tiles and
// orders each tile in LDS one bit at a time: after splitting by bits 0..a-1 of
// the group key (zeros first, stably) the tile is ordered by its reversed
// a-bit key (Observation 2), so level a's bits of every key form one
// contiguous run, and the ballots of bit a in that order are level a of the
// tile.  The waves hold consecutive parts of the current order in registers;
// per split they exchange their zero counts, write every symbol to its place
// in the next order and read their part back.  Each run is then copied to its
// interval start on the level (prefix order for the WT, bit-reversed order for
// the WM; Section 5.1).  Consecutive tiles put a key's runs next to each
// other, so the word a run ends in is kept in LDS and completed by the next
// tile's run of that key; only words shared with another range are filled by
// atomic OR.  With more than one group, the split by the group's last bit
// writes every symbol straight to its position in the next group's sequence.
#include "wt_tiles.h"

namespace wtg {

constexpr uint32_t kScatBufBytes = kTileBufBytes;
constexpr uint32_t kBitWords = kScatBufBytes / 64;  // bit words per level (1-byte symbols)
constexpr uint32_t kNoPend = 0xFFFFFFFFu;
constexpr uint32_t kForeignLow = 0x80000000u;  // pending word's low bits belong to another range

struct ScatSmem {
    uint8_t elem[kScatBufBytes];                    // the tile, in its current order
    uint64_t bits[kMaxGroupBits][kBitWords];        // level a of the tile, in order a
    uint32_t hist[kTileWaves][1u << kMaxGroupBits]; // per-wave key counts while loading
    TileTabs tb;
    uint32_t pend_w[kTab];  // word a key's coverage ends in (kNoPend: none)
    uint64_t pend_v[kTab];  // its bits so far
    uint32_t zc[kTileWaves];
};

// cnt (<= 64) bits of level a starting at tile-order bit s
__device__ inline uint64_t stream_bits(const uint64_t *src, uint32_t s, uint32_t cnt)
{
    const uint32_t sh = s & 63;
    uint64_t x = src[s >> 6] >> sh;
    if (sh + cnt > 64) x |= src[(s >> 6) + 1] << (64 - sh);
    if (cnt < 64) x &= (1ull << cnt) - 1;
    return x;
}

// largest key k < nk with wb[k] <= q (wb non-decreasing, wb[0] = 0): a
// 16-way probe, then a search inside the chosen segment
__device__ inline uint32_t key_of_word(const uint32_t *wb, uint32_t nk, uint32_t q)
{
    if (nk <= 16) {
        uint32_t k = 0;
#pragma unroll
        for (uint32_t i = 1; i < 16; i++)
            if (i < nk && wb[i] <= q) k = i;
        return k;
    }
    const uint32_t step = nk >> 4;
    uint32_t seg = 0;
#pragma unroll
    for (uint32_t i = 1; i < 16; i++)
        if (wb[i * step] <= q) seg = i;
    uint32_t k = seg * step;
    for (uint32_t i = 1; i < step; i++)
        if (wb[seg * step + i] <= q) k = seg * step + i;
    return k;
}

// words of level a that a run of this tile covers completely: plain stores
__device__ inline void copy_full_words(const TextDesc &d, uint32_t g, uint32_t a, const ScatSmem &sm)
{
    const uint32_t o = lvl_off(a), nk = 1u << a;
    const uint32_t words = sm.tb.words[a];
    uint64_t *out = level_ptr(d, g, a);
    const uint64_t *src = sm.bits[a];
    for (uint32_t q = threadIdx.x; q < words; q += kTileThreads) {
        const uint32_t e = o + key_of_word(sm.tb.wb + o, nk, q);
        const uint64_t gs = sm.tb.G[e], hh = sm.tb.h[e];
        const uint64_t gw = (gs >> 6) + (q - sm.tb.wb[e]);
        const uint64_t ws = gw << 6;
        if (gs <= ws && gs + hh >= ws + 64 && gw < d.W)
            out[gw] = stream_bits(src, sm.tb.lo[e] + (uint32_t)(ws - gs), 64);
    }
}

// first and last word of every run (one thread per run, all levels): merged
// with the word kept from earlier tiles of the range, stored when complete,
// kept otherwise
__device__ inline void run_end_words(const TextDesc &d, uint32_t g, uint32_t Kg, ScatSmem &sm)
{
    for (uint32_t e = threadIdx.x; e < lvl_off(Kg); e += kTileThreads) {
        const uint32_t hh = sm.tb.h[e];
        if (hh == 0) continue;
        const uint32_t a = 31 - __clz(e + 1);
        uint64_t *out = level_ptr(d, g, a);
        const uint64_t *src = sm.bits[a];
        const uint32_t ls = sm.tb.lo[e];
        const uint64_t gs = sm.tb.G[e], ge = gs + hh;
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

// FULL: the tile is complete, so every wave holds SW / 64 full chunks (every
// tile but possibly the text's last one) and the chunk loops test only the
// uniform chunk count.
template <typename E, uint32_t NCH, bool FULL>
__device__ void scatter_tile(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t t, ScatSmem &sm)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index: uniform
    const uint32_t S = 1u << d.log2S;
    const uint32_t SW = S / kTileWaves;  // positions per wave (<= 64 * NCH)
    const uint32_t RW = SW >> 6;         // chunks per wave
    const uint64_t start = (uint64_t)t << d.log2S;
    const uint32_t len = (uint32_t)min((uint64_t)S, d.n - start);
    const uint32_t wbeg = w * SW;
    const uint32_t wlen = FULL ? SW : (len > wbeg ? min(len - wbeg, SW) : 0u);
    const uint32_t nch = FULL ? (SW >> 6) : (wlen + 63) >> 6;  // chunks held (<= NCH)
    const uint32_t nfull = FULL ? (SW >> 6) : wlen >> 6;       // of which full
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint32_t nk = 1u << Kg, kmask = nk - 1u;
    const bool reorder = (g + 1 < d.G);
    const E *src = (const E *)seq_in(d, g) + start + wbeg;
    E *elem = (E *)sm.elem;

    // 1. the wave's part into registers (all loads in flight at once); key
    //    counts per wave
    uint32_t v[NCH];
#pragma unroll
    for (uint32_t c = 0; c < NCH; c++)
        v[c] = (FULL ? c < nch : c * 64 + lane < wlen) ? (uint32_t)src[c * 64 + lane] : 0u;
    uint32_t *hs = sm.hist[w];
    for (uint32_t k = lane; k < nk; k += 64) hs[k] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (uint32_t c = 0; c < NCH; c++)
        if (FULL ? c < nch : c * 64 + lane < wlen) atomicAdd(&hs[(v[c] >> shift) & kmask], 1u);
    __syncthreads();

    // 2. tile tables: counts merged upward, starts in reversed key order, words
    //    of every run
    for (uint32_t k = tid; k < nk; k += kTileThreads) {
        uint32_t s = 0;
#pragma unroll
        for (uint32_t ww = 0; ww < kTileWaves; ww++) s += sm.hist[ww][k];
        sm.tb.h[lvl_off(Kg) + k] = s;
    }
    __syncthreads();
    for (uint32_t a = Kg; a-- > 0;) {
        for (uint32_t k = tid; k < (1u << a); k += kTileThreads)
            sm.tb.h[lvl_off(a) + k] = sm.tb.h[lvl_off(a + 1) + 2 * k] + sm.tb.h[lvl_off(a + 1) + 2 * k + 1];
        __syncthreads();
    }
    for (uint32_t a = w; a <= Kg; a += kTileWaves) {
        const uint32_t o = lvl_off(a);
        wave_exscan_256(
            1u << a, [&](uint32_t i) { return sm.tb.h[o + rev_bits(i, a)]; },
            [&](uint32_t i, uint32_t x) { sm.tb.lo[o + rev_bits(i, a)] = x; });
    }
    run_words(Kg, sm.tb);  // ends with a barrier

    // 3. split the tile one bit at a time
    E *gout = (E *)seq_out(d, g);
    for (uint32_t a = 0; a < Kg; a++) {
        const uint32_t bit = 1u << (shift + Kg - 1 - a);  // bit (g*K + a) of the symbol
        const bool last = (a + 1 == Kg);
        const bool move = !last || reorder;
        // this level's bits in the current order (tile-order chunk w*RW + c),
        // and the wave's zero count
        uint32_t acc_lo = 0, acc_hi = 0, zeros = 0;
#pragma unroll
        for (uint32_t c = 0; c < NCH; c++) {
            if (c < nch) {
                const bool valid = FULL || c < nfull || (c * 64 + lane < wlen);
                const uint64_t B = __ballot(valid && (v[c] & bit));
                put_lane(acc_lo, acc_hi, B, c);
                zeros += ((FULL || c < nfull) ? 64u : wlen - c * 64) - (uint32_t)__popcll(B);
            }
        }
        if (lane < nch) sm.bits[a][w * RW + lane] = ((uint64_t)acc_hi << 32) | acc_lo;
        if (!move) break;
        if (lane == 0) sm.zc[w] = zeros;
        __syncthreads();
        uint32_t base0 = 0, base1 = 0;
#pragma unroll
        for (uint32_t ww = 0; ww < kTileWaves; ww++) {
            const uint32_t z = sm.zc[ww];
            base1 += z;
            if (ww < w) {
                base0 += z;
                base1 += min(SW, len > ww * SW ? len - ww * SW : 0u) - z;
            }
        }
        base0 = __builtin_amdgcn_readfirstlane(base0);
        base1 = __builtin_amdgcn_readfirstlane(base1);
#pragma unroll
        for (uint32_t c = 0; c < NCH; c++) {
            if (c < nfull) {
                const uint32_t x = v[c];
                const bool one = (x & bit) != 0;
                const uint64_t B = __ballot(one);
                const uint32_t ones = __popcll(B);
                const uint32_t d1 = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, base1));
                const uint32_t d0 = (base0 + base1) + lane - d1;
                const uint32_t dst = one ? d1 : d0;
                if (!last) {
                    elem[dst] = (E)x;
                } else {
                    const uint32_t key = (x >> shift) & kmask;
                    const uint32_t gi = sm.tb.G[lvl_off(Kg) + key] + (dst - sm.tb.lo[lvl_off(Kg) + key]);
                    if (gi < d.n) gout[gi] = (E)x;
                }
                base0 += 64u - ones;
                base1 += ones;
            } else if (!FULL && c == nfull && c < nch) {
                const bool valid = c * 64 + lane < wlen;
                const uint32_t x = v[c];
                const bool one = valid && (x & bit) != 0;
                const uint64_t B = __ballot(one);
                if (valid) {
                    const uint32_t d1 = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, base1));
                    const uint32_t d0 = (base0 + base1) + lane - d1;
                    const uint32_t dst = one ? d1 : d0;
                    if (!last) {
                        elem[dst] = (E)x;
                    } else {
                        const uint32_t key = (x >> shift) & kmask;
                        const uint32_t gi = sm.tb.G[lvl_off(Kg) + key] + (dst - sm.tb.lo[lvl_off(Kg) + key]);
                        if (gi < d.n) gout[gi] = (E)x;
                    }
                }
            }
        }
        if (last) break;
        __syncthreads();
#pragma unroll
        for (uint32_t c = 0; c < NCH; c++)
            if (FULL ? c < nch : c * 64 + lane < wlen) v[c] = elem[wbeg + c * 64 + lane];
    }
    __syncthreads();

    // 4. every level's runs to their interval starts
    for (uint32_t a = 0; a < Kg; a++) copy_full_words(d, g, a, sm);
    run_end_words(d, g, Kg, sm);
    __syncthreads();
    // the next tile's runs start where this tile's end
    for (uint32_t e = tid; e < lvl_off(Kg + 1); e += kTileThreads) sm.tb.G[e] += sm.tb.h[e];
    __syncthreads();
}

template <typename E, uint32_t NCH>
__device__ void scatter_range(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r, ScatSmem &sm)
{
    range_start_G(d, g, Kg, r, sm.tb.G);
    for (uint32_t e = threadIdx.x; e < kTab; e += kTileThreads) sm.pend_w[e] = kNoPend;
    __syncthreads();
    const uint32_t t0 = r * d.R, t1 = min(d.ntiles, t0 + d.R);
    for (uint32_t t = t0; t < t1; t++) {
        if (((uint64_t)(t + 1) << d.log2S) <= d.n) scatter_tile<E, NCH, true>(d, g, Kg, t, sm);
        else scatter_tile<E, NCH, false>(d, g, Kg, t, sm);
    }
    // words still open at the end of the range are shared with the next one
    for (uint32_t e = threadIdx.x; e < lvl_off(Kg); e += kTileThreads) {
        const uint32_t pw = sm.pend_w[e];
        if (pw == kNoPend) continue;
        const uint32_t a = 31 - __clz(e + 1);
        if ((pw & ~kForeignLow) < d.W)
            atomicOr((unsigned long long *)&level_ptr(d, g, a)[pw & ~kForeignLow],
                     (unsigned long long)sm.pend_v[e]);
    }
}

template <typename E>
__global__ __launch_bounds__(kTileThreads, 4) void k_scatter(const TextDesc *__restrict__ descs,
                                                             const uint32_t *__restrict__ bases,
                                                             uint32_t nd, uint32_t nitems, uint32_t g)
{
    __shared__ ScatSmem sm;
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t r = item - item_base(bases, nd, ti);
        if (d.b != sizeof(E) || g >= d.G || r >= d.nranges) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        scatter_range<E, kScatBufBytes / sizeof(E) / kTileWaves / 64>(d, g, Kg, r, sm);
        __syncthreads();
    }
}

hipError_t launch_scatter(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx)
{
    uint32_t grid = gl.nranges;
    if (gl.grid_cap && grid > gl.grid_cap) grid = gl.grid_cap;
    if (gl.bmask & 1u)
        hipLaunchKernelGGL(k_scatter<uint8_t>, dim3(grid), dim3(kTileThreads), 0, ctx.stream, d_descs,
                           gl.range_bases, gl.nd, gl.nranges, gl.g);
    if (gl.bmask & 2u)
        hipLaunchKernelGGL(k_scatter<uint16_t>, dim3(grid), dim3(kTileThreads), 0, ctx.stream,
                           d_descs, gl.range_bases, gl.nd, gl.nranges, gl.g);
    if (gl.bmask & 4u)
        hipLaunchKernelGGL(k_scatter<uint32_t>, dim3(grid), dim3(kTileThreads), 0, ctx.stream,
                           d_descs, gl.range_bases, gl.nd, gl.nranges, gl.g);
    if (ctx.after) ctx.after(ctx.user, KID_SCATTER);
    return hipGetLastError();
}

}  // namespace wtg
