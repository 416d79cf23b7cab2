// K2: the stable scatter of a range of tiles into every level of a group.
//
// Algorithm 1 places bit l of every symbol at the next free slot of its
// interval, scanning the text in order, so inside an interval the bits are in
// text order.  Here one workgroup walks a range of consecutive tiles; a tile
// is cut into one slice per wave, and every wave orders its own slice one bit
// at a time: after splitting by bits 0..a-1 of the group key (zeros first,
// stably) the slice is ordered by its reversed a-bit key (Observation 2), so
// level a's bits of every key form one contiguous run, and the ballot of bit a
// in that order is level a of the slice.  The zero count of each split comes
// from the slice's key histogram merged upward (Algorithm 1, Hist[i] =
// Hist[2i] + Hist[2i+1]).  Then the slices' runs are concatenated per key
// (slice order = text order) and copied to the key's interval start on the
// level (prefix order for the WT, bit-reversed order for the WM; Section
// 5.1).  Consecutive tiles put a key's runs next to each other, so the word a
// run ends in is kept in LDS and completed by the next tile's run of that key;
// only words shared with another range are filled by atomic OR.  With more
// than one group, the split by the group's last bit writes every symbol
// straight to its position in the next group's sequence.
#include "wt_tiles.h"

namespace wtg {

constexpr uint32_t kScatBufBytes = kTileBufBytes;  // one element buffer
constexpr uint32_t kBitWords = kScatBufBytes / 64;  // bit words per level (1-byte symbols)
constexpr uint32_t kNoPend = 0xFFFFFFFFu;
constexpr uint32_t kForeignLow = 0x80000000u;  // pending word's low bits belong to another range

struct ScatSmem {
    uint8_t elem[kScatBufBytes];
    // level bits per slice: bits[a][w * RW + c] = ballot of chunk c of slice w
    uint64_t bits[kMaxGroupBits][kBitWords];
    uint16_t hw[kTileWaves][kTab];  // per-slice key counts, every group level
    uint16_t lw[kTileWaves][kTab];  // per-slice key starts, reversed key order
    TileTabs tb;
    uint32_t pend_w[kTab];  // word a key's coverage ends in (kNoPend: none)
    uint64_t pend_v[kTab];  // its bits so far
};

// cnt (<= 64) bits of level a at offset off of the tile's run of table entry
// e: the slices' runs of the key, concatenated in slice order
__device__ inline uint64_t gather_bits(const ScatSmem &sm, uint32_t a, uint32_t e, uint32_t off,
                                       uint32_t cnt, uint32_t RW)
{
    const uint64_t *src = sm.bits[a];
    uint64_t val = 0;
    uint32_t filled = 0, before = 0;
    for (uint32_t w = 0; w < kTileWaves && filled < cnt; w++) {
        const uint32_t hk = sm.hw[w][e];
        if (off < before + hk) {
            uint32_t take = before + hk - off;
            if (take > cnt - filled) take = cnt - filled;
            const uint32_t s = w * RW * 64 + sm.lw[w][e] + (off - before);
            const uint32_t sh = s & 63;
            uint64_t x = src[s >> 6] >> sh;
            if (sh + take > 64) x |= src[(s >> 6) + 1] << (64 - sh);
            if (take < 64) x &= (1ull << take) - 1;
            val |= x << filled;
            filled += take;
            off += take;
        }
        before += hk;
    }
    return val;
}

// words of level a that a run of this tile covers completely: plain stores
__device__ inline void copy_full_words(const TextDesc &d, uint32_t g, uint32_t a, uint32_t RW,
                                       const ScatSmem &sm)
{
    const uint32_t o = lvl_off(a), nk = 1u << a;
    const uint32_t words = sm.tb.words[a];
    uint64_t *out = level_ptr(d, g, a);
    for (uint32_t q = threadIdx.x; q < words; q += kTileThreads) {
        uint32_t lo = 0, hi = nk;  // largest key whose first word index <= q
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (sm.tb.wb[o + mid] <= q) lo = mid;
            else hi = mid;
        }
        const uint32_t e = o + lo;
        const uint64_t gs = sm.tb.G[e], hh = sm.tb.h[e];
        const uint64_t gw = (gs >> 6) + (q - sm.tb.wb[e]);
        const uint64_t ws = gw << 6;
        if (gs <= ws && gs + hh >= ws + 64) out[gw] = gather_bits(sm, a, e, (uint32_t)(ws - gs), 64, RW);
    }
}

// first and last word of every run (one thread per run, all levels): merged
// with the word kept from earlier tiles of the range, stored when complete,
// kept otherwise
__device__ inline void run_end_words(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t RW,
                                     ScatSmem &sm)
{
    for (uint32_t e = threadIdx.x; e < lvl_off(Kg); e += kTileThreads) {
        const uint32_t hh = sm.tb.h[e];
        if (hh == 0) continue;
        const uint32_t a = 31 - __clz(e + 1);
        uint64_t *out = level_ptr(d, g, a);
        const uint64_t gs = sm.tb.G[e], ge = gs + hh;
        const uint64_t fw = gs >> 6, lw = (ge - 1) >> 6;
        uint32_t newp = kNoPend;
        uint64_t newv = 0;
        if ((gs & 63) != 0 || hh < 64) {
            const uint64_t b1 = ge < ((fw + 1) << 6) ? ge : ((fw + 1) << 6);
            uint64_t val = gather_bits(sm, a, e, 0, (uint32_t)(b1 - gs), RW) << (gs & 63);
            bool lowok = (gs & 63) == 0;
            const uint32_t pw = sm.pend_w[e];
            if (!lowok && pw != kNoPend && (pw & ~kForeignLow) == fw) {
                val |= sm.pend_v[e];
                lowok = (pw & kForeignLow) == 0;
            }
            if (b1 == ((fw + 1) << 6)) {
                if (lowok) out[fw] = val;
                else atomicOr((unsigned long long *)&out[fw], (unsigned long long)val);
            } else {
                newp = (uint32_t)fw | (lowok ? 0u : kForeignLow);
                newv = val;
            }
        }
        if (lw != fw && (ge & 63) != 0) {
            newp = (uint32_t)lw;
            newv = gather_bits(sm, a, e, (uint32_t)((lw << 6) - gs), (uint32_t)(ge - (lw << 6)), RW);
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

template <typename E, uint32_t NCH>
__device__ void scatter_tile(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t t, ScatSmem &sm)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t S = 1u << d.log2S;
    const uint32_t SW = S / kTileWaves;  // symbols per slice (<= 64 * NCH)
    const uint32_t RW = SW >> 6;         // bit words per slice
    const uint64_t start = (uint64_t)t << d.log2S;
    const uint32_t len = (uint32_t)min((uint64_t)S, d.n - start);
    const uint32_t wbeg = w * SW;
    const uint32_t wlen = len > wbeg ? min(len - wbeg, SW) : 0u;
    const uint32_t nch = (wlen + 63) >> 6;
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint32_t nk = 1u << Kg, kmask = nk - 1u;
    const bool reorder = (g + 1 < d.G);
    const E *src = (const E *)seq_in(d, g) + start + wbeg;
    E *cur = (E *)sm.elem + wbeg;
    uint16_t *hw = sm.hw[w];
    uint16_t *lw = sm.lw[w];

    // 1. the slice into registers (all loads in flight at once) and its key
    //    histogram (u32 scratch in the bit area, dead until the splits)
    uint32_t v[NCH];
#pragma unroll
    for (uint32_t c = 0; c < NCH; c++) v[c] = (c * 64 + lane < wlen) ? (uint32_t)src[c * 64 + lane] : 0u;
    uint32_t *hs = (uint32_t *)&sm.bits[0][0] + w * nk;
    for (uint32_t k = lane; k < nk; k += 64) hs[k] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (uint32_t c = 0; c < NCH; c++)
        if (c * 64 + lane < wlen) atomicAdd(&hs[(v[c] >> shift) & kmask], 1u);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();

    // 2. slice tables: key counts merged upward, starts in reversed key order
    for (uint32_t k = lane; k < nk; k += 64) hw[lvl_off(Kg) + k] = (uint16_t)hs[k];
    __builtin_amdgcn_wave_barrier();
    for (uint32_t a = Kg; a-- > 0;) {
        for (uint32_t k = lane; k < (1u << a); k += 64)
            hw[lvl_off(a) + k] = hw[lvl_off(a + 1) + 2 * k] + hw[lvl_off(a + 1) + 2 * k + 1];
        __builtin_amdgcn_wave_barrier();
    }
    for (uint32_t a = 0; a <= Kg; a++) {
        const uint32_t o = lvl_off(a);
        wave_exscan_256(
            1u << a, [&](uint32_t i) { return (uint32_t)hw[o + rev_bits(i, a)]; },
            [&](uint32_t i, uint32_t x) { lw[o + rev_bits(i, a)] = (uint16_t)x; });
    }
    __syncthreads();  // every slice's tables ready; the u32 scratch is dead

    // 3. tile counts per key and the words of every run
    for (uint32_t e = tid; e < lvl_off(Kg + 1); e += kTileThreads) {
        uint32_t s = 0;
#pragma unroll
        for (uint32_t ww = 0; ww < kTileWaves; ww++) s += sm.hw[ww][e];
        sm.tb.h[e] = s;
    }
    __syncthreads();
    run_words(Kg, sm.tb);  // ends with a barrier

    // zeros of the group's last bit in the slice, before its entry is reused
    const uint32_t z_last = lw[lvl_off(Kg) + 1];
    if (reorder) {
        // position of the slice's symbols among the tile's symbols of the same
        // deepest key, minus their start in the slice's order
        for (uint32_t x = lane; x < nk; x += 64) {
            uint32_t c = 0;
            for (uint32_t ww = 0; ww < w; ww++) c += sm.hw[ww][lvl_off(Kg) + x];
            lw[lvl_off(Kg) + x] = (uint16_t)(int16_t)((int32_t)c - (int32_t)lw[lvl_off(Kg) + x]);
        }
        __builtin_amdgcn_wave_barrier();
    }

    // 4. split the slice one bit at a time, symbols in registers.  Full
    //    chunks take the fast path; the slice's last chunk may be partial.
    E *gout = (E *)seq_out(d, g);
    const uint32_t nfull = wlen >> 6;
    for (uint32_t a = 0; a < Kg; a++) {
        const uint32_t bit = 1u << (shift + Kg - 1 - a);  // bit (g*K + a) of the symbol
        const bool last = (a + 1 == Kg);
        const bool move = !last || reorder;
        uint32_t base0 = 0;
        uint32_t base1 = __builtin_amdgcn_readfirstlane(last ? z_last : (uint32_t)lw[lvl_off(a + 1) + 1]);
        uint32_t acc_lo = 0, acc_hi = 0;
#pragma unroll
        for (uint32_t c = 0; c < NCH; c++) {
            if (c < nfull) {
                // every lane holds a symbol
                const uint32_t x = v[c];
                const bool one = (x & bit) != 0;
                const uint64_t B = __ballot(one);
                // lane c of acc keeps chunk c's word
                put_lane(acc_lo, acc_hi, B, c);
                if (move) {
                    const uint32_t ones = __popcll(B);
                    const uint32_t d1 = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, base1));
                    const uint32_t d0 = (base0 + base1) + lane - d1;
                    const uint32_t dst = one ? d1 : d0;
                    if (!last) {
                        cur[dst] = (E)x;
                    } else {
                        const uint32_t key = (x >> shift) & kmask;
                        const int32_t adj = (int16_t)lw[lvl_off(Kg) + key];
                        gout[(int64_t)sm.tb.G[lvl_off(Kg) + key] + adj + dst] = (E)x;
                    }
                    base0 += 64u - ones;
                    base1 += ones;
                }
            } else if (c == nfull && c < nch) {
                // the slice's last, partial chunk
                const bool valid = c * 64 + lane < wlen;
                const uint32_t x = v[c];
                const bool one = valid && (x & bit) != 0;
                const uint64_t B = __ballot(one);
                put_lane(acc_lo, acc_hi, B, c);
                if (move && valid) {
                    const uint32_t d1 = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, base1));
                    const uint32_t d0 = (base0 + base1) + lane - d1;
                    const uint32_t dst = one ? d1 : d0;
                    if (!last) {
                        cur[dst] = (E)x;
                    } else {
                        const uint32_t key = (x >> shift) & kmask;
                        const int32_t adj = (int16_t)lw[lvl_off(Kg) + key];
                        gout[(int64_t)sm.tb.G[lvl_off(Kg) + key] + adj + dst] = (E)x;
                    }
                }
            }
        }
        if (lane < nch) sm.bits[a][w * RW + lane] = ((uint64_t)acc_hi << 32) | acc_lo;
        if (move && !last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (uint32_t c = 0; c < NCH; c++)
                if (c * 64 + lane < wlen) v[c] = cur[c * 64 + lane];
        }
    }
    __syncthreads();

    // 5. every level's runs to their interval starts
    for (uint32_t a = 0; a < Kg; a++) copy_full_words(d, g, a, RW, sm);
    run_end_words(d, g, Kg, RW, sm);
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
    for (uint32_t t = t0; t < t1; t++) scatter_tile<E, NCH>(d, g, Kg, t, sm);
    // words still open at the end of the range are shared with the next one
    for (uint32_t e = threadIdx.x; e < lvl_off(Kg); e += kTileThreads) {
        const uint32_t pw = sm.pend_w[e];
        if (pw == kNoPend) continue;
        const uint32_t a = 31 - __clz(e + 1);
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
