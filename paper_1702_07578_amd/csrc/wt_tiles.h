// Per-range and per-tile tables shared by the border-zeroing and scatter
// kernels.
//   G[a][k]  interval start, on level a of the group, of key k's bits of the
//            current tile: the key's base (prefix order for the WT's own
//            levels, bit-reversed order otherwise; Section 3.2 and 5.1) plus
//            the key's count in every earlier tile (merged upward, Algorithm 1)
//   h[a][k]  the tile's count of key k on level a
//   lo[a][k] start of key k in the tile ordered by its reversed a-bit key
//            (Observation 2): keys in bit-reversed order
//   wb[a][k] first output word of key k's run, counting the words of the
//            tile's runs on level a in key order; words[a] the total
#pragma once

#include "wt_device.h"

namespace wtg {

constexpr uint32_t kTab = (2u << kMaxGroupBits);  // >= 2^(K+1) - 1 entries

struct TileTabs {
    uint32_t h[kTab];
    uint32_t G[kTab];
    uint32_t lo[kTab];  // start of key k inside the tile's order after a splits
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

// G at the first tile of range r: range prefix merged upward plus key bases.
// Block-wide; ends with a barrier.
__device__ inline void range_start_G(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r,
                                     uint32_t *G)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t nk = 1u << Kg;
    const uint32_t *TP = d.TP + (uint64_t)r * nk;
    for (uint32_t k = tid; k < nk; k += blockDim.x) G[lvl_off(Kg) + k] = TP[k];
    __syncthreads();
    for (uint32_t a = Kg; a-- > 0;) {
        for (uint32_t k = tid; k < (1u << a); k += blockDim.x)
            G[lvl_off(a) + k] = G[lvl_off(a + 1) + 2 * k] + G[lvl_off(a + 1) + 2 * k + 1];
        __syncthreads();
    }
    for (uint32_t a = 0; a <= Kg; a++) {
        const uint32_t *kb = (use_prefix_order(d, g, a, Kg) ? d.KBid : d.KBpi) + lvl_off(a);
        for (uint32_t k = tid; k < (1u << a); k += blockDim.x) G[lvl_off(a) + k] += kb[k];
    }
    __syncthreads();
}

// words of every run of the tile on levels 0..Kg-1 (one wave per level);
// reads h and G, writes wb and words.  Ends with a barrier.
__device__ inline void run_words(uint32_t Kg, TileTabs &tb)
{
    const uint32_t w = threadIdx.x >> 6;
    for (uint32_t a = w; a < Kg; a += blockDim.x >> 6) {
        const uint32_t o = lvl_off(a);
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
    __syncthreads();
}

}  // namespace wtg
