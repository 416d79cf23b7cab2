// Helpers shared by the border-zeroing and scatter kernels: the order in
// which a level's intervals are laid out, and G, the start of every key's
// bits at the first tile of a range of tiles:
//   G[a][k]  interval start, on level a of the group, of key k: the key's
//            base (prefix order for the WT's own levels, bit-reversed order
//            otherwise; Section 3.2 and 5.1) plus the key's count in every
//            earlier range (merged upward from the finest keys, Algorithm 1)
#pragma once

#include "wt_device.h"

namespace wtg {

constexpr uint32_t kTab = (2u << kMaxGroupBits);  // >= 2^(K+1) - 1 entries

__device__ inline bool use_prefix_order(const TextDesc &d, uint32_t g, uint32_t a, uint32_t Kg)
{
    // WT output levels of the first group use prefix order; everything else
    // (WM levels, the WT's temporary WM levels, the re-ordering target of the
    // next group) uses reversed order.
    return d.kind == WT_TREE && g == 0 && a < Kg;
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

}  // namespace wtg
