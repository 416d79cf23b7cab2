// Shared by the border and scatter kernels: the order in which a level's
// intervals are laid out.  The interval of key k on level a of a group starts
// at the key's base in that order (Section 3.2 and 5.1) plus the key's count
// in every earlier range (merged upward from the finest keys, Algorithm 1).
#pragma once

#include "wt_device.h"

namespace wtg {

__device__ inline bool use_prefix_order(const TextDesc &d, uint32_t g, uint32_t a, uint32_t Kg)
{
    // WT output levels of the first group use prefix order; everything else
    // (WM levels, the WT's temporary WM levels, the re-ordering target of the
    // next group) uses reversed order.
    return d.kind == WT_TREE && g == 0 && a < Kg;
}

}  // namespace wtg
