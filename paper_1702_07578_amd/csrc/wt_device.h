// Device helpers shared by the kernels: work-item to text mapping, level
// pointers, bit reversal, wave primitives and directory-based rank.
#pragma once

#include "wt_internal.h"

namespace wtg {

// Map a global work item to (text index, item inside the text).  bases holds
// ndesc + 1 prefix sums of the per-text item counts of this launch.
__device__ inline uint32_t find_text(const uint32_t *__restrict__ bases, uint32_t nd,
                                     uint32_t item)
{
    if (nd == 1) return 0;
    uint32_t lo = 0, hi = nd;  // largest i with bases[i] <= item
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (bases[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Largest index p in [0, hi) with key(p) <= pos, for a key that does not
// decrease and key(0) <= pos, found by one whole wave (every lane active, the
// same arguments in every lane): each round the 64 lanes probe evenly spaced
// indexes of the remaining range and a ballot keeps the last probe at or
// before pos, so 2^15 entries take three rounds of one load each instead of
// fifteen dependent loads.
template <typename Key>
__device__ inline uint64_t wave_search_last_le(uint64_t hi, uint64_t pos, Key key)
{
    const uint64_t lane = __lane_id();
    uint64_t lo = 0;
    while (hi - lo > 1) {
        const uint64_t step = (hi - lo + 63) >> 6;
        const uint64_t p = lo + lane * step;
        const bool le = p < hi && (uint64_t)key(p < hi ? p : hi - 1) <= pos;
        const uint64_t m = __ballot(le);  // a prefix of the lanes; lane 0 probes lo
        lo += (uint64_t)(63 - __clzll((long long)m)) * step;
        hi = lo + step < hi ? lo + step : hi;
    }
    return lo;
}

// The same among texts [a, b] (bases[a] <= item): for a workgroup whose
// items are known to lie in the texts of its first and last item.
__device__ inline uint32_t find_text_in(const uint32_t *__restrict__ bases, uint32_t a, uint32_t b,
                                        uint32_t item)
{
    uint32_t lo = a, hi = b + 1;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (bases[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Text of a workgroup's item, with the texts of the group's first and last
// items found once (by threads 0 and 1) and shared through `ends`; every
// thread of the group must call it.
__device__ inline uint32_t find_text_block(const uint32_t *__restrict__ bases, uint32_t nd, uint32_t nitems,
                                           uint32_t *ends)
{
    const uint32_t first = blockIdx.x * blockDim.x;
    const uint32_t last = min(nitems, first + blockDim.x) - 1;
    if (nd == 1) return 0;
    // the texts of the first and the last item, by waves 0 and 1 (the block
    // has at least 128 threads, every one of them active here)
    if (threadIdx.x < 128) {
        const uint32_t slot = threadIdx.x >> 6;
        const uint64_t r = wave_search_last_le(nd, slot ? last : first, [&](uint64_t m) { return bases[m]; });
        if ((threadIdx.x & 63) == 0) ends[slot] = (uint32_t)r;
    }
    __syncthreads();
    const uint32_t item = first + threadIdx.x;
    if (item >= nitems) return 0;
    return ends[0] == ends[1] ? ends[0] : find_text_in(bases, ends[0], ends[1], item);
}

__device__ inline uint32_t item_base(const uint32_t *__restrict__ bases, uint32_t nd, uint32_t text)
{
    return nd == 1 ? 0u : bases[text];
}

// pi_a(i): reverse the a low bits of i (bit-reversal permutation, Section 5)
__device__ inline uint32_t rev_bits(uint32_t i, uint32_t a)
{
    return a == 0 ? 0u : (__brev(i) >> (32u - a));
}

// Output (or temporary) bit vector of level a of group g.
__device__ inline uint64_t *level_ptr(const TextDesc &d, uint32_t g, uint32_t a)
{
    uint32_t l = g * d.K + a;
    if (d.kind == WT_TREE && g > 0) return d.tmp_bits + (uint64_t)(l - d.K) * d.W;
    return d.bits + (uint64_t)l * d.W;
}

// The sequence a group reads: the text for group 0, then the re-ordered
// copies (alternating buffers).
__device__ inline const void *seq_in(const TextDesc &d, uint32_t g)
{
    if (g == 0) return d.text;
    return (g & 1u) ? d.seqA : d.seqB;
}

__device__ inline void *seq_out(const TextDesc &d, uint32_t g)
{
    return ((g + 1u) & 1u) ? d.seqA : d.seqB;
}

// Global-memory views of device pointers.  A pointer read from a descriptor
// is generic to the compiler, which then emits flat instructions; a flat
// access counts against the LDS wait counter as well as the vector-memory
// one, so every later wait for an LDS result would also wait for it (a store
// in flight would stall the next LDS read).  Accesses through these views
// are global instructions.
// (The host pass of this source sees the plain type: host code never
// dereferences these pointers, and vector types have no address-space-
// qualified copy there.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gmem = __attribute__((address_space(1))) T;
#else
template <typename T>
using gmem = T;
#endif
template <typename T>
__device__ inline gmem<T> *gp(T *p)
{
    return (gmem<T> *)p;
}
// a 16-byte load marked non-temporal (data read once, which should not
// displace cache lines that are used again)
__device__ inline ulonglong2 load_nt(const gmem<ulonglong2> *p)
{
    typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
    const u64x2 v = __builtin_nontemporal_load((const gmem<u64x2> *)p);
    return make_ulonglong2(v.x, v.y);
}
__device__ inline void gatomic_or(uint64_t *p, uint64_t v)
{
    __hip_atomic_fetch_or(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// number of set bits of mask in lanes below the calling lane
__device__ inline uint32_t mbcnt64(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint32_t lane_id() { return mbcnt64(~0ull); }

// x of the lane k places below within its row of 16 lanes, 0 if there is
// none (DPP row_shr:k); the whole wave must be active
template <int K>
__device__ inline uint32_t dpp_row_shr(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x110 + K, 0xf, 0xf, false);
}

// lane 15 of the previous row in rows 1 and 3, else 0 (DPP row_bcast:15)
__device__ inline uint32_t dpp_bcast15(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
}

// lane 31 in rows 2 and 3, else 0 (DPP row_bcast:31)
__device__ inline uint32_t dpp_bcast31(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
}

// inclusive prefix sum over the 64 lanes of a wave (all lanes active):
// within rows of 16 by shifted adds, then across rows by broadcasts
__device__ inline uint32_t wave_incl_scan(uint32_t x)
{
    x += dpp_row_shr<1>(x);
    x += dpp_row_shr<2>(x);
    x += dpp_row_shr<4>(x);
    x += dpp_row_shr<8>(x);
    x += dpp_bcast15(x);
    x += dpp_bcast31(x);
    return x;
}

// inclusive prefix maximum over the 64 lanes of a wave (all lanes active)
__device__ inline uint32_t wave_incl_max(uint32_t x)
{
    x = max(x, dpp_row_shr<1>(x));
    x = max(x, dpp_row_shr<2>(x));
    x = max(x, dpp_row_shr<4>(x));
    x = max(x, dpp_row_shr<8>(x));
    x = max(x, dpp_bcast15(x));
    x = max(x, dpp_bcast31(x));
    return x;
}

// value of lane 63
__device__ inline uint32_t last_lane(uint32_t x) { return __builtin_amdgcn_readlane(x, 63); }

// ones in bits[0, i) using the 512-bit block directory rd
__device__ inline uint64_t rank1_dir(const uint64_t *__restrict__ bits, const uint32_t *__restrict__ rd,
                                     uint64_t i)
{
    const uint64_t blk = i >> 9;
    const uint32_t before = rd[blk];
    // words of the block before position i (the last one partly)
    const uint32_t wi = (uint32_t)(i >> 6) & 7u, rem = (uint32_t)(i & 63);
    const uint32_t need = wi + (rem != 0);
    uint32_t part = 0;
    if (need != 0) {
        // all loads issued before the first count; word k >= need re-reads
        // word need - 1 (no word past those the count reads) and is masked out
        const uint64_t *b = bits + blk * 8;
        uint64_t w[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) w[k] = b[min(k, need - 1)];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint64_t m = k < wi ? ~0ull : (k == wi ? (1ull << rem) - 1 : 0ull);
            part += __popcll(w[k] & m);
        }
    }
    return (uint64_t)before + part;
}

}  // namespace wtg
