// Construction by sorting (Section 3.2, "Using Sorting", Algorithm 2, and its
// WM version of Section 5.1): the second build strategy.
//
// The text is cut into P chunks of C symbols (the paper's per-core slices).
// One pass counts every chunk's symbols (Hist_c over the full L-bit symbols)
// and checks their range.  Then, level by level from the last level up:
//   * the chunk histograms of the level's prefixes are the sums of pairs of the
//     next level's (the prefix without its last bit);
//   * one zero-based prefix sum over (prefix, chunk), the prefixes in prefix
//     order for the WT and in bit-reversed order for the WM, gives every
//     chunk's start for every prefix in the sorted text;
//   * a stable counting sort of the text by the level's prefix writes the
//     sorted copy: one wave walks one chunk in text order, ranking each 64
//     symbols among equal prefixes by ballots over the prefix bits;
//   * the level's bit vector is bit l of the sorted copy, word by word.
// Level 0 is bit 0 of the text itself.  Every level's words are written whole
// by one writer, so no word is shared between writers.
#include <hip/hip_runtime.h>

#include "wt_device.h"
#include "wt_internal.h"

namespace wtg {

constexpr uint32_t kPsScanBlock = 4096;  // entries per block of the prefix sum

template <typename E>
__device__ inline uint32_t sym_load(const void *p, uint64_t i)
{
    return (uint32_t)((const E *)p)[i];
}

// ---------------------------------------------------------------------------
// chunk histograms of the full symbols (and the range check); one block per
// chunk, Hist[q * P + c].  Up to 8 interleaved copies of the histogram in LDS
// (fewer for large alphabets) spread the atomics of frequent symbols; 16-byte
// loads when the text is 16-byte aligned (chunk starts are multiples of 256
// symbols).
template <typename E>
__global__ __launch_bounds__(256) void k_ps_hist(PsDesc d, bool vec)
{
    extern __shared__ uint32_t hist[];
    constexpr uint32_t per = 16 / sizeof(E);
    const uint32_t c = blockIdx.x, t = threadIdx.x;
    const uint32_t ns = 1u << d.L;
    const uint32_t copies = ns <= 512 ? 8u : (4096u >> d.L);
    for (uint32_t q = t; q < ns * copies; q += 256) hist[q] = 0;
    __syncthreads();
    const uint64_t i0 = (uint64_t)c * d.C;
    const uint64_t i1 = min(d.n, i0 + d.C);
    const uint32_t mask = ns - 1, cp = t & (copies - 1);
    bool bad = false;
    uint64_t tail = i0;
    if (vec) {
        const uint64_t units = (i1 - i0) / per;
        const uint4 *src = (const uint4 *)((const E *)d.text + i0);
        for (uint64_t u = t; u < units; u += 256) {
            const uint4 v = src[u];
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
#pragma unroll
                for (uint32_t s = 0; s < 4 / sizeof(E); s++) {
                    const uint32_t a = sizeof(E) == 4 ? w4[k] : (w4[k] >> (s * 8 * sizeof(E))) & ((1u << (8 * sizeof(E))) - 1);
                    bad |= (d.L < 32) && (a >> d.L) != 0;
                    atomicAdd(&hist[(a & mask) * copies + cp], 1u);
                }
            }
        }
        tail = i0 + units * per;
    }
    for (uint64_t i = tail + t; i < i1; i += 256) {
        const uint32_t a = sym_load<E>(d.text, i);
        bad |= (d.L < 32) && (a >> d.L) != 0;
        atomicAdd(&hist[(a & mask) * copies + cp], 1u);
    }
    if (bad) atomicExch(d.status, (int32_t)WT_ERANGE);
    __syncthreads();
    for (uint32_t q = t; q < ns; q += 256) {
        uint32_t x = 0;
        for (uint32_t k = 0; k < copies; k++) x += hist[q * copies + k];
        d.H0[(uint64_t)q * d.P + c] = x;
    }
}

// histogram of the l-bit prefixes from that of the (l+1)-bit prefixes
__global__ __launch_bounds__(256) void k_ps_merge(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                                  uint32_t l, uint32_t P)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ((uint64_t)P << l)) return;
    const uint64_t q = e / P, c = e - q * P;
    dst[e] = src[(2 * q) * P + c] + src[(2 * q + 1) * P + c];
}

// entry of position i of the prefix sum: prefix k-th in the kind's order,
// then chunk
__device__ inline uint64_t ps_entry(uint64_t i, uint32_t P, uint32_t l, uint32_t kind)
{
    const uint64_t k = i / P, c = i - k * P;
    const uint64_t q = (kind == WT_TREE) ? k : rev_bits((uint32_t)k, l);
    return q * P + c;
}

// exclusive prefix sum over 1024 threads' values in LDS (Hillis-Steele)
__device__ inline uint32_t block_exscan(uint32_t v, uint32_t *part)
{
    const uint32_t t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t x = (t >= off) ? part[t - off] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    const uint32_t r = part[t] - v;
    __syncthreads();
    return r;
}

// block sums of the prefix sum (4096 entries per block)
__global__ __launch_bounds__(1024) void k_ps_scan_up(const uint32_t *__restrict__ H, uint32_t *__restrict__ bsum,
                                                     uint32_t l, uint32_t P, uint32_t kind)
{
    __shared__ uint32_t part[1024];
    const uint64_t E = (uint64_t)P << l;
    const uint64_t i0 = (uint64_t)blockIdx.x * kPsScanBlock + threadIdx.x * 4;
    uint32_t s = 0;
    for (uint32_t j = 0; j < 4; j++)
        if (i0 + j < E) s += H[ps_entry(i0 + j, P, l, kind)];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t off = 512; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = part[0];
}

// exclusive prefix sum of the block sums (at most 4096), one block
__global__ __launch_bounds__(1024) void k_ps_scan_top(uint32_t *bsum, uint32_t nblocks)
{
    __shared__ uint32_t part[1024];
    const uint32_t i0 = threadIdx.x * 4;
    uint32_t v[4], s = 0;
    for (uint32_t j = 0; j < 4; j++) {
        v[j] = (i0 + j < nblocks) ? bsum[i0 + j] : 0u;
        s += v[j];
    }
    uint32_t run = block_exscan(s, part);
    for (uint32_t j = 0; j < 4; j++) {
        if (i0 + j < nblocks) bsum[i0 + j] = run;
        run += v[j];
    }
}

// every entry replaced by its zero-based prefix sum in the kind's order
__global__ __launch_bounds__(1024) void k_ps_scan_down(uint32_t *H, const uint32_t *__restrict__ bsum, uint32_t l,
                                                       uint32_t P, uint32_t kind)
{
    __shared__ uint32_t part[1024];
    const uint64_t E = (uint64_t)P << l;
    const uint64_t i0 = (uint64_t)blockIdx.x * kPsScanBlock + threadIdx.x * 4;
    uint64_t at[4];
    uint32_t v[4], s = 0;
    for (uint32_t j = 0; j < 4; j++) {
        at[j] = (i0 + j < E) ? ps_entry(i0 + j, P, l, kind) : 0;
        v[j] = (i0 + j < E) ? H[at[j]] : 0u;
        s += v[j];
    }
    uint32_t run = block_exscan(s, part) + bsum[blockIdx.x];
    for (uint32_t j = 0; j < 4; j++) {
        if (i0 + j < E) H[at[j]] = run;
        run += v[j];
    }
}

// ---------------------------------------------------------------------------
// stable counting sort of the text by the l-bit prefix (l >= 1): one block
// per chunk, the chunk walked in segments of kPsSeg symbols.  Per segment:
//   1. wave w ranks the symbols of its quarter among equal prefixes (ballots
//      over the prefix bits, in text order) and counts them per prefix;
//   2. per prefix, the waves' offsets and the prefix's start in the segment
//      sorted by prefix (a scan over the prefixes);
//   3. the symbols go to that sorted order in LDS;
//   4. the staged segment is written out: a symbol at staged position p with
//      prefix q goes to cursor[q] + (p - start of q), so equal prefixes leave
//      as runs of consecutive addresses;
//   5. every cursor moves past its prefix's symbols of the segment.
constexpr uint32_t kPsSeg = 4096;
constexpr uint32_t kPsPer = kPsSeg / 256;  // symbols per lane and segment

// exclusive prefix sum over the 256 threads of a block; returns the total
__device__ inline uint32_t block256_exscan(uint32_t v, uint32_t *wsum, uint32_t &total)
{
    const uint32_t w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if ((threadIdx.x & 63) == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t k = 0; k < w; k++) before += wsum[k];
    total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return before + inc - v;
}

// one segment; FULL: all kPsSeg symbols present (no bounds tests)
template <typename E, bool FULL>
__device__ inline void ps_segment(const E *__restrict__ src, E *__restrict__ out, uint32_t len, uint32_t l,
                                  uint32_t shift, uint32_t *cursor, uint32_t *sstart, uint16_t *cnt, E *stage,
                                  uint32_t *wsum)
{
    const uint32_t nq = 1u << l;
    const uint32_t t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t per = (nq + 255) / 256;
    uint16_t *mycnt = cnt + w * nq;
    // 1. ranks within the wave's quarter
    // symbols, and their ranks (packed above 16-bit symbols: one register each)
    constexpr bool kPack = sizeof(E) <= 2;
    uint32_t a[kPsPer], rk[kPack ? 1 : kPsPer];
    const uint32_t base0 = w * (kPsSeg / 4) + lane;
#pragma unroll
    for (uint32_t j = 0; j < kPsPer; j++) {
        const uint32_t o = base0 + j * 64;
        a[j] = (FULL || o < len) ? (uint32_t)src[o] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kPsPer; j++) {
        const bool ok = FULL || base0 + j * 64 < len;
        const uint32_t q = (a[j] >> shift) & (nq - 1);
        uint64_t peers = FULL ? ~0ull : __ballot(ok);
        for (uint32_t k = 0; k < l; k++) {
            // inv: all ones when bit k of q is clear; the lanes that agree
            // with this one on bit k are the ballot, flipped by inv
            const int32_t inv = __builtin_amdgcn_sbfe((int32_t)~q, k, 1);
            const uint64_t m = __ballot(inv == 0);
            peers &= m ^ ((uint64_t)(uint32_t)inv << 32 | (uint32_t)inv);
        }
        const uint32_t rank = mbcnt64(peers);
        const uint32_t num = (uint32_t)__popcll(peers);
        uint32_t r = 0;
        if (ok) {
            const uint32_t base = mycnt[q];
            r = base + rank;
            if (rank + 1 == num) mycnt[q] = (uint16_t)(base + num);  // the last lane of the prefix
        }
        if constexpr (kPack) a[j] |= r << 16;
        else rk[j] = r;
    }
    __syncthreads();
    // 2. wave offsets per prefix, and the prefixes' starts in the segment
    //    (thread t scans prefixes [t * per, (t + 1) * per), per <= 8)
    uint32_t tot[8];
    uint32_t run = 0;
#pragma unroll
    for (uint32_t k = 0; k < 8; k++) {
        const uint32_t q = t * per + k;
        tot[k] = 0;
        if (k < per && q < nq) {
            const uint32_t c0 = cnt[q], c1 = cnt[nq + q], c2 = cnt[2 * nq + q], c3 = cnt[3 * nq + q];
            cnt[q] = 0;
            cnt[nq + q] = (uint16_t)c0;
            cnt[2 * nq + q] = (uint16_t)(c0 + c1);
            cnt[3 * nq + q] = (uint16_t)(c0 + c1 + c2);
            tot[k] = c0 + c1 + c2 + c3;
            run += tot[k];
        }
    }
    uint32_t total;
    uint32_t st = block256_exscan(run, wsum, total);
    // each wave's start of q in the staged segment (start of q plus the
    // wave's offset), and the cursor made relative to the staged position
#pragma unroll
    for (uint32_t k = 0; k < 8; k++) {
        const uint32_t q = t * per + k;
        if (k < per && q < nq) {
            sstart[q] = st;
            cursor[q] -= st;
#pragma unroll
            for (uint32_t ww = 0; ww < 4; ww++) cnt[ww * nq + q] = (uint16_t)(cnt[ww * nq + q] + st);
            st += tot[k];
        }
    }
    __syncthreads();
    // 3. stage in prefix order
#pragma unroll
    for (uint32_t j = 0; j < kPsPer; j++) {
        if (FULL || base0 + j * 64 < len) {
            const uint32_t x = kPack ? (a[j] & 0xffffu) : a[j];
            const uint32_t r = kPack ? (a[j] >> 16) : rk[kPack ? 0 : j];
            const uint32_t q = (x >> shift) & (nq - 1);
            stage[cnt[w * nq + q] + r] = (E)x;
        }
    }
    __syncthreads();
    // 4. write out in runs: staged position p of prefix q goes to
    //    cursor[q] + p (the cursor holds the global start minus the staged one)
#pragma unroll 4
    for (uint32_t p = t; p < (FULL ? kPsSeg : len); p += 256) {
        const uint32_t x = (uint32_t)stage[p];
        const uint32_t q = (x >> shift) & (nq - 1);
        out[cursor[q] + p] = (E)x;
    }
    __syncthreads();
    // 5. cursors past the segment (back to global positions), counts cleared
    for (uint32_t q = t; q < nq; q += 256) {
        const uint32_t end = (q + 1 < nq) ? sstart[q + 1] : len;
        cursor[q] += end;
        cnt[q] = cnt[nq + q] = cnt[2 * nq + q] = cnt[3 * nq + q] = 0;
    }
    __syncthreads();
}

template <typename E>
__global__ __launch_bounds__(256) void k_ps_sort(PsDesc d, uint32_t l, const uint32_t *__restrict__ B)
{
    extern __shared__ uint32_t sm[];
    __shared__ uint32_t wsum[4];
    const uint32_t nq = 1u << l;
    uint32_t *cursor = sm;             // [nq]: next global position of prefix q
    uint32_t *sstart = cursor + nq;    // [nq]: start of q in the staged segment
    uint16_t *cnt = (uint16_t *)(sstart + nq);  // [4][nq]: per wave counts, then offsets
    E *stage = (E *)(sm + 4 * nq);     // [kPsSeg], 16-byte aligned
    const uint32_t t = threadIdx.x;
    const uint32_t c = blockIdx.x;
    for (uint32_t q = t; q < nq; q += 256) {
        cursor[q] = B[(uint64_t)q * d.P + c];
        cnt[q] = cnt[nq + q] = cnt[2 * nq + q] = cnt[3 * nq + q] = 0;
    }
    __syncthreads();
    const uint64_t i0 = (uint64_t)c * d.C;
    const uint64_t i1 = min(d.n, i0 + d.C);
    const uint32_t shift = d.L - l;
    E *out = (E *)d.sorted;
    for (uint64_t seg = i0; seg < i1; seg += kPsSeg) {
        const uint32_t len = (uint32_t)min<uint64_t>(kPsSeg, i1 - seg);
        const E *src = (const E *)d.text + seg;
        if (len == kPsSeg)
            ps_segment<E, true>(src, out, len, l, shift, cursor, sstart, cnt, stage, wsum);
        else
            ps_segment<E, false>(src, out, len, l, shift, cursor, sstart, cnt, stage, wsum);
    }
}

// ---------------------------------------------------------------------------
// level l's words from a sequence in level order (the text for level 0, the
// sorted copy otherwise): each lane takes 16 bytes, 4b lanes form a word;
// grid-stride over the level's W words, Z added once per wave
template <typename E>
__device__ inline uint32_t unit_bits(const uint4 &u, uint32_t sh)
{
    const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
    uint32_t m = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) {
        uint32_t r;
        if (sizeof(E) == 1) {
            // bit sh of each byte, gathered into 4 bits by one multiply
            const uint32_t x = (w4[q] >> sh) & 0x01010101u;
            r = ((x * 0x01020408u) >> 24) & 0xfu;
        } else if (sizeof(E) == 2) {
            const uint32_t x = (w4[q] >> sh) & 0x00010001u;
            r = (x | (x >> 15)) & 3u;
        } else {
            r = (w4[q] >> sh) & 1u;
        }
        m |= r << (q * (4 / sizeof(E)));
    }
    return m;
}

template <int CTRL>
__device__ inline uint64_t dpp_or64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xf, 0xf, false);
    return x | ((uint64_t)hi << 32 | lo);
}

template <typename E>
__global__ __launch_bounds__(256) void k_ps_bits(const void *__restrict__ seq, uint64_t n, uint32_t L, uint32_t l,
                                                 uint64_t *__restrict__ words, uint64_t W, uint64_t *zeros,
                                                 bool vec)
{
    constexpr uint32_t per = 16 / sizeof(E);   // symbols per lane
    constexpr uint32_t group = 64 / per;       // lanes per word
    const uint32_t lane = lane_id();
    const uint32_t sh = L - 1 - l;  // bit l (MSB-first) of an element
    const uint64_t units = W * group;
    const uint64_t nwaves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    uint32_t zero_count = 0;
    for (uint64_t u0 = wave * 64; u0 < units; u0 += nwaves * 64) {
        const uint64_t u = u0 + lane;
        const uint64_t first = u * per;
        uint32_t m = 0, valid = 0;
        if (first < n) {
            valid = (uint32_t)min<uint64_t>(per, n - first);
            if (vec && valid == per) {
                m = unit_bits<E>(*(const uint4 *)((const E *)seq + first), sh);
            } else {
                for (uint32_t j = 0; j < valid; j++) m |= ((sym_load<E>(seq, first + j) >> sh) & 1u) << j;
            }
        }
        zero_count += valid - __popc(m);
        uint64_t x = (uint64_t)m << ((lane % group) * per);
        // OR over the group's lanes (4, 8 or 16 lanes inside a row of 16)
        x = dpp_or64<0xb1>(x);   // quad_perm [1,0,3,2]
        x = dpp_or64<0x4e>(x);   // quad_perm [2,3,0,1]
        if (group >= 8) x = dpp_or64<0x141>(x);   // row_half_mirror
        if (group >= 16) x = dpp_or64<0x140>(x);  // row_mirror
        if (lane % group == 0 && u < units) words[u / group] = x;
    }
    // Z: zeros of the wave's units, one atomic per wave
    uint32_t z = wave_incl_scan(zero_count);
    z = last_lane(z);
    if (lane == 0 && z) atomicAdd((unsigned long long *)zeros, (unsigned long long)z);
}

// ---------------------------------------------------------------------------
static inline uint32_t blocks_of(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

template <typename E>
static hipError_t launch_ps_t(const PsDesc &d, const LaunchCtx &ctx)
{
    const uint32_t L = d.L;
    const uint32_t copies = (1u << L) <= 512 ? 8u : (4096u >> L);
    hipLaunchKernelGGL(k_ps_hist<E>, dim3(d.P), dim3(256), (1u << L) * copies * 4, ctx.stream, d,
                       ((uintptr_t)d.text & 15) == 0);
    const uint32_t bits_blocks = (uint32_t)std::min<uint64_t>(2048, std::max<uint64_t>(1, blocks_of(d.W * 64, 256)));
    uint32_t *cur = d.H0, *nxt = d.H1;
    if (L >= 2) {
        hipLaunchKernelGGL(k_ps_merge, dim3(blocks_of((uint64_t)d.P << (L - 1), 256)), dim3(256), 0, ctx.stream,
                           cur, nxt, L - 1, d.P);
        std::swap(cur, nxt);
    }
    for (uint32_t l = L - 1; l >= 1 && l < L; l--) {
        if (l >= 2)
            hipLaunchKernelGGL(k_ps_merge, dim3(blocks_of((uint64_t)d.P << (l - 1), 256)), dim3(256), 0,
                               ctx.stream, cur, nxt, l - 1, d.P);
        const uint64_t E_l = (uint64_t)d.P << l;
        const uint32_t nb = blocks_of(E_l, kPsScanBlock);
        hipLaunchKernelGGL(k_ps_scan_up, dim3(nb), dim3(1024), 0, ctx.stream, cur, d.bsum, l, d.P, d.kind);
        hipLaunchKernelGGL(k_ps_scan_top, dim3(1), dim3(1024), 0, ctx.stream, d.bsum, nb);
        hipLaunchKernelGGL(k_ps_scan_down, dim3(nb), dim3(1024), 0, ctx.stream, cur, d.bsum, l, d.P, d.kind);
        // cursors and starts (u32), wave counts (u16), the staged segment
        const uint32_t lds = (1u << l) * 16 + kPsSeg * (uint32_t)sizeof(E);
        hipLaunchKernelGGL(k_ps_sort<E>, dim3(d.P), dim3(256), lds, ctx.stream, d, l, cur);
        hipLaunchKernelGGL(k_ps_bits<E>, dim3(bits_blocks), dim3(256), 0, ctx.stream, (const void *)d.sorted, d.n,
                           L, l, d.bits + (uint64_t)l * d.W, d.W, d.zeros + l, true);
        std::swap(cur, nxt);
    }
    if (L >= 1)
        hipLaunchKernelGGL(k_ps_bits<E>, dim3(bits_blocks), dim3(256), 0, ctx.stream, d.text, d.n, L, 0u, d.bits,
                           d.W, d.zeros, ((uintptr_t)d.text & 15) == 0);
    return hipGetLastError();
}

hipError_t launch_ps(const PsDesc &d, const LaunchCtx &ctx)
{
    if (d.b == 1) return launch_ps_t<uint8_t>(d, ctx);
    if (d.b == 2) return launch_ps_t<uint16_t>(d, ctx);
    return launch_ps_t<uint32_t>(d, ctx);
}

}  // namespace wtg
