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
        if (d.pair) *d.status2 = WT_OK;
    }
    for (uint32_t l = threadIdx.x; l < d.L; l += blockDim.x) {
        d.zeros[l] = 0;
        if (d.pair) d.zeros2[l] = 0;
    }
}

// pair (WT and WM of one text from one pass): both descriptors in one
// launch, stored next to each other (the WM's serves its directories), and
// both status words and Z cleared
__global__ void k_init_pair(TextDesc d, TextDesc d2, TextDesc *dst)
{
    if (threadIdx.x == 0) {
        dst[0] = d;
        dst[1] = d2;
        *d.status = WT_OK;
        *d2.status = WT_OK;
    }
    for (uint32_t l = threadIdx.x; l < d.L; l += blockDim.x) {
        d.zeros[l] = 0;
        d2.zeros[l] = 0;
    }
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

// counters per wave in the histogram's shared array: 2^11, eight copies of
// each of 256 keys
constexpr uint32_t kHistLog2PerWave = 11;

// himask: the bits at or above L of every symbol in a 32-bit word (0 when no
// check is needed); key of a symbol: its bits from `shift` up, kw of them
// (the key's bits above the symbol's width are zero)
template <typename E, uint32_t lc>
__device__ inline void count_unit(const uint4 &u, uint32_t shift, uint32_t kw, uint32_t himask,
                                  bool &bad, uint32_t *hist)
{
    const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (uint32_t q = 0; q < 4; q++) {
        bad |= (w4[q] & himask) != 0;
#pragma unroll
        for (uint32_t s = 0; s < 4 / sizeof(E); s++)
            atomicAdd(&hist[__builtin_amdgcn_ubfe(w4[q], s * 8 * sizeof(E) + shift, kw) << lc], 1u);
    }
}

template <typename E, uint32_t lc>
__device__ void hist_range(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r, uint32_t *sh)
{
    const uint32_t tid = threadIdx.x, w = tid >> 6;
    const uint32_t nk = 1u << Kg, mask = nk - 1u;
    // every wave counts into 2^lc interleaved copies of each key (copy = lane
    // mod 2^lc), so lanes with equal keys mostly hit different words in
    // different banks: 8 copies for 64 keys or more (measured best for 128
    // and 256 keys), one per lane for 32 keys or fewer
    const uint32_t per_wave = nk << lc;
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint64_t span = (uint64_t)d.R << d.log2S;
    const uint64_t start = (uint64_t)r * span;
    const uint64_t len = min(span, d.n - start);
    const E *src = (const E *)seq_in(d, g) + start;
    uint32_t *hist = sh + w * per_wave + (tid & ((1u << lc) - 1u));

    for (uint32_t i = tid; i < kTileWaves * per_wave; i += kTileThreads) sh[i] = 0;
    __syncthreads();
    bool bad = false;
    const bool check = (g == 0) && (d.L < 32);
    // bits at or above L of every symbol of a 32-bit word
    // key bits that lie inside the symbol (a key may reach above its width)
    const uint32_t width = 8 * sizeof(E);
    const uint32_t kw = shift >= width ? 0u : min(Kg, width - shift);
    const uint32_t kshift = shift >= width ? 0u : shift;
    uint32_t himask = 0;
    if (check && d.L < 8 * sizeof(E)) {
        const uint32_t one = (sizeof(E) == 4) ? 0xFFFFFFFFu : ((1u << (8 * sizeof(E))) - 1u);
        const uint32_t m = one & ~((1u << d.L) - 1u);
        himask = (sizeof(E) == 1) ? m * 0x01010101u : (sizeof(E) == 2 ? m * 0x00010001u : m);
    }
    const uint32_t per_unit = 16 / sizeof(E);
    uint64_t done = 0;
    if (((uintptr_t)src & 15) == 0) {
        const gmem<uint4> *u = gp((const uint4 *)src);
        const uint64_t nu = len / per_unit;
        uint64_t i = tid;
        // four units per step, the next four loaded before the current ones
        // are counted
        if (i + 3 * kTileThreads < nu) {
            uint4 a0 = u[i], a1 = u[i + kTileThreads], a2 = u[i + 2 * kTileThreads], a3 = u[i + 3 * kTileThreads];
            for (i += 4 * kTileThreads; i + 3 * kTileThreads < nu; i += 4 * kTileThreads) {
                const uint4 b0 = u[i], b1 = u[i + kTileThreads], b2 = u[i + 2 * kTileThreads],
                            b3 = u[i + 3 * kTileThreads];
                count_unit<E, lc>(a0, kshift, kw, himask, bad, hist);
                count_unit<E, lc>(a1, kshift, kw, himask, bad, hist);
                count_unit<E, lc>(a2, kshift, kw, himask, bad, hist);
                count_unit<E, lc>(a3, kshift, kw, himask, bad, hist);
                a0 = b0;
                a1 = b1;
                a2 = b2;
                a3 = b3;
            }
            count_unit<E, lc>(a0, kshift, kw, himask, bad, hist);
            count_unit<E, lc>(a1, kshift, kw, himask, bad, hist);
            count_unit<E, lc>(a2, kshift, kw, himask, bad, hist);
            count_unit<E, lc>(a3, kshift, kw, himask, bad, hist);
        }
        for (; i < nu; i += kTileThreads) count_unit<E, lc>(u[i], kshift, kw, himask, bad, hist);
        done = nu * per_unit;
    }
    for (uint64_t i = done + tid; i < len; i += kTileThreads) {
        const uint32_t e = gp(src)[i];
        if (check && (e >> d.L) != 0) bad = true;
        atomicAdd(&hist[((e >> shift) & mask) << lc], 1u);
    }
    if (bad) {
        atomicExch(d.status, (int32_t)WT_ERANGE);
        if (d.pair) atomicExch(d.status2, (int32_t)WT_ERANGE);
    }
    __syncthreads();
    // sum every key's copies in all waves: thread (k, p), p < P = threads
    // per key, adds every P-th of them; the P parts are then halved in place
    // until one is left
    uint32_t *H = d.H + (uint64_t)r * nk;
    if (lc == 3) {  // 64 keys or more: one thread sums all copies of a key
        for (uint32_t k = tid; k < nk; k += kTileThreads) {
            uint32_t t = 0;
#pragma unroll
            for (uint32_t j = 0; j < (kTileWaves << lc); j++) t += sh[(j >> lc) * per_wave + (k << lc) + (j & 7)];
            gp(H)[k] = t;
        }
        return;
    }
    const uint32_t P = kTileThreads / nk, k = tid % nk, p = tid / nk;
    const uint32_t J = kTileWaves << lc;  // counters of one key
    uint32_t part = 0;
    for (uint32_t j = p; j < J; j += P) part += sh[(j >> lc) * per_wave + (k << lc) + (j & ((1u << lc) - 1u))];
    if (P == 1) {
        gp(H)[k] = part;
        return;
    }
    __syncthreads();
    sh[tid] = part;  // part p of key k at p nk + k
    __syncthreads();
    for (uint32_t half = P >> 1; half > 0; half >>= 1) {
        if (tid < half * nk) sh[tid] += sh[tid + half * nk];
        __syncthreads();
    }
    if (tid < nk) gp(H)[tid] = sh[tid];
}

__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_hist(const TextDesc *__restrict__ descs,
                                                       const uint32_t *__restrict__ bases,
                                                       uint32_t nd, uint32_t nitems, uint32_t g)
{
    __shared__ uint32_t sh[kTileWaves << kHistLog2PerWave];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t r = item - item_base(bases, nd, ti);
        if (g >= d.G || r >= d.nranges) continue;
        const uint32_t Kg = group_bits(d, g);
        static_assert(kMaxGroupBits + 3 <= kHistLog2PerWave && 5 + 6 <= kHistLog2PerWave, "copies fit");
        if (Kg >= 6) {
            if (d.b == 1) hist_range<uint8_t, 3>(d, g, Kg, r, sh);
            else if (d.b == 2) hist_range<uint16_t, 3>(d, g, Kg, r, sh);
            else hist_range<uint32_t, 3>(d, g, Kg, r, sh);
        } else {
            if (d.b == 1) hist_range<uint8_t, 6>(d, g, Kg, r, sh);
            else if (d.b == 2) hist_range<uint16_t, 6>(d, g, Kg, r, sh);
            else hist_range<uint32_t, 6>(d, g, Kg, r, sh);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K1a: per chunk of kBorderChunk ranges, column sums of the range histograms.
// The block's threads are P parts of each of the nk keys (thread p nk + k is
// part p of key k, P nk = the block size); a part adds up to kPartRanges
// ranges, with all of its loads issued before the first add.

constexpr uint32_t kSumThreads = 1024;
constexpr uint32_t kPartRanges = 8;
static_assert(kBorderChunk <= kPartRanges * (kSumThreads >> kMaxGroupBits),
              "a part adds at most kPartRanges ranges of a chunk");

// Sum of the P parts of every key, left in buf[k]; thread p nk + k brings
// part p of key k (P a power of two, P nk = the block size).
__device__ inline void parts_reduce(uint32_t s, uint32_t nk, uint32_t P, uint32_t *buf)
{
    const uint32_t tid = threadIdx.x, p = tid / nk;
    buf[tid] = s;
    __syncthreads();
    for (uint32_t half = P >> 1; half > 0; half >>= 1) {
        if (p < half) buf[tid] += buf[tid + half * nk];
        __syncthreads();
    }
}

// Inclusive sum of parts 0..p of the thread's key (same layout), in
// log2(P) steps.
__device__ inline uint32_t parts_incl_scan(uint32_t s, uint32_t nk, uint32_t P, uint32_t *buf)
{
    const uint32_t tid = threadIdx.x, p = tid / nk;
    buf[tid] = s;
    __syncthreads();
    for (uint32_t off = 1; off < P; off <<= 1) {
        const uint32_t v = p >= off ? buf[tid - off * nk] : 0u;
        __syncthreads();
        s += v;
        buf[tid] = s;
        __syncthreads();
    }
    return s;
}

__global__ __launch_bounds__(kSumThreads) void k_chunk_sum(const TextDesc *__restrict__ descs,
                                                           const uint32_t *__restrict__ bases, uint32_t nd,
                                                           uint32_t nitems, uint32_t g)
{
    __shared__ uint32_t part[kSumThreads];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t c = item - item_base(bases, nd, ti);
        if (g >= d.G || c >= d.nchunks) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        const uint32_t nk = 1u << Kg, P = kSumThreads / nk;
        const uint32_t k = threadIdx.x % nk, p = threadIdx.x / nk;
        const uint32_t r0 = c * kBorderChunk, r1 = min(d.nranges, r0 + kBorderChunk);  // r0 < r1
        uint32_t s = 0;
#pragma unroll
        for (uint32_t i = 0; i < kPartRanges; i++) {
            const uint32_t r = r0 + p + i * P;
            const uint32_t x = gp(d.H)[(uint64_t)min(r, r1 - 1) * nk + k];
            s += r < r1 ? x : 0u;
        }
        parts_reduce(s, nk, P, part);
        if (p == 0) gp(d.CS)[(uint64_t)c * nk + k] = part[k];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K1b: per chunk of ranges, everything the scatter needs before it starts
// (Algorithm 1: merged histograms and borders; Section 3.2: borders
// interleaved over slices; Section 5.1: bit-reversed order and Z):
//   - the chunk's prefix and the totals of every finest key, from all chunk sums
//   - totals of every shorter key (merged upward) and the key bases of every
//     level in prefix and in bit-reversed order (computed by every block; the
//     text's first block also publishes them, with Z and, for a deep WT, the
//     first row of the interval walk)
//   - TP, the range-exclusive prefix of every finest key for the chunk's ranges
//   - the output words shared between ranges: a range's run of key k on a
//     level starts at G (the subtree sum of TP plus the key's base); when G is
//     not word-aligned its word also holds bits of the previous range (or
//     key), both sides fill it by atomic OR, and it is cleared here; the
//     text's first range also clears the padding words.

constexpr uint32_t kBorderThreads = 1024;
constexpr uint32_t kBorderWaves = kBorderThreads / 64;
static_assert(kBorderChunk <= kPartRanges * (kBorderThreads >> kMaxGroupBits),
              "a part takes at most kPartRanges ranges of a chunk");

__global__ __launch_bounds__(kBorderThreads) void k_borders(const TextDesc *__restrict__ descs,
                                                            const uint32_t *__restrict__ bases,
                                                            uint32_t nd, uint32_t nitems,
                                                            uint32_t g)
{
    constexpr uint32_t kK = 1u << kMaxGroupBits;
    __shared__ uint32_t part[kBorderThreads];
    __shared__ uint32_t pre[kK];
    __shared__ uint32_t tot[2 * kK];
    __shared__ uint32_t kbid[2 * kK], kbpi[2 * kK];
    __shared__ uint32_t S[kBorderWaves][kK + 1];
    __shared__ uint32_t tpl[kBorderChunk * kK];  // TP of the chunk's ranges
    const uint32_t tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t c = item - item_base(bases, nd, ti);
        if (g >= d.G || c >= d.nchunks) continue;
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0) continue;
        const uint32_t nk = 1u << Kg, P = kBorderThreads / nk;
        const uint32_t k = tid % nk, p = tid / nk;

        // chunk prefix and totals of the finest keys
        uint32_t before = 0, all = 0;
        // a part's chunks c2 = p + i P, eight loads issued before their adds
        for (uint32_t cb = p; cb < d.nchunks; cb += kPartRanges * P) {
            uint32_t xs[kPartRanges];
#pragma unroll
            for (uint32_t i = 0; i < kPartRanges; i++)
                xs[i] = gp(d.CS)[(uint64_t)min(cb + i * P, d.nchunks - 1) * nk + k];
#pragma unroll
            for (uint32_t i = 0; i < kPartRanges; i++) {
                const uint32_t c2 = cb + i * P;
                const uint32_t x = c2 < d.nchunks ? xs[i] : 0u;
                all += x;
                before += c2 < c ? x : 0u;
            }
        }
        parts_reduce(before, nk, P, part);
        if (p == 0) pre[k] = part[k];
        __syncthreads();
        parts_reduce(all, nk, P, part);
        if (p == 0) tot[lvl_off(Kg) + k] = part[k];
        __syncthreads();
        for (uint32_t a = Kg; a-- > 0;) {
            for (uint32_t kk = tid; kk < (1u << a); kk += kBorderThreads)
                tot[lvl_off(a) + kk] = tot[lvl_off(a + 1) + 2 * kk] + tot[lvl_off(a + 1) + 2 * kk + 1];
            __syncthreads();
        }
        // key bases: one wave per (level, order), keys visited in that order
        for (uint32_t job = w; job < 2 * (Kg + 1); job += kBorderWaves) {
            const uint32_t a = job >> 1;
            const bool rev = job & 1;
            uint32_t *kb = (rev ? kbpi : kbid) + lvl_off(a);
            const uint32_t *ht = tot + lvl_off(a);
            uint32_t carry = 0;
            for (uint32_t base = 0; base < (1u << a); base += 64) {
                const uint32_t i = base + lane;
                const uint32_t key = (i < (1u << a)) ? (rev ? rev_bits(i, a) : i) : 0u;
                const uint32_t x = (i < (1u << a)) ? ht[key] : 0u;
                const uint32_t incl = wave_incl_scan(x);
                if (i < (1u << a)) kb[key] = carry + incl - x;
                carry += last_lane(incl);
            }
        }
        __syncthreads();
        if (c == 0) {
            for (uint32_t e = tid; e < lvl_off(Kg + 1); e += kBorderThreads) {
                d.HT[e] = tot[e];
                d.KBid[e] = kbid[e];
                d.KBpi[e] = kbpi[e];
            }
            // Z of the group's levels: zeros of level a = symbols whose next
            // bit is 0, the even keys one level deeper (Section 5.1)
            if (tid < Kg) {
                uint64_t z = 0;
                for (uint32_t kk = 0; kk < (2u << tid); kk += 2) z += tot[lvl_off(tid + 1) + kk];
                d.zeros[g * d.K + tid] = z;
                if (d.pair) d.zeros2[g * d.K + tid] = z;
            }
            // deep WT: intervals of the K-bit prefixes (level K) seed the walk
            // (of this WT, or of the WT paired with this WM)
            if (d.G > 1 && g == 0 && (d.kind == WT_TREE || d.pair)) {
                uint32_t *tab = d.kind == WT_TREE ? d.walk : d.walk2;  // walk_off(K, K) == 0
                for (uint32_t q = tid; q < nk; q += kBorderThreads) {
                    tab[q] = kbpi[lvl_off(Kg) + q];
                    tab[nk + q] = tot[lvl_off(Kg) + q];
                    tab[2 * nk + q] = kbid[lvl_off(Kg) + q];
                }
            }
        }
        // TP of the chunk's ranges: each part of a key takes up to kPartRanges
        // consecutive ranges, loaded together; the chunk's TP is also kept in
        // LDS for the shared words below
        const uint32_t r0 = c * kBorderChunk, r1 = min(d.nranges, r0 + kBorderChunk);  // r0 < r1
        const uint32_t per = (kBorderChunk + P - 1) / P;
        const uint32_t q0 = min(r1, r0 + p * per), q1 = min(r1, q0 + per);
        uint32_t x[kPartRanges], s = 0;
#pragma unroll
        for (uint32_t i = 0; i < kPartRanges; i++) {
            const uint32_t r = q0 + i;
            x[i] = gp(d.H)[(uint64_t)min(r, r1 - 1) * nk + k];
            x[i] = r < q1 ? x[i] : 0u;
            s += x[i];
        }
        uint32_t run = pre[k] + parts_incl_scan(s, nk, P, part) - s;
#pragma unroll
        for (uint32_t i = 0; i < kPartRanges; i++) {
            const uint32_t r = q0 + i;
            if (r < q1) {
                gp(d.TP)[(uint64_t)r * nk + k] = run;
                tpl[(r - r0) * nk + k] = run;
            }
            run += x[i];
        }
        __syncthreads();
        // shared words of every range of the chunk (one wave per range)
        for (uint32_t r = r0 + w; r < r1; r += kBorderWaves) {
            const uint32_t *tp = tpl + (r - r0) * nk;
            uint32_t *sw = S[w];
            uint32_t carry = 0;
            for (uint32_t base = 0; base < nk; base += 64) {
                const uint32_t j = base + lane;
                const uint32_t v = (j < nk) ? tp[j] : 0u;
                const uint32_t incl = wave_incl_scan(v);
                if (j < nk) sw[j] = carry + incl - v;
                carry += last_lane(incl);
            }
            if (lane == 0) sw[nk] = carry;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (uint32_t e = lane; e < lvl_off(Kg); e += 64) {
                const uint32_t a = 31 - __clz(e + 1), kk = e - lvl_off(a), sh = Kg - a;
                const uint32_t *kb = use_prefix_order(d, g, a, Kg) ? kbid : kbpi;
                const uint32_t raw = sw[(kk + 1) << sh] - sw[kk << sh];
                const uint32_t gs = raw + kb[e];
                if ((gs & 63) != 0 && (gs >> 6) < d.W) gp(level_ptr(d, g, a))[gs >> 6] = 0;
                if (d.pair && g == 0) {  // the pair's other structure, in its order
                    const uint32_t gs2 = raw + (d.kind == WT_MATRIX ? kbid : kbpi)[e];
                    if ((gs2 & 63) != 0 && (gs2 >> 6) < d.W) gp(d.bits2)[(uint64_t)a * d.W + (gs2 >> 6)] = 0;
                }
            }
            if (r == 0) {
                // padding words, and the word holding position n (its bits
                // past n must stay zero; the run ending there fills it by OR)
                for (uint32_t a = 0; a < Kg; a++) {
                    uint64_t *out = level_ptr(d, g, a);
                    for (uint64_t wd = (d.n >> 6) + lane; wd < d.W; wd += 64) out[wd] = 0;
                    if (d.pair && g == 0)
                        for (uint64_t wd = (d.n >> 6) + lane; wd < d.W; wd += 64) d.bits2[(uint64_t)a * d.W + wd] = 0;
                }
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
    __shared__ uint32_t ends[2];
    const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ti = find_text_block(bases, nd, nitems, ends);
    if (item >= nitems) return;
    const TextDesc &d = descs[ti];
    const uint32_t p = item - item_base(bases, nd, ti);
    // the fields the test needs, loaded together (no branch between loads);
    // l + 1 < L <= 32 before the shift
    const uint32_t kind = d.kind, G = d.G, L = d.L, l = d.K + step;
    if (((kind != WT_TREE) | (G <= 1) | (l + 1 >= L)) || p >= (1u << l)) return;
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

// Gather: every word of WT level l >= K from the WM level's intervals; one
// thread fills kGatherWords consecutive words, keeping the interval of the
// previous piece (the next piece is in the same interval or the next
// non-empty one far more often than not), so most pieces need no search.
__global__ __launch_bounds__(256) void k_gather(const TextDesc *__restrict__ descs,
                                                const uint32_t *__restrict__ bases, uint32_t nd,
                                                uint32_t nitems)
{
    // the intervals of the first and the last word of the block (when they
    // belong to the same text and level, every word of the block between
    // them lies in an interval between theirs)
    __shared__ uint32_t b_ti[2], b_l[2], b_p[2], ends[2];
    __shared__ uint64_t b_pos[2];
    const uint32_t first = blockIdx.x * blockDim.x;
    const uint32_t item = first + threadIdx.x;
    const uint32_t last = min(nitems, first + blockDim.x) - 1;
    bool ok = item < nitems;
    uint32_t ti = find_text_block(bases, nd, nitems, ends), l = 0, np = 1;
    uint64_t w0 = 0;
    const TextDesc *dp = nullptr;
    const gmem<uint32_t> *tab = nullptr;
    if (ok) {
        dp = &descs[ti];
        const uint64_t idx = item - item_base(bases, nd, ti);
        ok = dp->kind == WT_TREE && dp->G > 1;
        if (ok) {
            const uint64_t Wg = dp->W / kGatherWords;  // W is a multiple of 8
            l = dp->K + (uint32_t)(idx / Wg);
            ok = l < dp->L;
            w0 = (idx % Wg) * kGatherWords;
            np = 1u << l;
            tab = gp(dp->walk + walk_off(dp->K, l));
        }
    }
    // largest p in [a, b) with wt_start[p] <= pos (wt_start[a] <= pos)
    auto search = [&](uint64_t pos, uint32_t a, uint32_t b) -> uint32_t {
        while (b - a > 1) {
            const uint32_t mid = (a + b) >> 1;
            if (tab[2 * np + mid] <= pos) a = mid;
            else b = mid;
        }
        return a;
    };
    // slot 0: the block's first item, slot 1: its last (the same thread when
    // the block holds one item)
    for (uint32_t slot = 0; slot < 2; slot++) {
        if (item != (slot ? last : first)) continue;
        b_ti[slot] = ok ? ti : 0xFFFFFFFFu;
        b_l[slot] = l;
        b_pos[slot] = (w0 << 6) + (slot ? kGatherWords * 64 - 1 : 0);
    }
    __syncthreads();
    // one text and level for the whole block: the two ends are searched once,
    // by wave 0 and wave 1 (positions past the text end clamp to n - 1)
    const bool one = b_ti[0] != 0xFFFFFFFFu && b_ti[0] == b_ti[1] && b_l[0] == b_l[1];
    if (one && threadIdx.x < 128) {
        const uint32_t slot = threadIdx.x >> 6;
        const TextDesc &d0 = descs[b_ti[0]];
        const uint32_t np0 = 1u << b_l[0];
        const uint32_t *tab0 = d0.walk + walk_off(d0.K, b_l[0]);
        const uint64_t r = wave_search_last_le(np0, min(b_pos[slot], d0.n - 1),
                                               [&](uint64_t p) { return tab0[2 * np0 + p]; });
        if ((threadIdx.x & 63) == 0) b_p[slot] = (uint32_t)r;
    }
    __syncthreads();
    if (!ok) return;
    const TextDesc &d = *dp;
    uint32_t ra = 0, rb = np;  // search range of the first piece of a word
    if (one) {
        ra = b_p[0];
        rb = b_p[1] + 1;
    }
    gmem<uint64_t> *out = gp(d.bits + (uint64_t)l * d.W);
    const gmem<uint64_t> *wm = gp(d.tmp_bits + (uint64_t)(l - d.K) * d.W);
    uint32_t lo = np;  // interval of the previous piece (none yet)
    for (uint32_t k = 0; k < kGatherWords; k++) {
        const uint64_t ws = (w0 + k) << 6;
        const uint64_t we = min(ws + 64, d.n);
        uint64_t val = 0;
        uint64_t pos = ws;
        while (pos < we) {
            // the non-empty interval holding pos: the previous one or the
            // next one when they hold it, else a search
            if (lo < np && tab[2 * np + lo] <= pos && pos < (uint64_t)tab[2 * np + lo] + tab[np + lo]) {
            } else if (lo + 1 < np && tab[2 * np + lo + 1] == pos && tab[np + lo + 1] != 0) {
                lo = lo + 1;
            } else if (lo < np) {
                // empty intervals follow the previous one: a bracket that
                // doubles from it until an interval starts past pos, then a
                // search inside it (log of the gap, not of the range)
                uint32_t a = lo, b = lo + 1, step = 1;
                while (b < rb && tab[2 * np + b] <= pos) {
                    a = b;
                    step <<= 1;
                    b = a + step;
                }
                lo = search(pos, a, max(min(b, rb), a + 1));  // never empty
            } else {
                lo = search(pos, ra, rb);
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
        out[w0 + k] = val;
    }
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

hipError_t launch_init_pair(const TextDesc &d, const TextDesc &d2, TextDesc *d_dst, const LaunchCtx &ctx)
{
    hipLaunchKernelGGL(k_init_pair, dim3(1), dim3(64), 0, ctx.stream, d, d2, d_dst);
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
    hipLaunchKernelGGL(k_chunk_sum, dim3(grid_for(gl.nchunks, gl.grid_cap)), dim3(kSumThreads), 0,
                       ctx.stream, d_descs, gl.chunk_bases, nd, gl.nchunks, g);
    after(ctx, KID_CHUNK_SUM);
    hipLaunchKernelGGL(k_borders, dim3(grid_for(gl.nchunks, gl.grid_cap)), dim3(kBorderThreads), 0,
                       ctx.stream, d_descs, gl.chunk_bases, nd, gl.nchunks, g);
    after(ctx, KID_BORDERS);
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
