// Batched access / rank / select over a built wavelet tree or wavelet matrix,
// one lane per query, L dependent steps each (Section 2 and Section 5: the
// indexes answer these in O(lg sigma) with binary rank/select on the levels).
//
// Level-wise WT: the node of a prefix occupies the same range [s, e) on every
// deeper level; its left child is [s, s + z) and its right child [s + z, e),
// z = zeros of the node on the current level.
// WM (definition of Section 5): a position i of level l with bit b moves to
// rank_0(BV_l, i) (b = 0) or Z[l] + rank_1(BV_l, i) (b = 1) on level l + 1.
#include "wt_device.h"

namespace wtg {

struct QLevel {
    const uint64_t *bits;
    const uint32_t *rd;
    const uint32_t *sel0;
    const uint32_t *sel1;
};

__device__ inline QLevel qlevel(const wt_levels &s, uint32_t l)
{
    QLevel q;
    q.bits = s.bits + (uint64_t)l * s.words_per_level;
    q.rd = s.rank_dir + (uint64_t)l * s.rank_stride;
    q.sel0 = s.sel0 + (uint64_t)l * s.sel_stride;
    q.sel1 = s.sel1 + (uint64_t)l * s.sel_stride;
    return q;
}

__device__ inline uint32_t getbit(const uint64_t *bits, uint64_t i)
{
    return (uint32_t)((bits[i >> 6] >> (i & 63)) & 1u);
}

__device__ inline uint64_t rank1(const QLevel &q, uint64_t i) { return rank1_dir(q.bits, q.rd, i); }

// 0-based position of the r-th (1-based) set bit of x; x has at least r ones
__device__ inline uint32_t select_in_word(uint64_t x, uint32_t r)
{
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t width = 32; width >= 1; width >>= 1) {
        const uint64_t lowmask = (width == 64) ? ~0ull : ((1ull << width) - 1);
        const uint32_t c = __popcll(x & lowmask);
        if (r > c) {
            r -= c;
            x >>= width;
            pos += width;
        }
    }
    return pos;
}

// position of the k-th (1-based) b-bit among positions < n; the caller
// guarantees 1 <= k <= number of b-bits in [0, n)
__device__ uint64_t select_b(const QLevel &q, uint64_t n, uint64_t nb, uint64_t k, uint32_t b)
{
    const uint32_t *smp = b ? q.sel1 : q.sel0;
    // guard against a k past the level's count (never the case for a
    // consistent structure)
    const uint64_t ones = q.rd[nb];
    const uint64_t count = b ? ones : n - ones;
    if (k == 0 || k > count || nb == 0) return ~0ull;
    const uint64_t qi = (k - 1) / WT_SEL_SPACING;
    uint64_t lo = smp[qi];
    uint64_t hi = smp[qi + 1];
    if (lo >= nb) lo = nb - 1;
    if (hi == 0xFFFFFFFFull || hi >= nb) hi = nb - 1;
    if (hi < lo) hi = lo;
    // b-bits before block j
    auto before = [&](uint64_t j) -> uint64_t {
        const uint64_t ones = q.rd[j];
        if (b) return ones;
        const uint64_t s = j * 512;
        return (s < n ? s : n) - ones;
    };
    // largest j in [lo, hi] with before(j) < k
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (before(mid) < k) lo = mid;
        else hi = mid - 1;
    }
    uint64_t r = k - before(lo);
    // the block's 8 words (lo < nb: the block lies inside the level), all
    // loaded before the scan
    const uint64_t *wp = q.bits + lo * 8;
    uint64_t w[8];
#pragma unroll
    for (uint32_t i = 0; i < 8; i++) w[i] = wp[i];
#pragma unroll
    for (uint32_t i = 0; i < 8; i++) {
        const uint64_t x = b ? w[i] : ~w[i];
        const uint32_t c = __popcll(x);
        if (r <= c) return lo * 512 + i * 64 + select_in_word(x, (uint32_t)r);
        r -= c;
    }
    return ~0ull;  // unreachable for valid k
}

__global__ __launch_bounds__(256) void k_access(wt_levels s, const uint64_t *__restrict__ pos,
                                                uint64_t m, uint32_t *__restrict__ out)
{
    const uint64_t qi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= m) return;
    uint64_t i = pos[qi];
    if (i >= s.n) {
        out[qi] = 0xFFFFFFFFu;
        return;
    }
    uint32_t c = 0;
    uint64_t st = 0, en = s.n;
    for (uint32_t l = 0; l < s.lg_sigma; l++) {
        const QLevel q = qlevel(s, l);
        const uint32_t b = getbit(q.bits, i);
        c = (c << 1) | b;
        if (s.kind == WT_MATRIX) {
            const uint64_t r1 = rank1(q, i);
            i = b ? s.zeros[l] + r1 : i - r1;
        } else {
            const uint64_t r1s = rank1(q, st), r1e = rank1(q, en), r1i = rank1(q, i);
            const uint64_t z = (en - st) - (r1e - r1s);
            if (b == 0) {
                i = st + ((i - r1i) - (st - r1s));
                en = st + z;
            } else {
                i = st + z + (r1i - r1s);
                st = st + z;
            }
        }
    }
    out[qi] = c;
}

__global__ __launch_bounds__(256) void k_rank(wt_levels s, const uint32_t *__restrict__ sym,
                                              const uint64_t *__restrict__ pos, uint64_t m,
                                              uint64_t *__restrict__ out)
{
    const uint64_t qi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= m) return;
    const uint64_t c = sym[qi];
    uint64_t p = pos[qi];
    const uint32_t L = s.lg_sigma;
    if (p > s.n) {
        out[qi] = ~0ull;
        return;
    }
    if (L < 32 && (c >> L) != 0) {
        out[qi] = 0;
        return;
    }
    uint64_t st = 0, en = s.n;
    for (uint32_t l = 0; l < L; l++) {
        const QLevel q = qlevel(s, l);
        const uint32_t b = (uint32_t)((c >> (L - 1 - l)) & 1u);
        if (s.kind == WT_MATRIX) {
            const uint64_t r1p = rank1(q, p), r1s = rank1(q, st);
            if (b) {
                p = s.zeros[l] + r1p;
                st = s.zeros[l] + r1s;
            } else {
                p = p - r1p;
                st = st - r1s;
            }
        } else {
            const uint64_t r1s = rank1(q, st), r1e = rank1(q, en), r1p = rank1(q, p);
            const uint64_t z = (en - st) - (r1e - r1s);
            if (b == 0) {
                p = st + ((p - r1p) - (st - r1s));
                en = st + z;
            } else {
                p = st + z + (r1p - r1s);
                st = st + z;
            }
        }
    }
    out[qi] = p - st;
}

__global__ __launch_bounds__(256) void k_select(wt_levels s, const uint32_t *__restrict__ sym,
                                                const uint64_t *__restrict__ kk, uint64_t m,
                                                uint64_t *__restrict__ out)
{
    const uint64_t qi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (qi >= m) return;
    const uint64_t c = sym[qi];
    const uint64_t k = kk[qi];
    const uint32_t L = s.lg_sigma;
    const uint64_t nb = s.words_per_level / 8;
    if (k == 0 || (L < 32 && (c >> L) != 0)) {
        out[qi] = ~0ull;
        return;
    }
    uint64_t sv[32];
    uint64_t st = 0, en = s.n;
    for (uint32_t l = 0; l < L; l++) {
        const QLevel q = qlevel(s, l);
        const uint32_t b = (uint32_t)((c >> (L - 1 - l)) & 1u);
        sv[l] = st;
        const uint64_t r1s = rank1(q, st), r1e = rank1(q, en);
        if (s.kind == WT_MATRIX) {
            if (b) {
                st = s.zeros[l] + r1s;
                en = s.zeros[l] + r1e;
            } else {
                st = st - r1s;
                en = en - r1e;
            }
        } else {
            const uint64_t z = (en - st) - (r1e - r1s);
            if (b == 0) en = st + z;
            else st = st + z;
        }
    }
    if (k > en - st) {
        out[qi] = ~0ull;
        return;
    }
    uint64_t p = (s.kind == WT_MATRIX) ? st + k - 1 : k - 1;
    for (uint32_t l = L; l-- > 0;) {
        const QLevel q = qlevel(s, l);
        const uint32_t b = (uint32_t)((c >> (L - 1 - l)) & 1u);
        if (s.kind == WT_MATRIX) {
            p = b ? select_b(q, s.n, nb, p - s.zeros[l] + 1, 1) : select_b(q, s.n, nb, p + 1, 0);
        } else {
            const uint64_t sl = sv[l];
            const uint64_t r1s = rank1(q, sl);
            const uint64_t rb = b ? r1s : sl - r1s;
            p = select_b(q, s.n, nb, rb + p + 1, b) - sl;
        }
    }
    out[qi] = p;
}

// Lemma 5: WT position i of level l -> WM position (one lane per query).
// select_1(U, i+1) has exactly i ones before it, so rank_0 there is
// select_1(U, i+1) - i; select_0(U, k) has k-1 zeros before it, so rank_1
// there is select_0(U, k) - (k-1).
__global__ __launch_bounds__(256) void k_posmap(wt_posmap m, uint32_t level,
                                                const uint64_t *__restrict__ pos, uint64_t count,
                                                uint64_t *__restrict__ out)
{
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const uint64_t i = pos[q];
    if (i >= m.n || level >= m.lg_sigma) {
        out[q] = ~0ull;
        return;
    }
    if (level <= 1) {
        out[q] = i;
        return;
    }
    QLevel u;
    u.bits = m.U;
    u.rd = m.rank_dir;
    u.sel0 = m.sel0;
    u.sel1 = m.sel1;
    const uint64_t nb = m.u_words / 8;
    const uint64_t c = select_b(u, m.u_len, nb, i + 1, 1) - i;
    const uint32_t sh = m.lg_sigma - level;
    const uint64_t bp = c >> sh;
    if (bp >= (1ull << level)) {  // never for a consistent map
        out[q] = ~0ull;
        return;
    }
    const uint64_t k = bp << sh;
    const uint64_t before = k ? select_b(u, m.u_len, nb, k, 0) - (k - 1) : 0;
    out[q] = (uint64_t)m.X[((1ull << level) - 1) + bp] + (i - before);
}

hipError_t launch_posmap_query(const wt_posmap &m, uint32_t level, const uint64_t *d_pos,
                               uint64_t count, uint64_t *d_out, const LaunchCtx &ctx)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_posmap, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, ctx.stream, m,
                       level, d_pos, count, d_out);
    if (ctx.after) ctx.after(ctx.user, KID_QUERY);
    return hipGetLastError();
}

hipError_t launch_queries(const wt_levels &s, int op, const uint32_t *d_sym, const uint64_t *d_arg,
                          uint64_t m, void *d_out, const LaunchCtx &ctx)
{
    if (m == 0) return hipSuccess;
    const uint64_t blocks = (m + 255) / 256;
    if (op == 0)
        hipLaunchKernelGGL(k_access, dim3((uint32_t)blocks), dim3(256), 0, ctx.stream, s, d_arg, m,
                           (uint32_t *)d_out);
    else if (op == 1)
        hipLaunchKernelGGL(k_rank, dim3((uint32_t)blocks), dim3(256), 0, ctx.stream, s, d_sym, d_arg,
                           m, (uint64_t *)d_out);
    else
        hipLaunchKernelGGL(k_select, dim3((uint32_t)blocks), dim3(256), 0, ctx.stream, s, d_sym,
                           d_arg, m, (uint64_t *)d_out);
    if (ctx.after) ctx.after(ctx.user, KID_QUERY);
    return hipGetLastError();
}

}  // namespace wtg
