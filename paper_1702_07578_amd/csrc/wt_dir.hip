// Rank/select directories of the level bit vectors.
//
// The paper augments every level with binary rank and select structures
// (Section 2 and Section 5) without fixing a layout.  This library's layout:
//   rank_dir[j]  ones in bits [0, 512 j) of the level, j = 0 .. W/8;
//   sel_b[q]     index of the 512-bit block that holds the (4096 q + 1)-th b
//                among positions < n; 0xFFFFFFFF for q past the last sample.
// Built in two launches per set of levels: ones per block and per chunk of
// 1024 blocks (and the select samples reset), then the block scan that
// writes rank_dir and the select samples, each chunk adding up the counts of
// the chunks before it.
#include "wt_device.h"

namespace wtg {

// levels of a text covered by a directory launch
__device__ inline uint32_t dir_levels(const TextDesc &d, bool tmp)
{
    if (!tmp) return d.L;
    return (d.kind == WT_TREE && d.G > 1) ? d.L - d.K : 0u;
}

__device__ inline const uint64_t *dir_bits(const TextDesc &d, bool tmp, uint32_t l)
{
    return tmp ? d.tmp_bits + (uint64_t)l * d.W : d.bits + (uint64_t)l * d.W;
}

__device__ inline uint32_t *dir_rank(const TextDesc &d, bool tmp, uint32_t l)
{
    return (tmp ? d.tmp_rank : d.rank_dir) + (uint64_t)l * d.rank_stride;
}

// ones per 512-bit block and per chunk
__global__ __launch_bounds__(256) void k_dir_count(const TextDesc *__restrict__ descs,
                                                   const uint32_t *__restrict__ bases, uint32_t nd,
                                                   uint32_t nitems, uint32_t tmp)
{
    __shared__ uint32_t red[256 / 64];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t idx = item - item_base(bases, nd, ti);
        if (d.dir_chunks == 0) continue;
        const uint32_t l = idx / d.dir_chunks, c = idx % d.dir_chunks;
        if (l >= dir_levels(d, tmp)) continue;
        const uint64_t *bits = dir_bits(d, tmp, l);
        uint16_t *bc = d.dir_bc + (uint64_t)l * d.nb;
        // The chunk's blocks as 16-byte units, four per block, lane-
        // interleaved (consecutive lanes read consecutive units); the four
        // lanes of a block add their counts across the quad.
        constexpr uint32_t kUnits = kDirChunk * 4, kIters = kUnits / 256;
        const gmem<ulonglong2> *p = gp((const ulonglong2 *)bits) + (uint64_t)c * kUnits;
        const uint64_t nblk = min((uint64_t)kDirChunk, d.nb - (uint64_t)c * kDirChunk);
        const uint32_t units = (uint32_t)nblk * 4;
        // every load of the thread is issued before the first count: units
        // past the chunk's end re-read its last unit (no branch per load)
        uint32_t x[kIters];
        if (units != 0) {
#pragma unroll
            for (uint32_t r = 0; r < kIters; r++) {
                const uint32_t u = r * 256 + threadIdx.x;
                const ulonglong2 v = load_nt(p + min(u, units - 1));  // each level word is read once here
                x[r] = u < units ? __popcll(v.x) + __popcll(v.y) : 0u;
            }
        } else {
#pragma unroll
            for (uint32_t r = 0; r < kIters; r++) x[r] = 0;
        }
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t r = 0; r < kIters; r++) {
            const uint32_t u = r * 256 + threadIdx.x;
            uint32_t v = x[r];
            v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
            v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
            if ((threadIdx.x & 3) == 0 && u < units) {
                gp(bc)[(uint64_t)c * kDirChunk + (u >> 2)] = (uint16_t)v;
                sum += v;
            }
        }
        // block sum
        for (uint32_t off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t s = 0;
            for (uint32_t i = 0; i < 256 / 64; i++) s += red[i];
            gp(d.dir_cs)[(uint64_t)l * d.dir_chunks + c] = s;
        }
        // the chunk's share of the level's select samples reset to "absent"
        // (the directory write sets the sampled ones)
        if (!tmp) {
            const uint32_t per = (uint32_t)((d.sel_stride + d.dir_chunks - 1) / d.dir_chunks);
            const uint64_t q0 = (uint64_t)c * per, q1 = min((uint64_t)d.sel_stride, q0 + per);
            gmem<uint32_t> *s0 = gp(d.sel0 + (uint64_t)l * d.sel_stride);
            gmem<uint32_t> *s1 = gp(d.sel1 + (uint64_t)l * d.sel_stride);
            for (uint64_t q = q0 + threadIdx.x; q < q1; q += 256) {
                s0[q] = 0xFFFFFFFFu;
                s1[q] = 0xFFFFFFFFu;
            }
        }
        __syncthreads();
    }
}

// block scan of one chunk: rank_dir entries and select samples
__global__ __launch_bounds__(256) void k_dir_write(const TextDesc *__restrict__ descs,
                                                   const uint32_t *__restrict__ bases, uint32_t nd,
                                                   uint32_t nitems, uint32_t tmp)
{
    __shared__ uint32_t wsum[256 / 64], wbefore[256 / 64];
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t idx = item - item_base(bases, nd, ti);
        if (d.dir_chunks == 0) continue;
        const uint32_t l = idx / d.dir_chunks, c = idx % d.dir_chunks;
        if (l >= dir_levels(d, tmp)) continue;
        const uint16_t *bc = d.dir_bc + (uint64_t)l * d.nb;
        uint32_t *rd = dir_rank(d, tmp, l);
        const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
        // each thread: 4 consecutive blocks
        const uint64_t j0 = (uint64_t)c * kDirChunk + tid * 4;
        uint32_t v[4], s = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            v[r] = (j0 + r < d.nb) ? gp(bc)[j0 + r] : 0u;
            s += v[r];
        }
        // ones of the level before this chunk: the sum of the earlier chunks'
        // counts, added up by the whole block
        const gmem<uint32_t> *cs = gp(d.dir_cs + (uint64_t)l * d.dir_chunks);
        uint32_t before = 0;
        // eight loads issued before their adds (indices past c - 1 re-read it)
        for (uint32_t i0 = tid; i0 < c; i0 += 8 * 256) {
            uint32_t xs[8];
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) xs[k] = cs[min(i0 + k * 256, c - 1)];
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) before += i0 + k * 256 < c ? xs[k] : 0u;
        }
        before = wave_incl_scan(before);
        const uint32_t incl = wave_incl_scan(s);
        if (lane == 63) {
            wsum[w] = incl;
            wbefore[w] = before;
        }
        __syncthreads();
        uint32_t pre = 0;
        for (uint32_t ww = 0; ww < 256 / 64; ww++) pre += wbefore[ww];
        // the last chunk also writes the level's final rank entry (its total)
        if (c + 1 == d.dir_chunks && tid == 0) {
            uint32_t all = pre;
            for (uint32_t ww = 0; ww < 256 / 64; ww++) all += wsum[ww];
            gp(rd)[d.nb] = all;
        }
        for (uint32_t ww = 0; ww < w; ww++) pre += wsum[ww];
        pre += incl - s;
        uint32_t *s0 = d.sel0 + (uint64_t)l * d.sel_stride;
        uint32_t *s1 = d.sel1 + (uint64_t)l * d.sel_stride;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint64_t j = j0 + r;
            if (j < d.nb) {
                gp(rd)[j] = pre;
                if (!tmp) {
                    // the (4096 q + 1)-th one lies in block j iff pre < 4096 q + 1 <= pre + v
                    const uint64_t q1 = ((uint64_t)pre + WT_SEL_SPACING - 1) / WT_SEL_SPACING;
                    if (q1 * WT_SEL_SPACING < (uint64_t)pre + v[r]) gp(s1)[q1] = (uint32_t)j;
                    const uint64_t bstart = j * 512;
                    const uint64_t valid = bstart >= d.n ? 0 : min((uint64_t)512, d.n - bstart);
                    const uint64_t zpre = min(bstart, d.n) - pre;
                    const uint64_t zc = valid - v[r];
                    const uint64_t q0 = (zpre + WT_SEL_SPACING - 1) / WT_SEL_SPACING;
                    if (q0 * WT_SEL_SPACING < zpre + zc) gp(s0)[q0] = (uint32_t)j;
                }
            }
            pre += v[r];
        }
        __syncthreads();
    }
}

}  // namespace wtg

namespace wtg {

hipError_t launch_dirs(const TextDesc *d_descs, const uint32_t *bases, uint32_t nd, uint32_t nitems,
                       uint32_t max_levels, bool tmp, uint32_t grid_cap, const LaunchCtx &ctx)
{
    if (max_levels == 0) return hipSuccess;
    if (nitems) {
        uint32_t grid = (grid_cap && nitems > grid_cap) ? grid_cap : nitems;
        hipLaunchKernelGGL(k_dir_count, dim3(grid), dim3(256), 0, ctx.stream, d_descs, bases, nd,
                           nitems, (uint32_t)tmp);
        if (ctx.after) ctx.after(ctx.user, KID_DIR_COUNT);
    }
    if (nitems) {
        uint32_t grid = (grid_cap && nitems > grid_cap) ? grid_cap : nitems;
        hipLaunchKernelGGL(k_dir_write, dim3(grid), dim3(256), 0, ctx.stream, d_descs, bases, nd,
                           nitems, (uint32_t)tmp);
        if (ctx.after) ctx.after(ctx.user, KID_DIR_WRITE);
    }
    return hipGetLastError();
}

}  // namespace wtg
