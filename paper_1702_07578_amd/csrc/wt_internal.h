// Internal declarations of the GPU library: per-text build descriptor, plan
// of the workspace, constants and the kernel launchers shared between the
// translation units.  Not part of the public ABI (include/wt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wt.h"

namespace wtg {

// The histogram runs 256 threads (4 wave64s) per range of consecutive tiles:
// with 8 interleaved copies of 256 keys per wave that is 32 KiB of LDS, five
// workgroups per CU.
constexpr uint32_t kTileThreads = 256;
constexpr uint32_t kTileWaves = kTileThreads / 64;
// The scatter gives every wave a range of its own and walks it one tile at a
// time; a tile is at most kWaveTile symbols (held in registers, 32 per lane).
constexpr uint32_t kWaveTile = 2048;
// Largest number of levels handled by one pass over the (re-ordered) text.
constexpr uint32_t kMaxGroupBits = 8;
// Ranges per text when the text is long enough: three rounds of the 4096
// scatter waves resident at four per SIMD on 256 CUs (the five-wave pair
// kernel measured no faster with other counts).
constexpr uint32_t kTargetRanges = 12288;
// Ranges per chunk of the column scans over the range histograms.
constexpr uint32_t kBorderChunk = 32;
constexpr uint32_t kGatherWords = 1;  // words per thread of the WT gather (divides W, a multiple of 8)
// Directory: 512-bit blocks, chunks of kDirChunk blocks per workgroup.
constexpr uint32_t kDirChunk = 1024;

// Everything a kernel needs to know about one text of a build.  Lives in the
// workspace (device memory); one entry per text of a batch.
struct TextDesc {
    // input
    const void *text;
    uint64_t n;
    uint32_t b;     // bytes per symbol (1, 2, 4)
    uint32_t L;     // levels
    uint32_t kind;  // WT_TREE / WT_MATRIX
    uint32_t K;     // levels per group (pass over the text)
    uint32_t G;     // number of groups
    uint32_t log2S; // log2 symbols per tile
    uint32_t ntiles;
    uint32_t R;          // tiles per range; one scatter wave walks a range in order
    uint32_t nchunks;    // chunks of kBorderChunk ranges (column scan)
    uint32_t dir_chunks; // directory chunks per level
    uint32_t nranges;
    uint64_t W;  // words per level
    uint64_t nb; // 512-bit blocks per level (W / 8)
    uint64_t rank_stride, sel_stride;
    // outputs
    uint64_t *bits;
    uint64_t *zeros;
    uint32_t *rank_dir;
    uint32_t *sel0, *sel1;
    int32_t *status;
    // workspace
    uint32_t *H;   // [nranges][2^K] per-range histogram of the group key
    uint32_t *TP;  // [nranges][2^K] range-exclusive prefix of H per key
    uint32_t *CS;  // [nchunks][2^K] chunk sums
    uint32_t *KBid, *KBpi; // [2^(K+1)] key bases per group level, prefix / reversed order
    uint32_t *HT;  // [2^(K+1)] per group level key totals
    void *seqA, *seqB;     // reordered text between groups (n symbols each)
    uint64_t *tmp_bits;    // WT only, G > 1: WM levels K..L-1, [L-K][W]
    uint32_t *tmp_rank;    // [L-K][rank_stride]
    uint32_t *walk;        // WT only, G > 1: per level l in [K,L): 3 x 2^l u32
    uint16_t *dir_bc;      // [Lall][nb] ones per 512-bit block
    uint32_t *dir_cs;      // [Lall][dir_chunks] chunk sums -> prefixes
    // pair build: the other structure of the same text is written as well,
    // from the same splits of group 0, into these outputs (a WT desc of one
    // group writes its WM; a WM desc of several groups writes its WT's levels
    // of group 0 and seeds that WT's interval walk, walk2; the WT gathers its
    // deeper levels from the WM's)
    uint32_t pair;
    uint64_t *bits2;
    uint64_t *zeros2;
    int32_t *status2;
    uint32_t *walk2;
};

// Construction by sorting (the second strategy): text cut into P chunks of C
// symbols; H0/H1 hold chunk histograms [prefix][chunk] (2^L * P entries
// each), bsum the prefix sum's block sums, sorted the sorted copy (n symbols).
constexpr uint32_t kPsMaxLevels = 12;
struct PsDesc {
    const void *text;
    uint64_t n;
    uint32_t b, L, kind, P;
    uint64_t C;
    uint32_t *H0, *H1, *bsum;
    void *sorted;
    uint64_t *bits;  // level l at bits + l * W
    uint64_t W;
    uint64_t *zeros;
    int32_t *status;
};

// Host-side plan of one text: the descriptor plus workspace size.
struct Plan {
    TextDesc d;
    size_t ws_bytes;  // bytes of workspace used by this text (excluding descriptor)
};

// level a of a group: number of keys 2^a, table offset 2^a - 1
__host__ __device__ inline uint32_t lvl_off(uint32_t a) { return (1u << a) - 1u; }

__host__ __device__ inline uint32_t group_bits(const TextDesc &d, uint32_t g)
{
    uint32_t done = g * d.K;
    if (done >= d.L) return 0;
    uint32_t r = d.L - done;
    return r < d.K ? r : d.K;
}

// walk table of level l (WT deep levels): wm_start, len, wt_start
__host__ __device__ inline uint64_t walk_off(uint32_t K, uint32_t l)
{
    // sum over k in [K, l) of 3 * 2^k
    return 3ull * ((1ull << l) - (1ull << K));
}

// kernel ids for profiling
enum KernelId : uint32_t {
    KID_INIT = 0,
    KID_HIST,
    KID_CHUNK_SUM,
    KID_BORDERS,
    KID_SCATTER,
    KID_DIR_COUNT,
    KID_DIR_SCAN,  // no longer launched (the chunk scan is part of the write); kept so ids stay stable
    KID_DIR_WRITE,
    KID_WALK,
    KID_GATHER,
    KID_QUERY,
    KID_COUNT_
};

// Launch hook: called after every kernel launch (profiling); may be null.
struct LaunchCtx {
    hipStream_t stream;
    void (*after)(void *user, uint32_t kid);
    void *user;
};

// Launchers (wt_build.hip, wt_dir.hip, wt_query.hip)
struct GroupLaunch {
    uint32_t g;
    uint32_t nd;
    const uint32_t *range_bases;  // device, nd + 1 entries (unused when nd == 1)
    const uint32_t *chunk_bases;
    uint32_t nranges;  // total range items of the launch
    uint32_t nchunks;  // total chunk items
    bool any_levels;   // some text has at least one level in this group
    uint32_t bmask;    // symbol widths present: bit 0 (1 byte), 1 (2 bytes), 2 (4 bytes)
    uint32_t rmask;    // bit 0: some text ends with group g; bit 1: some text goes on
    uint32_t grid_cap; // 0: one workgroup per item
    // scatter instantiations to launch: bit 0 single structures, bit 1 pairs
    // (WT and WM of one text, one group) of at most 7 levels, bit 2 pairs of
    // 8, bit 3 pairs whose text goes on to more groups (group 0 only)
    uint32_t pmask = 1;
};

hipError_t launch_init(const TextDesc &d, TextDesc *d_dst, const LaunchCtx &ctx);
hipError_t launch_init_pair(const TextDesc &d, const TextDesc &d2, TextDesc *d_dst, const LaunchCtx &ctx);
hipError_t launch_init_batch(const TextDesc *d_descs, uint32_t nd, const LaunchCtx &ctx);
hipError_t launch_group(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx);
hipError_t launch_scatter(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx);
hipError_t launch_walk(const TextDesc *d_descs, const uint32_t *bases, uint32_t nd,
                       uint32_t nitems, uint32_t step, const LaunchCtx &ctx);
hipError_t launch_gather(const TextDesc *d_descs, const uint32_t *bases, uint32_t nd,
                         uint32_t nitems, const LaunchCtx &ctx);
hipError_t launch_dirs(const TextDesc *d_descs, const uint32_t *bases, uint32_t nd, uint32_t nitems,
                       uint32_t max_levels, bool tmp, uint32_t grid_cap, const LaunchCtx &ctx);
hipError_t launch_convert_walk(const wt_levels &src, uint32_t *d_tab, uint32_t levels,
                               bool need_wm_starts, const LaunchCtx &ctx);
hipError_t launch_convert_gather(const wt_levels &src, const wt_levels &dst, const uint32_t *d_tab,
                                 const LaunchCtx &ctx);
hipError_t launch_merge(const wt_levels *d_parts, uint32_t count, uint32_t *d_tabs, uint64_t stride,
                        uint32_t *d_mtab, const wt_levels &dst, const LaunchCtx &ctx);
hipError_t launch_export_nodes(const wt_levels &wt, const uint32_t *d_tab, uint64_t *d_nodes,
                               uint64_t *d_pool, uint64_t pool_words, const LaunchCtx &ctx);
hipError_t launch_ps(const PsDesc &d, const LaunchCtx &ctx);
hipError_t launch_posmap_fill(const wt_posmap &m, const uint32_t *d_tab, const LaunchCtx &ctx);
hipError_t launch_posmap_query(const wt_posmap &m, uint32_t level, const uint64_t *d_pos,
                               uint64_t count, uint64_t *d_out, const LaunchCtx &ctx);
hipError_t launch_queries(const wt_levels &s, int op, const uint32_t *d_sym, const uint64_t *d_arg,
                          uint64_t m, void *d_out, const LaunchCtx &ctx);

}  // namespace wtg
