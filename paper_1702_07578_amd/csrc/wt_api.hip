// C ABI (include/wt.h): argument checks, sizing, output binding, workspace
// planning and the launch sequence of a build.  No device memory is allocated
// here; every buffer comes from the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "wt_internal.h"

namespace wtg {

static inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }
static inline uint64_t cdiv64(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

static inline uint64_t words_per_level(uint64_t n) { return align_up(cdiv64(n, 64), 8); }
// directory chunks of a level of nb 512-bit blocks: at least one, which also
// writes the level's final rank entry when the level is empty
static inline uint32_t dir_chunks_of(uint64_t nb) { return (uint32_t)std::max<uint64_t>(1, cdiv64(nb, kDirChunk)); }
static inline uint64_t rank_stride(uint64_t n) { return align_up(words_per_level(n) / 8 + 1, 16); }
static inline uint64_t sel_stride(uint64_t n) { return align_up(cdiv64(n, WT_SEL_SPACING) + 1, 16); }

static uint32_t log2_floor(uint64_t x)
{
    uint32_t r = 0;
    while (x > 1) {
        x >>= 1;
        r++;
    }
    return r;
}

static int check_args(uint64_t n, uint32_t b, uint32_t L, uint32_t kind)
{
    if (b != 1 && b != 2 && b != 4) return WT_EINVAL;
    if (L > 32) return WT_EINVAL;
    if (n >= (1ull << 32)) return WT_EINVAL;
    if (kind != WT_TREE && kind != WT_MATRIX) return WT_EINVAL;
    if (kind == WT_TREE && L > WT_MAX_TREE_LEVELS) return WT_ENOTSUP;
    return WT_OK;
}

// Output layout, offsets relative to a 256-byte aligned start.
struct OutLayout {
    uint64_t W, rs, ss;
    uint64_t o_bits, o_zeros, o_rank, o_sel0, o_sel1, o_status, total;
};

static OutLayout out_layout(uint64_t n, uint32_t L)
{
    OutLayout o;
    o.W = words_per_level(n);
    o.rs = rank_stride(n);
    o.ss = sel_stride(n);
    uint64_t off = 0;
    o.o_bits = off;
    off = align_up(off + (uint64_t)L * o.W * 8, 256);
    o.o_zeros = off;
    off = align_up(off + (uint64_t)L * 8, 256);
    o.o_rank = off;
    off = align_up(off + (uint64_t)L * o.rs * 4, 256);
    o.o_sel0 = off;
    off = align_up(off + (uint64_t)L * o.ss * 4, 256);
    o.o_sel1 = off;
    off = align_up(off + (uint64_t)L * o.ss * 4, 256);
    o.o_status = off;
    off = align_up(off + 4, 256);
    o.total = off;
    return o;
}

// Workspace plan of one text: descriptor fields and region offsets relative
// to the text's region start.
struct WsPlan {
    TextDesc d;  // pointer fields hold offsets until bound
    uint64_t o_H, o_TP, o_CS, o_KBid, o_KBpi, o_HT, o_seqA, o_seqB, o_tmpb, o_tmpr, o_walk,
        o_bc, o_cs;
    uint64_t bytes;
};

static int plan_text(uint64_t n, uint32_t b, uint32_t L, uint32_t kind, const wt_tune *tune,
                     WsPlan &p)
{
    int rc = check_args(n, b, L, kind);
    if (rc != WT_OK) return rc;
    std::memset(&p, 0, sizeof(p));
    TextDesc &d = p.d;
    d.n = n;
    d.b = b;
    d.L = L;
    d.kind = kind;
    uint32_t K = (tune && tune->group_bits) ? std::min<uint32_t>(tune->group_bits, kMaxGroupBits)
                                            : kMaxGroupBits;
    if (K == 0) K = 1;
    if (L > 0 && K > L) K = L;
    d.K = K;
    d.G = (L == 0) ? 1 : (uint32_t)cdiv64(L, K);
    // tiles are always kWaveTile symbols (the scatter holds one in registers)
    d.log2S = log2_floor(kWaveTile);
    const uint32_t ls = d.log2S;
    d.ntiles = (uint32_t)cdiv64(n, 1ull << ls);
    // consecutive tiles form a range, walked in order by one workgroup
    const uint32_t target = (tune && tune->grid) ? tune->grid : kTargetRanges;
    d.R = (uint32_t)std::max<uint64_t>(1, cdiv64(d.ntiles, target));
    d.nranges = (uint32_t)cdiv64(d.ntiles, d.R);
    d.nchunks = (uint32_t)cdiv64(d.nranges, kBorderChunk);
    d.W = words_per_level(n);
    d.nb = d.W / 8;
    d.rank_stride = rank_stride(n);
    d.sel_stride = sel_stride(n);
    d.dir_chunks = dir_chunks_of(d.nb);

    const uint64_t nk = 1ull << K;
    const bool deep_wt = (kind == WT_TREE && d.G > 1);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    p.o_H = take((uint64_t)d.nranges * nk * 4);
    p.o_TP = take((uint64_t)d.nranges * nk * 4);
    p.o_CS = take((uint64_t)d.nchunks * nk * 4);
    p.o_KBid = take((2 * nk) * 4);
    p.o_KBpi = take((2 * nk) * 4);
    p.o_HT = take((2 * nk) * 4);
    p.o_seqA = take(d.G > 1 ? n * b : 0);
    p.o_seqB = take(d.G > 2 ? n * b : 0);
    p.o_tmpb = take(deep_wt ? (uint64_t)(L - K) * d.W * 8 : 0);
    p.o_tmpr = take(deep_wt ? (uint64_t)(L - K) * d.rank_stride * 4 : 0);
    p.o_walk = take(deep_wt ? walk_off(K, L) * 4 : 0);
    p.o_bc = take((uint64_t)L * d.nb * 2);
    p.o_cs = take((uint64_t)L * d.dir_chunks * 4);
    p.bytes = off;
    return WT_OK;
}

static void bind_ws(WsPlan &p, uint8_t *base)
{
    TextDesc &d = p.d;
    d.H = (uint32_t *)(base + p.o_H);
    d.TP = (uint32_t *)(base + p.o_TP);
    d.CS = (uint32_t *)(base + p.o_CS);
    d.KBid = (uint32_t *)(base + p.o_KBid);
    d.KBpi = (uint32_t *)(base + p.o_KBpi);
    d.HT = (uint32_t *)(base + p.o_HT);
    d.seqA = base + p.o_seqA;
    d.seqB = base + p.o_seqB;
    d.tmp_bits = (uint64_t *)(base + p.o_tmpb);
    d.tmp_rank = (uint32_t *)(base + p.o_tmpr);
    d.walk = (uint32_t *)(base + p.o_walk);
    d.dir_bc = (uint16_t *)(base + p.o_bc);
    d.dir_cs = (uint32_t *)(base + p.o_cs);
}

static void bind_out(TextDesc &d, const wt_levels &o)
{
    d.bits = o.bits;
    d.zeros = o.zeros;
    d.rank_dir = o.rank_dir;
    d.sel0 = o.sel0;
    d.sel1 = o.sel1;
    d.status = o.status;
}

static int check_out(const wt_levels *out, uint64_t n, uint32_t L, uint32_t kind)
{
    if (!out) return WT_EINVAL;
    if (out->n != n || out->lg_sigma != L || out->kind != kind) return WT_EINVAL;
    if (!out->status) return WT_EINVAL;
    if (L > 0 && (!out->bits || !out->zeros || !out->rank_dir || !out->sel0 || !out->sel1))
        return WT_EINVAL;
    if (out->words_per_level != words_per_level(n) || out->rank_stride != rank_stride(n) ||
        out->sel_stride != sel_stride(n))
        return WT_EINVAL;
    return WT_OK;
}

// Launch counts of a set of texts (one build or a batch).
struct Sched {
    uint32_t nd = 0;
    uint32_t gmax = 0;
    uint32_t nranges = 0, nchunks = 0;
    std::vector<bool> any_levels;  // per group
    std::vector<uint32_t> rmask;   // per group: bit 0 last group of a text, bit 1 not last
    uint32_t bmask = 0;            // symbol widths present
    uint32_t pmask = 0;            // scatter instantiations (GroupLaunch::pmask)
    uint32_t dir_items = 0, tmpdir_items = 0, max_levels = 0, max_tmp_levels = 0;
    std::vector<uint32_t> walk_items;  // per step
    uint32_t gather_items = 0;
    // host prefix arrays (nd + 1 each), only needed for nd > 1
    std::vector<uint32_t> b_ranges, b_chunks, b_dir, b_tmpdir, b_gather;
    std::vector<std::vector<uint32_t>> b_walk;
};

static int schedule(const std::vector<TextDesc> &ds, Sched &s)
{
    s.nd = (uint32_t)ds.size();
    uint32_t max_steps = 0;
    for (const TextDesc &d : ds) {
        s.gmax = std::max(s.gmax, d.G);
        if (d.kind == WT_TREE && d.G > 1) max_steps = std::max(max_steps, d.L - d.K - 1);
    }
    s.any_levels.assign(s.gmax, false);
    s.rmask.assign(s.gmax, 0u);
    s.walk_items.assign(max_steps, 0);
    s.b_walk.assign(max_steps, {});
    auto push = [](std::vector<uint32_t> &v, uint64_t &acc, uint64_t add) {
        v.push_back((uint32_t)acc);
        acc += add;
    };
    uint64_t at = 0, ac = 0, adir = 0, atmp = 0, aga = 0;
    std::vector<uint64_t> aw(max_steps, 0);
    for (const TextDesc &d : ds) {
        const bool deep = (d.kind == WT_TREE && d.G > 1);
        push(s.b_ranges, at, d.nranges);
        push(s.b_chunks, ac, d.nchunks);
        push(s.b_dir, adir, (uint64_t)d.L * d.dir_chunks);
        push(s.b_tmpdir, atmp, deep ? (uint64_t)(d.L - d.K) * d.dir_chunks : 0);
        push(s.b_gather, aga, deep ? (uint64_t)(d.L - d.K) * (d.W / kGatherWords) : 0);
        for (uint32_t st = 0; st < max_steps; st++) {
            const bool has = deep && (d.K + st + 1 < d.L);
            push(s.b_walk[st], aw[st], has ? (1ull << (d.K + st)) : 0);
        }
        for (uint32_t g = 0; g < d.G; g++) {
            if (group_bits(d, g) > 0) s.any_levels[g] = true;
            s.rmask[g] |= (g + 1 < d.G) ? 2u : 1u;
        }
        s.bmask |= (d.b == 1) ? 1u : (d.b == 2 ? 2u : 4u);
        if (d.pair && d.G > 1) s.pmask |= 8u | 1u;  // group 0 paired, the rest single
        else if (d.pair) s.pmask |= (d.K <= 7) ? 2u : 4u;
        else if (d.nranges) s.pmask |= 1u;
        s.max_levels = std::max(s.max_levels, d.L);
        if (deep) s.max_tmp_levels = std::max(s.max_tmp_levels, d.L - d.K);
    }
    s.b_ranges.push_back((uint32_t)at);
    s.b_chunks.push_back((uint32_t)ac);
    s.b_dir.push_back((uint32_t)adir);
    s.b_tmpdir.push_back((uint32_t)atmp);
    s.b_gather.push_back((uint32_t)aga);
    for (uint32_t st = 0; st < max_steps; st++) s.b_walk[st].push_back((uint32_t)aw[st]);
    const uint64_t lim = 0xFFFFFFFFull;
    if (at > lim || ac > lim || adir > lim || atmp > lim || aga > lim) return WT_ENOTSUP;
    for (uint64_t x : aw)
        if (x > lim) return WT_ENOTSUP;
    s.nranges = (uint32_t)at;
    s.nchunks = (uint32_t)ac;
    s.dir_items = (uint32_t)adir;
    s.tmpdir_items = (uint32_t)atmp;
    s.gather_items = (uint32_t)aga;
    for (uint32_t st = 0; st < max_steps; st++) s.walk_items[st] = (uint32_t)aw[st];
    return WT_OK;
}

// Device copies of the prefix arrays (batch only); all null for one text.
struct DevBases {
    const uint32_t *ranges = nullptr, *chunks = nullptr, *dir = nullptr, *tmpdir = nullptr,
                   *gather = nullptr;
    std::vector<const uint32_t *> walk;
};

static hipError_t run_build(const TextDesc *d_descs, const Sched &s, const DevBases &b,
                            uint32_t grid_cap, const LaunchCtx &ctx)
{
    hipError_t e;
    for (uint32_t g = 0; g < s.gmax; g++) {
        GroupLaunch gl;
        gl.pmask = s.pmask;
        gl.g = g;
        gl.nd = s.nd;
        gl.range_bases = b.ranges;
        gl.chunk_bases = b.chunks;
        gl.nranges = s.nranges;
        gl.nchunks = s.nchunks;
        gl.any_levels = s.any_levels[g];
        gl.bmask = s.bmask;
        gl.rmask = s.rmask[g];
        gl.grid_cap = grid_cap;
        if ((e = launch_group(d_descs, gl, ctx)) != hipSuccess) return e;
    }
    if (s.max_tmp_levels) {
        if ((e = launch_dirs(d_descs, b.tmpdir, s.nd, s.tmpdir_items, s.max_tmp_levels, true,
                             grid_cap, ctx)) != hipSuccess)
            return e;
        for (uint32_t st = 0; st < s.walk_items.size(); st++)
            if ((e = launch_walk(d_descs, b.walk.empty() ? nullptr : b.walk[st], s.nd,
                                 s.walk_items[st], st, ctx)) != hipSuccess)
                return e;
        if ((e = launch_gather(d_descs, b.gather, s.nd, s.gather_items, ctx)) != hipSuccess)
            return e;
    }
    return launch_dirs(d_descs, b.dir, s.nd, s.dir_items, s.max_levels, false, grid_cap, ctx);
}

static int build_one(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes,
                     uint32_t lg_sigma, wt_levels *out, void *d_ws, size_t ws_bytes,
                     const wt_tune *tune, const LaunchCtx &ctx)
{
    WsPlan p;
    int rc = plan_text(n, sym_bytes, lg_sigma, kind, tune, p);
    if (rc != WT_OK) return rc;
    if ((rc = check_out(out, n, lg_sigma, kind)) != WT_OK) return rc;
    if (n > 0 && !d_text) return WT_EINVAL;
    if ((uintptr_t)d_text % sym_bytes) return WT_EINVAL;
    if (!d_ws) return WT_EINVAL;
    const uint64_t need = p.bytes + align_up(sizeof(TextDesc), 256) + 256;
    if (ws_bytes < need) return WT_ENOSPACE;
    uint8_t *base = (uint8_t *)align_up((uintptr_t)d_ws, 256);
    TextDesc *d_desc = (TextDesc *)base;
    bind_ws(p, base + align_up(sizeof(TextDesc), 256));
    p.d.text = d_text;
    bind_out(p.d, *out);
    std::vector<TextDesc> ds{p.d};
    Sched s;
    if ((rc = schedule(ds, s)) != WT_OK) return rc;
    if (launch_init(p.d, d_desc, ctx) != hipSuccess) return WT_EHIP;
    DevBases b;
    b.walk.assign(s.walk_items.size(), nullptr);
    const uint32_t cap = tune ? tune->persist : 0;
    if (run_build(d_desc, s, b, cap, ctx) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

}  // namespace wtg
// the conversion with a launch context (defined with the C entry points)
static int convert_one(const wt_levels *src, wt_levels *dst, void *d_ws, size_t ws_bytes,
                       const wtg::LaunchCtx &ctx);
namespace wtg {

// workspace head of a one-pass pair build: the two descriptors
static size_t pair_head_bytes() { return align_up(2 * sizeof(TextDesc), 256); }

// Both structures of one text.  With one group, the WT's build also writes
// the WM from the same tile splits (the two differ only in where each run of
// a level goes: prefix order or bit-reversed order, Section 5.1); with more
// groups, the WM is built and the WT gathered from its intervals (the
// conversion), which costs less than a second multi-group build.
static int pair_one(const void *d_text, uint64_t n, uint32_t b, uint32_t L, wt_levels *wt,
                    wt_levels *wm, void *d_ws, size_t ws_bytes, const wt_tune *tune, const LaunchCtx &ctx)
{
    WsPlan p;
    int rc = plan_text(n, b, L, WT_TREE, tune, p);
    if (rc != WT_OK) return rc;
    if ((rc = check_out(wt, n, L, WT_TREE)) != WT_OK) return rc;
    if ((rc = check_out(wm, n, L, WT_MATRIX)) != WT_OK) return rc;
    if (n > 0 && !d_text) return WT_EINVAL;
    if ((uintptr_t)d_text % b) return WT_EINVAL;
    if (!d_ws) return WT_EINVAL;
    if (L == 0) {
        if ((rc = build_one(WT_TREE, d_text, n, b, L, wt, d_ws, ws_bytes, tune, ctx)) != WT_OK) return rc;
        return build_one(WT_MATRIX, d_text, n, b, L, wm, d_ws, ws_bytes, tune, ctx);
    }
    if (p.d.G != 1) {
        if ((rc = build_one(WT_MATRIX, d_text, n, b, L, wm, d_ws, ws_bytes, tune, ctx)) != WT_OK) return rc;
        // the build's workspace is free again once the stream passes it
        return ::convert_one(wm, wt, d_ws, ws_bytes, ctx);
    }
    if (ws_bytes < p.bytes + pair_head_bytes() + 256) return WT_ENOSPACE;
    uint8_t *base = (uint8_t *)align_up((uintptr_t)d_ws, 256);
    // the two descriptors next to each other (the WT's, then the WM's)
    TextDesc *d_desc = (TextDesc *)base, *d_desc2 = d_desc + 1;
    bind_ws(p, base + pair_head_bytes());
    p.d.text = d_text;
    bind_out(p.d, *wt);
    TextDesc d2 = p.d;  // the WM, for its directories
    d2.kind = WT_MATRIX;
    bind_out(d2, *wm);
    p.d.pair = 1;
    p.d.bits2 = wm->bits;
    p.d.zeros2 = wm->zeros;
    p.d.status2 = wm->status;
    std::vector<TextDesc> ds{p.d};
    Sched s;
    if ((rc = schedule(ds, s)) != WT_OK) return rc;
    if (launch_init_pair(p.d, d2, d_desc, ctx) != hipSuccess) return WT_EHIP;
    DevBases bb;
    bb.walk.assign(s.walk_items.size(), nullptr);
    const uint32_t cap = tune ? tune->persist : 0;
    if (run_build(d_desc, s, bb, cap, ctx) != hipSuccess) return WT_EHIP;
    // the WM's directories after the WT's: the two share the workspace's
    // block-count arrays
    if (launch_dirs(d_desc2, nullptr, 1, s.dir_items, s.max_levels, false, cap, ctx) != hipSuccess)
        return WT_EHIP;
    return WT_OK;
}

static size_t pair_ws_bytes(uint64_t n, uint32_t b, uint32_t L, const wt_tune *tune)
{
    WsPlan p;
    if (plan_text(n, b, L, WT_TREE, tune, p) != WT_OK) return 0;
    if (p.d.G == 1 && L > 0) return p.bytes + pair_head_bytes() + 256;
    WsPlan q;
    if (plan_text(n, b, L, WT_MATRIX, tune, q) != WT_OK) return 0;
    size_t need = q.bytes + align_up(sizeof(TextDesc), 256) + 256;
    if (L > 0) {
        const size_t conv = wt_convert_workspace_bytes(n, L);
        if (conv == 0) return 0;
        need = std::max(need, conv);
    } else {
        need = std::max<size_t>(need, p.bytes + align_up(sizeof(TextDesc), 256) + 256);
    }
    return need;
}

}  // namespace wtg

using namespace wtg;

extern "C" {

size_t wt_output_bytes(uint64_t n, uint32_t lg_sigma)
{
    if (lg_sigma > 32 || n >= (1ull << 32)) return 0;
    return out_layout(n, lg_sigma).total + 256;
}

size_t wt_workspace_bytes_tuned(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_kind kind,
                                const wt_tune *tune)
{
    WsPlan p;
    if (plan_text(n, sym_bytes, lg_sigma, (uint32_t)kind, tune, p) != WT_OK) return 0;
    return p.bytes + align_up(sizeof(TextDesc), 256) + 256;
}

size_t wt_workspace_bytes(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_kind kind)
{
    return wt_workspace_bytes_tuned(n, sym_bytes, lg_sigma, kind, nullptr);
}

int wt_levels_bind(wt_levels *out, void *d_mem, size_t bytes, uint64_t n, uint32_t lg_sigma,
                   wt_kind kind)
{
    if (!out || !d_mem) return WT_EINVAL;
    if (lg_sigma > 32 || n >= (1ull << 32)) return WT_EINVAL;
    if (kind != WT_TREE && kind != WT_MATRIX) return WT_EINVAL;
    OutLayout o = out_layout(n, lg_sigma);
    uint8_t *base = (uint8_t *)align_up((uintptr_t)d_mem, 256);
    if ((uint64_t)(base - (uint8_t *)d_mem) + o.total > bytes) return WT_ENOSPACE;
    out->n = n;
    out->lg_sigma = lg_sigma;
    out->kind = (uint32_t)kind;
    out->words_per_level = o.W;
    out->rank_stride = o.rs;
    out->sel_stride = o.ss;
    out->bits = (uint64_t *)(base + o.o_bits);
    out->zeros = (uint64_t *)(base + o.o_zeros);
    out->rank_dir = (uint32_t *)(base + o.o_rank);
    out->sel0 = (uint32_t *)(base + o.o_sel0);
    out->sel1 = (uint32_t *)(base + o.o_sel1);
    out->status = (int32_t *)(base + o.o_status);
    return WT_OK;
}

int wt_build_tuned(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes,
                   uint32_t lg_sigma, wt_levels *out, void *d_ws, size_t ws_bytes,
                   const wt_tune *tune, hipStream_t stream)
{
    LaunchCtx ctx{stream, nullptr, nullptr};
    return build_one(kind, d_text, n, sym_bytes, lg_sigma, out, d_ws, ws_bytes, tune, ctx);
}

size_t wt_pair_workspace_bytes(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma)
{
    return pair_ws_bytes(n, sym_bytes, lg_sigma, nullptr);
}

size_t wt_pair_workspace_bytes_tuned(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, const wt_tune *tune)
{
    return pair_ws_bytes(n, sym_bytes, lg_sigma, tune);
}

int wt_pair_build(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_levels *wt,
                  wt_levels *wm, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    LaunchCtx ctx{stream, nullptr, nullptr};
    return pair_one(d_text, n, sym_bytes, lg_sigma, wt, wm, d_ws, ws_bytes, nullptr, ctx);
}

int wt_pair_build_tuned(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_levels *wt,
                        wt_levels *wm, void *d_ws, size_t ws_bytes, const wt_tune *tune, hipStream_t stream)
{
    LaunchCtx ctx{stream, nullptr, nullptr};
    return pair_one(d_text, n, sym_bytes, lg_sigma, wt, wm, d_ws, ws_bytes, tune, ctx);
}

}  // extern "C"

// Workspace of the allocation-free pair build: a file-scope device array, one
// copy per GPU (loaded with this file's code object, held until the process
// ends).  In host code its name is only a host-side stand-in: the device
// address of the current GPU's copy comes from hipGetSymbolAddress, taken
// once per device and kept here; only that address is handed to kernels.
static __device__ __align__(256) uint8_t scratch[WT_NOALLOC_SCRATCH_BYTES];
static constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices];

// address of the current device's scratch, or null if the runtime refuses
static void *scratch_for_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

extern "C" {

int wt_pair_build_noalloc(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma, wt_levels *wt,
                          wt_levels *wm, hipStream_t stream)
{
    // sizes are checked before the device is touched
    const size_t need = pair_ws_bytes(n, sym_bytes, lg_sigma, nullptr);
    if (need == 0) return WT_EINVAL;
    if (need > (size_t)WT_NOALLOC_SCRATCH_BYTES) return WT_ENOSPACE;
    void *ws = scratch_for_current_device();
    if (!ws) return WT_EHIP;
    LaunchCtx ctx{stream, nullptr, nullptr};
    return pair_one(d_text, n, sym_bytes, lg_sigma, wt, wm, ws, (size_t)WT_NOALLOC_SCRATCH_BYTES, nullptr, ctx);
}

int wt_build(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
             wt_levels *out, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    return wt_build_tuned(WT_TREE, d_text, n, sym_bytes, lg_sigma, out, d_ws, ws_bytes, nullptr,
                          stream);
}

int wm_build(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
             wt_levels *out, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    return wt_build_tuned(WT_MATRIX, d_text, n, sym_bytes, lg_sigma, out, d_ws, ws_bytes, nullptr,
                          stream);
}

static int query_common(const wt_levels *s, int op, const uint32_t *d_sym, const uint64_t *d_arg,
                        uint64_t m, void *d_out, hipStream_t stream)
{
    if (!s || (m > 0 && (!d_arg || !d_out || (op != 0 && !d_sym)))) return WT_EINVAL;
    if (s->kind != WT_TREE && s->kind != WT_MATRIX) return WT_EINVAL;
    if (s->lg_sigma > 32 || s->n >= (1ull << 32)) return WT_EINVAL;
    if (m >= (1ull << 38)) return WT_EINVAL;
    LaunchCtx ctx{stream, nullptr, nullptr};
    return launch_queries(*s, op, d_sym, d_arg, m, d_out, ctx) == hipSuccess ? WT_OK : WT_EHIP;
}

int wt_access(const wt_levels *s, const uint64_t *d_pos, uint64_t m, uint32_t *d_out,
              hipStream_t stream)
{
    return query_common(s, 0, nullptr, d_pos, m, d_out, stream);
}

int wt_rank(const wt_levels *s, const uint32_t *d_sym, const uint64_t *d_pos, uint64_t m,
            uint64_t *d_out, hipStream_t stream)
{
    return query_common(s, 1, d_sym, d_pos, m, d_out, stream);
}

int wt_select(const wt_levels *s, const uint32_t *d_sym, const uint64_t *d_k, uint64_t m,
              uint64_t *d_out, hipStream_t stream)
{
    return query_common(s, 2, d_sym, d_k, m, d_out, stream);
}

// ---- conversion between the WT and the WM, and the position map ----------

// Workspace of a conversion or a position-map build: the interval walk of
// levels 0..L, one descriptor (for the directory kernels), and the directory
// scratch of either the L destination levels or U.
struct ConvWs {
    uint32_t *tab;
    TextDesc *desc;
    uint16_t *dir_bc;
    uint32_t *dir_cs;
    uint64_t *zeros;  // scratch Z and status for U's descriptor
    int32_t *status;
};

static uint64_t conv_plan(uint64_t n, uint32_t L, uint8_t *base, ConvWs *w)
{
    const uint64_t ulen = n + (1ull << L);
    const uint64_t nb = words_per_level(n) / 8, nbu = words_per_level(ulen) / 8;
    const uint64_t bc = std::max<uint64_t>((uint64_t)L * nb, nbu);
    const uint64_t cs = std::max<uint64_t>((uint64_t)L * dir_chunks_of(nb), dir_chunks_of(nbu));
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + std::max<uint64_t>(bytes, 1), 256);
        return o;
    };
    const uint64_t o_tab = take(3ull * ((2ull << L) - 1) * 4);
    const uint64_t o_desc = take(sizeof(TextDesc));
    const uint64_t o_bc = take(bc * 2);
    const uint64_t o_cs = take(cs * 4);
    const uint64_t o_z = take(16);
    if (w) {
        w->tab = (uint32_t *)(base + o_tab);
        w->desc = (TextDesc *)(base + o_desc);
        w->dir_bc = (uint16_t *)(base + o_bc);
        w->dir_cs = (uint32_t *)(base + o_cs);
        w->zeros = (uint64_t *)(base + o_z);
        w->status = (int32_t *)(base + o_z + 8);
    }
    return off + 256;
}

static bool view_ok(const wt_levels *v)
{
    return v && check_out(v, v->n, v->lg_sigma, v->kind) == WT_OK;
}

size_t wt_convert_workspace_bytes(uint64_t n, uint32_t lg_sigma)
{
    if (lg_sigma > WT_MAX_TREE_LEVELS || n >= (1ull << 32)) return 0;
    return conv_plan(n, lg_sigma, nullptr, nullptr);
}

// descriptor that lets the directory kernels run over `levels` bit vectors
static TextDesc dir_desc(uint64_t n, uint32_t levels, uint64_t *bits, uint32_t *rank_dir, uint32_t *sel0,
                         uint32_t *sel1, uint64_t *zeros, int32_t *status, const ConvWs &w)
{
    TextDesc d{};
    d.n = n;
    d.b = 1;
    d.L = levels;
    d.kind = WT_MATRIX;
    d.K = levels ? levels : 1;
    d.G = 1;
    d.W = words_per_level(n);
    d.nb = d.W / 8;
    d.rank_stride = rank_stride(n);
    d.sel_stride = sel_stride(n);
    d.dir_chunks = dir_chunks_of(d.nb);
    d.bits = bits;
    d.zeros = zeros;
    d.rank_dir = rank_dir;
    d.sel0 = sel0;
    d.sel1 = sel1;
    d.status = status;
    d.dir_bc = w.dir_bc;
    d.dir_cs = w.dir_cs;
    return d;
}

int wt_convert(const wt_levels *src, wt_levels *dst, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    LaunchCtx ctx{stream, nullptr, nullptr};
    return convert_one(src, dst, d_ws, ws_bytes, ctx);
}

}  // extern "C"

static int convert_one(const wt_levels *src, wt_levels *dst, void *d_ws, size_t ws_bytes,
                       const wtg::LaunchCtx &ctx)
{
    if (!view_ok(src) || !view_ok(dst) || !d_ws) return WT_EINVAL;
    if (src->n != dst->n || src->lg_sigma != dst->lg_sigma || src->kind == dst->kind) return WT_EINVAL;
    const uint64_t n = src->n;
    const uint32_t L = src->lg_sigma;
    if (L > WT_MAX_TREE_LEVELS) return WT_ENOTSUP;
    const size_t need = wt_convert_workspace_bytes(n, L);
    if (need == 0) return WT_ENOTSUP;
    if (ws_bytes < need) return WT_ENOSPACE;
    ConvWs w;
    conv_plan(n, L, (uint8_t *)align_up((uintptr_t)d_ws, 256), &w);
    // the descriptor (and the destination's status and Z cleared) first
    TextDesc d = dir_desc(n, L, dst->bits, dst->rank_dir, dst->sel0, dst->sel1, dst->zeros, dst->status, w);
    if (launch_init(d, w.desc, ctx) != hipSuccess) return WT_EHIP;
    if (L == 0) return WT_OK;
    if (n > 0) {
        if (launch_convert_walk(*src, w.tab, L, true, ctx) != hipSuccess) return WT_EHIP;
        if (launch_convert_gather(*src, *dst, w.tab, ctx) != hipSuccess) return WT_EHIP;
    }
    if (launch_dirs(w.desc, nullptr, 1, L * d.dir_chunks, L, false, 0, ctx) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

extern "C" {

// merge of partial structures: the walk of every piece (levels 0..L), the
// (prefix, piece) starts of every level, the pieces' views, a descriptor and
// the directory scratch of the whole
static uint64_t merge_plan(uint64_t n, uint32_t L, uint32_t count, uint8_t *base, ConvWs *w,
                           uint32_t **mtab, wt_levels **views, uint64_t *stride)
{
    const uint64_t st = 3ull * ((2ull << L) - 1);
    const uint64_t nb = words_per_level(n) / 8;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + std::max<uint64_t>(bytes, 1), 256);
        return o;
    };
    const uint64_t o_tab = take(st * count * 4);
    const uint64_t o_m = take((uint64_t)count * ((1ull << L) - 1) * 4);
    const uint64_t o_v = take((uint64_t)count * sizeof(wt_levels));
    const uint64_t o_desc = take(sizeof(TextDesc));
    const uint64_t o_bc = take((uint64_t)L * nb * 2);
    const uint64_t o_cs = take((uint64_t)L * dir_chunks_of(nb) * 4);
    if (w) {
        w->tab = (uint32_t *)(base + o_tab);
        w->desc = (TextDesc *)(base + o_desc);
        w->dir_bc = (uint16_t *)(base + o_bc);
        w->dir_cs = (uint32_t *)(base + o_cs);
        w->zeros = nullptr;
        w->status = nullptr;
        *mtab = (uint32_t *)(base + o_m);
        *views = (wt_levels *)(base + o_v);
        *stride = st;
    }
    return off + 256;
}

size_t wt_merge_workspace_bytes(uint64_t n, uint32_t lg_sigma, uint32_t count)
{
    if (lg_sigma > WT_MAX_TREE_LEVELS || n >= (1ull << 32) || count == 0) return 0;
    // tables of count * 2^(lg_sigma + 1) entries per piece set
    if ((uint64_t)count << (lg_sigma + 1) > (1ull << 30)) return 0;
    return merge_plan(n, lg_sigma, count, nullptr, nullptr, nullptr, nullptr, nullptr);
}

int wt_merge(const wt_levels *parts, uint32_t count, wt_levels *dst, void *d_ws, size_t ws_bytes,
             hipStream_t stream)
{
    if (!parts || count == 0 || !view_ok(dst) || !d_ws) return WT_EINVAL;
    uint64_t total = 0;
    for (uint32_t c = 0; c < count; c++) {
        if (!view_ok(&parts[c]) || parts[c].kind != dst->kind || parts[c].lg_sigma != dst->lg_sigma)
            return WT_EINVAL;
        total += parts[c].n;
    }
    if (total != dst->n) return WT_EINVAL;
    const uint32_t L = dst->lg_sigma;
    const size_t need = wt_merge_workspace_bytes(dst->n, L, count);
    if (need == 0) return WT_ENOTSUP;
    if (ws_bytes < need) return WT_ENOSPACE;
    ConvWs w;
    uint32_t *mtab;
    wt_levels *views;
    uint64_t stride;
    merge_plan(dst->n, L, count, (uint8_t *)align_up((uintptr_t)d_ws, 256), &w, &mtab, &views, &stride);
    LaunchCtx ctx{stream, nullptr, nullptr};
    // the pieces' views to the device (the host array may go once this returns)
    if (hipMemcpyAsync(views, parts, count * sizeof(wt_levels), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return WT_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return WT_EHIP;
    TextDesc d = dir_desc(dst->n, L, dst->bits, dst->rank_dir, dst->sel0, dst->sel1, dst->zeros,
                          dst->status, w);
    if (launch_init(d, w.desc, ctx) != hipSuccess) return WT_EHIP;
    if (L == 0) return WT_OK;
    if (launch_merge(views, count, w.tab, stride, mtab, *dst, ctx) != hipSuccess) return WT_EHIP;
    if (launch_dirs(w.desc, nullptr, 1, L * d.dir_chunks, L, false, 0, ctx) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

// ---- construction by sorting ------------------------------------------------

// chunks: at most kTargetRanges, and few enough that a level's (prefix, chunk)
// table stays within 2^23 entries (the prefix sum's two-level reach)
static void ps_chunks(uint64_t n, uint32_t L, uint32_t *P, uint64_t *C)
{
    const uint64_t pmax = std::max<uint64_t>(1, std::min<uint64_t>(kTargetRanges, (1ull << 23) >> (L ? L - 1 : 0)));
    const uint64_t c = align_up(std::max<uint64_t>(cdiv64(std::max<uint64_t>(n, 1), pmax), 1), 256);
    *C = c;
    *P = (uint32_t)std::max<uint64_t>(1, cdiv64(n, c));
}

struct PsWs {
    TextDesc *desc;
    uint16_t *dir_bc;
    uint32_t *dir_cs;
    uint32_t *H0, *H1, *bsum;
    void *sorted;
};

static uint64_t ps_plan(uint64_t n, uint32_t b, uint32_t L, uint8_t *base, PsWs *w)
{
    uint32_t P;
    uint64_t C;
    ps_chunks(n, L, &P, &C);
    const uint64_t nb = words_per_level(n) / 8;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = off;
        off = align_up(off + std::max<uint64_t>(bytes, 1), 256);
        return o;
    };
    const uint64_t o_desc = take(sizeof(TextDesc));
    const uint64_t o_bc = take((uint64_t)L * nb * 2);
    const uint64_t o_cs = take((uint64_t)L * dir_chunks_of(nb) * 4);
    const uint64_t o_h0 = take(((uint64_t)P << L) * 4);
    const uint64_t o_h1 = take(((uint64_t)P << L) * 4);
    const uint64_t o_bs = take(4096 * 4);
    const uint64_t o_sorted = take(n * b + 16);
    if (w) {
        w->desc = (TextDesc *)(base + o_desc);
        w->dir_bc = (uint16_t *)(base + o_bc);
        w->dir_cs = (uint32_t *)(base + o_cs);
        w->H0 = (uint32_t *)(base + o_h0);
        w->H1 = (uint32_t *)(base + o_h1);
        w->bsum = (uint32_t *)(base + o_bs);
        w->sorted = base + o_sorted;
    }
    return off + 256;
}

size_t wt_ps_workspace_bytes(uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma)
{
    if (check_args(n, sym_bytes, lg_sigma, WT_MATRIX) != WT_OK || lg_sigma > kPsMaxLevels) return 0;
    return ps_plan(n, sym_bytes, lg_sigma, nullptr, nullptr);
}

int wt_ps_build(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
                wt_levels *out, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    int rc = check_args(n, sym_bytes, lg_sigma, kind);
    if (rc != WT_OK) return rc;
    if (lg_sigma > kPsMaxLevels) return WT_ENOTSUP;
    if ((rc = check_out(out, n, lg_sigma, kind)) != WT_OK) return rc;
    if (!d_ws || (n > 0 && !d_text)) return WT_EINVAL;
    if (((uintptr_t)d_text % sym_bytes) != 0) return WT_EINVAL;
    const size_t need = wt_ps_workspace_bytes(n, sym_bytes, lg_sigma);
    if (ws_bytes < need) return WT_ENOSPACE;
    const uint32_t L = lg_sigma;
    PsWs w;
    ps_plan(n, sym_bytes, L, (uint8_t *)align_up((uintptr_t)d_ws, 256), &w);
    ConvWs cw{};
    cw.dir_bc = w.dir_bc;
    cw.dir_cs = w.dir_cs;
    LaunchCtx ctx{stream, nullptr, nullptr};
    TextDesc d = dir_desc(n, L, out->bits, out->rank_dir, out->sel0, out->sel1, out->zeros, out->status, cw);
    if (launch_init(d, w.desc, ctx) != hipSuccess) return WT_EHIP;
    if (L == 0) return WT_OK;
    PsDesc p{};
    p.text = d_text;
    p.n = n;
    p.b = sym_bytes;
    p.L = L;
    p.kind = kind;
    ps_chunks(n, L, &p.P, &p.C);
    p.H0 = w.H0;
    p.H1 = w.H1;
    p.bsum = w.bsum;
    p.sorted = w.sorted;
    p.bits = out->bits;
    p.W = out->words_per_level;
    p.zeros = out->zeros;
    p.status = out->status;
    if (launch_ps(p, ctx) != hipSuccess) return WT_EHIP;
    if (launch_dirs(w.desc, nullptr, 1, L * d.dir_chunks, L, false, 0, ctx) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

uint64_t wt_export_pool_words(uint64_t n, uint32_t lg_sigma)
{
    if (lg_sigma > WT_MAX_TREE_LEVELS || lg_sigma == 0) return 0;
    // a node of h bits takes ceil(h/64) <= h/64 + 1 words; a level holds n bits
    return (uint64_t)lg_sigma * cdiv64(n, 64) + ((1ull << lg_sigma) - 1);
}

int wt_export_nodes(const wt_levels *wt, uint64_t *d_nodes, uint64_t *d_pool, uint64_t pool_words,
                    void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    if (!view_ok(wt) || wt->kind != WT_TREE || !d_nodes || !d_pool || !d_ws) return WT_EINVAL;
    const uint32_t L = wt->lg_sigma;
    if (L > WT_MAX_TREE_LEVELS) return WT_ENOTSUP;
    if (L == 0) return WT_OK;
    if (pool_words < wt_export_pool_words(wt->n, L)) return WT_ENOSPACE;
    const size_t need = wt_convert_workspace_bytes(wt->n, L);
    if (need == 0) return WT_ENOTSUP;
    if (ws_bytes < need) return WT_ENOSPACE;
    ConvWs w;
    conv_plan(wt->n, L, (uint8_t *)align_up((uintptr_t)d_ws, 256), &w);
    LaunchCtx ctx{stream, nullptr, nullptr};
    if (launch_convert_walk(*wt, w.tab, L, false, ctx) != hipSuccess) return WT_EHIP;
    // pool words past the nodes' runs are left as they are
    const uint64_t used = wt_export_pool_words(wt->n, L);
    if (launch_export_nodes(*wt, w.tab, d_nodes, d_pool, used, ctx) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

struct PmLayout {
    uint64_t ulen, uw, rs, ss, o_rd, o_s0, o_s1, o_x, total;
};

static PmLayout pm_layout(uint64_t n, uint32_t L)
{
    PmLayout p;
    p.ulen = n + (1ull << L);
    p.uw = words_per_level(p.ulen);
    p.rs = rank_stride(p.ulen);
    p.ss = sel_stride(p.ulen);
    p.o_rd = align_up(p.uw * 8, 256);
    p.o_s0 = p.o_rd + align_up(p.rs * 4, 256);
    p.o_s1 = p.o_s0 + align_up(p.ss * 4, 256);
    p.o_x = p.o_s1 + align_up(p.ss * 4, 256);
    p.total = p.o_x + align_up(std::max<uint64_t>((1ull << L) - 1, 1) * 4, 256);
    return p;
}

size_t wt_posmap_bytes(uint64_t n, uint32_t lg_sigma)
{
    if (lg_sigma > WT_MAX_TREE_LEVELS || n + (1ull << lg_sigma) >= (1ull << 32)) return 0;
    return pm_layout(n, lg_sigma).total + 256;
}

int wt_posmap_bind(wt_posmap *m, void *d_mem, size_t bytes, uint64_t n, uint32_t lg_sigma)
{
    if (!m || !d_mem) return WT_EINVAL;
    const size_t need = wt_posmap_bytes(n, lg_sigma);
    if (need == 0) return WT_ENOTSUP;
    if (bytes < need) return WT_ENOSPACE;
    const PmLayout p = pm_layout(n, lg_sigma);
    uint8_t *base = (uint8_t *)align_up((uintptr_t)d_mem, 256);
    m->n = n;
    m->lg_sigma = lg_sigma;
    m->reserved = 0;
    m->u_len = p.ulen;
    m->u_words = p.uw;
    m->rank_stride = p.rs;
    m->sel_stride = p.ss;
    m->U = (uint64_t *)base;
    m->rank_dir = (uint32_t *)(base + p.o_rd);
    m->sel0 = (uint32_t *)(base + p.o_s0);
    m->sel1 = (uint32_t *)(base + p.o_s1);
    m->X = (uint32_t *)(base + p.o_x);
    return WT_OK;
}

static bool posmap_ok(const wt_posmap *m)
{
    if (!m || !m->U) return false;
    const PmLayout p = pm_layout(m->n, m->lg_sigma);
    return m->u_len == p.ulen && m->u_words == p.uw && m->rank_stride == p.rs && m->sel_stride == p.ss;
}

int wt_posmap_build(const wt_levels *s, wt_posmap *m, void *d_ws, size_t ws_bytes, hipStream_t stream)
{
    if (!view_ok(s) || !posmap_ok(m) || !d_ws) return WT_EINVAL;
    if (s->n != m->n || s->lg_sigma != m->lg_sigma) return WT_EINVAL;
    const uint32_t L = s->lg_sigma;
    if (wt_posmap_bytes(s->n, L) == 0) return WT_ENOTSUP;
    const size_t need = wt_convert_workspace_bytes(s->n, L);
    if (need == 0) return WT_ENOTSUP;
    if (ws_bytes < need) return WT_ENOSPACE;
    ConvWs w;
    conv_plan(s->n, L, (uint8_t *)align_up((uintptr_t)d_ws, 256), &w);
    LaunchCtx ctx{stream, nullptr, nullptr};
    // the walk down to the leaves: symbol counts, and the WM starts (X)
    if (launch_convert_walk(*s, w.tab, L, true, ctx) != hipSuccess) return WT_EHIP;
    TextDesc d = dir_desc(m->u_len, 1, m->U, m->rank_dir, m->sel0, m->sel1, w.zeros, w.status, w);
    if (launch_init(d, w.desc, ctx) != hipSuccess) return WT_EHIP;
    if (launch_posmap_fill(*m, w.tab, ctx) != hipSuccess) return WT_EHIP;
    if (launch_dirs(w.desc, nullptr, 1, d.dir_chunks, 1, false, 0, ctx) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

int wt_posmap_query(const wt_posmap *m, uint32_t level, const uint64_t *d_pos, uint64_t count,
                    uint64_t *d_out, hipStream_t stream)
{
    if (!posmap_ok(m)) return WT_EINVAL;
    if (count > 0 && (!d_pos || !d_out)) return WT_EINVAL;
    LaunchCtx ctx{stream, nullptr, nullptr};
    return launch_posmap_query(*m, level, d_pos, count, d_out, ctx) == hipSuccess ? WT_OK : WT_EHIP;
}

int wt_get_status(const wt_levels *s, hipStream_t stream)
{
    if (!s || !s->status) return WT_EINVAL;
    int32_t st = 0;
    if (hipMemcpyAsync(&st, s->status, sizeof(st), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return WT_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return WT_EHIP;
    return st;
}

const char *wt_strerror(int code)
{
    switch (code) {
    case WT_OK: return "ok";
    case WT_EINVAL: return "invalid argument";
    case WT_ENOSPACE: return "buffer too small";
    case WT_ERANGE: return "symbol out of range for lg_sigma";
    case WT_EHIP: return "HIP runtime error";
    case WT_ENOTSUP: return "unsupported configuration";
    default: return "unknown error";
    }
}

// ---- batch -----------------------------------------------------------------

struct BatchPlan {
    std::vector<WsPlan> plans;
    std::vector<int64_t> partner;  // for a WT paired with the WM of the same text: the WM's index
    uint64_t o_desc, o_bases, n_bases, o_texts, total;
};

// WT and WM items of the same text (same pointer, length, width, levels) are
// built as a pair.  One group of levels: the WT's descriptor writes both, the
// WM's keeps its outputs and directories but gets no build work items.  More
// groups (of the full width): the WM's descriptor writes the WT's levels of
// group 0 as well and seeds its walk; the WT's gets no scatter work and
// gathers its deeper levels from the WM's (its temporary levels are the
// WM's levels).
static void pair_items(const wt_batch_item *items, uint32_t count, BatchPlan &bp)
{
    bp.partner.assign(count, -1);
    using Key = std::tuple<uintptr_t, uint64_t, uint32_t, uint32_t>;
    std::map<Key, std::vector<uint32_t>> wms;  // unpaired WM items per text, in item order
    for (uint32_t j = count; j-- > 0;)
        if (items[j].kind == WT_MATRIX)
            wms[Key((uintptr_t)items[j].d_text, items[j].n, items[j].sym_bytes, items[j].lg_sigma)].push_back(j);
    for (uint32_t i = 0; i < count; i++) {
        const TextDesc &di = bp.plans[i].d;
        if (items[i].kind != WT_TREE || di.L == 0 || di.n == 0) continue;
        if (di.G > 1 && di.K != kMaxGroupBits) continue;
        auto it = wms.find(Key((uintptr_t)items[i].d_text, items[i].n, items[i].sym_bytes, items[i].lg_sigma));
        if (it == wms.end() || it->second.empty()) continue;
        const uint32_t j = it->second.back();
        it->second.pop_back();
        if (di.G == 1) {
            bp.partner[i] = j;  // the WT writes the WM too
            bp.plans[i].d.pair = 1;
            bp.plans[j].d.nranges = 0;
            bp.plans[j].d.nchunks = 0;
        } else {
            bp.partner[j] = i;  // the WM writes the WT's first group
            bp.plans[j].d.pair = 1;
            bp.plans[i].d.nranges = 0;
            bp.plans[i].d.nchunks = 0;
        }
    }
}

static int plan_batch(const wt_batch_item *items, uint32_t count, const wt_tune *tune,
                      BatchPlan &bp, Sched *sched)
{
    if (!items || count == 0) return WT_EINVAL;
    bp.plans.resize(count);
    std::vector<TextDesc> ds(count);
    uint64_t off_texts = 0;
    std::vector<uint64_t> text_off(count);
    for (uint32_t i = 0; i < count; i++) {
        int rc = plan_text(items[i].n, items[i].sym_bytes, items[i].lg_sigma, items[i].kind, tune,
                           bp.plans[i]);
        if (rc != WT_OK) return rc;
        text_off[i] = off_texts;
        off_texts = align_up(off_texts + bp.plans[i].bytes, 256);
    }
    pair_items(items, count, bp);
    for (uint32_t i = 0; i < count; i++) ds[i] = bp.plans[i].d;
    Sched s;
    int rc = schedule(ds, s);
    if (rc != WT_OK) return rc;
    uint64_t nb = 5ull * (count + 1) + (uint64_t)s.walk_items.size() * (count + 1);
    bp.o_desc = 0;
    bp.o_bases = align_up((uint64_t)count * sizeof(TextDesc), 256);
    bp.n_bases = nb;
    bp.o_texts = align_up(bp.o_bases + nb * 4, 256);
    bp.total = bp.o_texts + off_texts + 256;
    // stash text offsets in the plan (reuse the bytes field as offset)
    for (uint32_t i = 0; i < count; i++) bp.plans[i].bytes = text_off[i];
    if (sched) *sched = std::move(s);
    return WT_OK;
}

size_t wt_batch_workspace_bytes(const wt_batch_item *items, uint32_t count, const wt_tune *tune)
{
    BatchPlan bp;
    if (plan_batch(items, count, tune, bp, nullptr) != WT_OK) return 0;
    return bp.total;
}

// Binds every text of the batch to the workspace and builds the host image
// of descriptors and work-item prefix arrays (uploaded by prepare).
struct BatchImage {
    std::vector<uint8_t> img;
    const TextDesc *d_descs;
    DevBases db;
    Sched s;
};

static int batch_image(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                       const wt_tune *tune, BatchImage &bi)
{
    BatchPlan bp;
    int rc = plan_batch(items, count, tune, bp, &bi.s);
    if (rc != WT_OK) return rc;
    if (!d_ws) return WT_EINVAL;
    if (ws_bytes < bp.total) return WT_ENOSPACE;
    uint8_t *base = (uint8_t *)align_up((uintptr_t)d_ws, 256);
    std::vector<TextDesc> ds(count);
    for (uint32_t i = 0; i < count; i++) {
        const wt_batch_item &it = items[i];
        if ((rc = check_out(it.out, it.n, it.lg_sigma, it.kind)) != WT_OK) return rc;
        if (it.n > 0 && !it.d_text) return WT_EINVAL;
        if ((uintptr_t)it.d_text % it.sym_bytes) return WT_EINVAL;
        WsPlan &p = bp.plans[i];
        bind_ws(p, base + bp.o_texts + p.bytes);
        p.d.text = it.d_text;
        bind_out(p.d, *it.out);
        ds[i] = p.d;
    }
    // pairs: the primary writes the partner's outputs; a deep WT partner takes
    // the WM's levels as its temporary levels
    for (uint32_t i = 0; i < count; i++) {
        if (bp.partner[i] < 0) continue;
        TextDesc &d = ds[i];
        TextDesc &o = ds[bp.partner[i]];
        d.bits2 = o.bits;
        d.zeros2 = o.zeros;
        d.status2 = o.status;
        if (d.kind == WT_MATRIX) {
            d.walk2 = o.walk;
            o.tmp_bits = d.bits + (uint64_t)d.K * d.W;
            o.tmp_rank = d.rank_dir + (uint64_t)d.K * d.rank_stride;
        }
    }
    bi.img.assign(bp.o_texts, 0);
    std::memcpy(bi.img.data() + bp.o_desc, ds.data(), count * sizeof(TextDesc));
    uint32_t *bases = (uint32_t *)(bi.img.data() + bp.o_bases);
    uint32_t *dbases = (uint32_t *)(base + bp.o_bases);
    uint64_t k = 0;
    auto put = [&](const std::vector<uint32_t> &v) {
        std::memcpy(bases + k, v.data(), v.size() * 4);
        const uint32_t *p = dbases + k;
        k += v.size();
        return p;
    };
    bi.db.ranges = put(bi.s.b_ranges);
    bi.db.chunks = put(bi.s.b_chunks);
    bi.db.dir = put(bi.s.b_dir);
    bi.db.tmpdir = put(bi.s.b_tmpdir);
    bi.db.gather = put(bi.s.b_gather);
    for (auto &w : bi.s.b_walk) bi.db.walk.push_back(put(w));
    bi.d_descs = (const TextDesc *)(base + bp.o_desc);
    return WT_OK;
}

static int batch_prepare(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                         const wt_tune *tune, hipStream_t stream)
{
    BatchImage bi;
    int rc = batch_image(items, count, d_ws, ws_bytes, tune, bi);
    if (rc != WT_OK) return rc;
    uint8_t *base = (uint8_t *)align_up((uintptr_t)d_ws, 256);
    // on the caller's stream, so that the copy waits for nothing else; the
    // host image lives until the stream has passed it
    if (hipMemcpyAsync(base, bi.img.data(), bi.img.size(), hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return WT_EHIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

static int batch_launch(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                        const wt_tune *tune, const LaunchCtx &ctx)
{
    BatchImage bi;
    int rc = batch_image(items, count, d_ws, ws_bytes, tune, bi);
    if (rc != WT_OK) return rc;
    if (launch_init_batch(bi.d_descs, count, ctx) != hipSuccess) return WT_EHIP;
    const uint32_t cap = tune ? tune->persist : 0;
    if (run_build(bi.d_descs, bi.s, bi.db, cap, ctx) != hipSuccess) return WT_EHIP;
    return WT_OK;
}

int wt_batch_prepare(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                     const wt_tune *tune, hipStream_t stream)
{
    return batch_prepare(items, count, d_ws, ws_bytes, tune, stream);
}

int wt_batch_launch(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                    const wt_tune *tune, hipStream_t stream)
{
    LaunchCtx ctx{stream, nullptr, nullptr};
    return batch_launch(items, count, d_ws, ws_bytes, tune, ctx);
}

int wt_batch_build(const wt_batch_item *items, uint32_t count, void *d_ws, size_t ws_bytes,
                   const wt_tune *tune, hipStream_t stream)
{
    int rc = batch_prepare(items, count, d_ws, ws_bytes, tune, stream);
    if (rc != WT_OK) return rc;
    LaunchCtx ctx{stream, nullptr, nullptr};
    return batch_launch(items, count, d_ws, ws_bytes, tune, ctx);
}

// ---- profiling ---------------------------------------------------------------

struct ProfState {
    hipStream_t stream;
    std::vector<hipEvent_t> ev;
    std::vector<uint32_t> kid;
    bool failed = false;
};

static void prof_after(void *user, uint32_t kid)
{
    ProfState *ps = (ProfState *)user;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
        ps->failed = true;
        return;
    }
    if (hipEventRecord(e, ps->stream) != hipSuccess) ps->failed = true;
    ps->ev.push_back(e);
    ps->kid.push_back(kid);
}

int wt_build_profiled(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes,
                      uint32_t lg_sigma, wt_levels *out, void *d_ws, size_t ws_bytes,
                      const wt_tune *tune, hipStream_t stream, double *ms_by_kernel,
                      uint32_t *launches_by_kernel, uint32_t n_ids)
{
    if (!ms_by_kernel || !launches_by_kernel || n_ids < KID_COUNT_) return WT_EINVAL;
    ProfState ps;
    ps.stream = stream;
    hipEvent_t e0;
    if (hipEventCreate(&e0) != hipSuccess) return WT_EHIP;
    if (hipEventRecord(e0, stream) != hipSuccess) return WT_EHIP;
    LaunchCtx ctx{stream, prof_after, &ps};
    int rc = build_one(kind, d_text, n, sym_bytes, lg_sigma, out, d_ws, ws_bytes, tune, ctx);
    if (hipEventSynchronize(ps.ev.empty() ? e0 : ps.ev.back()) != hipSuccess) rc = WT_EHIP;
    if (rc == WT_OK && !ps.failed) {
        hipEvent_t prev = e0;
        for (size_t i = 0; i < ps.ev.size(); i++) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, prev, ps.ev[i]) != hipSuccess) rc = WT_EHIP;
            ms_by_kernel[ps.kid[i]] += ms;
            launches_by_kernel[ps.kid[i]] += 1;
            prev = ps.ev[i];
        }
    }
    (void)hipEventDestroy(e0);
    for (hipEvent_t e : ps.ev) (void)hipEventDestroy(e);
    if (ps.failed && rc == WT_OK) rc = WT_EHIP;
    return rc;
}

const char *wt_kernel_name(uint32_t id)
{
    static const char *names[] = {"init",      "hist",      "chunk_sum", "borders",
                                  "scatter",   "dir_count", "dir_scan",  "dir_write",
                                  "walk",      "gather",    "query"};
    return id < sizeof(names) / sizeof(names[0]) ? names[id] : "unknown";
}

}  // extern "C"

// ---- caller-event recording ----------------------------------------------------

namespace {
struct RecState {
    hipStream_t stream;
    hipEvent_t *events;
    uint32_t *ids;
    uint32_t cap;
    uint32_t count;
    bool failed;
};

void rec_after(void *user, uint32_t kid)
{
    RecState *r = (RecState *)user;
    if (r->count < r->cap) {
        if (hipEventRecord(r->events[r->count], r->stream) != hipSuccess) r->failed = true;
        r->ids[r->count] = kid;
    }
    r->count++;
}
}  // namespace

extern "C" int wt_pair_build_recorded(const void *d_text, uint64_t n, uint32_t sym_bytes, uint32_t lg_sigma,
                                      wt_levels *wt, wt_levels *wm, void *d_ws, size_t ws_bytes,
                                      hipStream_t stream, hipEvent_t *events, uint32_t *kernel_ids,
                                      uint32_t capacity, uint32_t *recorded)
{
    if ((capacity && (!events || !kernel_ids)) || !recorded) return WT_EINVAL;
    RecState r{stream, events, kernel_ids, capacity, 0, false};
    LaunchCtx ctx{stream, rec_after, &r};
    int rc = pair_one(d_text, n, sym_bytes, lg_sigma, wt, wm, d_ws, ws_bytes, nullptr, ctx);
    *recorded = r.count;
    if (rc == WT_OK && r.failed) rc = WT_EHIP;
    return rc;
}

extern "C" int wt_build_recorded(wt_kind kind, const void *d_text, uint64_t n, uint32_t sym_bytes,
                                 uint32_t lg_sigma, wt_levels *out, void *d_ws, size_t ws_bytes,
                                 const wt_tune *tune, hipStream_t stream, hipEvent_t *events,
                                 uint32_t *kernel_ids, uint32_t capacity, uint32_t *recorded)
{
    if ((capacity && (!events || !kernel_ids)) || !recorded) return WT_EINVAL;
    RecState r{stream, events, kernel_ids, capacity, 0, false};
    LaunchCtx ctx{stream, rec_after, &r};
    int rc = build_one(kind, d_text, n, sym_bytes, lg_sigma, out, d_ws, ws_bytes, tune, ctx);
    *recorded = r.count;
    if (rc == WT_OK && r.failed) rc = WT_EHIP;
    return rc;
}
