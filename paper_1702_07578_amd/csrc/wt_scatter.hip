// K2: the stable scatter of a range of tiles into every level of a group.
//
// Algorithm 1 places bit l of every symbol at the next free slot of its
// interval, scanning the text in order, so inside an interval the bits are in
// text order.  Here every wave owns one range of consecutive tiles and walks
// it tile by tile, with no barrier shared with other waves.  A tile (at most
// kWaveTile symbols) sits in the wave's LDS element buffer; it is ordered one
// bit at a time: after splitting by bits 0..a-1 of the group key (zeros
// first, stably) the tile is ordered by its reversed a-bit key (Observation
// 2), so level a's bits of every key form one contiguous run.  Each pass has
// every lane own 8 consecutive positions of each of the tile's 4 blocks: the
// lane packs their bits into one byte of level a's stream, and the ones
// before each of them (its own count plus a wave scan of the lanes' counts)
// give every symbol its place in the next order.  The tile's key counts (one
// LDS histogram) give the length of every run and its start in each level's
// order.  Each run is then copied to its interval start on the level (prefix
// order for the WT, bit-reversed order for the WM; Section 5.1).  Consecutive
// tiles put a key's runs next to each other, so the word a run ends in is
// kept in LDS and completed by the next tile's run of that key; only words
// shared with another range are filled by atomic OR.  With more than one
// group, the split by the group's last bit writes every symbol straight to
// its position in the next group's sequence.
#include <type_traits>

#include "wt_tiles.h"

namespace wtg {

constexpr uint32_t kChunks = kWaveTile / 64;              // chunks of 64 symbols per tile
// state of the word a key's run ends in (that word is G >> 6 of the key's
// next run): none, kept in LDS, or kept with low bits that belong to
// another range (that word is then completed by atomic OR)
constexpr uint8_t kNoPend = 0, kPend = 1, kPendForeign = 2;

// One wave's LDS.  Tables of levels 0..Kg-1 are indexed lvl_off(a) + key.
// REORDER (the group's symbols move on to the next group's sequence) adds
// the tables of level Kg, the finest key.
template <typename E, bool REORDER, bool PAIR, uint32_t KB>
struct WaveSmem {
    static constexpr uint32_t kRunsB = (1u << KB) - 1;  // (level, key) pairs of levels 0..KB-1
    static constexpr uint32_t kKeysB = 1u << KB;        // keys of level KB (the finest)
    static constexpr uint32_t kWordsB = KB * kChunks;   // full output words of one tile
    static constexpr uint32_t kScanPer = (kKeysB + 63) / 64;  // table entries per lane in a scan
    static_assert(kRunsB <= 256, "a run index fits one byte");
    // level a of the tile in order a; while the tables are built (and at a
    // range start) it holds the finest key counts and their prefix sums
    uint64_t bits[KB][kChunks];
    uint64_t pend_v[kRunsB];  // bits so far of the word a key's run ends in
    uint64_t pend_v2[PAIR ? kRunsB : 1];  // the same for the pair's WM
    uint32_t G[kRunsB];       // global start of the key's bits for this tile
    uint32_t G2[PAIR ? kRunsB : 1];       // the same in the pair's WM
    uint16_t h[kRunsB];       // the tile's count of every key
    uint16_t lo[kRunsB];      // start of the key in the tile order of its level
    uint8_t pend[kRunsB];     // state of that word
    uint8_t pend2[PAIR ? kRunsB : 1];
    uint32_t lvw[KB];  // word offset of level a from the group's base pointer
    uint32_t GK[REORDER ? kKeysB : 1];
    uint16_t hK[REORDER ? kKeysB : 1];
    uint16_t loK[REORDER ? kKeysB : 1];
    union alignas(16) {
        E elem[kWaveTile];  // the tile, in its next order (loading and splits)
        struct {            // copy-out, after the splits
            uint8_t kw[kWordsB];   // run of every full word
            // per run: its first full word's bit in the level streams and
            // its word on the output, each minus (64 or 1) x its first word
            // number, so that word q of the numbering takes bit rec.x + 64 q
            // to word rec.y + q
            uint2 rec[kRunsB];
        } co;
    };

    __device__ uint32_t *tmp32() { return (uint32_t *)&bits[0][0]; }              // kKeysB entries
    __device__ uint16_t *tmp16() { return (uint16_t *)(tmp32() + kKeysB); }       // kKeysB + 1 entries
    static_assert(sizeof(uint64_t) * KB * kChunks >= 4 * kKeysB + 2 * (kKeysB + 1),
                  "level buffer too small for the table scratch");
};

// orders the wave's LDS accesses (the wave runs in lockstep; no s_barrier)
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exclusive scan of n <= 64 PER values by one wave, PER consecutive values
// per lane; get(i) / put(i, x, value i); returns the total
template <uint32_t PER, typename Get, typename Put>
__device__ inline uint32_t wave_exscan_n(uint32_t n, Get get, Put put)
{
    const uint32_t lane = lane_id();
    uint32_t v[PER];
    uint32_t s = 0;
#pragma unroll
    for (uint32_t r = 0; r < PER; r++) {
        const uint32_t i = lane * PER + r;
        v[r] = (i < n) ? get(i) : 0u;
        s += v[r];
    }
    const uint32_t incl = wave_incl_scan(s);
    uint32_t ex = incl - s;
#pragma unroll
    for (uint32_t r = 0; r < PER; r++) {
        const uint32_t i = lane * PER + r;
        if (i < n) put(i, ex, v[r]);
        ex += v[r];
    }
    return last_lane(incl);
}

// level of table entry e (entries lvl_off(a) .. lvl_off(a+1)-1 are level a)
__device__ inline uint32_t level_of(uint32_t e) { return 31 - __clz(e + 1); }

// The 64 bits of the tile's level streams starting at bit s (all levels in
// one array, level a at bit a * kWaveTile): three 32-bit words and two
// funnel shifts.  The third word is read only to be shifted out when s is a
// multiple of 32; reads past the last level stay inside the wave's LDS.
__device__ inline uint64_t stream64(const uint64_t *levels, uint32_t s)
{
    const uint32_t *w = (const uint32_t *)levels + (s >> 5);
    const uint32_t d0 = w[0], d1 = w[1], d2 = w[2], sh = s & 31;
    return ((uint64_t)__builtin_amdgcn_alignbit(d2, d1, sh) << 32) | __builtin_amdgcn_alignbit(d1, d0, sh);
}

// the low cnt bits of x, 0 < cnt <= 64
__device__ inline uint64_t low_bits(uint64_t x, uint32_t cnt) { return x & (~0ull >> (64 - cnt)); }

// f(integral_constant<I>) for I = B .. N-1, unrolled at compile time
template <uint32_t I, uint32_t N, typename F>
__device__ __attribute__((always_inline)) inline void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<uint32_t, I>{});
        static_for<I + 1, N>(f);
    }
}

// Base of the bit vectors group g writes: the output levels, or, for the
// WT's later groups, its temporary WM levels; level a of the group starts
// sm.lvw[a] words after it.  Word offsets fit 32 bits (L W < 2^31).
__device__ inline uint64_t *group_base(const TextDesc &d, uint32_t g)
{
    return (d.kind == WT_TREE && g > 0) ? d.tmp_bits : d.bits;
}
__device__ inline uint32_t group_level0(const TextDesc &d, uint32_t g)
{
    return (d.kind == WT_TREE && g > 0) ? (g - 1) * d.K : g * d.K;
}

// G at the first tile of range r: the range prefix of every finest key merged
// upward, plus the key bases of each level.
template <typename E, bool REORDER, bool PAIR, uint32_t KB>
__device__ inline void wave_range_start(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r,
                                        WaveSmem<E, REORDER, PAIR, KB> &sm)
{
    const uint32_t lane = lane_id();
    const uint32_t nk = 1u << Kg;
    const uint32_t *TP = d.TP + (uint64_t)r * nk;
    uint32_t *T = sm.tmp32();
    for (uint32_t k = lane; k < nk; k += 64) T[k] = gp(TP)[k];
    wave_sync();
    for (uint32_t a = Kg; a-- > 0;) {
        const uint32_t *up = (a + 1 == Kg) ? T : sm.G + lvl_off(a + 1);
        for (uint32_t k = lane; k < (1u << a); k += 64)
            sm.G[lvl_off(a) + k] = up[2 * k] + up[2 * k + 1];
        wave_sync();
    }
    for (uint32_t a = 0; a < Kg; a++) {
        const uint32_t *kb = (use_prefix_order(d, g, a, Kg) ? d.KBid : d.KBpi) + lvl_off(a);
        for (uint32_t k = lane; k < (1u << a); k += 64) {
            const uint32_t raw = sm.G[lvl_off(a) + k];
            sm.G[lvl_off(a) + k] = raw + gp(kb)[k];
            // the other structure: bit-reversed order for a WM, prefix order for a WT
            if (PAIR) sm.G2[lvl_off(a) + k] = raw + gp(d.kind == WT_MATRIX ? d.KBid : d.KBpi)[lvl_off(a) + k];
        }
    }
    if (REORDER) {
        const uint32_t *kb = d.KBpi + lvl_off(Kg);
        for (uint32_t k = lane; k < nk; k += 64) sm.GK[k] = T[k] + gp(kb)[k];
    }
    if (lane < Kg) sm.lvw[lane] = (group_level0(d, g) + lane) * (uint32_t)d.W;
    wave_sync();
}

// full words of a run: [ceil(G/64), floor((G+h)/64)), none past word W
__device__ inline uint32_t full_words(uint32_t gs, uint32_t hh, uint32_t W)
{
    const uint32_t f = (gs + 63) >> 6, l = min((uint32_t)(((uint64_t)gs + hh) >> 6), W);
    return l > f ? l - f : 0u;
}

// One output of the scatter: the global starts of the runs, the words kept
// at run ends, and the base of the group's bit vectors.
struct Side {
    uint32_t *G;
    uint8_t *pend;
    uint64_t *pend_v;
    uint64_t *base;
};

// Words that a run of this tile covers completely, all levels at once, by
// plain stores: the full words of all runs are numbered run by run, and the
// lanes take consecutive words.
template <typename E, bool REORDER, bool PAIR, uint32_t KB>
__device__ __attribute__((always_inline)) inline void copy_full_words(const TextDesc &d, uint32_t Kg,
                                                                      WaveSmem<E, REORDER, PAIR, KB> &sm,
                                                                      const Side &sd)
{
    const uint32_t lane = lane_id();
    const uint32_t nr = lvl_off(Kg);
    const uint32_t *G = sd.G;
    const uint32_t W = (uint32_t)d.W;
    constexpr uint32_t kWords = KB * kChunks;  // words of one tile, all levels
    static_assert(kWords % 4 == 0 && kWords / 4 <= 64, "one dword of the word table per lane");
    // run of every word: the run whose first word it is, 0 elsewhere
    if (lane < kWords / 4) ((uint32_t *)sm.co.kw)[lane] = 0u;
    wave_sync();
    const uint32_t total = wave_exscan_n<WaveSmem<E, REORDER, PAIR, KB>::kScanPer>(
        nr, [&](uint32_t e) { return full_words(G[e], sm.h[e], W); },
        [&](uint32_t e, uint32_t x, uint32_t cnt) {
            const uint32_t a = level_of(e), gs = G[e], gw = (gs + 63) >> 6;
            sm.co.rec[e] = make_uint2(a * kWaveTile + sm.lo[e] + ((gw << 6) - gs) - 64u * x,
                                      sm.lvw[a] + gw - x);
            if (cnt != 0) sm.co.kw[x] = (uint8_t)e;
        });
    wave_sync();
    // the lane's words q = lane + 64 i: the run carried forward to each (the
    // largest run index at or before q, scanned row by row), then the stores
    constexpr uint32_t NQ = (kWords + 63) / 64;
    uint32_t rq[NQ], carry = 0;
#pragma unroll
    for (uint32_t i = 0; i < NQ; i++) {
        const uint32_t q = lane + 64 * i;
        const uint32_t k = q < total ? (uint32_t)sm.co.kw[q] : 0u;
        rq[i] = max(wave_incl_max(k), carry);
        carry = last_lane(rq[i]);
    }
    uint64_t *base = sd.base;
#pragma unroll
    for (uint32_t i = 0; i < NQ; i++) {
        const uint32_t q = lane + 64 * i;
        if (q < total) {
            const uint2 r = sm.co.rec[rq[i]];
            gp(base)[r.y + q] = stream64(&sm.bits[0][0], r.x + 64u * q);
        }
    }
    wave_sync();
}

// First and last word of every run (one lane per run, all levels): merged
// with the word kept from earlier tiles of the range, stored when complete,
// kept otherwise.  The pair does both of its outputs in the same pass over
// the runs (the run's length, its place in the streams and its first 64
// bits are the same for both).
template <uint32_t NS, typename E, bool REORDER, bool PAIR, uint32_t KB>
__device__ __attribute__((always_inline)) inline void run_end_words(const TextDesc &d, uint32_t Kg,
                                                                    WaveSmem<E, REORDER, PAIR, KB> &sm,
                                                                    const Side (&sides)[NS])
{
    const uint32_t W = (uint32_t)d.W;
    for (uint32_t e = lane_id(); e < lvl_off(Kg); e += 64) {
        const uint32_t hh = sm.h[e];
        if (hh == 0) continue;
        const uint32_t a = level_of(e);
        const uint32_t sb = a * kWaveTile + sm.lo[e];  // the run's first bit in the streams
        const uint64_t first = stream64(&sm.bits[0][0], sb);
        const uint32_t lvw = sm.lvw[a];
#pragma unroll
        for (uint32_t k = 0; k < NS; k++) {
            const Side &sd = sides[k];
            uint64_t *base = sd.base;
            // positions are below n < 2^32; ge may equal n
            const uint32_t gs = sd.G[e], ge = gs + hh;
            const uint32_t fw = gs >> 6, lw = (ge - 1) >> 6;
            const uint32_t off = gs & 63;
            // the first word, when the run does not cover it from its bit 0
            // to its top (the full words are stored by copy_full_words)
            const bool head = off != 0 || hh < 64;
            const uint32_t cnt = min(hh, 64u - off);  // bits of the run in word fw
            uint64_t hv = low_bits(first, cnt) << off;
            const uint8_t pw = sd.pend[e];
            const bool merge = off != 0 && pw != kNoPend;  // the kept word is fw
            if (merge) hv |= sd.pend_v[e];
            const bool lowok = off == 0 || pw == kPend;
            const bool head_full = off + cnt == 64;
            if (head && head_full && fw < W) {
                if (lowok) gp(base)[lvw + fw] = hv;
                else gatomic_or(&base[lvw + fw], hv);
            }
            // the last word, when it is not the first and the run ends inside it
            const bool tail = lw != fw && (ge & 63) != 0;
            const uint64_t tv = low_bits(stream64(&sm.bits[0][0], sb + ((lw << 6) - gs)), (ge - 1) % 64 + 1);
            const bool keep_head = head && !head_full;
            sd.pend[e] = tail ? kPend : (keep_head ? (lowok ? kPend : kPendForeign) : kNoPend);
            sd.pend_v[e] = tail ? tv : (keep_head ? hv : 0ull);
        }
    }
}

// The split of a tile, with every lane owning runs of 8 consecutive
// positions: block b (of 4) of the tile order holds positions [512 b, 512 b +
// 512), and lane l holds positions 512 b + 8 l + j, j = 0..7, as 8 symbols
// in 2, 4 or 8 32-bit words (1-, 2- or 4-byte symbols).  Per block a lane
// then knows the bits of its own 8 positions: they form one byte of level
// a's word stream (byte 64 b + l), and its ones before each of them come from
// a count of its own plus a wave scan of the lanes' counts.  A symbol at
// position p with r ones before it in the tile goes to base1 + r when its bit
// is one and to p - r when it is zero (base1 = zeros of the bit in the tile).

// One symbol of a lane's run: VCC := its bit (byte J of the flag word f is
// nonzero); the zero's place is K - X1 + i (K > X1 always; v_sad_u32 gives
// |K - X1| + i); dest := bit ? X1 : that; X1 += bit.  VCC is the only scalar
// register written; the sad sits between the compare and the first read of
// VCC, which gives the one wait state a vector read of a vector-written
// scalar register needs on this chip.
template <uint32_t J, uint32_t I>
__device__ __attribute__((always_inline)) inline uint32_t split_step(uint32_t f, uint32_t K, uint32_t &X1)
{
    uint32_t d;
    asm volatile(
        "v_cmp_ne_u32_sdwa vcc, %[f], 0 src0_sel:BYTE_%c[j] src1_sel:DWORD\n\t"
        "v_sad_u32 %[d], %[K], %[x], %[i]\n\t"
        "v_cndmask_b32_e32 %[d], %[d], %[x], vcc\n\t"
        "v_addc_co_u32_e32 %[x], vcc, 0, %[x], vcc"
        : [d] "=&v"(d), [x] "+v"(X1)
        : [f] "v"(f), [K] "v"(K), [j] "n"(J), [i] "n"(I)
        : "vcc");
    return d;
}

// symbol j of a lane's run (j = 0..7) from its 32-bit words q, to the LDS
// element at byte address dd
template <typename E, uint32_t J>
__device__ __attribute__((always_inline)) inline void put_elem(uint32_t dd, const uint32_t *q, const uint32_t *sq)
{
    typedef __attribute__((address_space(3))) uint8_t lds_u8;
    typedef __attribute__((address_space(3))) uint16_t lds_u16;
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    if constexpr (sizeof(E) == 1) {
        // bytes 0 and 2 of a word directly, 1 and 3 from the word rotated by 8
        constexpr uint32_t w = J / 4, by = J % 4;
        const uint32_t x = (by & 1) ? sq[w] : q[w];
        *(lds_u8 *)(uintptr_t)dd = (uint8_t)((by & 2) ? (x >> 16) : x);
    } else if constexpr (sizeof(E) == 2) {
        constexpr uint32_t w = J / 2;
        *(lds_u16 *)(uintptr_t)dd = (uint16_t)((J & 1) ? (q[w] >> 16) : q[w]);
    } else {
        *(lds_u32 *)(uintptr_t)dd = q[J];
    }
}

// Ballots (SPLIT false) or split (SPLIT true) of the tile by bit bp of the
// symbols; level a's word stream goes to sm.bits[a].  The tile's zero count
// of the bit comes from its own count, not from a table.
template <typename E, bool REORDER, bool PAIR, uint32_t KB, bool SPLIT>
__device__ __attribute__((always_inline)) inline void split_pass_lm(uint32_t a, uint32_t bp,
                                                                    WaveSmem<E, REORDER, PAIR, KB> &sm)
{
    static_assert(kWaveTile == 2048, "tiles of 4 blocks of 512");
    typedef __attribute__((address_space(3))) uint8_t lds_u8;
    constexpr uint32_t EB = sizeof(E), NW = 2 * EB;  // 32-bit words of a lane's run
    const uint32_t lane = lane_id();
    const uint32_t ebase = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) E *)sm.elem;
    uint32_t q[4][NW];
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) {
        const uint32_t *src = (const uint32_t *)(sm.elem + 512 * b + 8 * lane);
        if constexpr (NW == 2) {
            const uint2 u = *(const uint2 *)src;
            q[b][0] = u.x;
            q[b][1] = u.y;
        } else {
#pragma unroll
            for (uint32_t i = 0; i < NW; i += 4) {
                const uint4 u = *(const uint4 *)(src + i);
                q[b][i] = u.x;
                q[b][i + 1] = u.y;
                q[b][i + 2] = u.z;
                q[b][i + 3] = u.w;
            }
        }
    }
    // The flags: per 4 symbols one word whose byte j is nonzero iff symbol j's
    // bit bp is set.  For wider symbols, the byte of each symbol that holds
    // bit bp is gathered first (v_perm_b32: one per 4 16-bit symbols, two and
    // an OR per 4 32-bit ones).  Bits past the symbol width (a key above a
    // narrow symbol) are 0.
    const uint32_t m8 = bp >= 8 * EB ? 0u : 0x01010101u << (bp & 7);
    const uint32_t kb = (bp >> 3) & 3u;  // the byte of a symbol that holds bit bp
    uint32_t f[4][2];
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) {
        if constexpr (EB == 1) {
            f[b][0] = q[b][0] & m8;
            f[b][1] = q[b][1] & m8;
        } else if constexpr (EB == 2) {
            // symbols 2w, 2w+1 in word w: byte kb of symbol s is byte 2 s + kb
            // of the word pair
            const uint32_t sel = kb | ((2u + kb) << 8) | ((4u + kb) << 16) | ((6u + kb) << 24);
            f[b][0] = __builtin_amdgcn_perm(q[b][1], q[b][0], sel) & m8;
            f[b][1] = __builtin_amdgcn_perm(q[b][3], q[b][2], sel) & m8;
        } else {
            // symbol s in word s; selector byte 12 gives a zero byte
            const uint32_t lo = kb | ((4u + kb) << 8) | 0x0C0C0000u;
            const uint32_t hi = 0x00000C0Cu | (kb << 16) | ((4u + kb) << 24);
#pragma unroll
            for (uint32_t h = 0; h < 2; h++)
                f[b][h] = (__builtin_amdgcn_perm(q[b][4 * h + 1], q[b][4 * h], lo) |
                           __builtin_amdgcn_perm(q[b][4 * h + 3], q[b][4 * h + 2], hi)) & m8;
        }
    }
    // the lane's byte of the level word in each block (bit j: symbol j), by
    // two 4-way dot products of the flag bytes with 2^j, and its count
    uint32_t cnt[4];
    lds_u8 *lvl = (lds_u8 *)(uintptr_t)(uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint64_t *)sm.bits[a];
    const uint32_t bsh = bp & 7;
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) {
        const uint32_t w = __builtin_amdgcn_udot4(f[b][0], 0x08040201u,
                                                  __builtin_amdgcn_udot4(f[b][1], 0x80402010u, 0u, false), false) >> bsh;
        cnt[b] = __builtin_popcount(w);
        lvl[64 * b + lane] = (uint8_t)w;
    }
    if (!SPLIT) return;
    // ones before the lane's run of each block: two scans of 16-bit pairs
    const uint32_t c01 = cnt[0] | (cnt[1] << 16), c23 = cnt[2] | (cnt[3] << 16);
    const uint32_t i01 = wave_incl_scan(c01), i23 = wave_incl_scan(c23);
    const uint32_t t01 = last_lane(i01), t23 = last_lane(i23);
    const uint32_t e01 = i01 - c01, e23 = i23 - c23;
    const uint32_t T0 = t01 & 0xFFFFu, T01 = T0 + (t01 >> 16), T012 = T01 + (t23 & 0xFFFFu);
    const uint32_t ones = T012 + (t23 >> 16);
    const uint32_t P1[4] = {e01 & 0xFFFFu, T0 + (e01 >> 16), T01 + (e23 & 0xFFFFu), T012 + (e23 >> 16)};
    // Ones go to base1 + (ones before), base1 = zeros of the bit.  The places
    // are LDS byte addresses for 1-byte symbols; for wider ones they are
    // symbol positions plus 16 (so that K - X1 >= 16 - 7 > 0), scaled to
    // addresses at the store.
    const uint32_t bias = EB == 1 ? ebase : 16u;
    const uint32_t X1base = bias + kWaveTile - ones;
    const uint32_t abase = ebase - 16u * EB;  // address of biased position 0 (EB > 1)
    // everything the lane reads is loaded; the writes below may overwrite it
    wave_sync();
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) {
        uint32_t X1 = X1base + P1[b];
        const uint32_t K = X1base + bias + 512 * b + 8 * lane;
        uint32_t sq[2] = {0, 0};
        if constexpr (EB == 1) {
            // bytes 1 and 3 of each word: the low byte and byte 2 of the word
            // rotated by 8.  The rotation is opaque to the compiler, which
            // would otherwise shift byte 3 down on its own instead of storing
            // it from the upper half.
            asm("v_alignbit_b32 %0, %1, %1, 8" : "=v"(sq[0]) : "v"(q[b][0]));
            asm("v_alignbit_b32 %0, %1, %1, 8" : "=v"(sq[1]) : "v"(q[b][1]));
        }
        static_for<0, 8>([&](auto jj) {
            constexpr uint32_t j = decltype(jj)::value;
            const uint32_t pos = split_step<j % 4, j>(f[b][j / 4], K, X1);
            put_elem<E, j>(EB == 1 ? pos : abase + pos * EB, q[b], sq);
        });
    }
}

// One tile of kWaveTile symbols (the text's last tile may be shorter; it is
// padded).
// 16-byte units of a whole tile per lane, and the tile's units as loaded by
// the wave (lane-interleaved: unit u * 64 + lane)
template <typename E>
struct TileUnits {
    static constexpr uint32_t kPerLane = kWaveTile * sizeof(E) / 16 / 64;
    uint4 q[kPerLane];
    __device__ void load(const E *tile)
    {
        const gmem<uint4> *u = gp((const uint4 *)tile);
        const uint32_t lane = lane_id();
#pragma unroll
        for (uint32_t i = 0; i < kPerLane; i++) q[i] = u[i * 64 + lane];
    }
};

// Tiles whose units are loaded one tile ahead (16-byte text, symbols of one
// byte): while a tile is split, the next one is on its way.
template <typename E>
constexpr bool kPrefetch = sizeof(E) == 1;

template <typename E, bool REORDER, bool PAIR, uint32_t KB, typename EIN>
__device__ __attribute__((always_inline)) inline void wave_tile(const TextDesc &d, uint32_t g,
                                                                uint32_t Kg, uint32_t t,
                                                                WaveSmem<E, REORDER, PAIR, KB> &sm,
                                                                TileUnits<EIN> &tu, bool vec,
                                                                bool have, uint32_t t1)
{
    // KEYS: the text's symbols are wider than the tile's elements, which
    // hold the group key alone (the last group of a wider text: its key is
    // the symbol's low Kg <= 8 bits, shift 0)
    constexpr bool KEYS = sizeof(EIN) != sizeof(E);
    static_assert(!KEYS || (sizeof(E) == 1 && !REORDER), "keys are bytes, and only the last group drops the symbol");
    const uint32_t lane = lane_id();
    const uint64_t start = (uint64_t)t * kWaveTile;
    const uint32_t len = (uint32_t)min((uint64_t)kWaveTile, d.n - start);
    const bool padded = len < kWaveTile;
    const uint32_t shift = d.L - g * d.K - Kg;
    const uint32_t nk = 1u << Kg, kmask = nk - 1u;
    const gmem<EIN> *src = gp((const EIN *)seq_in(d, g) + start + lane);
    uint32_t *cnt = sm.tmp32();
    uint16_t *P = sm.tmp16();

    // 1. the tile, in text order, through registers into LDS, counting the
    //    finest keys by LDS atomics on the way (the registers are free while
    //    the tables are built).  With few keys, each key has 2^cb copies of
    //    its counter (lane l adds to copy l mod 2^cb), so that the lanes of
    //    one atomic instruction do not all meet on a handful of words.
    const uint32_t cb = min(4u, KB - Kg), lane_copy = lane & ((1u << cb) - 1u);
    // the lane's counter of key k: byte offset k << (cb + 2) from its copy 0
    char *const cnt_lane = (char *)(cnt + lane_copy);
    const uint32_t csh = cb + 2;
    for (uint32_t k = lane; k < (nk << cb); k += 64) cnt[k] = 0;
    wave_sync();
    if (!padded && vec) {
        // whole tile of a 16-byte aligned sequence: 16-byte units; with
        // prefetch they were loaded during the previous tile
        if (!kPrefetch<EIN> || !have) tu.load((const EIN *)seq_in(d, g) + start);
        if constexpr (!KEYS) {
            uint4 *eu = (uint4 *)sm.elem;
#pragma unroll
            for (uint32_t i = 0; i < TileUnits<E>::kPerLane; i++) eu[i * 64 + lane] = tu.q[i];
            // the key's bits that lie inside the symbol (the rest are zero)
            constexpr uint32_t width = 8 * sizeof(E);
            const uint32_t kw = shift >= width ? 0u : min(Kg, width - shift);
            const uint32_t ks = shift >= width ? 0u : shift;
#pragma unroll
            for (uint32_t i = 0; i < TileUnits<E>::kPerLane; i++) {
                const uint32_t w4[4] = {tu.q[i].x, tu.q[i].y, tu.q[i].z, tu.q[i].w};
#pragma unroll
                for (uint32_t j = 0; j < 4; j++)
#pragma unroll
                    for (uint32_t s = 0; s < 4 / sizeof(E); s++)
                        atomicAdd((uint32_t *)(cnt_lane + (__builtin_amdgcn_ubfe(w4[j], s * width + ks, kw) << csh)),
                                  1u);
            }
        } else {
            // the low byte of every symbol (v_perm_b32), masked to the key:
            // 8 keys per unit of 16-bit symbols, 4 per unit of 32-bit ones,
            // stored at the unit's symbol positions
            const uint32_t km4 = kmask * 0x01010101u;
#pragma unroll
            for (uint32_t i = 0; i < TileUnits<EIN>::kPerLane; i++) {
                const uint4 u = tu.q[i];
                uint32_t kq[2];
                if constexpr (sizeof(EIN) == 2) {
                    kq[0] = __builtin_amdgcn_perm(u.y, u.x, 0x06040200u) & km4;
                    kq[1] = __builtin_amdgcn_perm(u.w, u.z, 0x06040200u) & km4;
                    *(uint2 *)(sm.elem + 8 * (i * 64 + lane)) = make_uint2(kq[0], kq[1]);
                } else {
                    kq[0] = (__builtin_amdgcn_perm(u.y, u.x, 0x0C0C0400u) |
                             __builtin_amdgcn_perm(u.w, u.z, 0x04000C0Cu)) & km4;
                    *(uint32_t *)(sm.elem + 4 * (i * 64 + lane)) = kq[0];
                }
#pragma unroll
                for (uint32_t j = 0; j < 16 / sizeof(EIN); j++)
                    atomicAdd((uint32_t *)(cnt_lane + (__builtin_amdgcn_ubfe(kq[j / 4], 8 * (j % 4), 8) << csh)), 1u);
            }
        }
        if (kPrefetch<EIN>) {
            // the next tile of the range, when it is whole
            const uint64_t nstart = start + kWaveTile;
            if (t + 1 < t1 && nstart + kWaveTile <= d.n) tu.load((const EIN *)seq_in(d, g) + nstart);
        }
    } else {
        // a key alone keeps only its bits (padding: all ones, after every key)
        const uint32_t keep = KEYS ? kmask : ~0u;
        uint32_t v[kChunks];
        if (!padded) {
#pragma unroll
            for (uint32_t c = 0; c < kChunks; c++) v[c] = (uint32_t)src[c * 64] & keep;
#pragma unroll
            for (uint32_t c = 0; c < kChunks; c++) atomicAdd(&cnt[(((v[c] >> shift) & kmask) << cb) | lane_copy], 1u);
        } else {
#pragma unroll
            for (uint32_t c = 0; c < kChunks; c++)
                v[c] = (c * 64 + lane < len) ? ((uint32_t)src[c * 64] & keep) : (uint32_t)(E)~0u;
#pragma unroll
            for (uint32_t c = 0; c < kChunks; c++)
                if (c * 64 + lane < len) atomicAdd(&cnt[(((v[c] >> shift) & kmask) << cb) | lane_copy], 1u);
        }
#pragma unroll
        for (uint32_t c = 0; c < kChunks; c++) sm.elem[c * 64 + lane] = (E)v[c];
    }
    wave_sync();

    // 2. the tile's count of every key of levels 0..Kg-1, as differences of
    //    the prefix sums P of the finest counts (padding not counted)
    // (a key's count: the sum of its copies)
    auto key_count = [&](uint32_t k) {
        uint32_t x = 0;
        for (uint32_t c = 0; c < (1u << cb); c++) x += cnt[(k << cb) + c];
        return x;
    };
    wave_exscan_n<WaveSmem<E, REORDER, PAIR, KB>::kScanPer>(
        nk, key_count, [&](uint32_t k, uint32_t x, uint32_t) { P[k] = (uint16_t)x; });
    if (lane == 0) P[nk] = (uint16_t)len;
    if (REORDER)
        for (uint32_t k = lane; k < nk; k += 64) sm.hK[k] = (uint16_t)key_count(k);
    wave_sync();
    // 3. start of every key in the tile order of its level (keys in reversed
    //    order), with the counts of step 2 taken on the way
    //    One scan runs over levels 1..Kg-1 one after the other: each level's
    //    counts add up to len, so level a starts at (a - 1) len.
    if (lane == 0) {
        sm.lo[0] = 0;
        sm.h[0] = (uint16_t)len;
    }
    wave_exscan_n<WaveSmem<E, REORDER, PAIR, KB>::kScanPer>(
        lvl_off(Kg) - 1,
        [&](uint32_t i) {
            const uint32_t a = level_of(i + 1), k = rev_bits(i + 1 - lvl_off(a), a), sh = Kg - a;
            return (uint32_t)(P[(k + 1) << sh] - P[k << sh]);
        },
        [&](uint32_t i, uint32_t x, uint32_t cnt) {
            const uint32_t a = level_of(i + 1), e = lvl_off(a) + rev_bits(i + 1 - lvl_off(a), a);
            sm.lo[e] = (uint16_t)(x - (a - 1) * len);
            sm.h[e] = (uint16_t)cnt;
        });
    if (REORDER)
        wave_exscan_n<WaveSmem<E, REORDER, PAIR, KB>::kScanPer>(
            nk, [&](uint32_t i) { return (uint32_t)sm.hK[rev_bits(i, Kg)]; },
            [&](uint32_t i, uint32_t x, uint32_t) { sm.loK[rev_bits(i, Kg)] = (uint16_t)x; });
    wave_sync();

    // 4. split by one bit at a time; each pass's bits are level a in the
    //    tile order of level a (Observation 2: after the splits by bits
    //    0..a-1 the tile is ordered by its reversed a-bit key)
    for (uint32_t a = 0; a + 1 < Kg; a++) {
        split_pass_lm<E, REORDER, PAIR, KB, true>(a, shift + Kg - 1 - a, sm);
        wave_sync();
    }
    split_pass_lm<E, REORDER, PAIR, KB, REORDER>(Kg - 1, shift, sm);
    wave_sync();
    if (REORDER) {
        // the last split ordered the tile by its reversed Kg-bit key: each
        // key's symbols, in text order, go to the key's place in the next
        // group's sequence (padding sorts last and is dropped)
        E *gout = (E *)seq_out(d, g);
        for (uint32_t p = lane; p < len; p += 64) {
            const E x = sm.elem[p];
            const uint32_t k = (x >> shift) & kmask;
            const uint32_t gi = sm.GK[k] + (p - sm.loK[k]);
            if (gi < d.n) gp(gout)[gi] = x;
        }
        wave_sync();
    }

    // 5. every level's runs to their interval starts (and, for the pair, to
    //    the WM's)
    const Side s1{sm.G, sm.pend, sm.pend_v, group_base(d, g)};
    copy_full_words(d, Kg, sm, s1);
    if constexpr (PAIR) {
        const Side s2{sm.G2, sm.pend2, sm.pend_v2, d.bits2};
        copy_full_words(d, Kg, sm, s2);
        const Side both[2] = {s1, s2};
        run_end_words(d, Kg, sm, both);
    } else {
        const Side one[1] = {s1};
        run_end_words(d, Kg, sm, one);
    }
    wave_sync();
    // the next tile's runs start where this tile's end
    for (uint32_t e = lane; e < lvl_off(Kg); e += 64) {
        sm.G[e] += sm.h[e];
        if (PAIR) sm.G2[e] += sm.h[e];
    }
    if (REORDER)
        for (uint32_t k = lane; k < nk; k += 64) sm.GK[k] += sm.hK[k];
    wave_sync();
}

template <typename E, bool REORDER, bool PAIR, uint32_t KB, typename EIN>
__device__ void wave_range(const TextDesc &d, uint32_t g, uint32_t Kg, uint32_t r,
                           WaveSmem<E, REORDER, PAIR, KB> &sm)
{
    const uint32_t lane = lane_id();
    wave_range_start(d, g, Kg, r, sm);
    for (uint32_t e = lane; e < (1u << KB) - 1; e += 64) {
        sm.pend[e] = kNoPend;
        if (PAIR) sm.pend2[e] = kNoPend;
    }
    wave_sync();
    const uint32_t t0 = r * d.R, t1 = min(d.ntiles, t0 + d.R);
    const EIN *seq = (const EIN *)seq_in(d, g);
    const bool vec = ((uintptr_t)seq & 15) == 0;
    TileUnits<EIN> tu;
    for (uint32_t t = t0; t < t1; t++) wave_tile<E, REORDER, PAIR, KB, EIN>(d, g, Kg, t, sm, tu, vec, t > t0, t1);
    // words still open at the end of the range are shared with the next one
    for (uint32_t e = lane; e < lvl_off(Kg); e += 64) {
        if (sm.pend[e] != kNoPend) {
            const uint32_t wd = sm.G[e] >> 6;
            if (wd < (uint32_t)d.W)
                gatomic_or(&group_base(d, g)[sm.lvw[level_of(e)] + wd], sm.pend_v[e]);
        }
        if (PAIR && sm.pend2[e] != kNoPend) {
            const uint32_t wd = sm.G2[e] >> 6;
            if (wd < (uint32_t)d.W)
                gatomic_or(&d.bits2[sm.lvw[level_of(e)] + wd], sm.pend_v2[e]);
        }
    }
    wave_sync();
}

// Waves per scatter workgroup.  LDS is granted per workgroup: groups of
// four waves keep neighbouring ranges on one CU and its SIMDs evenly loaded,
// but when single waves pack a CU's 160 KiB markedly tighter (by a quarter or
// more: eleven instead of eight waves of the 13.5 KiB re-ordering pair
// kernel, for instance) each workgroup is one wave.
constexpr uint32_t kCuLdsBytes = 160 * 1024;
template <typename E, bool REORDER, bool PAIR, uint32_t KB>
constexpr uint32_t scat_block_waves()
{
    constexpr uint32_t S = sizeof(WaveSmem<E, REORDER, PAIR, KB>);
    constexpr uint32_t w4 = 4 * (kCuLdsBytes / (4 * S)), w1 = kCuLdsBytes / S;
    return (4 * w1 >= 5 * w4) ? 1u : 4u;
}

// Waves per SIMD the registers are held to: the byte-symbol pair kernel with
// 7-level tables (7.5 KiB of LDS) to five, where only values used by a padded
// last tile spill; the single byte-symbol kernel to four (its LDS allows four);
// the re-ordering pair kernel of 1- and 2-byte symbols to three.  The others
// keep the compiler's choice.
template <typename E, bool REORDER, bool PAIR, uint32_t KB>
constexpr uint32_t kScatMinWaves = (sizeof(E) == 1 && PAIR && !REORDER && KB == 7)   ? 5
                                   : (sizeof(E) == 1 && !PAIR && !REORDER)            ? 4
                                   : (PAIR && REORDER && sizeof(E) <= 2)              ? 3
                                                                                      : 1;

// Work item = (text, range); wave w of workgroup b takes item b BW + w,
// then strides by the whole grid.  The REORDER variant takes the texts whose
// symbols move on to another group after group g.
template <typename E, bool REORDER, bool PAIR, uint32_t KB, typename EIN = E>
__global__ __launch_bounds__((scat_block_waves<E, REORDER, PAIR, KB>() * 64)) __attribute__((amdgpu_waves_per_eu(kScatMinWaves<E, REORDER, PAIR, KB>))) void k_scatter(const TextDesc *__restrict__ descs,
                                                             const uint32_t *__restrict__ bases,
                                                             uint32_t nd, uint32_t nitems, uint32_t g)
{
    constexpr uint32_t BW = scat_block_waves<E, REORDER, PAIR, KB>();
    __shared__ WaveSmem<E, REORDER, PAIR, KB> sm[BW];
    const uint32_t w = BW == 1 ? 0u : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (uint32_t item = blockIdx.x * BW + w; item < nitems; item += gridDim.x * BW) {
        const uint32_t ti = find_text(bases, nd, item);
        const TextDesc &d = descs[ti];
        const uint32_t r = item - item_base(bases, nd, ti);
        if (d.b != sizeof(EIN) || g >= d.G || r >= d.nranges || (g + 1 < d.G) != REORDER) continue;
        if ((d.pair != 0 && g == 0) != PAIR) continue;  // pairs' group 0 goes to the pair instantiations
        const uint32_t Kg = group_bits(d, g);
        if (Kg == 0 || Kg > KB) continue;  // the tables hold KB levels (the host picks KB >= Kg)
        if (PAIR && KB == kMaxGroupBits && Kg < KB) continue;  // the 7-bit pair kernel takes those
        wave_range<E, REORDER, PAIR, KB, EIN>(d, g, Kg, r, sm[w]);
    }
}

// one instantiation over all items: one wave per item, or, with a cap, a
// persistent grid of grid_cap workgroups of four waves (the same number of
// waves whatever the instantiation's workgroup size)
template <typename E, bool REORDER, bool PAIR, uint32_t KB, typename EIN = E>
static void launch_one(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx)
{
    constexpr uint32_t BW = scat_block_waves<E, REORDER, PAIR, KB>();
    uint32_t grid = (gl.nranges + BW - 1) / BW;
    const uint32_t cap = gl.grid_cap * (4 / BW);
    if (cap && grid > cap) grid = cap;
    hipLaunchKernelGGL((k_scatter<E, REORDER, PAIR, KB, EIN>), dim3(grid), dim3(BW * 64), 0, ctx.stream, d_descs,
                       gl.range_bases, gl.nd, gl.nranges, gl.g);
}

template <typename E>
static void launch_width(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx)
{
    constexpr uint32_t K8 = kMaxGroupBits;
    // pairs: WT and WM of one text (one group) from the same splits
    if (gl.g == 0 && (gl.pmask & 2u)) launch_one<E, false, true, 7>(d_descs, gl, ctx);
    if (gl.g == 0 && (gl.pmask & 4u)) launch_one<E, false, true, K8>(d_descs, gl, ctx);
    if (gl.g == 0 && (gl.pmask & 8u)) launch_one<E, true, true, K8>(d_descs, gl, ctx);
    if (!(gl.pmask & 1u)) return;
    // the last group of a text of wider symbols splits its key bytes alone
    if (gl.rmask & 1u) launch_one<uint8_t, false, false, K8, E>(d_descs, gl, ctx);
    if (gl.rmask & 2u) launch_one<E, true, false, K8>(d_descs, gl, ctx);
}

hipError_t launch_scatter(const TextDesc *d_descs, const GroupLaunch &gl, const LaunchCtx &ctx)
{
    if (gl.bmask & 1u) launch_width<uint8_t>(d_descs, gl, ctx);
    if (gl.bmask & 2u) launch_width<uint16_t>(d_descs, gl, ctx);
    if (gl.bmask & 4u) launch_width<uint32_t>(d_descs, gl, ctx);
    if (ctx.after) ctx.after(ctx.user, KID_SCATTER);
    return hipGetLastError();
}

}  // namespace wtg
