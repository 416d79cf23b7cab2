"""Pins for the oracle: checks against what the paper and plain mathematics fix,
each written independently of the oracle's C code.

Every ``check_*`` function takes an ``oracle.Oracle`` and raises AssertionError
on a mismatch.  ``tests/test_oracle_pins.py`` runs them on the oracle;
``tests/test_oracle_mutations.py`` runs them on deliberately broken copies of
the oracle to show that each planted mistake is caught.

Independent formulations used here (pure Python, small inputs only):
  * WT level l = bit l of the text stably sorted by the l-bit prefix
    (Section 2, Observation 1), with Python's stable ``sorted``;
  * WM level l = bit l of the text stably sorted by the bit-reversed l-bit
    prefix (Section 5, Observation 2), with ``sorted``;
  * WM level l by the defining recursion of Section 5 (zeros move to
    rank_0 positions, ones to Z + rank_1 positions), with counting ranks;
  * rank/select/access by counting over the text (Section 2).
"""
from __future__ import annotations

import itertools
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "running_example.txt")

WT, WM = 0, 1


# -- brute-force formulations ---------------------------------------------------

def bit(L, k, a):
    return (a >> (L - 1 - k)) & 1


def prefix(L, k, a):
    return 0 if k == 0 else a >> (L - k)


def rev(x, k):
    return int(format(x, f"0{k}b")[::-1], 2) if k else 0


def levels_by_sort(kind, T, L):
    """Observation 1 (WT) / Observation 2 (WM): stable sort by the (reversed) prefix."""
    out = []
    for l in range(L):
        if kind == WT:
            seq = sorted(T, key=lambda a: prefix(L, l, a))
        else:
            seq = sorted(T, key=lambda a: rev(prefix(L, l, a), l))
        out.append([bit(L, l, a) for a in seq])
    return out


def wm_by_recursion(T, L):
    """The WM definition of Section 5: level 0 is the MSBs in text order; the
    symbol at position i of level l-1 goes to rank_0(BV_{l-1}, i) if its bit is
    0, else to Z[l-1] + rank_1(BV_{l-1}, i)."""
    n = len(T)
    seq = list(T)
    levels, zeros = [], []
    for l in range(L):
        bv = [bit(L, l, a) for a in seq]
        levels.append(bv)
        z = bv.count(0)
        zeros.append(z)
        nxt = [None] * n
        for i, a in enumerate(seq):
            r1 = sum(bv[:i])
            r0 = i - r1
            nxt[z + r1 if bv[i] else r0] = a
        seq = nxt
    return levels, zeros


def pack(bits_list, W):
    words = np.zeros(W, dtype=np.uint64)
    for p, b in enumerate(bits_list):
        if b:
            words[p // 64] |= np.uint64(1) << np.uint64(p % 64)
    return words


def unpack(words, n):
    return [int((int(words[p // 64]) >> (p % 64)) & 1) for p in range(n)]


def words_per_level(n):
    return ((n + 63) // 64 + 7) // 8 * 8


def read_golden():
    g = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            g[k] = v
    return g


# -- checks -----------------------------------------------------------------------

def check_golden(o):
    g = read_golden()
    T = np.array([int(x) for x in g["text"].split()], dtype=np.uint8)
    L = int(g["lg_sigma"])
    for kind, tag in ((WT, "wt"), (WM, "wm")):
        bits, zeros = o.build(kind, T, L)
        for l in range(L):
            want = [int(c) for c in g[f"{tag}_level{l}"]]
            assert unpack(bits[l], len(T)) == want, (tag, l)
        assert [hex(int(w[0])) for w in bits] == g[f"{tag}_hex"].split(), tag
        assert [int(z) for z in zeros] == [int(x) for x in g["zeros"].split()], tag
    assert [int(x) for x in o.hist(T, L, 3)] == [int(x) for x in g["hist3"].split()]
    assert [int(x) for x in o.hist(T, L, 1)] == [int(x) for x in g["hist1"].split()]
    h2 = o.hist(T, L, 2)
    assert [int(x) for x in h2] == [int(x) for x in g["hist2"].split()]
    assert [int(x) for x in o.spos(WT, h2, 2)] == [int(x) for x in g["spos_wt2"].split()]
    assert [int(x) for x in o.spos(WM, h2, 2)] == [int(x) for x in g["spos_wm2"].split()]

    def triples(key):
        for item in g[key].split():
            lhs, res = item.split("=")
            yield lhs, int(res)

    for kind in (WT, WM):
        bits, zeros = o.build(kind, T, L)
        for lhs, res in triples("rank"):
            c, i = (int(x) for x in lhs.split(":"))
            assert int(o.queries_def(T, L, 1, [c], [i])[0]) == res, ("rank", lhs)
            assert int(o.queries_walk(kind, bits, zeros, len(T), L, 1, [c], [i])[0]) == res
        for lhs, res in triples("select"):
            c, k = (int(x) for x in lhs.split(":"))
            assert int(o.queries_def(T, L, 2, [c], [k])[0]) == res, ("select", lhs)
            assert int(o.queries_walk(kind, bits, zeros, len(T), L, 2, [c], [k])[0]) == res
        for lhs, res in triples("access"):
            i = int(lhs)
            assert int(o.queries_def(T, L, 0, None, [i])[0]) == res
            assert int(o.queries_walk(kind, bits, zeros, len(T), L, 0, None, [i])[0]) == res


def check_printed_small_facts(o):
    # bits(3) = 011 with 3 bits (Section 2): bit(k, 3) for k = 0, 1, 2
    assert [bit(3, k, 3) for k in range(3)] == [0, 1, 1]
    # reverse(001) = 100 (Section 5)
    assert o.reverse_bits(0b001, 3) == 0b100
    # pi_2 = (0, 2, 1, 3) (Section 5)
    assert [o.reverse_bits(i, 2) for i in range(4)] == [0, 2, 1, 3]
    # recurrences: pi_{k+1} = (2 pi_k(0..), 2 pi_k(0..) + 1) and pi_k = pi_{k+1}/2
    for k in range(1, 13):
        pk = [o.reverse_bits(i, k) for i in range(1 << k)]
        pk1 = [o.reverse_bits(i, k + 1) for i in range(1 << (k + 1))]
        assert pk1 == [2 * x for x in pk] + [2 * x + 1 for x in pk]
        assert [x >> 1 for x in pk1[: 1 << k]] == pk


def _small_cases(seed=11, count=120, max_n=70, max_L=7):
    rng = np.random.default_rng(seed)
    cases = []
    for _ in range(count):
        L = int(rng.integers(1, max_L + 1))
        n = int(rng.integers(0, max_n + 1))
        dtype = np.uint8 if L <= 8 else (np.uint16 if L <= 16 else np.uint32)
        T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(dtype)
        cases.append((T, L))
    return cases


def check_levels_brute(o, exhaustive=True):
    """Levels equal the stable-sort formulations; the WM equals its recursion."""
    cases = _small_cases()
    if exhaustive:
        for L in (1, 2, 3):
            for n in range(0, 5):
                for tup in itertools.product(range(1 << L), repeat=n):
                    cases.append((np.array(tup, dtype=np.uint8), L))
    for T, L in cases:
        n = len(T)
        W = words_per_level(n)
        Tl = [int(x) for x in T]
        for kind in (WT, WM):
            bits, zeros = o.build(kind, T, L)
            assert bits.shape == (L, W)
            want = levels_by_sort(kind, Tl, L)
            for l in range(L):
                assert np.array_equal(bits[l], pack(want[l], W)), (kind, l, Tl, L)
                assert int(zeros[l]) == want[l].count(0)
        rl, rz = wm_by_recursion(Tl, L)
        bits, zeros = o.build(WM, T, L)
        for l in range(L):
            assert unpack(bits[l], n) == rl[l]
        assert [int(z) for z in zeros] == rz


def check_wide_symbols(o):
    """16-, 20- and 32-level texts of 16/32-bit symbols against the sort formulation."""
    rng = np.random.default_rng(5)
    for L, dtype in ((16, np.uint16), (20, np.uint32), (32, np.uint32)):
        for n in (1, 37, 150):
            T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(dtype)
            Tl = [int(x) for x in T]
            for kind in (WT, WM):
                bits, zeros = o.build(kind, T, L)
                want = levels_by_sort(kind, Tl, L)
                for l in range(L):
                    assert unpack(bits[l], n) == want[l], (L, kind, l)


def check_invariants(o):
    """Invariants the paper states: WT and WM agree on levels 0 and 1
    (Section 5.2); level l holds as many ones as symbols with bit l set;
    Z[l] = SPos_WM^{l+1}[1] (Section 5.1, zeros from even prefixes) and
    Z[L-1] = number of even symbols; the WT level is the WM level with its
    intervals moved from bit-reversed to prefix order (Section 5.1);
    histograms merge pairwise (Section 3.1) and sum to n."""
    rng = np.random.default_rng(7)
    for _ in range(40):
        L = int(rng.integers(1, 9))
        n = int(rng.integers(1, 400))
        T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(np.uint8 if L <= 8 else np.uint16)
        Tl = [int(x) for x in T]
        bt, zt = o.build(WT, T, L)
        bm, zm = o.build(WM, T, L)
        for l in range(min(L, 2)):
            assert np.array_equal(bt[l], bm[l])
        assert np.array_equal(zt, zm)
        for l in range(L):
            ones = sum(bit(L, l, a) for a in Tl)
            assert sum(unpack(bt[l], n)) == ones
            assert sum(unpack(bm[l], n)) == ones
            # padding bits beyond n are zero
            W = bt.shape[1]
            assert unpack(bt[l], W * 64)[n:] == [0] * (W * 64 - n)
            assert unpack(bm[l], W * 64)[n:] == [0] * (W * 64 - n)
        for l in range(L):
            h = o.hist(T, L, l)
            assert int(h.sum()) == n
            assert [int(x) for x in h] == [sum(1 for a in Tl if prefix(L, l, a) == p) for p in range(1 << l)]
            if l + 1 <= L:
                h1 = o.hist(T, L, l + 1)
                assert np.array_equal(h, h1[0::2] + h1[1::2])
        for l in range(L - 1):
            h1 = o.hist(T, L, l + 1)
            assert int(zm[l]) == int(o.spos(WM, h1, l + 1)[1])
        assert int(zm[L - 1]) == sum(1 for a in Tl if a % 2 == 0)
        # WT level l = WM level l with intervals re-ordered
        for l in range(L):
            h = o.hist(T, L, l)
            st, sm = o.spos(WT, h, l), o.spos(WM, h, l)
            ut, um = unpack(bt[l], n), unpack(bm[l], n)
            for p in range(1 << l):
                a, b, c = int(st[p]), int(sm[p]), int(h[p])
                assert ut[a:a + c] == um[b:b + c]


def check_queries(o):
    """Query definitions against counting, and the walks over the oracle's own
    levels against the definitions, on both structures."""
    rng = np.random.default_rng(9)
    for _ in range(30):
        L = int(rng.integers(0, 7))
        n = int(rng.integers(0, 200))
        T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(np.uint8)
        Tl = [int(x) for x in T]
        sig = 1 << L
        pos = list(range(n + 2))
        acc = o.queries_def(T, L, 0, None, pos)
        assert [int(x) for x in acc] == Tl + [0xFFFFFFFF] * 2
        cs, is_, ks = [], [], []
        for c in range(sig + 1):
            for i in range(0, n + 2, max(1, n // 7)):
                cs.append(c)
                is_.append(i)
            for k in range(0, Tl.count(c) + 2):
                ks.append((c, k))
        rk = o.queries_def(T, L, 1, cs, is_)
        for c, i, r in zip(cs, is_, rk):
            want = 2**64 - 1 if i > n else (0 if c >= sig else Tl[:i].count(c))
            assert int(r) == want, ("rank", c, i)
        sc = o.queries_def(T, L, 2, [c for c, _ in ks], [k for _, k in ks])
        for (c, k), r in zip(ks, sc):
            occ = [j for j, a in enumerate(Tl) if a == c]
            want = occ[k - 1] if 1 <= k <= len(occ) else 2**64 - 1
            assert int(r) == want, ("select", c, k)
        for kind in (WT, WM):
            bits, zeros = o.build(kind, T, L)
            assert np.array_equal(o.queries_walk(kind, bits, zeros, n, L, 0, None, pos), acc)
            assert np.array_equal(o.queries_walk(kind, bits, zeros, n, L, 1, cs, is_), rk)
            assert np.array_equal(o.queries_walk(kind, bits, zeros, n, L, 2,
                                                 [c for c, _ in ks], [k for _, k in ks]), sc)


def check_rank_scan(o):
    """The one-scan rank (for long texts) against counting over the text
    (Section 2: rank_c(i) = occurrences of c in T[0, i)), with the queries
    in no particular order, repeated positions, symbols that never occur,
    c >= 2^L and i > n."""
    rng = np.random.default_rng(23)
    for _ in range(40):
        L = int(rng.integers(0, 9))
        n = int(rng.integers(0, 300))
        dt = np.uint8 if L <= 8 else np.uint16
        T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(dt)
        Tl = [int(x) for x in T]
        m = int(rng.integers(1, 60))
        cs = [int(c) for c in rng.integers(0, (1 << L) + 2, size=m)]
        ps = [int(p) for p in rng.integers(0, n + 3, size=m)]
        got = o.rank_scan(T, L, cs, ps)
        for c, p, r in zip(cs, ps, got):
            want = 2**64 - 1 if p > n else (0 if c >= (1 << L) else Tl[:p].count(c))
            assert int(r) == want, ("rank_scan", L, n, c, p, int(r), want)


def check_par_build(o):
    """The all-cores builder equals the single-threaded one (itself pinned by
    the checks above) for many thread counts, including more threads than
    64-symbol slices, empty texts, one level and no levels; it refuses an
    out-of-range symbol."""
    import oracle
    rng = np.random.default_rng(29)
    cases = [(0, 3), (1, 1), (63, 2), (64, 7), (65, 8), (700, 5), (5000, 12), (3000, 16), (2000, 20)]
    for _ in range(12):
        cases.append((int(rng.integers(0, 3000)), int(rng.integers(0, 11))))
    for n, L in cases:
        dt = np.uint8 if L <= 8 else (np.uint16 if L <= 16 else np.uint32)
        T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(dt)
        if n > 10 and L > 1:
            T[: n // 3] = T[0]  # a long run of one symbol (one node holds many slices)
        for kind in (WT, WM):
            want_b, want_z = o.build(kind, T, L)
            for threads in (1, 2, 3, 7, 16):
                b, z = o.par_build(kind, T, L, threads)
                assert np.array_equal(b, want_b), ("par_build levels", kind, n, L, threads)
                assert np.array_equal(z, want_z), ("par_build zeros", kind, n, L, threads)
    try:
        o.par_build(WM, np.array([0, 9, 1], dtype=np.uint8), 3, 2)
    except oracle.OracleError as e:
        assert e.code == oracle.ERANGE
    else:
        raise AssertionError("symbol 9 with 3 levels must be rejected")


def check_rank_select_bv(o):
    rng = np.random.default_rng(13)
    for n in (0, 1, 63, 64, 65, 200, 700):
        bl = [int(x) for x in rng.integers(0, 2, size=n)]
        w = pack(bl, max(1, words_per_level(n)))
        for i in range(n + 1):
            assert o.rank_bv(w, i, 1) == sum(bl[:i])
            assert o.rank_bv(w, i, 0) == i - sum(bl[:i])
        ones = [p for p, b in enumerate(bl) if b]
        zer = [p for p, b in enumerate(bl) if not b]
        for k in range(1, len(ones) + 1):
            assert o.select_bv(w, n, k, 1) == ones[k - 1]
        for k in range(1, len(zer) + 1):
            assert o.select_bv(w, n, k, 0) == zer[k - 1]


def check_directory(o):
    """rank_dir[j] = ones before bit 512 j; sel_b[q] = block of the
    (4096 q + 1)-th b; unused sample slots hold 0xFFFFFFFF."""
    rng = np.random.default_rng(17)
    for n, p1 in ((0, 0.5), (1, 1.0), (511, 0.5), (512, 0.5), (513, 0.9), (9000, 0.5),
                  (20000, 0.97), (20000, 0.03)):
        bl = (rng.random(n) < p1).astype(np.int64)
        W = words_per_level(n)
        w = pack(bl, max(W, 1))[:W]
        rd, s0, s1 = o.directory(w, n)
        assert rd.size == W // 8 + 1
        cum = np.concatenate([[0], np.cumsum(bl)])
        for j in range(W // 8 + 1):
            assert int(rd[j]) == int(cum[min(512 * j, n)])
        ones = np.flatnonzero(bl == 1)
        zer = np.flatnonzero(bl == 0)
        cap = (n + 4095) // 4096 + 1
        assert s0.size == cap and s1.size == cap
        for arr, pos in ((s1, ones), (s0, zer)):
            want = [int(pos[q * 4096]) // 512 for q in range((len(pos) + 4095) // 4096)]
            want += [0xFFFFFFFF] * (cap - len(want))
            assert [int(x) for x in arr] == want


def check_sample_level(o):
    """The per-position formulation agrees with the full levels."""
    rng = np.random.default_rng(19)
    for L, n in ((1, 50), (3, 300), (6, 1000), (9, 777)):
        T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(np.uint16)
        for kind in (WT, WM):
            bits, _ = o.build(kind, T, L)
            for l in range(L):
                pos = rng.integers(0, n, size=64)
                got = o.sample_level(kind, T, L, l, pos)
                want = [unpack(bits[l], n)[p] for p in pos]
                assert [int(x) for x in got] == want


def check_map_wt_to_wm(o):
    """The WT-to-WM position map (Section 5.1, Lemma 5): the hand-worked
    running example, identity on levels 0 and 1, a bijection on every level,
    and it carries every WT bit to an equal WM bit."""
    g = read_golden()
    T = np.array([int(x) for x in g["text"].split()], dtype=np.uint8)
    got = o.map_wt_to_wm(T, 3, 2, np.arange(T.size))
    assert [int(x) for x in got] == [int(x) for x in g["map_wt_to_wm2"].split()]
    rng = np.random.default_rng(23)
    for L, n in ((2, 100), (3, 500), (5, 2000), (8, 3000), (11, 1500)):
        T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(np.uint16)
        if L == 11:  # a skewed text with empty intervals
            T = (T % 37) * 53 % (1 << L)
        wt, _ = o.build(WT, T, L)
        wm, _ = o.build(WM, T, L)
        for l in range(L):
            j = o.map_wt_to_wm(T, L, l, np.arange(n))
            if l <= 1:
                assert np.array_equal(j, np.arange(n, dtype=np.uint64))
            assert np.array_equal(np.sort(j), np.arange(n, dtype=np.uint64)), (L, l)
            bt, bm = unpack(wt[l], n), unpack(wm[l], n)
            assert all(bt[i] == bm[int(j[i])] for i in range(n)), (L, l)


def check_pointer_tree(o):
    """The pointer-based WT (Section 2): the hand-worked nodes of the running
    example, every node against a filter of the text on tiny inputs, each
    node's zeros and ones sizing its two children, whole-word runs in entry
    order, and the nodes of a level side by side forming the WT level."""
    g = read_golden()
    T = np.array([int(x) for x in g["text"].split()], dtype=np.uint8)
    nodes, pool = o.pointer_tree(T, 3)
    want = g["ptree_nodes"].split()
    assert ["".join(map(str, o.node_bits(nodes, pool, e))) for e in range(7)] == want
    rng = np.random.default_rng(31)
    cases = [(rng.integers(0, 1 << L, size=n).astype(np.uint16), L)
             for L, n in ((1, 7), (2, 70), (3, 130), (4, 64), (5, 300), (7, 1000))]
    cases.append((((np.arange(700) * 53) % 37 * 3 % 512).astype(np.uint16), 9))  # empty nodes
    cases.append((np.zeros(0, dtype=np.uint8), 3))
    for T, L in cases:
        nodes, pool = o.pointer_tree(T, L)
        wt, _ = o.build(WT, T, L)
        w = 0
        for l in range(L):
            row = []
            for p in range(1 << l):
                e = (1 << l) - 1 + p
                got = o.node_bits(nodes, pool, e)
                if T.size <= 300:
                    assert got == [bit(L, l, int(a)) for a in T if prefix(L, l, int(a)) == p], (L, l, p)
                assert int(nodes[e, 0]) == w
                w += (len(got) + 63) // 64
                # bits past the node's length stay clear
                if len(got) % 64:
                    assert int(pool[int(nodes[e, 0]) + len(got) // 64]) >> (len(got) % 64) == 0
                if l + 1 < L:
                    assert int(nodes[2 * e + 1, 1]) == got.count(0)
                    assert int(nodes[2 * e + 2, 1]) == got.count(1)
                row += got
            assert row == unpack(wt[l], T.size), (L, l)
    assert int(nodes[0, 1]) == T.size


def check_errors(o):
    import oracle
    T = np.array([0, 1, 8], dtype=np.uint8)
    for kind in (WT, WM):
        try:
            o.build(kind, T, 3)
        except oracle.OracleError as e:
            assert e.code == oracle.ERANGE
        else:
            raise AssertionError("symbol 8 with 3 levels must be rejected")
    # L = 0: only symbol 0 allowed, no levels
    bits, zeros = o.build(WM, np.zeros(5, dtype=np.uint8), 0)
    assert bits.shape[0] == 0 and zeros.size == 0


ALL_CHECKS = [check_golden, check_printed_small_facts, check_levels_brute, check_wide_symbols,
              check_invariants, check_queries, check_rank_scan, check_par_build, check_rank_select_bv, check_directory,
              check_sample_level, check_map_wt_to_wm, check_pointer_tree, check_errors]
