"""Batched build of many independent texts in one sequence of launches:
every text of the batch must equal the oracle (levels, Z, directories) and
the standalone build of the same text; the launch-only entry point is
captured in a HIP graph and every replay is checked."""
import numpy as np
import pytest

from tests.gpu_util import assert_matches_oracle, gpu_build, lib

pytestmark = pytest.mark.gpu

WT, WM = 0, 1


def _batch(count, seed, lo_exp, hi_exp, extra=()):
    from paper_1702_07578_amd import inputs
    texts = []
    for i, sp in enumerate(inputs.batch_specs(count, seed=seed, lo_exp=lo_exp, hi_exp=hi_exp)):
        T, L = inputs.batch_text(sp)
        texts.append((T, L, i % 2))
    texts.extend(extra)
    return texts


def _items(texts, dev):
    import torch
    B = lib()
    items = []
    for T, L, kind in texts:
        d = B.to_device(T, dev) if T.size else torch.zeros(8, dtype=torch.uint8, device=dev)
        s = B.Structure(T.size, L, kind, device=dev)
        items.append((d, T.size, T.dtype.itemsize, L, kind, s))
    return items


def _garble(items):
    for it in items:
        it[5].buf.fill_(0xA5)


def _defined(s, n):
    """The parts of a structure the interface defines: every level word, Z,
    rank entries 0..W/8 and the select samples up to ceil(n/4096)+1 (the
    stride padding after them is unspecified)."""
    bits, zeros, rd, s0, s1 = s.host_arrays()
    W = bits.shape[1] if bits.ndim == 2 else 0
    cap = -(-n // 4096) + 1
    return (bits.copy(), zeros.copy(), rd[:, : W // 8 + 1].copy(), s0[:, :cap].copy(),
            s1[:, :cap].copy())


def _snapshot(items):
    return [_defined(it[5], it[1]) for it in items]


def _edge_texts():
    rng = np.random.default_rng(5)
    return [
        (np.zeros(0, np.uint8), 3, WT),
        (np.zeros(0, np.uint8), 3, WM),
        (np.array([7], np.uint8), 3, WT),
        (np.array([200, 3], np.uint8), 8, WM),
        (rng.integers(0, 1 << 12, 5000).astype(np.uint16), 12, WT),
        (rng.integers(0, 1 << 12, 5000).astype(np.uint16), 12, WM),
        (rng.integers(0, 1 << 20, 3000).astype(np.uint32), 20, WT),
        (np.zeros(4097, np.uint8), 0, WM),
    ]


@pytest.mark.parametrize("persist", [0, 40])
def test_batch_matches_oracle_and_standalone(orc, persist):
    import torch
    B = lib()
    dev = torch.device("cuda:0")
    texts = _batch(24, seed=11, lo_exp=6.0, hi_exp=15.0, extra=_edge_texts())
    items = _items(texts, dev)
    _garble(items)
    B.batch_build(items, tune=B.make_tune(persist=persist))
    torch.cuda.synchronize()
    for (T, L, kind), it in zip(texts, items):
        assert_matches_oracle(orc, T, L, kind, it[5])
        alone = gpu_build(T, L, kind)
        for a, b in zip(_defined(it[5], T.size), _defined(alone, T.size)):
            assert np.array_equal(a, b)


def test_batch_tuned_tiles(orc):
    """Small tiles and few ranges per text: several tiles per range in every
    text of the batch, levels in groups of 3."""
    import torch
    B = lib()
    dev = torch.device("cuda:0")
    texts = _batch(12, seed=12, lo_exp=11.0, hi_exp=16.0)
    items = _items(texts, dev)
    _garble(items)
    B.batch_build(items, tune=B.make_tune(tile_log2=10, group_bits=3, grid=3, persist=17))
    torch.cuda.synchronize()
    for (T, L, kind), it in zip(texts, items):
        assert_matches_oracle(orc, T, L, kind, it[5])


def test_batch_graph_replays(orc):
    """prepare once, capture launch in a graph, replay it several times with
    the outputs overwritten in between; every replay equals the eager build."""
    import torch
    B = lib()
    dev = torch.device("cuda:0")
    texts = _batch(16, seed=13, lo_exp=8.0, hi_exp=14.0, extra=_edge_texts()[2:6])
    items = _items(texts, dev)
    batch = B.Batch(items, tune=B.make_tune(persist=64))
    batch.build()
    torch.cuda.synchronize()
    want = _snapshot(items)
    for (T, L, kind), it in zip(texts, items):
        assert_matches_oracle(orc, T, L, kind, it[5], check_dirs=False)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        batch.prepare(side)
        with torch.cuda.graph(g, stream=side):
            batch.launch(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        _garble(items)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(items)
        for i, (a, b) in enumerate(zip(got, want)):
            for x, y in zip(a, b):
                assert np.array_equal(x, y), f"replay {rep} text {i}"
        # eager work between replays
        batch.build()
        torch.cuda.synchronize()


def test_batch_argument_errors():
    import torch
    B = lib()
    dev = torch.device("cuda:0")
    T = np.arange(100, dtype=np.uint8) % 8
    items = _items([(T, 3, WT)], dev)
    b = B.Batch(items)
    import ctypes
    small = torch.empty(64, dtype=torch.uint8, device=dev)
    for f in (B.wt_batch_prepare, B.wt_batch_launch, B.wt_batch_build):
        assert f(b.arr, 1, ctypes.c_void_p(small.data_ptr()), 64, None, None) == B.WT_ENOSPACE
        assert f(b.arr, 0, ctypes.c_void_p(small.data_ptr()), 64, None, None) == B.WT_EINVAL
    # a symbol out of range is reported in the text's own status word only
    T2 = np.array([1, 2, 9], dtype=np.uint8)
    items2 = _items([(T, 3, WM), (T2, 3, WM)], dev)
    B.batch_build(items2)
    torch.cuda.synchronize()
    assert items2[0][5].status() == 0
    assert items2[1][5].status() == B.WT_ERANGE
    b.build()
    torch.cuda.synchronize()
    assert items[0][5].status() == 0


def test_batch_pairs_share_one_pass(orc):
    """WT and WM items of the same device text are built as pairs inside a
    batch that also holds unpaired items: one group (one pass writes both; 7-
    and 8-level pair kernels), more groups (the WM writes the WT's first group
    and the WT gathers the rest from the WM: 12, 16 and 20 levels), a WT
    without its WM, a second WM or WT of a paired text, and texts of their
    own.  Every output equals the oracle and its standalone build, eagerly and
    on graph replays."""
    import torch
    B = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(29)
    shared = [
        (rng.integers(0, 1 << 7, 70001).astype(np.uint8), 7, (WT, WM)),
        (rng.integers(0, 1 << 8, 5000).astype(np.uint8), 8, (WM, WT)),
        (rng.integers(0, 1 << 3, 3).astype(np.uint8), 3, (WT, WM, WM)),
        (rng.integers(0, 1 << 5, 9000).astype(np.uint16), 5, (WT,)),
        (rng.integers(0, 1 << 12, 6000).astype(np.uint16), 12, (WT, WM)),
        (rng.integers(0, 1 << 20, 9001).astype(np.uint32), 20, (WM, WT)),
        ((np.arange(30000) * 7919 % 65521).astype(np.uint16), 16, (WT, WM, WT)),
        (rng.integers(0, 1 << 2, 2049).astype(np.uint8), 2, (WM, WT)),
    ]
    texts, items = [], []
    for T, L, kinds in shared:
        d = B.to_device(T, dev)
        for kind in kinds:
            texts.append((T, L, kind))
            items.append((d, T.size, T.dtype.itemsize, L, kind, B.Structure(T.size, L, kind, device=dev)))
    for T, L, kind in _batch(10, seed=31, lo_exp=8.0, hi_exp=14.0):
        texts.append((T, L, kind))
        items.append((B.to_device(T, dev), T.size, T.dtype.itemsize, L, kind, B.Structure(T.size, L, kind, device=dev)))
    _garble(items)
    batch = B.Batch(items, tune=B.make_tune(persist=48))
    batch.build()
    torch.cuda.synchronize()
    want = []
    for (T, L, kind), it in zip(texts, items):
        assert_matches_oracle(orc, T, L, kind, it[5])
        alone = gpu_build(T, L, kind)
        got = _defined(it[5], T.size)
        for a, b in zip(got, _defined(alone, T.size)):
            assert np.array_equal(a, b)
        want.append(got)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        batch.prepare(side)
        with torch.cuda.graph(g, stream=side):
            batch.launch(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for _ in range(2):
        _garble(items)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for w, it in zip(want, items):
            for a, b in zip(w, _defined(it[5], it[1])):
                assert np.array_equal(a, b)


def test_every_autotune_candidate_reproduces_the_oracle(orc):
    """The tuner keeps a candidate only when its outputs equal the default
    configuration's; here every candidate of its search space is built on a
    probe batch (mixed widths and alphabets, ranges of several tiles) and
    compared with the oracle, and the tuner accepts all of them."""
    import torch
    from paper_1702_07578_amd import autotune
    B = lib()
    dev = torch.device("cuda:0")
    texts = _batch(10, seed=13, lo_exp=8.0, hi_exp=17.0, extra=_edge_texts()[2:6])
    items = _items(texts, dev)
    tune, table = autotune.tune(items, reps=1)
    assert all(st == "ok" for _, _, _, st in table), table
    for g, p in autotune.CANDIDATES:
        _garble(items)
        print(f"[autotune] candidate grid={g} persist={p}", flush=True)
        B.batch_build(items, tune=B.make_tune(grid=g, persist=p))
        torch.cuda.synchronize()
        for (T, L, kind), it in zip(texts, items):
            assert_matches_oracle(orc, T, L, kind, it[5])
