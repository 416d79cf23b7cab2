"""Batched access / rank / select on the GPU against the oracle's plain
definitions over the text."""
import numpy as np
import pytest

from tests.gpu_util import gpu_build, lib

pytestmark = pytest.mark.gpu


def _queries(T, L, seed, m):
    rng = np.random.default_rng(seed)
    n = T.size
    pos = rng.integers(0, n + 3, size=m).astype(np.uint64)
    hi = min(1 << L, 1 << 32) if L < 32 else (1 << 32)
    # half the symbols drawn from the text (so select hits), some out of range
    syms = np.where(rng.random(m) < 0.6, T[rng.integers(0, max(n, 1), size=m)] if n else 0,
                    rng.integers(0, min(hi + 2, 1 << 32), size=m)).astype(np.uint64)
    syms = np.minimum(syms, (1 << 32) - 1).astype(np.uint32)
    ks = rng.integers(0, 6, size=m).astype(np.uint64)
    return pos, syms, ks


@pytest.mark.parametrize("L,n,dtype", [(3, 10, np.uint8), (1, 1000, np.uint8), (8, 70000, np.uint8),
                                       (7, 100000, np.uint8), (13, 40000, np.uint16),
                                       (20, 30000, np.uint32), (0, 500, np.uint8), (5, 0, np.uint8)])
@pytest.mark.parametrize("kind", [0, 1])
def test_queries_vs_definitions(orc, L, n, dtype, kind):
    import torch
    B = lib()
    rng = np.random.default_rng(L * 7 + n)
    T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(dtype) if L else np.zeros(n, dtype)
    s = gpu_build(T, L, kind)
    m = 20000
    pos, syms, ks = _queries(T, L, 5, m)
    # rank with every k = rank+1 for valid (c, i) so select is exercised on hits
    dpos = torch.from_numpy(pos.view(np.int64)).cuda()
    dsym = torch.from_numpy(syms.view(np.int32)).cuda()
    acc = s.access(dpos).cpu().numpy().view(np.uint32)
    want = orc.queries_def(T, L, 0, None, pos)
    assert np.array_equal(acc.astype(np.uint64), want)
    rk = s.rank(dsym, dpos).cpu().numpy().view(np.uint64)
    assert np.array_equal(rk, orc.queries_def(T, L, 1, syms, pos))
    # select: k from small values and from rank results (hits)
    kk = np.where(rng.random(m) < 0.5, ks, np.where(rk == np.uint64(2**64 - 1), 1, rk + 1)).astype(np.uint64)
    dk = torch.from_numpy(kk.view(np.int64)).cuda()
    sl = s.select(dsym, dk).cpu().numpy().view(np.uint64)
    assert np.array_equal(sl, orc.queries_def(T, L, 2, syms, kk))


def test_access_reconstructs_text():
    import torch
    from paper_1702_07578_amd import inputs
    T, L = inputs.make("markov96", 1 << 20)
    for kind in (0, 1):
        s = gpu_build(T, L, kind)
        pos = torch.arange(T.size, dtype=torch.int64, device="cuda")
        acc = s.access(pos).cpu().numpy().view(np.uint32)
        assert np.array_equal(acc, T.astype(np.uint32))


@pytest.mark.parametrize("n", [4096, 4097, 4159, 5119])
@pytest.mark.parametrize("kind", [0, 1])
def test_every_position_and_every_k(orc, n, kind):
    """rank of every symbol at every position 0..n (block starts, word starts,
    the ends of whole and ragged texts) and select of every symbol for every k
    from 1 to one past its count, against the oracle's definitions."""
    import torch
    L = 3
    rng = np.random.default_rng(n + kind)
    T = rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(np.uint8)
    s = gpu_build(T, L, kind)
    syms = np.repeat(np.arange(1 << L, dtype=np.uint32), n + 1)
    pos = np.tile(np.arange(n + 1, dtype=np.uint64), 1 << L)
    dev = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    rk = s.rank(dev(syms, np.int32), dev(pos, np.int64)).cpu().numpy().view(np.uint64)
    assert np.array_equal(rk, orc.queries_def(T, L, 1, syms, pos))
    counts = np.bincount(T, minlength=1 << L)
    ssym = np.concatenate([np.full(int(c) + 1, a, dtype=np.uint32) for a, c in enumerate(counts)])
    kk = np.concatenate([np.arange(1, int(c) + 2, dtype=np.uint64) for c in counts])
    sl = s.select(dev(ssym, np.int32), dev(kk, np.int64)).cpu().numpy().view(np.uint64)
    assert np.array_equal(sl, orc.queries_def(T, L, 2, ssym, kk))
