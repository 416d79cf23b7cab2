"""Ranges of several tiles, element by element against the oracle.

A scatter wave walks a range of consecutive 2048-symbol tiles in order and
carries, from one tile to the next, the word each key's run ends in; only the
words shared with another range are completed by atomic OR.  A text of n
symbols is cut into about 12288 ranges, so a range holds more than one tile
only past 12288 * 2048 symbols, or when tune.grid asks for fewer ranges.
These tests take both routes: short texts with a small grid (many tiles per
range, ragged last tile), and texts of 2^26 symbols in the default launch
configuration (three tiles per range), for the pair build (both structures
from one set of splits: Section 5.1) and the separate WT and WM builds.
Every level word, Z and every directory entry must equal the oracle's."""
import numpy as np
import pytest

from tests.gpu_util import assert_matches_oracle, lib

pytestmark = pytest.mark.gpu

WT, WM = 0, 1


def _rand(n, L, seed, dtype=None):
    rng = np.random.default_rng(seed)
    if dtype is None:
        dtype = np.uint8 if L <= 8 else (np.uint16 if L <= 16 else np.uint32)
    return rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(dtype)


def _text(kind, n, L, seed):
    """uniform symbols, or a text of long runs (a run of one symbol keeps a
    key's run open across many tiles)"""
    T = _rand(n, L, seed)
    if kind == "runs":
        rng = np.random.default_rng(seed + 1)
        cuts = np.sort(rng.integers(0, n, size=max(1, n // 3000)))
        for a, b in zip(cuts[::2], cuts[1::2]):
            T[a:b] = T[a]
    return T


def _pair(T, L, tune=None):
    import torch
    B = lib()
    wt, wm = B.pair_build(B.to_device(T), T.size, T.dtype.itemsize, L, tune=tune)
    torch.cuda.synchronize()
    return wt, wm


def _single(T, L, kind, tune=None):
    import torch
    B = lib()
    s = B.build(B.to_device(T), T.size, T.dtype.itemsize, L, kind, tune=tune)
    torch.cuda.synchronize()
    return s


def _plan_tiles_per_range(n, grid):
    tiles = -(-n // 2048)
    return max(1, -(-tiles // grid))


@pytest.mark.parametrize("text", ["uniform", "runs"])
@pytest.mark.parametrize("L", [1, 2, 3, 7, 8])
@pytest.mark.parametrize("n,grid", [(3 * 2048 * 5 + 37, 2), (2048 * 40 + 1, 3), (2048 * 64, 7),
                                    (2048 * 9 - 5, 1), (2048 * 130 + 999, 4)])
def test_forced_ranges(orc, n, grid, L, text):
    """tune.grid ranges per text: every range holds several tiles (the last
    one possibly short); pair build and both separate builds."""
    assert _plan_tiles_per_range(n, grid) > 1
    B = lib()
    tune = B.make_tune(grid=grid)
    T = _text(text, n, L, seed=n + 7 * L + grid)
    print(f"[multitile] forced n={n} grid={grid} L={L} text={text}", flush=True)
    wt, wm = _pair(T, L, tune)
    assert_matches_oracle(orc, T, L, WT, wt)
    assert_matches_oracle(orc, T, L, WM, wm)
    for kind in (WT, WM):
        assert_matches_oracle(orc, T, L, kind, _single(T, L, kind, tune))


@pytest.mark.parametrize("dtype,L", [(np.uint16, 11), (np.uint16, 16), (np.uint32, 20), (np.uint8, 8)])
def test_forced_ranges_several_groups(orc, dtype, L):
    """Several groups of levels (re-ordered text between groups; the WT's
    deep levels gathered from WM intervals) with ranges of many tiles."""
    B = lib()
    n = 2048 * 37 + 11
    T = _rand(n, L, seed=L + 100, dtype=dtype)
    for tune in (B.make_tune(grid=3), B.make_tune(grid=2, group_bits=3)):
        print(f"[multitile] groups L={L} b={T.dtype.itemsize} tune=({tune.grid},{tune.group_bits})", flush=True)
        wt, wm = _pair(T, L, tune)
        assert_matches_oracle(orc, T, L, WT, wt)
        assert_matches_oracle(orc, T, L, WM, wm)
        for kind in (WT, WM):
            assert_matches_oracle(orc, T, L, kind, _single(T, L, kind, tune))


def _same_levels(a, b):
    """level words and Z of two structures, compared on the device"""
    import torch
    va, vb = a.view, b.view
    L, W = a.L, va.words_per_level
    if not torch.equal(a._slice(va.bits, L * W, 8), b._slice(vb.bits, L * W, 8)):
        return False
    return torch.equal(a._slice(va.zeros, L, 8), b._slice(vb.zeros, L, 8))


@pytest.mark.slow
@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["markov96", "markov4", "uniform256", "uniform16"])
def test_default_launch_three_tiles_per_range(orc, name):
    """n = 2^26 in the default launch configuration: 32768 tiles in 10923
    ranges of three tiles.  markov96 and markov4 shapes (7 and 2 levels: the
    7-level pair kernel), uniform256 (8 levels: the 8-level pair kernel), a
    uniform 16-bit text (two groups: re-ordering scatter, WM build plus the WT
    gathered from it).  The pair build's WT and WM, level by level, Z and
    directories against the oracle; the separate builds equal them."""
    import torch
    from paper_1702_07578_amd import inputs
    B = lib()
    n = 1 << 26
    assert _plan_tiles_per_range(n, 12288) == 3
    T, L = inputs.make(name, n)
    print(f"[multitile] default launch {name}: n={n} b={T.dtype.itemsize} L={L}", flush=True)
    d = B.to_device(T)
    wt, wm = B.pair_build(d, n, T.dtype.itemsize, L)
    torch.cuda.synchronize()
    assert_matches_oracle(orc, T, L, WT, wt)
    assert_matches_oracle(orc, T, L, WM, wm)
    for kind, p in ((WT, wt), (WM, wm)):
        s = B.build(d, n, T.dtype.itemsize, L, kind)
        torch.cuda.synchronize()
        assert s.status() == 0
        assert _same_levels(s, p), f"separate build kind {kind} differs from the pair build"
        del s
    del wt, wm, d
    torch.cuda.empty_cache()
