"""GPU builds (C ABI, HIP kernels) against the oracle, element by element:
levels, zero counts and directories must be bit-identical."""
import numpy as np
import pytest

from tests.gpu_util import assert_matches_oracle, gpu_build, lib
from tests import pins

pytestmark = pytest.mark.gpu

WT, WM = 0, 1


def _rand(n, L, seed, dtype=None):
    rng = np.random.default_rng(seed)
    if dtype is None:
        dtype = np.uint8 if L <= 8 else (np.uint16 if L <= 16 else np.uint32)
    hi = 1 << L
    return rng.integers(0, hi, size=n, dtype=np.uint64).astype(dtype)


def test_running_example(orc):
    g = pins.read_golden()
    T = np.array([int(x) for x in g["text"].split()], dtype=np.uint8)
    for kind, tag in ((WT, "wt"), (WM, "wm")):
        s = gpu_build(T, 3, kind)
        bits, zeros, *_ = s.host_arrays()
        assert [hex(int(w[0])) for w in bits] == g[f"{tag}_hex"].split()
        assert [int(z) for z in zeros] == [5, 5, 5]
        assert_matches_oracle(orc, T, 3, kind, s)


@pytest.mark.parametrize("L", [0, 1, 2, 3, 7, 8])
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 511, 513, 1023, 1024, 1025, 4097])
def test_small_edges(orc, n, L):
    T = _rand(n, L, seed=1000 + n * 10 + L)
    for kind in (WT, WM):
        assert_matches_oracle(orc, T, L, kind, gpu_build(T, L, kind))


@pytest.mark.parametrize("grid", [2, 3])
@pytest.mark.parametrize("L", [2, 5, 7, 8])
def test_many_tiles_ragged_tail(orc, grid, L):
    """Ranges of several 2048-symbol tiles (tune.grid ranges per text) and a
    short last tile."""
    B = lib()
    n = 7 * 2048 + 37  # 8 tiles in grid ranges of 3 or 4 tiles
    T = _rand(n, L, seed=7 + L)
    for kind in (WT, WM):
        s = gpu_build(T, L, kind, tune=B.make_tune(grid=grid))
        assert_matches_oracle(orc, T, L, kind, s)


@pytest.mark.parametrize("group_bits", [1, 2, 3, 5, 8])
def test_group_bits(orc, group_bits):
    """Several passes over a re-ordered copy of the text (levels in groups)."""
    B = lib()
    for L, n in ((8, 20000), (13, 9000)):
        T = _rand(n, L, seed=31 + group_bits)
        for kind in (WT, WM):
            s = gpu_build(T, L, kind, tune=B.make_tune(tile_log2=10, group_bits=group_bits))
            assert_matches_oracle(orc, T, L, kind, s)


@pytest.mark.parametrize("L,dtype", [(9, np.uint16), (16, np.uint16), (20, np.uint32),
                                     (26, np.uint32), (12, np.uint32)])
def test_wide_symbols(orc, L, dtype):
    T = _rand(30000, L, seed=L, dtype=dtype)
    for kind in (WT, WM):
        assert_matches_oracle(orc, T, L, kind, gpu_build(T, L, kind))


def test_32_levels(orc):
    T = _rand(20000, 32, seed=3, dtype=np.uint32)
    assert_matches_oracle(orc, T, 32, WM, gpu_build(T, 32, WM))
    B = lib()
    with pytest.raises(B.WtError) as e:
        gpu_build(T, 32, WT)
    assert e.value.code == B.WT_ENOTSUP


@pytest.mark.parametrize("case", ["one_symbol", "two_extremes", "alternating", "sorted", "u8_wide_L"])
def test_degenerate_texts(orc, case):
    n, L = 50000, 8
    if case == "one_symbol":
        T = np.full(n, 77, dtype=np.uint8)
    elif case == "two_extremes":
        T = np.where(_rand(n, 1, 5) == 1, 255, 0).astype(np.uint8)
    elif case == "alternating":
        T = np.tile(np.array([0, 128, 64, 192, 1, 129], dtype=np.uint8), n // 6 + 1)[:n]
    elif case == "sorted":
        T = np.sort(_rand(n, L, 9))
    else:
        L = 11  # byte text, 11 levels: the three top bits are always zero
        T = _rand(n, 8, 10)
    for kind in (WT, WM):
        assert_matches_oracle(orc, T, L, kind, gpu_build(T, L, kind))


def test_sigma_not_power_of_two(orc):
    rng = np.random.default_rng(4)
    T = rng.integers(0, 97, size=70000).astype(np.uint8)
    for kind in (WT, WM):
        assert_matches_oracle(orc, T, 7, kind, gpu_build(T, 7, kind))


@pytest.mark.parametrize("name,n", [("uniform256", 1 << 20), ("markov96", 1 << 22),
                                    ("markov4", 1 << 22), ("zipf20", 1 << 20),
                                    ("uniform16", 1 << 21)])
def test_workload_shapes(orc, name, n):
    from paper_1702_07578_amd import inputs
    T, L = inputs.make(name, n)
    for kind in (WT, WM):
        assert_matches_oracle(orc, T, L, kind, gpu_build(T, L, kind))


def test_symbol_out_of_range_sets_status():
    B = lib()
    T = np.array([0, 1, 2, 8, 3], dtype=np.uint8)
    for kind in (WT, WM):
        s = gpu_build(T, 3, kind)
        assert s.status() == B.WT_ERANGE
    T = np.zeros(100, dtype=np.uint8)
    T[50] = 1
    assert gpu_build(T, 0, WM).status() == B.WT_ERANGE
    assert gpu_build(np.zeros(100, dtype=np.uint8), 0, WM).status() == 0
