"""Merging the structures of consecutive pieces of a text (domain
decomposition, Section 3.2, Lemma 4) gives the structure of the whole text: levels,
Z and directories equal the oracle's build of the concatenation."""
import numpy as np
import pytest

from tests.gpu_util import assert_matches_oracle, gpu_build, lib

pytestmark = pytest.mark.gpu

WT, WM = 0, 1


def _cases():
    from paper_1702_07578_amd import inputs
    rng = np.random.default_rng(51)
    yield "bytes", inputs.uniform(30000, 256, 1, 1), 8, [1000, 0, 1, 6427, 64, 2048 * 3 + 5, 16359]
    yield "markov", inputs.make("markov96", 50000)[0], 7, [25000, 25000]
    yield "dna", inputs.make("markov4", 40000)[0], 2, [7, 39993]
    yield "u16", inputs.zipf(20000, 1 << 16, 1.1, 2, 3), 16, [5000, 5001, 4999, 5000]
    yield "u32", rng.integers(0, 1 << 20, size=9000, dtype=np.uint64).astype(np.uint32), 20, [3000] * 3
    yield "single", inputs.uniform(4097, 8, 1, 2), 3, [4097]
    yield "empty_parts", inputs.uniform(500, 8, 1, 4), 3, [0, 500, 0]


@pytest.mark.parametrize("case", [c[0] for c in _cases()])
def test_merge_matches_oracle(orc, case):
    import torch
    B = lib()
    T, L, sizes = next((t, l, s) for name, t, l, s in _cases() if name == case)
    assert sum(sizes) == T.size
    cuts = np.cumsum([0] + sizes)
    for kind in (WT, WM):
        parts = [gpu_build(T[a:b], L, kind) for a, b in zip(cuts[:-1], cuts[1:])]
        whole = B.merge(parts)
        torch.cuda.synchronize()
        assert_matches_oracle(orc, T, L, kind, whole)


def test_merge_argument_errors():
    import ctypes
    B = lib()
    T = np.arange(200, dtype=np.uint8) % 8
    a = gpu_build(T[:100], 3, WT)
    b = gpu_build(T[100:], 3, WM)
    dst = B.Structure(200, 3, WT)
    arr = (B.WtLevels * 2)(a.view, b.view)
    rc = B.wt_merge(arr, 2, ctypes.byref(dst.view), ctypes.c_void_p(dst.buf.data_ptr()), 1 << 20, None)
    assert rc == B.WT_EINVAL  # kinds differ
    arr = (B.WtLevels * 1)(a.view)
    rc = B.wt_merge(arr, 1, ctypes.byref(dst.view), ctypes.c_void_p(dst.buf.data_ptr()), 1 << 20, None)
    assert rc == B.WT_EINVAL  # lengths do not add up
