"""Helpers for the GPU parity tests: build through the C ABI, copy back, and
compare element by element with the oracle."""
from __future__ import annotations

import numpy as np


def lib():
    from paper_1702_07578_amd import binding
    return binding


def gpu_build(T: np.ndarray, L: int, kind: int, tune=None):
    import torch
    B = lib()
    d = B.to_device(T)
    s = B.build(d, T.size, T.dtype.itemsize, L, kind, tune=tune)
    torch.cuda.synchronize()
    return s


def assert_matches_oracle(orc, T, L, kind, s, check_dirs=True):
    """Levels, Z and directories of the GPU structure s equal the oracle's."""
    n = T.size
    st = s.status()
    assert st == 0, f"status {st}"
    bits, zeros, rd, s0, s1 = s.host_arrays()
    ob, oz = orc.build(kind, T, L)
    assert bits.shape == ob.shape, (bits.shape, ob.shape)
    for l in range(L):
        if not np.array_equal(bits[l], ob[l]):
            bad = np.flatnonzero(bits[l] != ob[l])
            raise AssertionError(f"kind {kind} L {L} n {n}: level {l} differs in {bad.size} words, "
                                 f"first word {bad[0]}: gpu {bits[l][bad[0]]:#x} oracle {ob[l][bad[0]]:#x}")
    assert np.array_equal(zeros, oz), (zeros, oz)
    if check_dirs:
        W = ob.shape[1] if L else 0
        cap = orc.sel_capacity(n)
        for l in range(L):
            ord_, os0, os1 = orc.directory(ob[l], n)
            assert np.array_equal(rd[l][: W // 8 + 1], ord_), f"rank_dir level {l}"
            assert np.array_equal(s0[l][:cap], os0), f"sel0 level {l}"
            assert np.array_equal(s1[l][:cap], os1), f"sel1 level {l}"
