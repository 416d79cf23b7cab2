"""wt_pair_build_noalloc (the pair build with the library's per-GPU scratch
as workspace) against wt_pair_build (caller workspace) and the oracle.

Calls in a row share one scratch, which keeps the last call's contents, so
each case follows a larger one: a second call with a smaller text (and other
levels) must not see the first call's tables.  Every output the structure
defines (level words with their padding, Z, every directory entry, status)
must be equal, bit for bit."""
import numpy as np
import pytest

from tests.gpu_util import assert_matches_oracle, lib

pytestmark = pytest.mark.gpu

WT, WM = 0, 1


def _outputs(orc, s):
    """the defined part of every output array of a structure"""
    bits, zeros, rd, s0, s1 = s.host_arrays()
    W = s.view.words_per_level
    cap = orc.sel_capacity(s.n)
    return [bits, zeros, rd[:, : W // 8 + 1], s0[:, :cap], s1[:, :cap], np.array([s.status()])]


def _text(n, L, seed, dtype):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << L, size=n, dtype=np.uint64).astype(dtype)


def _both(T, L):
    import torch
    B = lib()
    n, b = T.size, T.dtype.itemsize
    d = B.to_device(T)
    ref = B.pair_build(d, n, b, L)
    torch.cuda.synchronize()
    out = (B.Structure(n, L, WT), B.Structure(n, L, WM))
    for s in out:  # the outputs start as garbage, as after an earlier build
        s.buf.fill_(0xA5)
    B.pair_build_noalloc(d, n, b, L, out)
    torch.cuda.synchronize()
    return ref, out


def _check(orc, T, L, with_oracle):
    print(f"[no_alloc] n={T.size} b={T.dtype.itemsize} L={L}", flush=True)
    ref, got = _both(T, L)
    for kind, r, g in ((WT, ref[0], got[0]), (WM, ref[1], got[1])):
        for i, (a, b) in enumerate(zip(_outputs(orc, r), _outputs(orc, g))):
            assert np.array_equal(a, b), f"kind {kind}: output array {i} differs from wt_pair_build"
        if with_oracle:
            assert_matches_oracle(orc, T, L, kind, g)


def test_two_calls_second_smaller(orc):
    """a long byte text (three tiles per scatter range), then a short one"""
    _check(orc, _text((1 << 26) + 777, 8, 11, np.uint8), 8, with_oracle=False)
    _check(orc, _text(70001, 5, 12, np.uint8), 5, with_oracle=True)


def test_several_groups_then_smaller(orc):
    """16-bit symbols over two groups of levels (WM build, then the WT
    gathered from it, both inside the scratch), then shorter texts"""
    _check(orc, _text(300007, 12, 13, np.uint16), 12, with_oracle=True)
    _check(orc, _text(4097, 3, 14, np.uint8), 3, with_oracle=True)
    _check(orc, _text(0, 3, 15, np.uint8), 3, with_oracle=True)


def test_too_large_is_refused():
    """more workspace than the scratch holds: WT_ENOSPACE, nothing enqueued"""
    B = lib()
    n, L = 1 << 26, 16
    assert B.wt_pair_workspace_bytes(n, 2, L) > B.WT_NOALLOC_SCRATCH_BYTES
    wt, wm = B.Structure(1, 1, WT), B.Structure(1, 1, WM)
    import ctypes
    rc = B.wt_pair_build_noalloc(ctypes.c_void_p(wt.buf.data_ptr()), n, 2, L, ctypes.byref(wt.view),
                                 ctypes.byref(wm.view), None)
    assert rc == B.WT_ENOSPACE
