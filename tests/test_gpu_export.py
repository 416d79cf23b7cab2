"""Export of a built WT to node-local bit vectors (the pointer-based tree of
Section 2) on the GPU, against the oracle's pointer tree: the node table and
every pool word, bit for bit."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import gpu_build, lib

pytestmark = pytest.mark.gpu

WT, WM = 0, 1


def _texts():
    from paper_1702_07578_amd import inputs
    rng = np.random.default_rng(43)
    yield "example", np.array([0, 1, 6, 7, 1, 5, 4, 2, 6, 3], np.uint8), 3
    yield "single", np.array([5], np.uint8), 3
    yield "empty", np.zeros(0, np.uint8), 4
    yield "uniform8", inputs.uniform(70001, 256, 1, 3), 8
    yield "markov96", inputs.make("markov96", 200000)[0], 7
    yield "zipf16", inputs.zipf(90000, 1 << 16, 1.1, 2, 5), 16
    yield "sparse20", (rng.integers(0, 300, size=40000, dtype=np.uint64) * 3001 % (1 << 20)).astype(np.uint32), 20
    yield "one_level", rng.integers(0, 2, size=5000, dtype=np.uint64).astype(np.uint8), 1


@pytest.mark.parametrize("case", [c[0] for c in _texts()])
def test_export_matches_oracle(orc, case):
    import torch
    B = lib()
    T, L = next((t, l) for name, t, l in _texts() if name == case)
    s = gpu_build(T, L, WT)
    nodes, pool = B.export_nodes(s)
    torch.cuda.synchronize()
    want_nodes, want_pool = orc.pointer_tree(T, L)
    got_nodes = nodes.cpu().numpy().view(np.uint64)
    assert np.array_equal(got_nodes, want_nodes), case
    got_pool = pool.cpu().numpy().view(np.uint64)
    assert got_pool.size == max(int(B.wt_export_pool_words(T.size, L)), 1)
    used = int(want_nodes[-1, 0] + (want_nodes[-1, 1] + 63) // 64) if want_nodes.size else 0
    assert np.array_equal(got_pool[:used], want_pool[:used]), case
    # the words past the last node's run are cleared
    assert not got_pool[used:want_pool.size].any()


def test_export_refuses_a_wavelet_matrix_and_short_pools():
    import torch
    B = lib()
    T = np.arange(1000, dtype=np.uint64).astype(np.uint8)
    m = gpu_build(T, 8, WM)
    buf = torch.zeros(1 << 16, dtype=torch.int64, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    need = int(B.wt_convert_workspace_bytes(1000, 8))
    assert B.wt_export_nodes(ctypes.byref(m.view), p, p, 1 << 12, p, need, None) == B.WT_EINVAL
    t = gpu_build(T, 8, WT)
    words = int(B.wt_export_pool_words(1000, 8))
    assert B.wt_export_nodes(ctypes.byref(t.view), p, p, words - 1, p, need, None) == B.WT_ENOSPACE
    assert B.wt_export_nodes(ctypes.byref(t.view), p, p, words, p, need - 1, None) == B.WT_ENOSPACE
    torch.cuda.synchronize()
