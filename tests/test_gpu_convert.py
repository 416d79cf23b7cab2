"""WT <-> WM conversion and the Lemma 5 position map on the GPU, against the
oracle: a converted structure equals the oracle's structure of the other
kind (levels, Z, directories), and the position map equals the oracle's map
on every position of every level."""
import numpy as np
import pytest

from tests.gpu_util import assert_matches_oracle, gpu_build, lib

pytestmark = pytest.mark.gpu

WT, WM = 0, 1


def _texts():
    from paper_1702_07578_amd import inputs
    rng = np.random.default_rng(41)
    yield "example", np.array([0, 1, 6, 7, 1, 5, 4, 2, 6, 3], np.uint8), 3
    yield "small", rng.integers(0, 8, size=1, dtype=np.uint64).astype(np.uint8), 3
    yield "uniform8", inputs.uniform(70000, 256, 1, 3), 8
    yield "markov96", inputs.make("markov96", 200000)[0], 7
    yield "zipf16", inputs.zipf(90000, 1 << 16, 1.1, 2, 5), 16
    yield "sparse20", (rng.integers(0, 300, size=40000, dtype=np.uint64) * 3001 % (1 << 20)).astype(np.uint32), 20
    yield "one_level", rng.integers(0, 2, size=5000, dtype=np.uint64).astype(np.uint8), 1


@pytest.mark.parametrize("case", [c[0] for c in _texts()])
def test_convert_matches_oracle(orc, case):
    import torch
    B = lib()
    T, L = next((t, l) for name, t, l in _texts() if name == case)
    for kind in (WT, WM):
        s = gpu_build(T, L, kind)
        other = B.convert(s)
        torch.cuda.synchronize()
        assert other.kind == 1 - kind
        assert_matches_oracle(orc, T, L, 1 - kind, other)


@pytest.mark.parametrize("case", [c[0] for c in _texts()])
def test_position_map_matches_oracle(orc, case):
    import torch
    B = lib()
    T, L = next((t, l) for name, t, l in _texts() if name == case)
    n = T.size
    pos = torch.arange(n, dtype=torch.int64, device="cuda")
    for kind in (WT, WM):
        pm = B.PosMap(gpu_build(T, L, kind))
        for l in range(L):
            got = pm.query(l, pos).cpu().numpy().view(np.uint64)
            want = orc.map_wt_to_wm(T, L, l, np.arange(n))
            assert np.array_equal(got, want), (case, kind, l)
        # out-of-range positions and levels
        bad = torch.tensor([n, n + 5], dtype=torch.int64, device="cuda")
        assert (pm.query(0, bad).cpu().numpy().view(np.uint64) == np.uint64(2**64 - 1)).all()
        assert (pm.query(L, pos[:1]).cpu().numpy().view(np.uint64) == np.uint64(2**64 - 1)).all()


def test_convert_argument_errors():
    import ctypes
    import torch
    B = lib()
    T = np.arange(100, dtype=np.uint8) % 8
    s = gpu_build(T, 3, WT)
    same = B.Structure(100, 3, WT)
    ws = torch.empty(int(B.wt_convert_workspace_bytes(100, 3)), dtype=torch.uint8, device="cuda")
    rc = B.wt_convert(ctypes.byref(s.view), ctypes.byref(same.view), ctypes.c_void_p(ws.data_ptr()),
                      ws.numel(), None)
    assert rc == B.WT_EINVAL  # same kind
    other = B.Structure(100, 3, WM)
    rc = B.wt_convert(ctypes.byref(s.view), ctypes.byref(other.view), ctypes.c_void_p(ws.data_ptr()), 16, None)
    assert rc == B.WT_ENOSPACE
    assert B.wt_convert_workspace_bytes(100, 27) == 0
