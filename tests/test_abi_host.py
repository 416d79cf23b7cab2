"""Host-side checks of the C ABI: the library loads, exports every function
include/wt.h declares, and its sizing, binding and argument checks behave
(no device work is enqueued by any call here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "wt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(w[tm]_[a-z_]+)\s*\(", src))
    return sorted(n for n in names if not n.startswith("wt_levels_t"))


def test_exports_every_declared_symbol():
    from paper_1702_07578_amd import binding as B
    names = _declared_functions()
    assert "wt_build" in names and "wm_build" in names and "wt_select" in names
    for n in names:
        assert hasattr(B.lib, n), n
        assert getattr(B.lib, n) is not None


def test_sizes_and_bind():
    from paper_1702_07578_amd import binding as B
    for n, L in ((0, 0), (10, 3), (1000, 8), (1 << 20, 8), (123457, 20)):
        nb = B.wt_output_bytes(n, L)
        W = ((n + 63) // 64 + 7) // 8 * 8
        assert nb >= L * W * 8
        v = B.WtLevels()
        fake = 1 << 40  # never dereferenced: binding only computes addresses
        assert B.wt_levels_bind(ctypes.byref(v), ctypes.c_void_p(fake), nb, n, L, 1) == 0
        assert v.words_per_level == W
        assert v.rank_stride >= W // 8 + 1 and v.sel_stride >= (n + 4095) // 4096 + 1
        assert v.bits == fake and v.status >= v.bits
        assert B.wt_levels_bind(ctypes.byref(v), ctypes.c_void_p(fake), nb - 257, n, L, 1) == B.WT_ENOSPACE
    assert B.wt_workspace_bytes(1 << 20, 1, 8, 0) > 0
    assert B.wt_workspace_bytes(1 << 20, 3, 8, 0) == 0
    assert B.wt_workspace_bytes(1 << 20, 4, 33, 1) == 0
    assert B.wt_workspace_bytes(1 << 32, 1, 8, 1) == 0


def test_argument_errors_return_before_device_work():
    from paper_1702_07578_amd import binding as B
    v = B.WtLevels()
    fake = ctypes.c_void_p(1 << 40)
    assert B.wt_levels_bind(ctypes.byref(v), fake, 1 << 20, 100, 3, 1) == 0
    # bad symbol width, too many levels, tree too deep, kind mismatch, no workspace
    assert B.wt_build_tuned(1, fake, 100, 3, 3, ctypes.byref(v), fake, 1 << 20, None, None) == B.WT_EINVAL
    assert B.wt_build_tuned(1, fake, 100, 1, 33, ctypes.byref(v), fake, 1 << 20, None, None) == B.WT_EINVAL
    assert B.wt_build_tuned(0, fake, 100, 4, 27, ctypes.byref(v), fake, 1 << 20, None, None) == B.WT_ENOTSUP
    assert B.wt_build_tuned(0, fake, 100, 1, 3, ctypes.byref(v), fake, 1 << 20, None, None) == B.WT_EINVAL
    assert B.wm_build(fake, 100, 1, 3, ctypes.byref(v), fake, 16, None) == B.WT_ENOSPACE
    assert B.wm_build(fake, 100, 1, 3, None, fake, 1 << 20, None) == B.WT_EINVAL
    assert B.wm_build(fake, 100, 1, 4, ctypes.byref(v), fake, 1 << 20, None) == B.WT_EINVAL
    assert B.wt_access(None, fake, 1, fake, None) == B.WT_EINVAL
    assert B.wt_strerror(B.WT_ERANGE).decode().startswith("symbol")
