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


def test_binding_constants_match_header():
    from paper_1702_07578_amd import binding as B
    src = open(os.path.join(ROOT, "include", "wt.h")).read()
    m = re.search(r"#define WT_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == B.WT_NOALLOC_SCRATCH_BYTES
    m = re.search(r"#define WT_MAX_TREE_LEVELS (\d+)", src)
    assert m and int(m.group(1)) == B.WT_MAX_TREE_LEVELS


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
    # the allocation-free pair build checks sizes before it looks for a device
    assert B.wt_pair_workspace_bytes(1 << 26, 2, 16) > B.WT_NOALLOC_SCRATCH_BYTES
    assert B.wt_pair_build_noalloc(fake, 1 << 26, 2, 16, ctypes.byref(v), ctypes.byref(v), None) == B.WT_ENOSPACE
    assert B.wt_pair_build_noalloc(fake, 100, 3, 3, ctypes.byref(v), ctypes.byref(v), None) == B.WT_EINVAL


def test_conversion_and_position_map_sizes():
    """Host-side sizing and binding of the conversion workspace and the
    position map (no device work)."""
    from paper_1702_07578_amd import binding as B
    assert B.wt_convert_workspace_bytes(1000, 8) > 3 * (2 ** 9) * 4
    assert B.wt_convert_workspace_bytes(1000, B.WT_MAX_TREE_LEVELS + 1) == 0
    assert B.wt_posmap_bytes(1000, 27) == 0
    assert B.wt_posmap_bytes((1 << 32) - 10, 4) == 0  # n + 2^L must stay below 2^32
    nbytes = B.wt_posmap_bytes(1000, 8)
    m = B.WtPosmap()
    assert B.wt_posmap_bind(ctypes.byref(m), ctypes.c_void_p(4096), nbytes, 1000, 8) == B.WT_OK
    assert m.u_len == 1000 + 256 and m.u_words % 8 == 0 and m.u_words * 64 >= m.u_len
    assert m.U % 256 == 0 and m.rank_dir > m.U and m.sel0 > m.rank_dir and m.sel1 > m.sel0 and m.X > m.sel1
    assert m.X + (256 - 1) * 4 <= 4096 + nbytes
    assert B.wt_posmap_bind(ctypes.byref(m), ctypes.c_void_p(4096), nbytes - 512, 1000, 8) == B.WT_ENOSPACE
    assert B.wt_posmap_bind(None, ctypes.c_void_p(4096), nbytes, 1000, 8) == B.WT_EINVAL
    # views that do not describe the same text are refused before any device work
    a, b = B.WtLevels(), B.WtLevels()
    out = B.wt_output_bytes(1000, 8)
    assert B.wt_levels_bind(ctypes.byref(a), ctypes.c_void_p(1 << 20), out, 1000, 8, 0) == B.WT_OK
    assert B.wt_levels_bind(ctypes.byref(b), ctypes.c_void_p(1 << 24), out, 1000, 8, 0) == B.WT_OK
    assert B.wt_convert(ctypes.byref(a), ctypes.byref(b), ctypes.c_void_p(1 << 28), 1 << 20, None) == B.WT_EINVAL


def test_export_sizes_and_refusals():
    """Pool bound of the node-local export and its refusals before any
    device work."""
    from paper_1702_07578_amd import binding as B
    assert B.wt_export_pool_words(1000, 8) == 8 * 16 + 255
    assert B.wt_export_pool_words(1000, 0) == 0
    assert B.wt_export_pool_words(1000, B.WT_MAX_TREE_LEVELS + 1) == 0
    v = B.WtLevels()
    out = B.wt_output_bytes(1000, 8)
    fake = ctypes.c_void_p(1 << 20)
    assert B.wt_levels_bind(ctypes.byref(v), fake, out, 1000, 8, 1) == B.WT_OK
    ws = B.wt_convert_workspace_bytes(1000, 8)
    assert B.wt_export_nodes(ctypes.byref(v), fake, fake, 1 << 12, fake, ws, None) == B.WT_EINVAL  # a WM
    assert B.wt_levels_bind(ctypes.byref(v), fake, out, 1000, 8, 0) == B.WT_OK
    assert B.wt_export_nodes(ctypes.byref(v), fake, fake, 100, fake, ws, None) == B.WT_ENOSPACE
    assert B.wt_export_nodes(ctypes.byref(v), fake, fake, 1 << 12, fake, ws - 1, None) == B.WT_ENOSPACE
    assert B.wt_export_nodes(ctypes.byref(v), None, fake, 1 << 12, fake, ws, None) == B.WT_EINVAL


def test_sorting_build_sizes_and_refusals():
    """Workspace of the sorting build and its host-side refusals."""
    from paper_1702_07578_amd import binding as B
    assert B.wt_ps_workspace_bytes(1 << 20, 1, 7) >= (1 << 20)  # the sorted copy
    assert B.wt_ps_workspace_bytes(1 << 20, 4, 12) >= 4 << 20
    assert B.wt_ps_workspace_bytes(1 << 20, 2, 13) == 0
    assert B.wt_ps_workspace_bytes(1 << 20, 3, 8) == 0
    v = B.WtLevels()
    fake = ctypes.c_void_p(1 << 20)
    assert B.wt_levels_bind(ctypes.byref(v), fake, B.wt_output_bytes(1000, 8), 1000, 8, 0) == B.WT_OK
    need = B.wt_ps_workspace_bytes(1000, 1, 8)
    assert B.wt_ps_build(0, fake, 1000, 1, 8, ctypes.byref(v), fake, need - 1, None) == B.WT_ENOSPACE
    assert B.wt_ps_build(1, fake, 1000, 1, 8, ctypes.byref(v), fake, need, None) == B.WT_EINVAL  # kind mismatch
    assert B.wt_ps_build(0, ctypes.c_void_p((1 << 20) + 1), 1000, 2, 8, ctypes.byref(v), fake, need,
                         None) == B.WT_EINVAL  # misaligned u16 text


def test_binding_uses_torchs_hip_runtime():
    """Importing the binding first (before torch) must still bind the library
    to the HIP runtime torch ships: two runtimes in one process would hand the
    library streams and memory it does not know."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1702_07578_amd import binding\n"
            "maps = [l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l]\n"
            "print('\\n'.join(sorted(set(maps))))\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    loaded = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(loaded) == 1, loaded
    assert os.sep + "torch" + os.sep in loaded[0], loaded
