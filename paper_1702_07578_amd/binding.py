"""ctypes binding of ``libwt.so`` (the C ABI of include/wt.h).

Argument marshalling only: every step of a build or a query runs in the HIP
kernels of the library.  PyTorch provides device memory and streams.  Importing
this module fails loudly when the library has not been built.

Names follow the C ABI: ``wt_output_bytes``, ``wt_workspace_bytes``,
``wt_levels_bind``, ``wt_build``, ``wm_build``, ``wt_build_tuned``,
``wt_access``, ``wt_rank``, ``wt_select``, ``wt_get_status``,
``wt_batch_workspace_bytes``, ``wt_batch_build``, ``wt_build_profiled``,
``wt_build_recorded``.
On top of them, ``Structure`` owns the torch buffers of one built index.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwt.so")

WT_TREE, WT_MATRIX = 0, 1
WT_OK, WT_EINVAL, WT_ENOSPACE, WT_ERANGE, WT_EHIP, WT_ENOTSUP = 0, -1, -2, -3, -4, -5
WT_MAX_TREE_LEVELS = 26
WT_SEL_SPACING = 4096
WT_NUM_KERNEL_IDS = 16
WT_NOALLOC_SCRATCH_BYTES = 64 << 20

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python __graft_entry__.py build or "
                      "python -m paper_1702_07578_amd.build_lib)")


class WtLevels(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("lg_sigma", ctypes.c_uint32),
        ("kind", ctypes.c_uint32),
        ("words_per_level", ctypes.c_uint64),
        ("rank_stride", ctypes.c_uint64),
        ("sel_stride", ctypes.c_uint64),
        ("bits", ctypes.c_void_p),
        ("zeros", ctypes.c_void_p),
        ("rank_dir", ctypes.c_void_p),
        ("sel0", ctypes.c_void_p),
        ("sel1", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


class WtTune(ctypes.Structure):
    _fields_ = [("tile_log2", ctypes.c_uint32), ("group_bits", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("persist", ctypes.c_uint32)]


class WtBatchItem(ctypes.Structure):
    _fields_ = [("d_text", ctypes.c_void_p), ("n", ctypes.c_uint64), ("sym_bytes", ctypes.c_uint32),
                ("lg_sigma", ctypes.c_uint32), ("kind", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("out", ctypes.POINTER(WtLevels))]


class WtPosmap(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("lg_sigma", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("u_len", ctypes.c_uint64), ("u_words", ctypes.c_uint64),
                ("rank_stride", ctypes.c_uint64), ("sel_stride", ctypes.c_uint64),
                ("U", ctypes.c_void_p), ("rank_dir", ctypes.c_void_p), ("sel0", ctypes.c_void_p),
                ("sel1", ctypes.c_void_p), ("X", ctypes.c_void_p)]


# PyTorch first: it ships the HIP runtime it was built for, under the same
# soname as the system's, and whichever is loaded first serves the whole
# process.  The library must use torch's, the runtime that owns the streams
# and the memory it is handed.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)
_v, _u64, _u32, _i, _sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
_LP = ctypes.POINTER(WtLevels)
_TP = ctypes.POINTER(WtTune)
_SIGS = {
    "wt_output_bytes": (_sz, [_u64, _u32]),
    "wt_workspace_bytes": (_sz, [_u64, _u32, _u32, _i]),
    "wt_workspace_bytes_tuned": (_sz, [_u64, _u32, _u32, _i, _TP]),
    "wt_levels_bind": (_i, [_LP, _v, _sz, _u64, _u32, _i]),
    "wt_build": (_i, [_v, _u64, _u32, _u32, _LP, _v, _sz, _v]),
    "wm_build": (_i, [_v, _u64, _u32, _u32, _LP, _v, _sz, _v]),
    "wt_build_tuned": (_i, [_i, _v, _u64, _u32, _u32, _LP, _v, _sz, _TP, _v]),
    "wt_access": (_i, [_LP, _v, _u64, _v, _v]),
    "wt_rank": (_i, [_LP, _v, _v, _u64, _v, _v]),
    "wt_select": (_i, [_LP, _v, _v, _u64, _v, _v]),
    "wt_get_status": (_i, [_LP, _v]),
    "wt_strerror": (ctypes.c_char_p, [_i]),
    "wt_batch_workspace_bytes": (_sz, [ctypes.POINTER(WtBatchItem), _u32, _TP]),
    "wt_batch_build": (_i, [ctypes.POINTER(WtBatchItem), _u32, _v, _sz, _TP, _v]),
    "wt_batch_prepare": (_i, [ctypes.POINTER(WtBatchItem), _u32, _v, _sz, _TP, _v]),
    "wt_batch_launch": (_i, [ctypes.POINTER(WtBatchItem), _u32, _v, _sz, _TP, _v]),
    "wt_build_profiled": (_i, [_i, _v, _u64, _u32, _u32, _LP, _v, _sz, _TP, _v,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint32), _u32]),
    "wt_kernel_name": (ctypes.c_char_p, [_u32]),
    "wt_convert_workspace_bytes": (_sz, [_u64, _u32]),
    "wt_convert": (_i, [_LP, _LP, _v, _sz, _v]),
    "wt_merge_workspace_bytes": (_sz, [_u64, _u32, _u32]),
    "wt_merge": (_i, [_LP, _u32, _LP, _v, _sz, _v]),
    "wt_pair_workspace_bytes": (_sz, [_u64, _u32, _u32]),
    "wt_pair_build": (_i, [_v, _u64, _u32, _u32, _LP, _LP, _v, _sz, _v]),
    "wt_pair_workspace_bytes_tuned": (_sz, [_u64, _u32, _u32, _TP]),
    "wt_pair_build_tuned": (_i, [_v, _u64, _u32, _u32, _LP, _LP, _v, _sz, _TP, _v]),
    "wt_pair_build_noalloc": (_i, [_v, _u64, _u32, _u32, _LP, _LP, _v]),
    "wt_pair_build_recorded": (_i, [_v, _u64, _u32, _u32, _LP, _LP, _v, _sz, _v, ctypes.POINTER(_v),
                                    ctypes.POINTER(_u32), _u32, ctypes.POINTER(_u32)]),
    "wt_ps_workspace_bytes": (_sz, [_u64, _u32, _u32]),
    "wt_ps_build": (_i, [_i, _v, _u64, _u32, _u32, _LP, _v, _sz, _v]),
    "wt_export_pool_words": (_u64, [_u64, _u32]),
    "wt_export_nodes": (_i, [_LP, _v, _v, _u64, _v, _sz, _v]),
    "wt_posmap_bytes": (_sz, [_u64, _u32]),
    "wt_posmap_bind": (_i, [ctypes.POINTER(WtPosmap), _v, _sz, _u64, _u32]),
    "wt_posmap_build": (_i, [_LP, ctypes.POINTER(WtPosmap), _v, _sz, _v]),
    "wt_posmap_query": (_i, [ctypes.POINTER(WtPosmap), _u32, _v, _u64, _v, _v]),
    "wt_build_recorded": (_i, [_i, _v, _u64, _u32, _u32, _LP, _v, _sz, _TP, _v,
                               ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint32),
                               _u32, ctypes.POINTER(ctypes.c_uint32)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class WtError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib.wt_strerror(code).decode()
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


def check(code: int, what: str):
    if code != WT_OK:
        raise WtError(code, what)


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_tune(tile_log2=0, group_bits=0, grid=0, persist=0):
    if not (tile_log2 or group_bits or grid or persist):
        return None
    return WtTune(tile_log2, group_bits, grid, persist)


def _tune_ptr(tune):
    return ctypes.byref(tune) if tune is not None else None


def sym_bytes_of(dtype) -> int:
    return {np.dtype(np.uint8): 1, np.dtype(np.uint16): 2, np.dtype(np.uint32): 4}[np.dtype(dtype)]


def to_device(arr: np.ndarray, device="cuda"):
    """Copy a numpy array to a device byte tensor (the library takes raw pointers)."""
    torch = _torch()
    a = np.ascontiguousarray(arr)
    t = torch.from_numpy(a.view(np.uint8).reshape(-1)) if a.size else torch.zeros(0, dtype=torch.uint8)
    return t.to(device)


def workspace_bytes(n, sym_bytes, L, kind, tune=None) -> int:
    return int(wt_workspace_bytes_tuned(n, sym_bytes, L, kind, _tune_ptr(tune)))


class Structure:
    """One WT or WM resident in device memory: its output buffer and view."""

    def __init__(self, n: int, L: int, kind: int, device="cuda"):
        torch = _torch()
        nbytes = int(wt_output_bytes(n, L))
        if nbytes == 0:
            raise WtError(WT_EINVAL, "wt_output_bytes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.view = WtLevels()
        check(wt_levels_bind(ctypes.byref(self.view), ctypes.c_void_p(self.buf.data_ptr()), nbytes, n,
                             L, kind), "wt_levels_bind")
        self.n, self.L, self.kind = n, L, kind

    @property
    def nbytes(self) -> int:
        return self.buf.numel()

    def _slice(self, ptr, count, itemsize):
        off = ptr - self.buf.data_ptr()
        return self.buf[off: off + count * itemsize]

    def host_arrays(self):
        """(bits [L,W] u64, zeros [L] u64, rank_dir [L,rank_stride] u32,
        sel0, sel1 [L,sel_stride] u32) copied to host numpy arrays."""
        v = self.view
        L, W = self.L, v.words_per_level
        host = self.buf.cpu().numpy()
        base = self.buf.data_ptr()

        def get(ptr, count, dt):
            off = ptr - base
            return host[off: off + count * np.dtype(dt).itemsize].view(dt)

        bits = get(v.bits, L * W, np.uint64).reshape(L, W)
        zeros = get(v.zeros, L, np.uint64)
        rd = get(v.rank_dir, L * v.rank_stride, np.uint32).reshape(L, v.rank_stride)
        s0 = get(v.sel0, L * v.sel_stride, np.uint32).reshape(L, v.sel_stride)
        s1 = get(v.sel1, L * v.sel_stride, np.uint32).reshape(L, v.sel_stride)
        return bits, zeros, rd, s0, s1

    def status(self, stream=None) -> int:
        return int(wt_get_status(ctypes.byref(self.view), _stream_handle(stream)))

    # -- queries (device tensors in, device tensors out) -----------------------
    def access(self, pos, stream=None):
        torch = _torch()
        pos = pos.contiguous()
        out = torch.empty(pos.numel(), dtype=torch.int32, device=pos.device)
        check(wt_access(ctypes.byref(self.view), ctypes.c_void_p(pos.data_ptr()), pos.numel(),
                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "wt_access")
        return out

    def rank(self, sym, pos, stream=None):
        torch = _torch()
        sym, pos = sym.contiguous(), pos.contiguous()
        out = torch.empty(pos.numel(), dtype=torch.int64, device=pos.device)
        check(wt_rank(ctypes.byref(self.view), ctypes.c_void_p(sym.data_ptr()),
                      ctypes.c_void_p(pos.data_ptr()), pos.numel(), ctypes.c_void_p(out.data_ptr()),
                      _stream_handle(stream)), "wt_rank")
        return out

    def select(self, sym, k, stream=None):
        torch = _torch()
        sym, k = sym.contiguous(), k.contiguous()
        out = torch.empty(k.numel(), dtype=torch.int64, device=k.device)
        check(wt_select(ctypes.byref(self.view), ctypes.c_void_p(sym.data_ptr()),
                        ctypes.c_void_p(k.data_ptr()), k.numel(), ctypes.c_void_p(out.data_ptr()),
                        _stream_handle(stream)), "wt_select")
        return out


def build(d_text, n: int, sym_bytes: int, L: int, kind: int, tune=None, stream=None, ws=None,
          out: Structure | None = None) -> Structure:
    """Build a WT (kind 0) or WM (kind 1) of the device byte tensor d_text
    (n symbols of sym_bytes bytes) and return its Structure."""
    torch = _torch()
    dev = d_text.device
    s = out if out is not None else Structure(n, L, kind, device=dev)
    need = workspace_bytes(n, sym_bytes, L, kind, tune)
    if need == 0:
        # invalid or unsupported configuration: the build call reports which,
        # from its host-side checks, before any device work
        check(wt_build_tuned(kind, ctypes.c_void_p(d_text.data_ptr() if n else 0), n, sym_bytes, L,
                             ctypes.byref(s.view), None, 0, _tune_ptr(tune), None),
              "wt_build_tuned")
        raise WtError(WT_EINVAL, "wt_workspace_bytes")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ptr = ctypes.c_void_p(d_text.data_ptr()) if n > 0 else ctypes.c_void_p(ws.data_ptr())
    check(wt_build_tuned(kind, ptr, n, sym_bytes, L, ctypes.byref(s.view),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _tune_ptr(tune),
                         _stream_handle(stream)), "wt_build_tuned")
    s._ws = ws  # keep alive until the caller synchronises
    return s


def pair_build(d_text, n: int, sym_bytes: int, L: int, stream=None, ws=None, out=None, tune=None):
    """The WT and the WM of one text (wt_pair_build, or wt_pair_build_tuned
    with tune): one pass writes both when L <= 8.  Returns (wt, wm)
    Structures; out = (wt, wm) reuses buffers."""
    torch = _torch()
    dev = d_text.device
    wt, wm = out if out is not None else (Structure(n, L, WT_TREE, device=dev), Structure(n, L, WT_MATRIX, device=dev))
    need = int(wt_pair_workspace_bytes_tuned(n, sym_bytes, L, _tune_ptr(tune)))
    if need == 0:
        check(wt_pair_build_tuned(ctypes.c_void_p(d_text.data_ptr() if n else 0), n, sym_bytes, L,
                                  ctypes.byref(wt.view), ctypes.byref(wm.view), None, 0, _tune_ptr(tune), None),
              "wt_pair_build")
        raise WtError(WT_EINVAL, "wt_pair_workspace_bytes")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ptr = ctypes.c_void_p(d_text.data_ptr()) if n > 0 else ctypes.c_void_p(ws.data_ptr())
    if tune is None:
        rc = wt_pair_build(ptr, n, sym_bytes, L, ctypes.byref(wt.view), ctypes.byref(wm.view),
                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream))
    else:
        rc = wt_pair_build_tuned(ptr, n, sym_bytes, L, ctypes.byref(wt.view), ctypes.byref(wm.view),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _tune_ptr(tune), _stream_handle(stream))
    check(rc, "wt_pair_build")
    wt._ws = ws
    return wt, wm


def pair_build_noalloc(d_text, n: int, sym_bytes: int, L: int, out, stream=None):
    """wt_pair_build_noalloc: both structures into out = (wt, wm), already
    bound Structures, with the library's own per-GPU scratch as workspace (no
    device allocation in the call)."""
    wt, wm = out
    ptr = ctypes.c_void_p(d_text.data_ptr() if n > 0 else 0)
    check(wt_pair_build_noalloc(ptr, n, sym_bytes, L, ctypes.byref(wt.view), ctypes.byref(wm.view),
                                _stream_handle(stream)), "wt_pair_build_noalloc")
    return wt, wm


def ps_build(d_text, n: int, sym_bytes: int, L: int, kind: int, stream=None, ws=None,
             out: Structure | None = None) -> Structure:
    """Build by sorting (wt_ps_build): the same structure as build(), by a
    counting sort of the text per level."""
    torch = _torch()
    dev = d_text.device
    s = out if out is not None else Structure(n, L, kind, device=dev)
    need = int(wt_ps_workspace_bytes(n, sym_bytes, L))
    if need == 0:
        check(wt_ps_build(kind, ctypes.c_void_p(d_text.data_ptr() if n else 0), n, sym_bytes, L,
                          ctypes.byref(s.view), None, 0, None), "wt_ps_build")
        raise WtError(WT_EINVAL, "wt_ps_workspace_bytes")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ptr = ctypes.c_void_p(d_text.data_ptr()) if n > 0 else ctypes.c_void_p(ws.data_ptr())
    check(wt_ps_build(kind, ptr, n, sym_bytes, L, ctypes.byref(s.view), ctypes.c_void_p(ws.data_ptr()),
                      ws.numel(), _stream_handle(stream)), "wt_ps_build")
    s._ws = ws
    return s


def build_profiled(d_text, n, sym_bytes, L, kind, tune=None, stream=None, ws=None, out=None):
    """One synchronous build with a HIP event after every kernel; returns
    (Structure, {kernel name: (ms, launches)})."""
    torch = _torch()
    dev = d_text.device
    s = out if out is not None else Structure(n, L, kind, device=dev)
    need = workspace_bytes(n, sym_bytes, L, kind, tune)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ms = (ctypes.c_double * WT_NUM_KERNEL_IDS)()
    cnt = (ctypes.c_uint32 * WT_NUM_KERNEL_IDS)()
    ptr = ctypes.c_void_p(d_text.data_ptr()) if n > 0 else ctypes.c_void_p(ws.data_ptr())
    check(wt_build_profiled(kind, ptr, n, sym_bytes, L, ctypes.byref(s.view),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _tune_ptr(tune),
                            _stream_handle(stream), ms, cnt, WT_NUM_KERNEL_IDS), "wt_build_profiled")
    res = {}
    for i in range(WT_NUM_KERNEL_IDS):
        if cnt[i]:
            res[wt_kernel_name(i).decode()] = (ms[i], cnt[i])
    s._ws = ws
    return s, res


def convert(s: Structure, stream=None) -> Structure:
    """The other structure (WT from a WM, WM from a WT) of the same text,
    gathered interval by interval (wt_convert)."""
    torch = _torch()
    dst = Structure(s.n, s.L, 1 - s.kind, device=s.buf.device)
    need = int(wt_convert_workspace_bytes(s.n, s.L))
    if need == 0:
        raise WtError(WT_ENOTSUP, "wt_convert_workspace_bytes")
    ws = torch.empty(need, dtype=torch.uint8, device=s.buf.device)
    check(wt_convert(ctypes.byref(s.view), ctypes.byref(dst.view), ctypes.c_void_p(ws.data_ptr()), need,
                     _stream_handle(stream)), "wt_convert")
    dst._ws = ws
    return dst


def merge(parts, stream=None) -> Structure:
    """The structure of the concatenated text from the structures of its
    consecutive pieces (same kind and levels), by wt_merge."""
    torch = _torch()
    n = sum(p.n for p in parts)
    L, kind = parts[0].L, parts[0].kind
    dst = Structure(n, L, kind, device=parts[0].buf.device)
    need = int(wt_merge_workspace_bytes(n, L, len(parts)))
    if need == 0:
        raise WtError(WT_ENOTSUP, "wt_merge_workspace_bytes")
    ws = torch.empty(need, dtype=torch.uint8, device=dst.buf.device)
    arr = (WtLevels * len(parts))(*[p.view for p in parts])
    check(wt_merge(arr, len(parts), ctypes.byref(dst.view), ctypes.c_void_p(ws.data_ptr()), need,
                   _stream_handle(stream)), "wt_merge")
    dst._ws = ws
    return dst


def export_nodes(s: Structure, stream=None):
    """Node-local bit vectors of a built WT (wt_export_nodes): a node table
    (int64 [2^L - 1, 2]: first pool word, bits; node 2^l - 1 + p is prefix p
    of length l) and the pool of words (int64) holding every node's bits from
    a fresh word."""
    torch = _torch()
    L = s.L
    dev = s.buf.device
    entries = (1 << L) - 1
    nodes = torch.empty((max(entries, 1), 2), dtype=torch.int64, device=dev)
    pool_words = int(wt_export_pool_words(s.n, L))
    pool = torch.empty(max(pool_words, 1), dtype=torch.int64, device=dev)
    need = int(wt_convert_workspace_bytes(s.n, L))
    if need == 0:
        raise WtError(WT_ENOTSUP, "wt_convert_workspace_bytes")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    check(wt_export_nodes(ctypes.byref(s.view), ctypes.c_void_p(nodes.data_ptr()),
                          ctypes.c_void_p(pool.data_ptr()), pool_words, ctypes.c_void_p(ws.data_ptr()), need,
                          _stream_handle(stream)), "wt_export_nodes")
    s._export_ws = ws
    return nodes[:entries], pool


class PosMap:
    """Lemma 5 position map of a built WT or WM: query(level, positions)
    returns, for WT positions of that level, the WM positions of the same
    bits."""

    def __init__(self, s: Structure, stream=None):
        torch = _torch()
        nbytes = int(wt_posmap_bytes(s.n, s.L))
        if nbytes == 0:
            raise WtError(WT_ENOTSUP, "wt_posmap_bytes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=s.buf.device)
        self.view = WtPosmap()
        check(wt_posmap_bind(ctypes.byref(self.view), ctypes.c_void_p(self.buf.data_ptr()), nbytes, s.n,
                             s.L), "wt_posmap_bind")
        need = int(wt_convert_workspace_bytes(s.n, s.L))
        ws = torch.empty(need, dtype=torch.uint8, device=s.buf.device)
        check(wt_posmap_build(ctypes.byref(s.view), ctypes.byref(self.view), ctypes.c_void_p(ws.data_ptr()),
                              need, _stream_handle(stream)), "wt_posmap_build")
        self._ws = ws

    def query(self, level: int, pos, stream=None):
        torch = _torch()
        pos = pos.contiguous()
        out = torch.empty(pos.numel(), dtype=torch.int64, device=pos.device)
        check(wt_posmap_query(ctypes.byref(self.view), level, ctypes.c_void_p(pos.data_ptr()), pos.numel(),
                              ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "wt_posmap_query")
        return out


class Batch:
    """A batch of texts bound to one workspace: prepare() uploads the
    descriptors (host call), launch() enqueues the kernels only (capturable in
    a graph), build() does both.  items: list of (d_text, n, sym_bytes, L,
    kind, Structure)."""

    @staticmethod
    def item_array(items):
        arr = (WtBatchItem * len(items))()
        for i, (t, n, b, L, kind, s) in enumerate(items):
            arr[i] = WtBatchItem(ctypes.c_void_p(t.data_ptr() if n > 0 else s.buf.data_ptr()), n, b, L,
                                 kind, 0, ctypes.pointer(s.view))
        return arr

    def __init__(self, items, tune=None, ws=None):
        torch = _torch()
        self.items = items
        self.tune = tune
        self.arr = Batch.item_array(items)
        need = int(wt_batch_workspace_bytes(self.arr, len(items), _tune_ptr(tune)))
        if need == 0:
            raise WtError(WT_EINVAL, "wt_batch_workspace_bytes")
        dev = items[0][5].buf.device
        self.ws = ws if (ws is not None and ws.numel() >= need) else torch.empty(need, dtype=torch.uint8,
                                                                                 device=dev)

    def _args(self, stream):
        return (self.arr, len(self.items), ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                _tune_ptr(self.tune), _stream_handle(stream))

    def prepare(self, stream=None):
        check(wt_batch_prepare(*self._args(stream)), "wt_batch_prepare")

    def launch(self, stream=None):
        check(wt_batch_launch(*self._args(stream)), "wt_batch_launch")

    def build(self, stream=None):
        check(wt_batch_build(*self._args(stream)), "wt_batch_build")


def batch_build(items, tune=None, stream=None, ws=None):
    """items: list of (d_text, n, sym_bytes, L, kind, Structure); returns the Batch."""
    b = Batch(items, tune=tune, ws=ws)
    b.build(stream)
    return b


class EventRecorder:
    """Caller-owned timing events for wt_build_recorded (torch events with
    timing enabled; their raw handles are passed to the library)."""

    def __init__(self, capacity: int):
        torch = _torch()
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(capacity)]
        for e in self.events:  # instantiate the underlying HIP events
            e.record()
        torch.cuda.synchronize()
        self.handles = (ctypes.c_void_p * capacity)(*[e.cuda_event for e in self.events])
        self.ids = (ctypes.c_uint32 * capacity)()
        self.capacity = capacity
        self.used = 0

    def build(self, d_text, n, sym_bytes, L, kind, structure, ws, tune=None, stream=None):
        """Enqueue one build, recording an event after each kernel."""
        rec = ctypes.c_uint32(0)
        cap = self.capacity - self.used
        if cap <= 0:
            raise WtError(WT_ENOSPACE, "EventRecorder full")
        hp = ctypes.cast(ctypes.byref(self.handles, self.used * ctypes.sizeof(ctypes.c_void_p)),
                         ctypes.POINTER(ctypes.c_void_p))
        ip = ctypes.cast(ctypes.byref(self.ids, self.used * 4), ctypes.POINTER(ctypes.c_uint32))
        ptr = ctypes.c_void_p(d_text.data_ptr()) if n > 0 else ctypes.c_void_p(ws.data_ptr())
        check(wt_build_recorded(kind, ptr, n, sym_bytes, L, ctypes.byref(structure.view),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _tune_ptr(tune),
                                _stream_handle(stream), hp, ip, cap, ctypes.byref(rec)),
              "wt_build_recorded")
        if rec.value > cap:
            raise WtError(WT_ENOSPACE, "EventRecorder capacity exceeded")
        first = self.used
        self.used += rec.value
        return first, self.used

    def pair_build(self, d_text, n, sym_bytes, L, wt, wm, ws, stream=None):
        """Enqueue one pair build (WT and WM), recording an event after each kernel."""
        rec = ctypes.c_uint32(0)
        cap = self.capacity - self.used
        if cap <= 0:
            raise WtError(WT_ENOSPACE, "EventRecorder full")
        hp = ctypes.cast(ctypes.byref(self.handles, self.used * ctypes.sizeof(ctypes.c_void_p)),
                         ctypes.POINTER(ctypes.c_void_p))
        ip = ctypes.cast(ctypes.byref(self.ids, self.used * 4), ctypes.POINTER(ctypes.c_uint32))
        ptr = ctypes.c_void_p(d_text.data_ptr()) if n > 0 else ctypes.c_void_p(ws.data_ptr())
        check(wt_pair_build_recorded(ptr, n, sym_bytes, L, ctypes.byref(wt.view), ctypes.byref(wm.view),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream), hp, ip,
                                     cap, ctypes.byref(rec)), "wt_pair_build_recorded")
        if rec.value > cap:
            raise WtError(WT_ENOSPACE, "EventRecorder capacity exceeded")
        first = self.used
        self.used += rec.value
        return first, self.used

    def kernel_times(self, start_event, first=0, last=None):
        """{kernel name: [ms of each launch]} for recorded launches [first, last);
        the launch before `first` (or start_event) marks the start."""
        last = self.used if last is None else last
        out = {}
        prev = start_event if first == 0 else self.events[first - 1]
        for i in range(first, last):
            name = wt_kernel_name(self.ids[i]).decode()
            out.setdefault(name, []).append(prev.elapsed_time(self.events[i]))
            prev = self.events[i]
        return out
