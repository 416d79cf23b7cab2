"""Reference oracle for wavelet tree / wavelet matrix construction.

TEST INFRASTRUCTURE ONLY.  A ctypes wrapper over ``wt_oracle.c``: plain,
single-threaded C that computes the level bit vectors, zero counts, prefix
histograms, interval starts, directories and queries straight from their
definitions in Fischer, Kurpicz, Loebel, arXiv 1702.07578 (Section 2 for the
wavelet tree and rank/select, Section 5 for the wavelet matrix).  Only the test
suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  It shares no code with the GPU library.

All arrays are numpy arrays in host memory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_PAR_SRC = os.path.join(_HERE, "wt_oracle_par.c")
_PAR_LIB = os.path.join(_HERE, "liboracle_par.so")

WT, WM = 0, 1
Q_ACCESS, Q_RANK, Q_SELECT = 0, 1, 2
SEL_SPACING = 4096
OK, EINVAL, ERANGE, ENOMEM = 0, -1, -3, -6


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def compile_library(src: str = _SRC, out: str = _LIB, extra_flags=()) -> str:
    """Compile the oracle with gcc into a shared library (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           *extra_flags, "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True, cwd=os.path.dirname(src))
    os.replace(out + ".tmp", out)
    return out


def compile_par_library(src: str = _PAR_SRC, out: str = _PAR_LIB, extra_flags=()) -> str:
    """Compile the all-cores form of the top-down builder (OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fopenmp", "-shared", "-fPIC",
           *extra_flags, "-o", out + ".tmp", src]
    subprocess.run(cmd, check=True, cwd=os.path.dirname(src))
    os.replace(out + ".tmp", out)
    return out


_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_int = ctypes.c_int


def _bind(lib):
    sig = {
        "orc_reverse_bits": (_u64, [_u64, _u32]),
        "orc_words_per_level": (_u64, [_u64]),
        "orc_sel_capacity": (_u64, [_u64]),
        "orc_check_symbols": (_int, [_vp, _u64, _u32, _u32]),
        "orc_build": (_int, [_int, _vp, _u64, _u32, _u32, _u64p, _u64, _u64p]),
        "orc_hist": (_int, [_vp, _u64, _u32, _u32, _u32, _u64p]),
        "orc_spos": (_int, [_int, _u64p, _u32, _u64p]),
        "orc_rank_bv": (_u64, [_u64p, _u64, _u32]),
        "orc_select_bv": (_u64, [_u64p, _u64, _u64, _u32]),
        "orc_directory": (_int, [_u64p, _u64, _u64, _u32p, _u32p, _u32p]),
        "orc_queries_def": (_int, [_vp, _u64, _u32, _u32, _int, _u32p, _u64p, _u64, _u64p]),
        "orc_rank_scan": (_int, [_vp, _u64, _u32, _u32, _u32p, _u64p, _u64, _u64p]),
        "orc_queries_walk": (_int, [_int, _u64p, _u64, _u64p, _u64, _u32, _int, _u32p, _u64p,
                                    _u64, _u64p]),
        "orc_sample_level": (_int, [_int, _vp, _u64, _u32, _u32, _u32, _u64p, _u64, _u8p]),
        "orc_map_wt_to_wm": (_int, [_vp, _u64, _u32, _u32, _u32, _u64p, _u64, _u64p]),
        "orc_pointer_tree": (_int, [_vp, _u64, _u32, _u32, _u64p, _u64p, _u64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


class Oracle:
    """One loaded copy of the oracle library (the default one, or a variant
    compiled from another source file, e.g. a deliberately broken copy used to
    show that the pins catch mistakes)."""

    def __init__(self, lib_path: str, par_path: str | None = None):
        self.lib = _bind(ctypes.CDLL(lib_path))
        self._par_path = par_path
        self._par = None

    def _par_lib(self):
        if self._par is None:
            path = self._par_path
            if path is None:
                if not os.path.exists(_PAR_LIB) or os.path.getmtime(_PAR_LIB) < os.path.getmtime(_PAR_SRC):
                    compile_par_library()
                path = _PAR_LIB
            lib = ctypes.CDLL(path)
            lib.orc_par_build.restype = _int
            lib.orc_par_build.argtypes = [_int, _vp, _u64, _u32, _u32, _u64p, _u64, _u64p, _int]
            lib.orc_par_max_threads.restype = _int
            lib.orc_par_max_threads.argtypes = []
            self._par = lib
        return self._par

    def par_threads(self) -> int:
        """Threads the all-cores builder uses by default (OpenMP's count)."""
        return int(self._par_lib().orc_par_max_threads())

    def par_build(self, kind: int, text, L: int, threads: int = 0):
        """The same levels and zero counts as build(), computed by the
        top-down algorithm on `threads` host threads (0: all OpenMP offers)."""
        t, b = self._text(text)
        n = t.size
        W = self.words_per_level(n)
        bits = np.zeros((max(L, 1), max(W, 1)), dtype=np.uint64)
        zeros = np.zeros(max(L, 1), dtype=np.uint64)
        rc = self._par_lib().orc_par_build(kind, t.ctypes.data, n, b, L, self._p(bits, _u64p), max(W, 1),
                                           self._p(zeros, _u64p), threads)
        if rc != OK:
            raise OracleError(rc, "par_build")
        return bits[:L, :W], zeros[:L].copy()

    # -- helpers -----------------------------------------------------------
    @staticmethod
    def _text(text):
        t = np.ascontiguousarray(text)
        if t.dtype not in (np.uint8, np.uint16, np.uint32):
            raise TypeError(f"text dtype must be uint8/16/32, got {t.dtype}")
        return t, t.dtype.itemsize

    @staticmethod
    def _p(a, typ):
        return a.ctypes.data_as(typ)

    def words_per_level(self, n: int) -> int:
        return int(self.lib.orc_words_per_level(n))

    def sel_capacity(self, n: int) -> int:
        return int(self.lib.orc_sel_capacity(n))

    def reverse_bits(self, x: int, k: int) -> int:
        return int(self.lib.orc_reverse_bits(x, k))

    # -- construction ------------------------------------------------------
    def build(self, kind: int, text, L: int):
        """Levels (uint64 [L, W]) and zero counts (uint64 [L]) of the WT or WM."""
        t, b = self._text(text)
        n = t.size
        W = self.words_per_level(n)
        bits = np.zeros((max(L, 1), max(W, 1)), dtype=np.uint64)
        zeros = np.zeros(max(L, 1), dtype=np.uint64)
        rc = self.lib.orc_build(kind, t.ctypes.data, n, b, L, self._p(bits, _u64p), max(W, 1),
                                self._p(zeros, _u64p))
        if rc != OK:
            raise OracleError(rc, "build")
        return bits[:L, :W].copy(), zeros[:L].copy()

    def hist(self, text, L: int, level: int):
        t, b = self._text(text)
        h = np.zeros(1 << level, dtype=np.uint64)
        rc = self.lib.orc_hist(t.ctypes.data, t.size, b, L, level, self._p(h, _u64p))
        if rc != OK:
            raise OracleError(rc, "hist")
        return h

    def spos(self, kind: int, hist, level: int):
        h = np.ascontiguousarray(hist, dtype=np.uint64)
        s = np.zeros(1 << level, dtype=np.uint64)
        rc = self.lib.orc_spos(kind, self._p(h, _u64p), level, self._p(s, _u64p))
        if rc != OK:
            raise OracleError(rc, "spos")
        return s

    # -- rank / select / directories --------------------------------------
    def rank_bv(self, words, i: int, b: int) -> int:
        w = np.ascontiguousarray(words, dtype=np.uint64)
        return int(self.lib.orc_rank_bv(self._p(w, _u64p), i, b))

    def select_bv(self, words, n: int, k: int, b: int) -> int:
        w = np.ascontiguousarray(words, dtype=np.uint64)
        return int(self.lib.orc_select_bv(self._p(w, _u64p), n, k, b))

    def directory(self, level_words, n: int):
        """(rank_dir uint32 [W/8+1], sel0 uint32 [cap], sel1 uint32 [cap]) of one level."""
        w = np.ascontiguousarray(level_words, dtype=np.uint64)
        W = w.size
        cap = self.sel_capacity(n)
        rd = np.zeros(W // 8 + 1, dtype=np.uint32)
        s0 = np.zeros(cap, dtype=np.uint32)
        s1 = np.zeros(cap, dtype=np.uint32)
        if W == 0:
            w = np.zeros(1, dtype=np.uint64)
        rc = self.lib.orc_directory(self._p(w, _u64p), n, W, self._p(rd, _u32p), self._p(s0, _u32p),
                                    self._p(s1, _u32p))
        if rc != OK:
            raise OracleError(rc, "directory")
        return rd, s0, s1

    # -- queries -----------------------------------------------------------
    def queries_def(self, text, L: int, op: int, syms, args):
        t, b = self._text(text)
        a = np.ascontiguousarray(args, dtype=np.uint64)
        s = np.ascontiguousarray(syms if syms is not None else np.zeros(a.size), dtype=np.uint32)
        out = np.zeros(max(a.size, 1), dtype=np.uint64)
        rc = self.lib.orc_queries_def(t.ctypes.data, t.size, b, L, op, self._p(s, _u32p),
                                      self._p(a, _u64p), a.size, self._p(out, _u64p))
        if rc != OK:
            raise OracleError(rc, "queries_def")
        return out[: a.size]

    def rank_scan(self, text, L: int, syms, positions):
        """rank_c(i) for pairs (syms[q], positions[q]) by one scan of the
        text (no occurrence lists; for long texts, L <= 26)."""
        t, b = self._text(text)
        p = np.ascontiguousarray(positions, dtype=np.uint64)
        s = np.ascontiguousarray(syms, dtype=np.uint32)
        out = np.zeros(max(p.size, 1), dtype=np.uint64)
        rc = self.lib.orc_rank_scan(t.ctypes.data, t.size, b, L, self._p(s, _u32p), self._p(p, _u64p), p.size,
                                    self._p(out, _u64p))
        if rc != OK:
            raise OracleError(rc, "rank_scan")
        return out[: p.size]

    def queries_walk(self, kind: int, bits, zeros, n: int, L: int, op: int, syms, args):
        bb = np.ascontiguousarray(bits, dtype=np.uint64)
        W = bb.shape[1] if bb.ndim == 2 else 0
        if bb.size == 0:
            bb = np.zeros((1, 1), dtype=np.uint64)
        z = np.ascontiguousarray(zeros if len(zeros) else np.zeros(1), dtype=np.uint64)
        a = np.ascontiguousarray(args, dtype=np.uint64)
        s = np.ascontiguousarray(syms if syms is not None else np.zeros(a.size), dtype=np.uint32)
        out = np.zeros(max(a.size, 1), dtype=np.uint64)
        rc = self.lib.orc_queries_walk(kind, self._p(bb, _u64p), W, self._p(z, _u64p), n, L, op,
                                       self._p(s, _u32p), self._p(a, _u64p), a.size,
                                       self._p(out, _u64p))
        if rc != OK:
            raise OracleError(rc, "queries_walk")
        return out[: a.size]

    def map_wt_to_wm(self, text, L: int, level: int, positions):
        """Positions in WM level `level` of the bits at the given WT positions."""
        t, b = self._text(text)
        p = np.ascontiguousarray(positions, dtype=np.uint64)
        out = np.zeros(max(p.size, 1), dtype=np.uint64)
        rc = self.lib.orc_map_wt_to_wm(t.ctypes.data, t.size, b, L, level, self._p(p, _u64p), p.size,
                                       self._p(out, _u64p))
        if rc != OK:
            raise OracleError(rc, "map_wt_to_wm")
        return out[: p.size]

    def pointer_tree(self, text, L: int):
        """Node table (uint64 [2^L - 1, 2]: first pool word, bits) and pool of
        the pointer-based WT (node e = 2^l - 1 + p holds prefix p of length l)."""
        t, b = self._text(text)
        n = t.size
        entries = (1 << L) - 1
        nodes = np.zeros((max(entries, 1), 2), dtype=np.uint64)
        pool_words = L * ((n + 63) // 64) + entries
        pool = np.zeros(max(pool_words, 1), dtype=np.uint64)
        rc = self.lib.orc_pointer_tree(t.ctypes.data, n, b, L, self._p(nodes, _u64p), self._p(pool, _u64p),
                                       pool.size)
        if rc != OK:
            raise OracleError(rc, "pointer_tree")
        return nodes[:entries].copy(), pool

    def node_bits(self, nodes, pool, e: int):
        """Bits (list of 0/1) of node e of a pointer_tree result."""
        w0, h = int(nodes[e, 0]), int(nodes[e, 1])
        return [int((int(pool[w0 + q // 64]) >> (q % 64)) & 1) for q in range(h)]

    def sample_level(self, kind: int, text, L: int, level: int, positions):
        t, b = self._text(text)
        p = np.ascontiguousarray(positions, dtype=np.uint64)
        out = np.zeros(max(p.size, 1), dtype=np.uint8)
        rc = self.lib.orc_sample_level(kind, t.ctypes.data, t.size, b, L, level, self._p(p, _u64p),
                                       p.size, self._p(out, _u8p))
        if rc != OK:
            raise OracleError(rc, "sample_level")
        return out[: p.size]


_default = None


def load() -> Oracle:
    """The oracle compiled from ``wt_oracle.c`` (compiled on first use if absent)."""
    global _default
    if _default is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            compile_library()
        _default = Oracle(_LIB)
    return _default
