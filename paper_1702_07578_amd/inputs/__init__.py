"""Seeded synthetic texts (random numbers only; no index arithmetic).

The same generators feed the oracle, the GPU library, the tests and the
benchmark.  They stand in for the paper's real texts (Pizza&Chili, 1000
Genomes, Common Crawl, a word-based news text; Section 4, Table 1), which are
not available here, by matching their shape: alphabet size, symbol width,
length, and a skewed or Markov distribution.

Streams: xoshiro256** seeded through splitmix64 from (seed, tag, chunk index),
in ``wt_inputs.c``; results do not depend on the number of threads.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wt_inputs.c")
_LIB = os.path.join(_HERE, "libwtinputs.so")
_lib = None


def compile_library() -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC,
           "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            compile_library()
        lib = ctypes.CDLL(_LIB)
        vp, u64, u32, dbl, i32 = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_double, ctypes.c_int)
        lib.gen_uniform.argtypes = [vp, u64, u32, u64, u64]
        lib.gen_uniform.restype = None
        lib.gen_markov2.argtypes = [vp, u64, u32, dbl, u64, u64]
        lib.gen_markov2.restype = i32
        lib.gen_zipf.argtypes = [vp, u64, u32, u64, dbl, u64, i32]
        lib.gen_zipf.restype = i32
        lib.gen_u64.argtypes = [vp, u64, u64, u64, u64]
        lib.gen_u64.restype = None
        lib.gen_unit.argtypes = [vp, u64, u64, u64]
        lib.gen_unit.restype = None
        _lib = lib
    return _lib


def _dtype_for(sym_bytes: int):
    return {1: np.uint8, 2: np.uint16, 4: np.uint32}[sym_bytes]


def lg_sigma(sigma: int) -> int:
    """Number of levels ceil(lg sigma) (0 for sigma = 1)."""
    return max(0, int(sigma - 1).bit_length())


def uniform(n: int, sigma: int, sym_bytes: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=_dtype_for(sym_bytes))
    _load().gen_uniform(out.ctypes.data, n, sym_bytes, sigma, seed)
    return out


def markov2(n: int, sigma: int, seed: int, alpha: float = 0.1, chain_len: int = 1 << 20) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    rc = _load().gen_markov2(out.ctypes.data, n, sigma, alpha, seed, chain_len)
    if rc != 0:
        raise ValueError(f"gen_markov2 failed ({rc})")
    return out


def zipf(n: int, sigma: int, s: float, sym_bytes: int, seed: int, permute: bool = True) -> np.ndarray:
    out = np.empty(n, dtype=_dtype_for(sym_bytes))
    rc = _load().gen_zipf(out.ctypes.data, n, sym_bytes, sigma, s, seed, 1 if permute else 0)
    if rc != 0:
        raise ValueError(f"gen_zipf failed ({rc})")
    return out


def u64(m: int, bound: int, seed: int, tag: int) -> np.ndarray:
    """m uniform integers in [0, bound) (bound 0: full 64-bit range)."""
    out = np.empty(m, dtype=np.uint64)
    _load().gen_u64(out.ctypes.data, m, bound, seed, tag)
    return out


def unit(m: int, seed: int, tag: int) -> np.ndarray:
    out = np.empty(m, dtype=np.float64)
    _load().gen_unit(out.ctypes.data, m, seed, tag)
    return out


# -- the workload recipes ------------------------------------------------------

# name: (generator, n, sigma, sym_bytes, seed, extra)
CONFIGS = {
    # single text, i.i.d. uniform over 256 symbols (8 levels)
    "uniform256": dict(kind="uniform", n=1 << 20, sigma=256, sym_bytes=1, seed=1),
    # text-like: order-2 Markov over 96 symbols (7 levels), XML/source-code shape
    "markov96": dict(kind="markov", n=1 << 30, sigma=96, sym_bytes=1, seed=2),
    # DNA-like: the same Markov family over 4 symbols (2 levels)
    "markov4": dict(kind="markov", n=1 << 31, sigma=4, sym_bytes=1, seed=3),
    # large alphabet: Zipf(1.1) over 2^20 permuted ids, uint32 (20 levels)
    "zipf20": dict(kind="zipf", n=1 << 28, sigma=1 << 20, sym_bytes=4, seed=4, s=1.1),
    # uint16 uniform over 2^16 (16 levels)
    "uniform16": dict(kind="uniform", n=1 << 29, sigma=1 << 16, sym_bytes=2, seed=5),
}


def make(name: str, n: int | None = None):
    """(text, lg_sigma) of a named recipe, optionally cut to length n (the
    same stream, so a shorter text is a prefix of the longer one for the
    uniform and Zipf recipes; Markov texts are prefixes chain by chain)."""
    c = CONFIGS[name]
    n = c["n"] if n is None else n
    if c["kind"] == "uniform":
        t = uniform(n, c["sigma"], c["sym_bytes"], c["seed"])
    elif c["kind"] == "markov":
        t = markov2(n, c["sigma"], c["seed"])
    else:
        t = zipf(n, c["sigma"], c["s"], c["sym_bytes"], c["seed"])
    return t, lg_sigma(c["sigma"])


def batch_specs(count: int = 4096, seed: int = 6, lo_exp: float = 10.0, hi_exp: float = 22.0):
    """Per-text specs of the batched workload: length floor(2^U(lo,hi)),
    sigma from {4, 256, 2^16} (uint8 up to 256, else uint16), uniform or
    Zipf(1.0) with permuted ids, 50/50.  Returns a list of dicts."""
    u = unit(3 * count, seed, 0).reshape(count, 3)
    specs = []
    for i in range(count):
        n = int(math.floor(2.0 ** (lo_exp + (hi_exp - lo_exp) * u[i, 0])))
        sigma = (4, 256, 1 << 16)[min(2, int(u[i, 1] * 3))]
        dist = "zipf" if u[i, 2] >= 0.5 else "uniform"
        specs.append(dict(n=n, sigma=sigma, sym_bytes=1 if sigma <= 256 else 2, dist=dist,
                          seed=(seed << 20) + i))
    return specs


def batch_text(spec) -> tuple[np.ndarray, int]:
    if spec["dist"] == "zipf":
        t = zipf(spec["n"], spec["sigma"], 1.0, spec["sym_bytes"], spec["seed"])
    else:
        t = uniform(spec["n"], spec["sigma"], spec["sym_bytes"], spec["seed"])
    return t, lg_sigma(spec["sigma"])
