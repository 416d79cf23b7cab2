"""Autotuner for batched builds.

A batch of texts of uneven length and alphabet is built by one sequence of
launches (wt_batch_launch).  Its speed depends on knobs that no single rule
fits for every mix: how many ranges of tiles each text is cut into (one
scatter wave walks a range) and how many workgroups a launch runs (a
persistent grid that loops over the work items).  The tuner times a small
set of candidates on the batch itself, keeps only the candidates whose
outputs are bit-identical to the default configuration's, and caches the
winner in a JSON file keyed by a coarse signature of the batch.

Everything here is host-side orchestration over the C ABI; every step of the
build runs in the library's kernels.
"""
from __future__ import annotations

import json
import math
import os

from . import binding as B

# (ranges per text, workgroups per launch); 0 means the library default
CANDIDATES = [(g, p) for g in (0, 1024, 128, 16) for p in (0, 4096, 1024)]


def signature(items) -> str:
    """Coarse description of a batch: count, total symbols (power of two),
    and the mix of (symbol width, levels, kind)."""
    total = sum(int(it[1]) for it in items)
    mix = {}
    for _, n, b, L, kind, _s in items:
        key = f"{b}:{L}:{kind}"
        mix[key] = mix.get(key, 0) + 1
    parts = ",".join(f"{k}x{v}" for k, v in sorted(mix.items()))
    return f"count={len(items)};log2sym={int(math.log2(max(total, 1)))};{parts}"


def _clear(items):
    for it in items:
        it[5].buf.zero_()


def _snapshot(items):
    return [it[5].buf.clone() for it in items]


def _same(items, ref) -> bool:
    import torch
    return all(torch.equal(it[5].buf, r) for it, r in zip(items, ref))


def _time_launch(batch, reps: int) -> float:
    """Median milliseconds of batch.launch() (descriptors already uploaded)."""
    import torch
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        batch.launch()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune(items, cache_path: str | None = None, reps: int = 3, candidates=CANDIDATES, log=None):
    """Best (grid, persist) for this batch and the table of timings.

    Each candidate's outputs must equal the default configuration's bit for
    bit (all output buffers, cleared before every build); a candidate that
    differs or fails is dropped.  Returns (tune, table) where tune is a
    binding.WtTune (or None for the defaults) and table lists
    (grid, persist, ms or None, status)."""
    import torch
    sig = signature(items)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if sig in cache:
            g, p = cache[sig]["grid"], cache[sig]["persist"]
            return B.make_tune(grid=g, persist=p), cache[sig].get("table", [])

    need = max(int(B.wt_batch_workspace_bytes(B.Batch.item_array(items), len(items),
                                              B._tune_ptr(B.make_tune(grid=g, persist=p))))
               for g, p in candidates)
    ws = torch.empty(need, dtype=torch.uint8, device=items[0][5].buf.device)

    ref_batch = B.Batch(items, tune=None, ws=ws)
    _clear(items)
    ref_batch.build()
    torch.cuda.synchronize()
    for it in items:
        st = it[5].status()
        if st != 0:
            raise B.WtError(st, "reference batch build")
    ref = _snapshot(items)

    table = []
    best = None
    for g, p in candidates:
        t = B.make_tune(grid=g, persist=p)
        try:
            batch = B.Batch(items, tune=t, ws=ws)
            _clear(items)
            batch.build()
            torch.cuda.synchronize()
            if not _same(items, ref):
                table.append((g, p, None, "outputs differ"))
                continue
            ms = _time_launch(batch, reps)
        except B.WtError as e:
            table.append((g, p, None, str(e)))
            continue
        table.append((g, p, ms, "ok"))
        if log:
            log(f"autotune grid={g} persist={p}: {ms:.3f} ms")
        if best is None or ms < best[2]:
            best = (g, p, ms)
    del ref
    if best is None:
        raise B.WtError(B.WT_EINVAL, "autotune: no candidate reproduced the default build")
    if cache_path:
        cache[sig] = {"grid": best[0], "persist": best[1], "ms": best[2], "table": table}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return B.make_tune(grid=best[0], persist=best[1]), table
