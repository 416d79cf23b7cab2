#!/usr/bin/env python3
"""Benchmark: wavelet tree + wavelet matrix construction on one MI355X.

Workload: the text-like plain build, n = 2^30 uint8 symbols over sigma = 96
(7 levels) from the seeded order-2 Markov recipe (see paper_1702_07578_amd/
inputs).  One step = one wavelet-tree build plus one wavelet-matrix build of
that text, each with its levels, Z and rank/select directories, inputs already
resident in HBM.  value = 2 n / step time (symbols built per second, counted
once per structure).

Per-kernel durations come from HIP events recorded by the library after every
kernel launch, on the build stream, inside the timed region.  The roofline
object reports the dominant kernel (the stable scatter) against the HBM peak
with its algorithmic bytes: the text re-read (n b) plus every level written
once (L W 8).  The oracle (plain C, one thread) is timed on a bounded prefix of
the same text as the CPU baseline.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "scatter_markov96_counters.json")
PAIR_COUNTERS = os.path.join(ROOT, "profiles", "pair_scatter_markov96_counters.json")
SCATTER_SRC = os.path.join(ROOT, "paper_1702_07578_amd", "csrc", "wt_scatter.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOAD_TEXT = {
    "markov96": "order-2 Markov text, sigma=96",
    "markov4": "order-2 Markov text, sigma=4",
    "uniform256": "i.i.d. uniform, sigma=256",
    "uniform16": "i.i.d. uniform, sigma=2^16",
    "zipf20": "Zipf(1.1) over 2^20 permuted ids",
}


def scatter_traffic(per_launch_alg_bytes, path=COUNTERS):
    """HBM bytes per scatter launch from the committed counter runs, or None
    when there are none or the kernel source changed since they were taken."""
    if not os.path.exists(path):
        return None
    c = json.load(open(path))
    src = hashlib.sha256(open(SCATTER_SRC, "rb").read()).hexdigest()
    if c.get("source_sha256") != src:
        return None
    return c.get("bytes_per_launch")


# the chip's vector-instruction issue rate: 256 CUs x 4 SIMDs, one wave64
# VALU instruction per SIMD every 4 cycles at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def src_sha():
    return hashlib.sha256(open(SCATTER_SRC, "rb").read()).hexdigest()


def alu_issue(workload, scatter_ms_per_step, path=None):
    """The pair step's scatter against the chip's VALU issue rate, from the
    committed instruction counters of that workload (rocprofv3 SQ_INSTS_VALU
    summed over one pair step's scatter dispatches), or None when there are
    none or the kernel source changed since they were taken."""
    path = path or os.path.join(ROOT, "profiles", f"scatter_issue_{workload}.json")
    if not os.path.exists(path):
        return None
    c = json.load(open(path))
    if c.get("source_sha256") != src_sha():
        return None
    ach = c["valu_per_step"] / (scatter_ms_per_step / 1e3)
    return {"achieved": round(ach / 1e9, 1), "peak": round(VALU_ISSUE_PEAK / 1e9, 1),
            "unit": "G wave64 VALU instructions/s", "frac": round(ach / VALU_ISSUE_PEAK, 4),
            "valu_per_64_symbols": c["valu_per_64_symbols"], "lds_per_64_symbols": c["lds_per_64_symbols"],
            "counters": os.path.relpath(path, ROOT)}


def single_alu_issue(avg_ms, path=COUNTERS):
    """The single build's scatter against the VALU issue rate, from the
    committed counters of its markov96 launches (same source only)."""
    if not os.path.exists(path):
        return None
    c = json.load(open(path))
    if c.get("source_sha256") != src_sha() or "sq" not in c:
        return None
    sq = c["sq"]
    ach = sq["per_dispatch_median"]["SQ_INSTS_VALU"] / (avg_ms / 1e3)
    return {"achieved": round(ach / 1e9, 1), "peak": round(VALU_ISSUE_PEAK / 1e9, 1),
            "unit": "G wave64 VALU instructions/s", "frac": round(ach / VALU_ISSUE_PEAK, 4),
            "valu_per_64_symbols": sq["valu_per_64_symbols"], "lds_per_64_symbols": sq["lds_per_64_symbols"],
            "counters": os.path.relpath(path, ROOT)}


def cpu_baseline(text, L, sample_n):
    import oracle
    orc = oracle.load()
    s = text[:sample_n]
    t0 = time.perf_counter()
    orc.build(1, s, L)
    orc.build(0, s, L)
    dt = time.perf_counter() - t0
    return {"value": 2 * sample_n / dt, "unit": "symbols/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_n} symbols of the same text, one WM and one WT build "
                      f"(levels and Z) in {dt:.2f} s"}


def host_info():
    """CPU model and core counts of the host the CPU baselines run on."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline_all_cores(text, L, sample_n):
    """The oracle's top-down builder parallelised over every thread OpenMP
    offers (the per-thread counts and interleaved prefix sum of Section 3.2
    applied to each level's split), on a bounded prefix of the text."""
    import oracle
    orc = oracle.load()
    s = text[:sample_n]
    threads = orc.par_threads()
    orc.par_build(1, s[: min(sample_n, 1 << 20)], L)  # warm the thread pool
    t0 = time.perf_counter()
    orc.par_build(1, s, L)
    orc.par_build(0, s, L)
    dt = time.perf_counter() - t0
    return {"value": 2 * sample_n / dt, "unit": "symbols/s", "cores": threads, "kind": "oracle (all cores)",
            "sample": f"first {sample_n} symbols of the same text, one WM and one WT build (levels and Z) "
                      f"with {threads} threads in {dt:.2f} s"}


# The paper's own construction times (Table 3: wavelet matrix, times in seconds,
# median of five runs, without rank/select support), for the rows whose texts the
# synthetic workloads stand in for.  Its hardware: two Intel Xeon E5-2686 v4 (up
# to 32 of their cores used), 256 GB RAM, g++ 6.2 -O3, OpenMP 4.5 (Section 4).
PAPER_TABLE3 = {
    "hardware": "2x Intel Xeon E5-2686 v4, up to 32 cores used, 256 GB RAM (Section 4)",
    "what": "wavelet matrix construction time in seconds, without rank/select (Table 3)",
    "rows": {
        "XML (n=2.9e8, sigma=97; markov96 stands in)": {
            "n": 2.9e8, "pcWM_1core_s": 4.737, "pcWM_32core_s": 0.988, "psWM_1core_s": 4.355,
            "psWM_32core_s": 0.531, "ddpcWM_32core_s": 0.468},
        "DNA (n=4.0e8, sigma=16; markov4 stands in by family)": {
            "n": 4.0e8, "pcWM_1core_s": 3.895, "pcWM_32core_s": 1.479, "psWM_1core_s": 4.293,
            "psWM_32core_s": 0.904, "ddpcWM_32core_s": 0.691},
        "1000G (n=88.2e8, sigma=4; markov4 stands in)": {
            "n": 88.2e8, "pcWM_1core_s": 32.322, "pcWM_32core_s": 4.900, "psWM_1core_s": 30.908,
            "psWM_32core_s": 6.969, "ddpcWM_32core_s": 2.429},
        "WORDS (n=1.4e8, sigma=2245405; zipf20 stands in)": {
            "n": 1.4e8, "pcWM_1core_s": 8.733, "pcWM_32core_s": 0.774, "psWM_1core_s": 13.394,
            "psWM_32core_s": 3.007, "ddpcWM_32core_s": 4.308},
    },
}


def paper_reference():
    """Table 3 times with their throughput (n / t, symbols/s, one structure)."""
    out = {"hardware": PAPER_TABLE3["hardware"], "what": PAPER_TABLE3["what"], "rows": {}}
    for name, r in PAPER_TABLE3["rows"].items():
        row = dict(r)
        for k in list(r):
            if k.endswith("_s"):
                row[k[:-2] + "_symbols_per_s"] = round(r["n"] / r[k], 1)
        out["rows"][name] = row
    return out


def pair_measure(B, d_text, n, b, L, steps, warmup, stream, dev, wt_s=None, wm_s=None):
    """K pair builds (the WT and the WM of the text by wt_pair_build) timed
    with HIP events; per-kernel durations from the events the library records
    after every launch.  Returns (record, wt, wm)."""
    import torch
    if wt_s is None:
        wt_s, wm_s = B.Structure(n, L, B.WT_TREE, device=dev), B.Structure(n, L, B.WT_MATRIX, device=dev)
    pws = torch.empty(int(B.wt_pair_workspace_bytes(n, b, L)), dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        B.pair_build(d_text, n, b, L, ws=pws, out=(wt_s, wm_s))
    torch.cuda.synchronize()
    probe = B.EventRecorder(512)
    probe.pair_build(d_text, n, b, L, wt_s, wm_s, pws)
    torch.cuda.synchronize()
    rec = B.EventRecorder(probe.used * steps + 8)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        rec.pair_build(d_text, n, b, L, wt_s, wm_s, pws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # the same steps without an event after every launch (for short texts
    # the recording itself is a visible part of the step)
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for _ in range(steps):
        B.pair_build(d_text, n, b, L, ws=pws, out=(wt_s, wm_s))
    p1.record(stream)
    torch.cuda.synchronize()
    ms_plain = p0.elapsed_time(p1) / steps
    kt = rec.kernel_times(e0)
    pk = {name: {"launches": len(v), "avg_ms": sum(v) / len(v)} for name, v in kt.items()}
    for s in (wt_s, wm_s):
        if s.status() != 0:
            raise SystemExit(f"pair build status {s.status()}")
    W = wt_s.view.words_per_level
    G = -(-L // 8) if L else 1
    # one group: the pair scatter writes both structures' levels; more
    # groups: the WM's scatter launches, one group each
    pbytes = n * b + 2 * L * W * 8 if L <= 8 else (n * b + L * W * 8) / G
    pach = pbytes / (pk["scatter"]["avg_ms"] / 1e3) / 1e9
    nb = W // 8
    dir_bytes = L * (nb + 1) * 4 + 2 * L * ((n + 4095) // 4096 + 1) * 4
    b_alg_build = 2 * n * b + L * W * 8 + dir_bytes
    build_gbs = 2 * b_alg_build / (ms / 1e3) / 1e9
    del pws
    return ({"ms_per_step": ms, "ms_per_step_unrecorded": ms_plain, "value": 2 * n / (ms / 1e3), "kernels": pk,
             "b_alg_build": b_alg_build,
             "build_alg_gbs": build_gbs,
             "scatter": {"kernel": ("scatter (pair: WT and WM runs from one set of splits)" if L <= 8 else
                                    "scatter (the WM's groups; the WT is gathered from the WM)"),
                         "achieved": pach, "alg_bytes_per_launch": int(pbytes),
                         "avg_launch_ms": pk["scatter"]["avg_ms"],
                         "ms_per_step": pk["scatter"]["avg_ms"] * pk["scatter"]["launches"] / steps}},
            wt_s, wm_s)


def bound_fields(workload, scatter_ms_per_step):
    """What bounds the scatter, from the committed counters of this kernel
    source: vector-instruction issue ("alu") when it runs at half the chip's
    issue rate or more, else latency (neither the issue rate nor HBM is
    saturated); the issue figures go under "alu".  Without matching counters
    the limiter is not measured.  The roofline's own figures stay algorithmic
    bytes against the HBM peak."""
    alu = alu_issue(workload, scatter_ms_per_step)
    if alu is None:
        return {"bound": "hbm", "limiter": "not measured on this kernel source (no matching instruction counters)"}
    if alu["frac"] >= 0.5:
        return {"bound": "alu", "alu": alu}
    return {"bound": "latency", "alu": alu,
            "limiter": "neither the VALU issue rate nor HBM is saturated (dependent LDS round trips and launch "
                       "latency of short work)"}


def config_line(B, name, steps, warmup, stream, dev, steady_args=None):
    """One workload's pair step at its full size: time, symbols/s, the
    scatter's roofline fraction and the whole step's fraction of the HBM peak
    (algorithmic bytes of both builds), after an access check of sampled
    positions against the text."""
    import numpy as np
    import torch

    from paper_1702_07578_amd import inputs
    t0 = time.time()
    text, L = inputs.make(name)
    n, b = text.size, text.dtype.itemsize
    d_text = B.to_device(text, dev)
    rec, wt_s, wm_s = pair_measure(B, d_text, n, b, L, steps, warmup, stream, dev)
    pos = torch.from_numpy(inputs.u64(1 << 16, n, 99, 0).view(np.int64)).to(dev)
    want = torch.from_numpy(text.astype(np.uint32).view(np.int32)).to(dev)[pos]
    for s in (wt_s, wm_s):
        if not torch.equal(s.access(pos), want):
            raise SystemExit(f"{name}: access check failed")
    sc = rec["scatter"]
    out = {"workload": f"{name}: {WORKLOAD_TEXT.get(name, 'text')}, n={n} uint{8 * b} symbols, {L} levels",
           "n": n, "sym_bytes": b, "lg_sigma": L, "steps": steps,
           "ms_per_step": round(rec["ms_per_step"], 4), "symbols_per_s": round(rec["value"], 1),
           "ms_per_step_unrecorded": round(rec["ms_per_step_unrecorded"], 4),
           "build_alg_gbs": round(rec["build_alg_gbs"], 1),
           "build_alg_frac": round(rec["build_alg_gbs"] / HBM_PEAK_GBS, 4),
           "scatter": {"kernel": sc["kernel"], "avg_launch_ms": round(sc["avg_launch_ms"], 4),
                       "alg_bytes_per_launch": sc["alg_bytes_per_launch"], "achieved_gbs": round(sc["achieved"], 1),
                       "frac": round(sc["achieved"] / HBM_PEAK_GBS, 4),
                       **bound_fields(name, sc["ms_per_step"])},
           "kernels": {k: {"avg_ms": round(v["avg_ms"], 4), "launches_per_step": v["launches"] // steps}
                       for k, v in rec["kernels"].items()}}
    if steady_args is not None:
        out["steady_state"] = steady_state_small(steady_args, B, n, L, rec["b_alg_build"], log)
    log(f"{name}: pair step {out['ms_per_step']} ms, scatter frac {out['scatter']['frac']}, "
        f"step frac {out['build_alg_frac']} ({time.time() - t0:.1f}s)")
    del wt_s, wm_s, d_text
    torch.cuda.empty_cache()
    return out


def run_batch(args):
    """Batched build of the 4096-text workload (WT and WM of every text) in
    one sequence of launches captured in a HIP graph, with autotuned knobs,
    against the same builds done one text at a time on the same stream."""
    import numpy as np
    import torch

    from paper_1702_07578_amd import autotune
    from paper_1702_07578_amd import binding as B
    from paper_1702_07578_amd import inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    specs = inputs.batch_specs(args.batch_count, seed=6)
    texts = [inputs.batch_text(sp) for sp in specs]
    total = sum(t.size for t, _ in texts)
    log(f"generated {len(texts)} texts, {total} symbols in {time.time() - t0:.1f}s")
    d_texts = [B.to_device(t, dev) for t, _ in texts]
    items, plain = [], []
    for (t, L), d in zip(texts, d_texts):
        for kind in (B.WT_TREE, B.WT_MATRIX):
            items.append((d, t.size, t.dtype.itemsize, L, kind, B.Structure(t.size, L, kind, device=dev)))
            plain.append(B.Structure(t.size, L, kind, device=dev))
    torch.cuda.synchronize()

    tune, table = autotune.tune(items, cache_path=args.tune_cache or None, log=log)
    batch = B.Batch(items, tune=tune)
    for it in items:
        it[5].buf.zero_()
    batch.prepare()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            batch.launch(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / args.steps
    for it in items:
        if it[5].status() != 0:
            raise SystemExit("batched build reported an error status")

    # the same builds, one text at a time on the same stream
    ws = torch.empty(max(B.workspace_bytes(n, b, L, k) for _, n, b, L, k, _ in items), dtype=torch.uint8,
                     device=dev)
    for s in plain:
        s.buf.zero_()

    def per_text():
        for (d, n, b, L, kind, _), s in zip(items, plain):
            B.build(d, n, b, L, kind, ws=ws, out=s)

    per_text()
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record()
    per_text()
    p1.record()
    torch.cuda.synchronize()
    plain_ms = p0.elapsed_time(p1)
    # every batched structure equals its one-at-a-time build (whole buffers,
    # both cleared before building)
    for it, s in zip(items, plain):
        if not torch.equal(it[5].buf, s.buf):
            raise SystemExit(f"batched output differs from the plain build (n={it[1]}, L={it[3]})")
    value = 2 * total / (batch_ms / 1e3)
    # algorithmic bytes of every structure of the batch: its text read twice,
    # every level written once, the directories written once
    alg = 0
    for _, n, b, L, _, s in items:
        W = s.view.words_per_level
        alg += 2 * n * b + L * W * 8 + L * (W // 8 + 1) * 4 + 2 * L * ((n + 4095) // 4096 + 1) * 4
    alg_gbs = alg / (batch_ms / 1e3) / 1e9
    out = {
        "metric": "batched WT+WM build throughput (symbols/s), one GPU",
        "value": round(value, 1), "unit": "symbols/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(batch_ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8/u16", "data": "synthetic",
        "config": {"workload": f"batch: {len(texts)} texts, lengths floor(2^U(10,22)), sigma in "
                               f"{{4, 256, 2^16}}, uniform or Zipf(1.0); WT and WM of every text in "
                               f"one graph-captured sequence of launches", "texts": len(texts),
                   "symbols": total, "tune": {"grid": tune.grid if tune else 0,
                                               "persist": tune.persist if tune else 0}},
        "roofline": {"kernel": "the whole batched build (every kernel of the graph replay)", "bound": "latency",
                     "limiter": "not HBM: the scatter is bound by instruction issue on long texts and the "
                                "16-level texts' interval walk and gather by dependent loads per prefix",
                     "achieved": round(alg_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": int(alg), "avg_launch_ms": round(batch_ms, 4)},
        "per_text_plain_ms": round(plain_ms, 3),
        "speedup_vs_per_text": round(plain_ms / batch_ms, 2),
        "autotune": [{"grid": g, "persist": p, "ms": ms, "status": st} for g, p, ms, st in table],
    }
    print(json.dumps(out), flush=True)


def steady_state_small(args, B, n, L, b_alg_build, log):
    """Many distinct texts of the small configuration back to back: the WT and
    the WM of each of `count` uniform texts (512 MiB of text in all, more than
    the 256 MB last-level cache), as one batched build in one graph replay;
    every structure is checked against its standalone build."""
    import torch

    from paper_1702_07578_amd import autotune
    from paper_1702_07578_amd import inputs

    dev = torch.device("cuda:0")
    count = args.steady_texts
    texts = [inputs.uniform(n, 256, 1, (1 << 16) + i) for i in range(count)]
    d_texts = [B.to_device(t, dev) for t in texts]
    items = [(d, n, 1, L, kind, B.Structure(n, L, kind, device=dev))
             for d in d_texts for kind in (B.WT_TREE, B.WT_MATRIX)]
    tune, _ = autotune.tune(items, log=log)
    batch = B.Batch(items, tune=tune)
    for it in items:
        it[5].buf.zero_()
    batch.prepare()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            batch.launch(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    ws = torch.empty(max(B.workspace_bytes(n, 1, L, k) for k in (B.WT_TREE, B.WT_MATRIX)), dtype=torch.uint8,
                     device=dev)
    alone = {k: B.Structure(n, L, k, device=dev) for k in (B.WT_TREE, B.WT_MATRIX)}
    for d, _, _, _, kind, s in items:
        if s.status() != 0:
            raise SystemExit("steady-state batch reported an error status")
        alone[kind].buf.zero_()
        B.build(d, n, 1, L, kind, ws=ws, out=alone[kind])
        if not torch.equal(s.buf, alone[kind].buf):
            raise SystemExit("steady-state batch output differs from the standalone build")
    alg = 2 * count * b_alg_build
    return {"texts": count, "symbols": count * n, "text_bytes": count * n,
            "build": "WT and WM of every text, one batched build, one graph replay",
            "tune": {"grid": tune.grid if tune else 0, "persist": tune.persist if tune else 0},
            "ms": round(ms, 4), "symbols_per_s": round(2 * count * n / (ms / 1e3), 1),
            "alg_bytes": int(alg), "alg_gbs": round(alg / (ms / 1e3) / 1e9, 1),
            "frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def run_serve(args):
    """Serving workload: Poisson arrivals of build requests (texts resident
    in HBM, lengths floor(2^U(12,26)), sigma in {256, 2^16}) mixed with query
    batches of 2^20 access/rank/select against resident structures, admitted
    by an HBM budget; latency p50/p99 and built symbols/s, at two loads, next
    to the same trace served one request at a time."""
    import numpy as np
    import torch

    from paper_1702_07578_amd import binding as B
    from paper_1702_07578_amd import inputs
    from paper_1702_07578_amd import serving as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    u = inputs.unit(2 * args.pool, 7, 0).reshape(args.pool, 2)
    pool = []
    for i in range(args.pool):
        n = int(2.0 ** (12 + 14 * u[i, 0]))
        sigma = 256 if u[i, 1] < 0.5 else 1 << 16
        T = inputs.uniform(n, sigma, 1 if sigma <= 256 else 2, (7 << 20) + i)
        pool.append((T, inputs.lg_sigma(sigma)))
    d_pool = [(B.to_device(T, dev), T.size, T.dtype.itemsize, L) for T, L in pool]
    mean_n = float(np.mean([T.size for T, _ in pool]))
    log(f"pool of {len(pool)} texts, mean length {mean_n:.0f}")

    # build capacity: every pool text once (WT and WM alternately), batched
    items = [(d, n, b, L, i % 2, B.Structure(n, L, i % 2, device=dev)) for i, (d, n, b, L) in enumerate(d_pool)]
    batch = B.Batch(items)
    batch.build()
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    batch.build()
    c1.record()
    torch.cuda.synchronize()
    capacity = sum(x[1] for x in d_pool) / (c0.elapsed_time(c1) / 1e3)
    qm = 1 << 20
    # query capacity: one 2^20 batch of each kind on the largest pool structure
    big = max(range(len(items)), key=lambda i: items[i][1])
    s_big = items[big][5]
    qpos = torch.from_numpy(inputs.u64(qm, items[big][1], 5, 0).view(np.int64)).to(dev)
    qsym = s_big.access(qpos)
    qk = s_big.rank(qsym, qpos) + 1  # select(T[j], rank + 1) = j
    torch.cuda.synchronize()
    q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    q0.record()
    s_big.access(qpos)
    s_big.rank(qsym, qpos)
    s_big.select(qsym, qk)
    q1.record()
    torch.cuda.synchronize()
    q_batch_s = q0.elapsed_time(q1) / 3 / 1e3
    del batch, items, s_big, qpos, qsym, qk
    torch.cuda.empty_cache()
    log(f"batched build capacity {capacity:.3e} symbols/s; one 2^20 query batch {q_batch_s * 1e3:.3f} ms")

    def trace(rho, seed):
        rng = np.random.default_rng(seed)
        # a build and a query batch arrive per pair; rho = the fraction of
        # the GPU's time the offered work needs
        lam = rho / (mean_n / capacity + q_batch_s)  # pairs per second
        reqs, builds, t = [], [], 0.0
        for rid in range(args.requests):
            t += float(rng.exponential(1.0 / (2 * lam)))  # builds and query batches, 1:1

            if builds and rng.random() < 0.5:
                target = int(rng.choice(builds[-64:]))
                op = int(rng.integers(0, 3))
                # positions drawn on the device at launch: j uniform, c = T[j],
                # select's k = rank(c, j) + 1 (it answers j)
                a = S.QuerySpec(m=qm, seed=(seed << 20) + rid)
                reqs.append(S.Request(rid=rid, kind=S.QUERY, arrival=t, target=target, op=op, args=a))
            else:
                reqs.append(S.Request(rid=rid, kind=S.BUILD, arrival=t, text=int(rng.integers(0, len(pool))),
                                      tree=int(rng.integers(0, 2))))
                builds.append(rid)
        return reqs

    def serve(reqs, slots, max_batch):
        ex = S.GpuExecutor(d_pool, slots)
        srv = S.Server(ex, int(args.budget_gib * (1 << 30)), slots=slots, max_batch=max_batch)
        w0 = time.perf_counter()
        done = srv.run(reqs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        built = sum(pool[r.text][0].size for r in done if r.kind == S.BUILD and r.status == 0)
        st = srv.stats()
        return {"build_p50_ms": round(st[S.BUILD]["p50_ms"], 3), "build_p99_ms": round(st[S.BUILD]["p99_ms"], 3),
                "query_p50_ms": round(st[S.QUERY]["p50_ms"], 3), "query_p99_ms": round(st[S.QUERY]["p99_ms"], 3),
                "builds": st[S.BUILD]["count"], "query_batches": st[S.QUERY]["count"],
                "failed": sum(r.status != 0 for r in done), "evictions": st["evictions"],
                "refused": st["refused"], "lost_queries": st["lost_queries"],
                "peak_gib": round(st["peak_bytes"] / 2 ** 30, 2), "wall_s": round(wall, 3),
                "built_symbols_per_s": round(built / wall, 1)}

    # warm-up: a short trace in both modes (first launches, allocator growth)
    serve(trace(0.5, 3)[:200], args.slots, 64)
    serve(trace(0.5, 3)[:200], 1, 1)
    results = {}
    for rho in (0.5, 0.9, 2.0):
        reqs = trace(rho, 11)
        results[f"load{rho}"] = {"continuous": serve(reqs, args.slots, 64)}
        reqs = trace(rho, 11)
        results[f"load{rho}"]["one_at_a_time"] = serve(reqs, 1, 1)
        log(f"load {rho}: {results[f'load{rho}']}")
    r5 = results["load0.5"]
    out = {
        "metric": "served WT/WM builds: built symbols/s and latency p50/p99 (ms), one GPU",
        "value": r5["continuous"]["built_symbols_per_s"], "unit": "symbols/s", "n_gpus": 1,
        "steps": args.requests, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8/u16", "data": "synthetic",
        "config": {"workload": f"serve: {args.requests} requests, Poisson arrivals offering 0.5 and 0.9 of "
                               f"the GPU's time (batched build capacity and 2^20-query batch time), builds "
                               f"and 2^20-query batches 1:1, pool of "
                               f"{len(pool)} resident texts (lengths floor(2^U(12,26)), sigma 256 or 2^16), "
                               f"HBM budget {args.budget_gib} GiB, {args.slots} stream slots",
                   "capacity_symbols_per_s": round(capacity, 1),
                   "query_batch_ms": round(q_batch_s * 1e3, 4)},
        "results": results,
        # below saturation the built rate follows the arrivals, so the gain
        # of continuous batching shows in the tail latency; past saturation
        # (offered load 2.0) it shows in the rate the server sustains
        "build_p99_gain_at_load0.9": round(results["load0.9"]["one_at_a_time"]["build_p99_ms"] /
                                           max(results["load0.9"]["continuous"]["build_p99_ms"], 1e-9), 2),
        "throughput_gain_at_load2.0": round(results["load2.0"]["continuous"]["built_symbols_per_s"] /
                                            max(results["load2.0"]["one_at_a_time"]["built_symbols_per_s"], 1e-9), 2),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="markov96")
    ap.add_argument("--n", type=int, default=0, help="override the text length")
    ap.add_argument("--cpu-sample", type=int, default=1 << 26)
    ap.add_argument("--cpu-sample-all", type=int, default=1 << 28,
                    help="symbols of the all-cores oracle baseline")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other plain configurations after the headline")
    ap.add_argument("--config-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--step-only", action="store_true",
                    help="only the pair step (warm-up, one probe step, then the timed steps twice): the "
                         "launches a counter run profiles")
    ap.add_argument("--tile-log2", type=int, default=0)
    ap.add_argument("--group-bits", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain elementwise copy of 1 GiB three times (the reference "
                         "kernel for scaling the HBM byte counters)")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--steady-texts", type=int, default=512,
                    help="uniform256: distinct texts of the steady-state measurement (0: skip)")
    ap.add_argument("--tune-cache", default="", help="JSON cache of the batch autotuner")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=4.0,
                    help="HBM budget of the serving workload (below its working set, so that admission "
                         "and eviction act)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch4096":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)

    import numpy as np
    import torch

    from paper_1702_07578_amd import binding as B
    from paper_1702_07578_amd import inputs

    t0 = time.time()
    text, L = inputs.make(args.workload, args.n or None)
    n = text.size
    b = text.dtype.itemsize
    log(f"generated {args.workload}: n={n} b={b} L={L} in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        # bitwise_not reads 1 GiB and writes 1 GiB in one elementwise kernel
        x = torch.zeros(1 << 28, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            torch.bitwise_not(x, out=y)
        torch.cuda.synchronize()
        del x, y
        log("copy calibration: 3 x bitwise_not over 2^28 int32 (1 GiB read + 1 GiB write each)")
    d_text = B.to_device(text, dev)
    if args.step_only:
        # warm-up steps, one probe step and the timed steps (recorded, then
        # unrecorded) of the pair build, nothing else: warmup + 1 + 2 steps
        # pair builds in all
        rec, _, _ = pair_measure(B, d_text, n, b, L, args.steps, args.warmup, stream, dev)
        print(json.dumps({"workload": args.workload, "n": n, "sym_bytes": b, "lg_sigma": L,
                          "pair_builds": args.warmup + 1 + 2 * args.steps, "ms_per_step": round(rec["ms_per_step"], 4),
                          "scatter_ms_per_step": round(rec["scatter"]["ms_per_step"], 4)}), flush=True)
        return
    tune = B.make_tune(tile_log2=args.tile_log2, group_bits=args.group_bits)
    structs = {k: B.Structure(n, L, k, device=dev) for k in (B.WT_TREE, B.WT_MATRIX)}
    ws_bytes = max(B.workspace_bytes(n, b, L, k, tune) for k in structs)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    spans = []  # (kind, first, last) recorded launches of every timed build

    def step(rec=None):
        for k in (B.WT_TREE, B.WT_MATRIX):
            if rec is None:
                B.build(d_text, n, b, L, k, tune=tune, ws=ws, out=structs[k])
            else:
                spans.append((k,) + rec.build(d_text, n, b, L, k, structs[k], ws, tune=tune))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k, s in structs.items():
        st = s.status()
        if st != 0:
            raise SystemExit(f"build status {st} for kind {k}")

    # launches per step, to size the event pool
    probe = B.EventRecorder(512)
    start_probe = torch.cuda.Event(enable_timing=True)
    start_probe.record()
    step(probe)
    torch.cuda.synchronize()
    per_step = probe.used
    rec = B.EventRecorder(per_step * args.steps + 8)

    # ---- timed region ----
    spans.clear()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step(rec)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    # ---- end timed region ----

    ms_per_step = total_ms / args.steps
    value = 2 * n / (ms_per_step / 1e3)
    kt = rec.kernel_times(ev0)
    # each structure on its own: its launches' durations, each measured from
    # the event before it (the builds run back to back on one stream)
    kind_ms = {}
    for k, first, last in spans:
        t = sum(sum(v) for v in rec.kernel_times(ev0, first, last).values())
        kind_ms[k] = kind_ms.get(k, 0.0) + t / args.steps
    kernels = {name: {"launches": len(v), "avg_ms": sum(v) / len(v), "total_ms_per_step": sum(v) / args.steps}
               for name, v in kt.items()}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms_per_step"])

    # algorithmic bytes per scatter launch: one launch per build here (one group)
    W = structs[0].view.words_per_level
    G = -(-L // 8) if L else 1
    scat = kernels.get("scatter", {"avg_ms": float("nan"), "launches": 0})
    per_launch_bytes = (n * b + L * W * 8) / max(1, G)
    achieved = per_launch_bytes / (scat["avg_ms"] / 1e3) / 1e9
    default_markov = args.workload == "markov96" and not args.n
    single_alu = single_alu_issue(scat["avg_ms"]) if default_markov else None
    roofline = {"kernel": "scatter",
                **({"bound": "alu", "alu": single_alu} if single_alu else
                   {"bound": "hbm", "limiter": "not measured on this workload or kernel source"}),
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": scatter_traffic(per_launch_bytes) if default_markov else None,
                "alg_bytes_per_launch": int(per_launch_bytes), "avg_launch_ms": round(scat["avg_ms"], 4)}
    # both structures by the pair build (wt_pair_build): one pass when the
    # levels fit one group, else the WM and the WT gathered from its
    # intervals; the same K steps, timed the same way
    pair = None
    if L and B.wt_pair_workspace_bytes(n, b, L):
        prec, _, _ = pair_measure(B, d_text, n, b, L, args.steps, args.warmup, stream, dev,
                                  structs[B.WT_TREE], structs[B.WT_MATRIX])
        sc = prec["scatter"]
        pair = {"ms_per_step": prec["ms_per_step"], "ms_per_step_unrecorded": prec["ms_per_step_unrecorded"],
                "value": prec["value"], "kernels": prec["kernels"],
                "roofline": {"kernel": sc["kernel"],
                             **(bound_fields(args.workload, sc["ms_per_step"]) if not args.n else
                                {"bound": "hbm", "limiter": "not measured at this text length"}),
                             "achieved": round(sc["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(sc["achieved"] / HBM_PEAK_GBS, 4),
                             "traffic": (scatter_traffic(sc["alg_bytes_per_launch"], PAIR_COUNTERS)
                                         if default_markov else None),
                             "alg_bytes_per_launch": sc["alg_bytes_per_launch"],
                             "avg_launch_ms": round(sc["avg_launch_ms"], 4)}}

    # whole-build roofline: B_alg = 2 n b + L W 8 + directories, per build
    nb = W // 8
    dir_bytes = L * (nb + 1) * 4 + 2 * L * ((n + 4095) // 4096 + 1) * 4
    b_alg_build = 2 * n * b + L * W * 8 + dir_bytes
    build_gbs = 2 * b_alg_build / (ms_per_step / 1e3) / 1e9

    # correctness property on the measured outputs: access reconstructs the text
    pos = torch.from_numpy(inputs.u64(1 << 16, n, 99, 0).view(np.int64)).to(dev)
    want = torch.from_numpy(text.astype(np.uint32).view(np.int32)).to(dev)[pos]
    for k, s in structs.items():
        got = s.access(pos)
        if not torch.equal(got, want):
            raise SystemExit(f"access check failed for kind {k}")

    # query throughput (extra): 2^20 access / rank / select on each structure
    # at random positions j: access(j), rank(c, j) and select(c, k) with
    # c = T[j] and k = rank(c, j) + 1 (so the select answers j)
    m = 1 << 20
    qpos_h = inputs.u64(m, n, 98, 1)
    qpos = torch.from_numpy(qpos_h.view(np.int64)).to(dev)
    qsym = torch.from_numpy(text[qpos_h.astype(np.int64)].astype(np.uint32).view(np.int32)).to(dev)
    qk = {k: s.rank(qsym, qpos) + 1 for k, s in structs.items()}
    torch.cuda.synchronize()
    qe0, qe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    qe0.record(stream)
    qres = {}
    for k, s in structs.items():
        qres[k] = (s.access(qpos), s.rank(qsym, qpos), s.select(qsym, qk[k]))
    qe1.record(stream)
    torch.cuda.synchronize()
    q_per_s = 6 * m / (qe0.elapsed_time(qe1) / 1e3)
    # self-check of the timed answers (Section 2 definitions): access
    # reconstructs T, select(c, rank(c, j) + 1) = j, rank(c, select(c, k)) = k - 1
    for k, s in structs.items():
        acc, rk, sel = qres[k]
        if not torch.equal(acc, qsym) or not torch.equal(rk + 1, qk[k]) or not torch.equal(sel, qpos):
            raise SystemExit(f"query self-check failed for kind {k}")
        if not torch.equal(s.rank(qsym, sel), qk[k] - 1):
            raise SystemExit(f"rank(select) self-check failed for kind {k}")
    del qres, qk

    # conversion between the two structures (Section 5.1) and the Lemma 5
    # position map, on the measured outputs: each converted structure must
    # equal the one built directly
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0e.record()
        r = fn()
        t1e.record()
        torch.cuda.synchronize()
        return r, t0e.elapsed_time(t1e)

    def same_levels(a, b):
        Wd = a.view.words_per_level
        return torch.equal(a.buf[: L * Wd * 8], b.buf[: L * Wd * 8])

    conv = {}
    for k_from, name in ((B.WT_MATRIX, "wm_to_wt_ms"), (B.WT_TREE, "wt_to_wm_ms")):
        other, ms = timed(lambda: B.convert(structs[k_from]))
        if not same_levels(other, structs[1 - k_from]) or other.status() != 0:
            raise SystemExit(f"conversion from kind {k_from} differs from the direct build")
        conv[name] = round(ms, 3)
        del other
    pm, pm_ms = timed(lambda: B.PosMap(structs[B.WT_TREE]))
    lvl = L - 1
    _, pq_ms = timed(lambda: pm.query(lvl, qpos))
    j = pm.query(lvl, qpos)
    wt_words = structs[B.WT_TREE].buf[: L * W * 8].view(torch.int64).view(L, W)[lvl]
    wm_words = structs[B.WT_MATRIX].buf[: L * W * 8].view(torch.int64).view(L, W)[lvl]
    bit_wt = (wt_words[qpos >> 6] >> (qpos & 63)) & 1
    bit_wm = (wm_words[j >> 6] >> (j & 63)) & 1
    if not torch.equal(bit_wt, bit_wm):
        raise SystemExit("position map does not carry WT bits to equal WM bits")
    # domain decomposition: the WM of 8 consecutive pieces, merged into the
    # WM of the whole text (must equal the direct build)
    pieces = 8
    cut = [(n * i) // pieces for i in range(pieces + 1)]
    parts = [B.build(d_text[cut[i] * b:cut[i + 1] * b], cut[i + 1] - cut[i], b, L, B.WT_MATRIX)
             for i in range(pieces)]
    merged, mg_ms = timed(lambda: B.merge(parts))
    if not same_levels(merged, structs[B.WT_MATRIX]) or merged.status() != 0:
        raise SystemExit("merged pieces differ from the direct build")
    conv["merge_8_pieces_ms"] = round(mg_ms, 3)
    del parts, merged
    # export of the WT to node-local bit vectors (pointer-based tree): every
    # sampled bit of every level must sit in its node at the same offset
    (xn, xp), x_ms = timed(lambda: B.export_nodes(structs[B.WT_TREE]))
    for lvl in range(L):
        e0 = (1 << lvl) - 1
        lens = xn[e0:e0 + (1 << lvl), 1]
        starts = torch.cumsum(lens, 0) - lens
        node = torch.searchsorted(starts, qpos, right=True) - 1
        k = qpos - starts[node]
        words = xn[e0 + node, 0] + (k >> 6)
        got = (xp[words] >> (k & 63)) & 1
        lv_words = structs[B.WT_TREE].buf[: L * W * 8].view(torch.int64).view(L, W)[lvl]
        if not torch.equal(got, (lv_words[qpos >> 6] >> (qpos & 63)) & 1):
            raise SystemExit(f"exported nodes of level {lvl} differ from the WT level")
    conv["export_nodes_ms"] = round(x_ms, 3)
    del xn, xp
    # the second build strategy (a counting sort of the text per level): its
    # time per build, and equality with the default build
    ps_ms = {}
    for k, name in (((B.WT_TREE, "sort_build_wt_ms"), (B.WT_MATRIX, "sort_build_wm_ms"))
                    if B.wt_ps_workspace_bytes(n, b, L) else ()):
        ps_out = B.Structure(n, L, k, device=dev)
        ps_ws = torch.empty(int(B.wt_ps_workspace_bytes(n, b, L)), dtype=torch.uint8, device=dev)
        _, t_ms = timed(lambda: B.ps_build(d_text, n, b, L, k, ws=ps_ws, out=ps_out))
        if not same_levels(ps_out, structs[k]) or ps_out.status() != 0:
            raise SystemExit(f"sorting build of kind {k} differs from the default build")
        ps_ms[name] = round(t_ms, 3)
        del ps_out, ps_ws
    # both structures when both are wanted: build the WM, convert it to the WT
    conv["wm_build_plus_convert_ms"] = round(ms_per_step / 2 + conv["wm_to_wt_ms"], 3)
    conv["posmap_build_ms"] = round(pm_ms, 3)
    conv["posmap_queries_per_s"] = round(m / (pq_ms / 1e3), 1)
    del pm

    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(text, L, min(args.cpu_sample, n))
        cpu_all = cpu_baseline_all_cores(text, L, min(args.cpu_sample_all, n))

    log(f"step {ms_per_step:.3f} ms; kernels per step: " +
        ", ".join(f"{k} {v['total_ms_per_step']:.3f}ms" for k, v in sorted(kernels.items(), key=lambda x: -x[1]['total_ms_per_step'])))
    # the headline step: the WT and the WM of the text by the pair build when
    # the levels fit one group (both structures from one pass), else by two
    # builds; the other way is reported beside it
    separate = {"ms_per_step": round(ms_per_step, 4), "value": round(value, 1),
                "wt_build_ms": round(kind_ms.get(B.WT_TREE, float("nan")), 4),
                "wm_build_ms": round(kind_ms.get(B.WT_MATRIX, float("nan")), 4), "roofline": roofline,
                "build_alg_gbs": round(build_gbs, 1),
                "kernels": {k: {"avg_ms": round(v["avg_ms"], 4), "launches_per_step": v["launches"] // args.steps}
                            for k, v in kernels.items()}}
    how = "WT build + WM build (wt_build, wm_build)"
    if pair is not None:
        ms_per_step, value, roofline = pair["ms_per_step"], pair["value"], pair["roofline"]
        kernels = {k: {"avg_ms": v["avg_ms"], "launches": v["launches"]} for k, v in pair["kernels"].items()}
        dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
        build_gbs = 2 * b_alg_build / (ms_per_step / 1e3) / 1e9
        how = ("the WT and the WM by one pass (wt_pair_build)" if L <= 8 else
               "the WM, then the WT gathered from its intervals (wt_pair_build)")
    out = {
        "metric": "WT+WM build throughput (symbols/s), one GPU",
        "value": round(value, 1),
        "unit": "symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"u{8 * b}",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_TEXT.get(args.workload, 'text')}, n={n} "
                               f"uint{8 * b} symbols, {L} levels; step = {how}, each with levels, Z and "
                               f"rank/select directories",
                   "n": n, "sym_bytes": b, "lg_sigma": L, "tile_log2": args.tile_log2 or "auto",
                   "group_bits": args.group_bits or "auto"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "host": host_info(),
        "paper_reference": paper_reference(),
        "build_alg_gbs": round(build_gbs, 1),
        "build_alg_frac": round(build_gbs / HBM_PEAK_GBS, 4),
        "kernels": {k: {"avg_ms": round(v["avg_ms"], 4), "launches_per_step": v["launches"] // args.steps}
                    for k, v in kernels.items()},
        "dominant_kernel": dom,
        "queries_per_s": round(q_per_s, 1),
        "conversion": conv,
        "sort_strategy": ps_ms,
        "separate_builds": separate if pair is not None else None,
        # the same pair steps without the per-launch events the timed region
        # records (value and the kernel durations come from the recorded ones)
        "ms_per_step_unrecorded": round(pair["ms_per_step_unrecorded"], 4) if pair is not None else None,
    }
    if args.workload == "uniform256" and not args.n and args.steady_texts:
        # the small configuration: its step above is the isolated latency; this
        # is the steady-state rate of many such texts
        out["steady_state"] = steady_state_small(args, B, n, L, b_alg_build, log)
    if default_markov and not args.no_configs:
        # the other plain configurations at their full sizes, each by the
        # pair step (the headline's structures and text are released first)
        del structs, ws, d_text, pos, want, qpos, qsym
        torch.cuda.empty_cache()
        out["configs"] = {}
        for name in ("uniform256", "markov4", "zipf20", "uniform16"):
            steady = args if (name == "uniform256" and args.steady_texts) else None
            out["configs"][name] = config_line(B, name, args.config_steps, args.warmup, stream, dev, steady)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
