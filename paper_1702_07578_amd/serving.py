"""Serving loop: builds and query batches admitted by HBM footprint.

Requests arrive over time.  A build request asks for the WT or WM of a text
already resident in HBM; a query request asks for a batch of access, rank
or select queries against a built, resident structure.  The server keeps a
budget of device memory: a request is admitted only when its footprint
(output buffer plus workspace for a build, answer buffers for queries) fits
into the budget minus what resident structures and requests in flight
already hold; resident structures are evicted oldest first when a build
would not fit otherwise (never one that a query in flight reads).

Continuous batching: whenever a stream slot is free, every admitted build
waiting at that moment is launched together as one batched build
(wt_batch_launch builds all of them in one sequence of launches), and
query batches take slots of their own, so queries overlap builds.  While
query batches are in flight or waiting, builds are launched on a capped
persistent grid, so they leave compute units free for the queries instead
of filling the chip ahead of them.  A request's latency runs from its
arrival to the moment the server sees its completion event.

A query batch either brings its input tensors or a QuerySpec (count and
seed): then its positions are drawn on the device when it is launched,
symbol c = T[j] for every position j, and for select k = rank(c, j) + 1 (so
select answers j); its footprint counts its inputs and its answers.

The scheduling logic is independent of the GPU: it talks to an executor
(GpuExecutor here; the tests also drive it with a simulated one).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any

BUILD, QUERY = "build", "query"
ACCESS, RANK, SELECT = 0, 1, 2


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                  # BUILD or QUERY
    arrival: float             # seconds on the server clock
    text: int = -1             # BUILD: index of a resident text
    tree: int = 1              # BUILD: 0 WT, 1 WM
    target: int = -1           # QUERY: rid of the build whose structure is queried
    op: int = ACCESS           # QUERY: ACCESS, RANK or SELECT
    args: Any = None           # QUERY: device tensors (op-specific) or a QuerySpec
    inputs: Any = None         # QUERY: the input tensors the batch ran on
    footprint: int = 0
    admitted: float = -1.0
    done: float = -1.0
    result: Any = None
    status: int = 0


@dataclasses.dataclass
class QuerySpec:
    """Inputs of a query batch drawn on the device at launch: m positions
    uniform over the text (seeded), their symbols, and for select the k that
    makes select answer each position."""
    m: int
    seed: int


def percentile(xs, q: float) -> float:
    """q-th percentile (0..100) by linear interpolation between closest ranks."""
    if not xs:
        return float("nan")
    s = sorted(xs)
    if len(s) == 1:
        return float(s[0])
    pos = (len(s) - 1) * q / 100.0
    lo = int(pos)
    hi = min(lo + 1, len(s) - 1)
    return float(s[lo] + (s[hi] - s[lo]) * (pos - lo))


class Server:
    """Admission by memory budget, slot-based continuous batching."""

    def __init__(self, executor, budget_bytes: int, slots: int = 4, max_batch: int = 64):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = [None] * slots   # in-flight handle per slot
        self.max_batch = max_batch
        self.queries_inflight = 0
        self.refused = 0              # requests that can never fit the budget
        self.lost_queries = 0         # queries whose structure was evicted or failed
        self.waiting = collections.deque()
        self.resident = collections.OrderedDict()  # build rid -> (structure, bytes)
        self.resident_bytes = 0
        self.inflight_bytes = 0
        self.readers = collections.Counter()       # build rid -> queries in flight
        self.finished = []
        self.gone = set()                          # evicted or failed builds
        self.peak_bytes = 0
        self.evictions = 0

    # -- accounting ------------------------------------------------------------
    def _held(self) -> int:
        return self.resident_bytes + self.inflight_bytes

    def _evict_for(self, need: int, protect: int = -1) -> bool:
        """Make room for need bytes by evicting resident structures (never
        one that a query in flight reads, nor `protect`): only when evicting
        all of them would make room; oldest first among the structures no
        waiting query targets, then oldest first among the others."""
        short = self._held() + need - self.budget
        if short <= 0:
            return True
        movable = [r for r in self.resident if self.readers[r] == 0 and r != protect]
        if sum(self.resident[r][1] for r in movable) < short:
            return False  # nothing is evicted for a request that still would not fit
        wanted = {r.target for r in self.waiting if r.kind == QUERY}
        for victim in [r for r in movable if r not in wanted] + [r for r in movable if r in wanted]:
            if self._held() + need <= self.budget:
                break
            _, nbytes = self.resident.pop(victim)
            self.resident_bytes -= nbytes
            self.gone.add(victim)
            self.ex.free_structure(victim)
            self.evictions += 1
        return True

    # -- the loop ---------------------------------------------------------------
    def submit(self, req: Request, now: float = 0.0):
        req.footprint = self.ex.footprint(req)
        if req.footprint > self.budget:
            # can never fit: refused at once
            req.status, req.admitted, req.done = -2, now, now
            self.refused += 1
            self.finished.append(req)
            if req.kind == BUILD:
                self.gone.add(req.rid)
            return
        self.waiting.append(req)

    def _complete(self, handle, now):
        reqs, nbytes = handle["reqs"], handle["bytes"]
        self.inflight_bytes -= nbytes
        for r in reqs:
            r.done = now
            self.finished.append(r)
            if r.kind == BUILD:
                s, keep = self.ex.take_structure(handle, r)
                r.status = self.ex.status(s)
                if r.status == 0:
                    self.resident[r.rid] = (s, keep)
                    self.resident_bytes += keep
                else:
                    self.gone.add(r.rid)
                    self.ex.free_structure(r.rid)
            else:
                self.readers[r.target] -= 1
                self.queries_inflight -= 1

    def poll(self, now: float):
        for i, h in enumerate(self.slots):
            if h is not None and self.ex.done(h):
                self._complete(h, now)
                self.slots[i] = None

    def admit(self, now: float):
        """Launch what fits on free slots: each query batch on a slot of its
        own, the waiting builds (first come, first served) together on one."""
        free = [i for i, h in enumerate(self.slots) if h is None]
        if not free or not self.waiting:
            return
        launched = set()
        for r in self.waiting:
            if r.kind != QUERY:
                continue
            if r.target in self.gone:
                # the structure was evicted (or its build failed)
                r.status, r.admitted, r.done = -1, now, now
                self.lost_queries += 1
                self.finished.append(r)
                launched.add(r.rid)
                continue
            if r.target not in self.resident or not free:
                continue  # target still being built, or no slot: wait
            if (self._held() + r.footprint > self.budget and
                    not self._evict_for(r.footprint, protect=r.target)):
                continue
            r.admitted = now
            self.readers[r.target] += 1
            self.queries_inflight += 1
            self.inflight_bytes += r.footprint
            s, _ = self.resident[r.target]
            self.resident.move_to_end(r.target)
            slot = free.pop(0)
            self.slots[slot] = self.ex.launch_query(slot, r, s)
            launched.add(r.rid)
        if free:
            builds, need = [], 0
            for r in self.waiting:
                if r.kind != BUILD:
                    continue
                if len(builds) >= self.max_batch:
                    break
                if (self._held() + need + r.footprint <= self.budget or
                        self._evict_for(need + r.footprint)):
                    builds.append(r)
                    need += r.footprint
                else:
                    break  # a build that does not fit holds back later builds
            if builds:
                slot = free.pop(0)
                for r in builds:
                    r.admitted = now
                    launched.add(r.rid)
                self.inflight_bytes += need
                # share the chip while query batches run or wait
                share = self.queries_inflight > 0 or any(
                    r.kind == QUERY and r.rid not in launched for r in self.waiting)
                self.slots[slot] = self.ex.launch_builds(slot, builds, share)
        if launched:
            self.waiting = collections.deque(r for r in self.waiting if r.rid not in launched)
        self.peak_bytes = max(self.peak_bytes, self._held())

    def run(self, requests, clock=time.perf_counter, idle=None, stall_s: float = 60.0):
        """Serve requests (arrival in seconds from the start of the run).
        Returns the finished requests.  Raises RuntimeError if nothing
        completes for stall_s seconds while work is waiting."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        t0 = clock()
        last = 0.0
        done = 0
        while pending or self.waiting or any(h is not None for h in self.slots):
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft(), now)
            self.poll(now)
            self.admit(now)
            if len(self.finished) != done:
                done, last = len(self.finished), now
            elif now - last > stall_s and not pending:
                raise RuntimeError(f"serving loop stalled: {len(self.waiting)} waiting")
            if idle is not None:
                idle(self, now)
        return self.finished

    def stats(self):
        out = {}
        for kind in (BUILD, QUERY):
            lat = [r.done - r.arrival for r in self.finished if r.kind == kind and r.status == 0]
            out[kind] = {"count": len(lat), "p50_ms": percentile(lat, 50) * 1e3,
                         "p99_ms": percentile(lat, 99) * 1e3}
        out["peak_bytes"] = self.peak_bytes
        out["evictions"] = self.evictions
        out["refused"] = self.refused
        out["lost_queries"] = self.lost_queries
        return out


class GpuExecutor:
    """Runs admitted work on the GPU through the C ABI, one stream per slot
    (all at the default priority)."""

    # workgroups of a build launched while queries run (of 256 compute units)
    SHARED_PERSIST = 96

    def __init__(self, texts, slots: int, device="cuda:0", share_persist: int = SHARED_PERSIST):
        import torch

        from . import binding as B
        self.B = B
        self.torch = torch
        self.texts = texts  # list of (d_text, n, sym_bytes, L)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.device = device
        self.structs = {}
        self.shared_tune = B.make_tune(persist=share_persist) if share_persist else None
        self.builds = {}  # build rid -> text index

    def footprint(self, r: Request) -> int:
        B = self.B
        if r.kind == BUILD:
            _, n, b, L = self.texts[r.text]
            return int(B.wt_output_bytes(n, L)) + int(B.workspace_bytes(n, b, L, r.tree))
        answer = 4 if r.op == ACCESS else 8
        if isinstance(r.args, QuerySpec):
            # positions (8), symbols (4), k for select (8), answers
            return r.args.m * (8 + (4 if r.op != ACCESS else 0) + (8 if r.op == SELECT else 0) + answer)
        return sum(int(t.numel()) * t.element_size() for t in r.args) + r.args[0].numel() * answer

    def launch_builds(self, slot: int, reqs, share: bool = False):
        B, torch = self.B, self.torch
        st = self.streams[slot]
        items = []
        for r in reqs:
            d, n, b, L = self.texts[r.text]
            items.append((d, n, b, L, r.tree, B.Structure(n, L, r.tree, device=self.device)))
            self.builds[r.rid] = r.text
        with torch.cuda.stream(st):
            batch = B.Batch(items, tune=self.shared_tune if share else None)
            batch.build(st)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"reqs": reqs, "bytes": sum(r.footprint for r in reqs), "event": ev,
                "batch": batch, "items": items}

    def query_inputs(self, r: Request, s, st):
        """The batch's input tensors: its own, or drawn from its QuerySpec on
        stream st (same seed, same inputs)."""
        torch = self.torch
        if not isinstance(r.args, QuerySpec):
            return r.args
        d, n, b, _ = self.texts[self.builds[r.target]]
        g = torch.Generator(device=self.device)
        g.manual_seed(int(r.args.seed))
        pos = torch.randint(0, max(n, 1), (r.args.m,), generator=g, device=self.device, dtype=torch.int64)
        if r.op == ACCESS:
            return (pos,)
        # the text is a byte tensor: its symbols as 1-, 2- or 4-byte values
        if b == 1:
            sym = d[pos].to(torch.int32)
        elif b == 2:
            sym = d.view(torch.int16)[pos].to(torch.int32) & 0xFFFF
        else:
            sym = d.view(torch.int32)[pos]
        if r.op == RANK:
            return (sym, pos)
        return (sym, s.rank(sym, pos, stream=st) + 1)

    def launch_query(self, slot: int, r: Request, s):
        torch = self.torch
        st = self.streams[slot]
        with torch.cuda.stream(st):
            args = r.inputs = self.query_inputs(r, s, st)
            if r.op == ACCESS:
                r.result = s.access(args[0], stream=st)
            elif r.op == RANK:
                r.result = s.rank(args[0], args[1], stream=st)
            else:
                r.result = s.select(args[0], args[1], stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"reqs": [r], "bytes": r.footprint, "event": ev, "inputs": args}

    def done(self, h) -> bool:
        return h["event"].query()

    def take_structure(self, h, r):
        i = h["reqs"].index(r)
        s = h["items"][i][5]
        self.structs[r.rid] = s
        return s, s.nbytes

    def status(self, s) -> int:
        return s.status()

    def free_structure(self, rid):
        self.structs.pop(rid, None)
