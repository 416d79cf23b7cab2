"""Serving loop scheduling on the CPU, with a simulated executor: admission
by memory budget, batching of waiting builds, queries waiting for their
structure, eviction order, refusal, and the latency percentiles."""
import numpy as np
import pytest

from paper_1702_07578_amd import serving as S


class FakeExecutor:
    """Every build takes `build_s` seconds per launch (whatever its size),
    every query batch `query_s`; footprints are given per request."""

    def __init__(self, clock, build_s=0.010, query_s=0.002):
        self.clock = clock
        self.build_s, self.query_s = build_s, query_s
        self.launches = []
        self.freed = []

    def footprint(self, r):
        return r.args["fp"]

    def launch_builds(self, slot, reqs, share=False):
        self.launches.append(("build", slot, [r.rid for r in reqs]))
        self.shared = getattr(self, "shared", []) + [share]
        return {"reqs": reqs, "bytes": sum(r.footprint for r in reqs),
                "end": self.clock.t + self.build_s}

    def launch_query(self, slot, r, s):
        self.launches.append(("query", slot, [r.rid]))
        r.result = ("answer", s)
        return {"reqs": [r], "bytes": r.footprint, "end": self.clock.t + self.query_s}

    def done(self, h):
        return self.clock.t >= h["end"]

    def take_structure(self, h, r):
        return ("structure", r.rid), r.args["keep"]

    def status(self, s):
        return 0

    def free_structure(self, rid):
        self.freed.append(rid)


class Clock:
    """Simulated time: every reading advances it by dt."""

    def __init__(self, dt=0.0005):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


def build(rid, t, fp=100, keep=60):
    return S.Request(rid=rid, kind=S.BUILD, arrival=t, text=0, args={"fp": fp, "keep": keep})


def query(rid, t, target, fp=10):
    return S.Request(rid=rid, kind=S.QUERY, arrival=t, target=target, args={"fp": fp})


def run(reqs, budget, slots=4, max_batch=64, dt=0.0005):
    clock = Clock(dt)
    ex = FakeExecutor(clock)
    srv = S.Server(ex, budget, slots=slots, max_batch=max_batch)
    peak = [0]

    def watch(s, now):
        peak[0] = max(peak[0], s.resident_bytes + s.inflight_bytes)
    done = srv.run(reqs, clock=clock, idle=watch)
    return srv, ex, done, peak[0]


def test_everything_finishes_within_budget():
    rng = np.random.default_rng(1)
    reqs, t = [], 0.0
    for i in range(60):
        t += float(rng.exponential(0.003))
        if i % 3 == 2:
            reqs.append(query(i, t, target=i - 1 - (i % 2)))
        else:
            reqs.append(build(i, t, fp=int(rng.integers(50, 200)), keep=int(rng.integers(20, 50))))
    srv, ex, done, peak = run(reqs, budget=600)
    assert len(done) == len(reqs)
    assert peak <= 600 and srv.peak_bytes <= 600
    for r in done:
        assert r.done >= r.admitted >= r.arrival
    st = srv.stats()
    assert st[S.BUILD]["count"] + st[S.QUERY]["count"] + sum(r.status != 0 for r in done) == len(reqs)


def test_waiting_builds_launch_together():
    # ten builds arrive while the only slot is busy: they go in one launch
    reqs = [build(0, 0.0)] + [build(i, 0.001 + 0.0001 * i) for i in range(1, 11)]
    srv, ex, done, _ = run(reqs, budget=10_000, slots=1)
    builds = [l for l in ex.launches if l[0] == "build"]
    assert builds[0][2] == [0]
    assert builds[1][2] == list(range(1, 11))


def test_max_batch_and_fifo():
    reqs = [build(0, 0.0)] + [build(i, 0.001) for i in range(1, 8)]
    srv, ex, done, _ = run(reqs, budget=10_000, slots=1, max_batch=3)
    order = [rid for kind, _, rids in ex.launches for rid in rids]
    assert order == list(range(8))
    assert max(len(rids) for _, _, rids in ex.launches) <= 3


def test_query_waits_for_its_structure():
    reqs = [build(0, 0.0), query(1, 0.0001, target=0)]
    srv, ex, done, _ = run(reqs, budget=10_000)
    q = next(r for r in done if r.rid == 1)
    b = next(r for r in done if r.rid == 0)
    assert q.status == 0 and q.admitted >= b.done
    assert q.result == ("answer", ("structure", 0))


def test_eviction_oldest_first_and_refusal():
    # each build keeps 60 of a 150 budget: the third build evicts the first
    reqs = [build(0, 0.0, fp=80, keep=60), build(1, 0.02, fp=80, keep=60),
            build(2, 0.04, fp=80, keep=60), query(3, 0.06, target=0),
            build(4, 0.07, fp=1000)]
    srv, ex, done, peak = run(reqs, budget=150)
    assert ex.freed[0] == 0
    by = {r.rid: r for r in done}
    assert by[3].status == -1      # its structure was evicted
    assert by[4].status == -2      # can never fit
    assert peak <= 150


def test_query_in_flight_pins_its_structure():
    # a long query on structure 0 while a build needs room: structure 1 goes
    reqs = [build(0, 0.0, fp=50, keep=40), build(1, 0.02, fp=50, keep=40),
            query(2, 0.04, target=0, fp=10)]
    clock = Clock()
    ex = FakeExecutor(clock, query_s=0.05)
    srv = S.Server(ex, 110, slots=4)
    reqs.append(build(3, 0.045, fp=60, keep=40))
    srv.run(reqs, clock=clock)
    assert 0 not in ex.freed[:1]
    assert ex.freed and ex.freed[0] == 1


@pytest.mark.parametrize("q", [0, 1, 50, 90, 99, 100])
def test_percentile_matches_numpy(q):
    xs = list(np.random.default_rng(3).exponential(1.0, size=101))
    assert S.percentile(xs, q) == pytest.approx(float(np.percentile(xs, q)))


def _server_with(resident, budget, waiting=(), readers=()):
    """A server in a given state: resident {rid: bytes} (oldest first),
    waiting requests, and structures that queries in flight read."""
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = S.Server(ex, budget, slots=2)
    for rid, nbytes in resident.items():
        srv.resident[rid] = (("structure", rid), nbytes)
        srv.resident_bytes += nbytes
    srv.waiting.extend(waiting)
    for rid in readers:
        srv.readers[rid] += 1
    return srv, ex


def test_nothing_evicted_when_eviction_cannot_make_room():
    # 100 of 150 held; 100 more needed; only 40 of the held bytes are
    # movable (structure 1 is read by a query in flight): no eviction at all
    srv, ex = _server_with({0: 40, 1: 60}, 150, readers=[1])
    assert not srv._evict_for(100)
    assert ex.freed == [] and srv.evictions == 0 and set(srv.resident) == {0, 1}
    # once the query is done, both go (oldest first) and the request fits
    srv.readers[1] -= 1
    assert srv._evict_for(100)
    assert ex.freed == [0, 1]


def test_structures_that_waiting_queries_target_are_evicted_last():
    # oldest is 0, but a waiting query targets it: 1 goes first
    srv, ex = _server_with({0: 50, 1: 50, 2: 50}, 150, waiting=[query(9, 0.0, target=0)])
    assert srv._evict_for(50)
    assert ex.freed == [1]
    assert srv._evict_for(150)
    assert ex.freed == [1, 2, 0]


def test_builds_share_the_chip_while_queries_run():
    # a long query on structure 0 is in flight when build 2 launches: that
    # build takes the capped grid; build 1, launched alone, does not
    clock = Clock()
    ex = FakeExecutor(clock, query_s=0.05)
    srv = S.Server(ex, 10_000, slots=4)
    reqs = [build(0, 0.0), build(1, 0.02), query(2, 0.04, target=0), build(3, 0.05)]
    srv.run(reqs, clock=clock)
    assert ex.shared == [False, False, True]


def test_refusals_and_lost_queries_are_counted():
    reqs = [build(0, 0.0, fp=80, keep=60), build(1, 0.02, fp=80, keep=60),
            build(2, 0.04, fp=80, keep=60), query(3, 0.06, target=0),
            build(4, 0.07, fp=1000)]
    srv, ex, done, _ = run(reqs, budget=150)
    st = srv.stats()
    assert st["refused"] == 1 and st["lost_queries"] == 1 and st["evictions"] >= 1
