"""Serving scheduler on a simulated clock with a modelled device (host only)."""
import numpy as np
import pytest

import mdwf_synth as S
from paper_1810_01609_amd.serve import Request, Scheduler, merge_chunks, percentiles, simulate, split_requests

GBS = 4000e9  # modelled sustained bandwidth


class FakeBackend:
    """Each RHS needs `iters` iterations; an iteration moves ~2 kB per 5D
    site per RHS; fused RHS share one launch."""

    def __init__(self, iters=100):
        self.iters = iters
        self.begun = []
        self.max_slots_seen = {}

    def footprint(self, r):
        # FP16 inner state (~550 B per even 5D site) + complex128 source and solution
        V = int(np.prod(r.volume))
        return r.nsrc * V * r.L5 * (550 // 2 + 2 * 192)

    def begin(self, r):
        self.begun.append(r.id)
        return {"req": r, "left": self.iters}

    def step(self, lane, jobs, iters):
        nslots = sum(j["req"].nsrc for j in jobs)
        self.max_slots_seen[lane] = max(self.max_slots_seen.get(lane, 0), nslots)
        V = int(np.prod(lane[0])) // 2
        n = min(iters, max(j["left"] for j in jobs))
        for j in jobs:
            j["left"] -= n
        return n * (nslots * V * lane[1] * 2000.0 / GBS + 40e-6)

    def poll(self, j):
        done = j["left"] <= 0
        return done, [{"converged": 1, "iters": self.iters}] * j["req"].nsrc if done else []

    def end(self, j):
        pass


def _trace(n=60, rate=20.0, seed=5):
    vols = [(8, 8, 8, 16), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]
    t = S.poisson_trace(n, rate, seed, vols, [8, 12, 16], (0.005, 0.05), (1, 12))
    return [Request(id=d["id"], t_arrival=d["t_arrival"], volume=d["volume"], L5=d["L5"], mq=d["mq"],
                    nsrc=d["nsrc"], seed=100000 + d["id"]) for d in t]


def test_all_requests_complete_within_budget():
    be = FakeBackend()
    tr = _trace()
    budget = 280 * 10 ** 9
    sched = simulate(tr, be, budget)
    assert len(sched.done) == len(tr)
    assert sched.peak_used <= budget
    assert sched.used == 0
    for r in sched.done:
        assert r.t_arrival <= r.t_admit <= r.t_done
    # admission follows arrival order
    admits = [r.t_admit for r in sorted(sched.done, key=lambda r: r.t_arrival)]
    assert all(a <= b for a, b in zip(admits, admits[1:]))
    p = percentiles(sched.done)
    assert 0 < p["p50_ms"] <= p["p99_ms"]


def test_continuous_batching_joins_running_batch():
    be = FakeBackend(iters=400)
    V = (8, 8, 8, 16)
    tr = [Request(0, 0.0, V, 8, 0.01, 2), Request(1, 0.001, V, 8, 0.02, 3), Request(2, 0.002, V, 8, 0.03, 1)]
    sched = simulate(tr, be, 1 << 40, iters_per_step=10)
    r0, r1, r2 = sorted(sched.done, key=lambda r: r.id)
    # later arrivals were admitted while the first was still iterating
    assert r1.t_admit < r0.t_done and r2.t_admit < r0.t_done
    assert be.max_slots_seen[(V, 8)] == 6


def test_budget_serialises_when_tight():
    be = FakeBackend()
    V = (16, 16, 16, 32)
    mk = lambda: [Request(i, 0.0, V, 12, 0.01, 4) for i in range(4)]
    tr = mk()
    one = be.footprint(tr[0])
    sched = simulate(tr, be, one + one // 2)
    assert sched.peak_used == one
    done = sorted(sched.done, key=lambda r: r.t_done)
    for a, b in zip(done, done[1:]):
        assert b.t_admit >= a.t_done - 1e-12
    wide = simulate(mk(), FakeBackend(), 8 * one)
    assert percentiles(wide.done)["p99_ms"] < percentiles(sched.done)["p99_ms"]


def test_oversized_request_is_rejected():
    be = FakeBackend()
    s = Scheduler(1000, be.footprint)
    with pytest.raises(ValueError):
        s.arrive(Request(0, 0.0, (8, 8, 8, 16), 8, 0.01, 1))


def test_slot_cap_per_lane():
    be = FakeBackend()
    V = (8, 8, 8, 16)
    tr = [Request(i, 0.0, V, 8, 0.01, 12) for i in range(4)]
    simulate(tr, be, 1 << 40, max_slots_per_lane=24)
    assert be.max_slots_seen[(V, 8)] <= 24


def test_split_and_merge_chunks():
    tr = [Request(7, 0.5, (8, 8, 8, 16), 8, 0.01, 12, seed=3), Request(8, 0.6, (8, 8, 8, 16), 8, 0.01, 2)]
    parts = split_requests(tr, 5)
    assert [(p.id, p.nsrc, p.src_offset, p.parent) for p in parts] == [
        (7000, 5, 0, 7), (7001, 5, 5, 7), (7002, 2, 10, 7), (8000, 2, 0, 8)]
    # no part shares an id with another, whatever the ids of whole and split requests
    many = split_requests([Request(i, 0.0, (8, 8, 8, 16), 8, 0.01, 1 + 5 * (i % 3)) for i in range(40)], 4)
    assert len({p.id for p in many}) == len(many)
    sched = simulate(parts, FakeBackend(), 1 << 40)
    merged = {r.id: r for r in merge_chunks(sched.done)}
    assert merged[7].nsrc == 12 and merged[8].nsrc == 2
    assert merged[7].t_done == max(r.t_done for r in sched.done if r.parent == 7)


def test_real_time_loop_frees_idle_lanes_and_keeps_budget():
    """serve_gpu, the threaded real-time loop, on a host-only backend: every
    request of a mixed trace completes, the admitted bytes never exceed the
    budget, every part of a split request keeps its own handle (no job is
    stepped twice in one call), and a lane whose last job ends is told to
    release its workspace."""
    import threading

    from paper_1810_01609_amd.serve import serve_gpu

    class ThreadedFake(FakeBackend):
        def __init__(self):
            super().__init__(iters=30)
            self.idled = []
            self.lock = threading.Lock()

        def step(self, lane, jobs, iters):
            assert len({id(j) for j in jobs}) == len(jobs), "a job listed twice in one step"
            super().step(lane, jobs, iters)
            return 0.0

        def idle(self, lane):
            with self.lock:
                self.idled.append(lane)

    tr = split_requests(_trace(n=24, rate=200.0), 4)
    be = ThreadedFake()
    budget = 200 * 10 ** 9
    sched, _, wall = serve_gpu(tr, be, budget, iters_per_step=10, max_slots_per_lane=16)
    assert len(sched.done) == len(tr)
    assert sched.peak_used <= budget and sched.used == 0
    assert set(be.idled) == {r.lane for r in tr}
    assert len(merge_chunks(sched.done)) == 24
