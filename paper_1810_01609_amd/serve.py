"""Continuous-batching serving loop for propagator solves.

Requests (a lattice volume, L5, quark mass and 1-12 complex Z2 sources)
arrive over time.  Gauge fields stay resident in HBM, one per volume.  A
request is admitted when its device footprint (``mdwf_job_footprint``) fits
the HBM budget that is left; admitted requests join a *lane* -- one lane per
(volume, L5), each with its own context and HIP stream -- and every lane
steps all of its in-flight jobs together through ``mdwf_job_step``, so new
requests join the running batch at the next iteration boundary and finished
ones leave it, freeing budget for the queue.  Lanes run in their own host
threads (the library releases the GIL), so work of different volumes
overlaps on the device.  Latency is completion minus arrival.

The paper's job manager does the same at machine scale ("Management and
Backfilling of Tasks": a map of resources consumed by running jobs, ready
jobs matched to open resources); here the resource is one GPU's HBM.

The scheduling core is independent of the device: ``Scheduler`` keeps the
queue, budget and lane membership and is driven either by ``serve_gpu``
(threads, wall clock, the HIP library) or by ``simulate`` (single thread,
simulated clock, a modelled backend) for host-only tests.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Request:
    id: int
    t_arrival: float
    volume: tuple
    L5: int
    mq: float
    nsrc: int
    seed: int = 0
    parent: int = -1  # id of the request a chunk belongs to (-1: a whole request)
    src_offset: int = 0  # index of the chunk's first source within its request
    # filled by the scheduler
    t_admit: float = -1.0
    t_done: float = -1.0
    stats: list = field(default_factory=list)
    footprint: int = 0

    @property
    def lane(self):
        return (tuple(self.volume), int(self.L5))

    @property
    def latency(self):
        return self.t_done - self.t_arrival


def split_requests(trace, max_rhs):
    """Split requests with more than `max_rhs` sources into chunks that are
    admitted and batched independently (a 12-source request on the largest
    volume would otherwise have to hold the whole GPU).  Every part, a whole
    request included, gets the id (request id * 1000 + chunk index), so no
    chunk shares an id with another request; `parent` names the request."""
    out = []
    for r in trace:
        if r.nsrc > 1000 * max_rhs:
            raise ValueError(f"request {r.id}: more than 1000 chunks")
        for k, off in enumerate(range(0, r.nsrc, max_rhs)):
            out.append(Request(id=r.id * 1000 + k, t_arrival=r.t_arrival, volume=r.volume, L5=r.L5, mq=r.mq,
                               nsrc=min(max_rhs, r.nsrc - off), seed=r.seed, parent=r.id, src_offset=off))
    return out


def merge_chunks(done):
    """Per original request: arrival, first admission, last completion."""
    by = {}
    for r in done:
        key = r.parent if r.parent >= 0 else r.id
        if key not in by:
            by[key] = Request(id=key, t_arrival=r.t_arrival, volume=r.volume, L5=r.L5, mq=r.mq, nsrc=0,
                              seed=r.seed, t_admit=r.t_admit, t_done=r.t_done)
        m = by[key]
        m.nsrc += r.nsrc
        m.t_admit = min(m.t_admit, r.t_admit)
        m.t_done = max(m.t_done, r.t_done)
        m.stats = m.stats + list(r.stats)
    return list(by.values())


class Scheduler:
    """Admission by HBM footprint, FIFO per arrival, lanes by (volume, L5)."""

    def __init__(self, budget_bytes: int, footprint, max_slots_per_lane: int = 64):
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak_used = 0
        self.footprint = footprint
        self.max_slots = max_slots_per_lane
        self.queue: deque[Request] = deque()
        self.starting: dict = {}  # lane -> admitted requests not yet begun on the device
        self.active: dict = {}  # lane -> list of in-flight requests
        self.done: list[Request] = []
        self.lock = threading.Lock()

    def arrive(self, req: Request):
        with self.lock:
            req.footprint = int(self.footprint(req))
            if req.footprint > self.budget:
                raise ValueError(f"request {req.id} needs {req.footprint} B, more than the whole budget")
            self.queue.append(req)

    def admit(self, now: float, lane=None):
        """Admit queued requests in arrival order while they fit.  A request
        that does not fit blocks the ones behind it (no starvation).  With
        `lane`, only that lane's head-of-line requests are considered."""
        out = []
        with self.lock:
            while self.queue:
                r = self.queue[0]
                if lane is not None and r.lane != lane:
                    break
                slots = sum(x.nsrc for x in self.active.get(r.lane, []) + self.starting.get(r.lane, []))
                if self.used + r.footprint > self.budget or slots + r.nsrc > self.max_slots:
                    break
                self.queue.popleft()
                self.used += r.footprint
                self.peak_used = max(self.peak_used, self.used)
                r.t_admit = now
                self.starting.setdefault(r.lane, []).append(r)
                out.append(r)
        return out

    def take_starting(self, lane):
        """Admitted requests of a lane that still have to be begun."""
        with self.lock:
            out = self.starting.get(lane, [])
            self.starting[lane] = []
            return out

    def activate(self, r: Request):
        with self.lock:
            self.active.setdefault(r.lane, []).append(r)

    def lanes_busy(self):
        with self.lock:
            return any(self.active.values()) or any(self.starting.values())

    def retire(self, r: Request, now: float, stats):
        with self.lock:
            self.active[r.lane].remove(r)
            self.used -= r.footprint
            r.t_done = now
            r.stats = stats
            self.done.append(r)

    def lane_jobs(self, lane):
        with self.lock:
            return list(self.active.get(lane, []))


def percentiles(reqs):
    import numpy as np

    lat = np.array([r.latency for r in reqs])
    wait = np.array([r.t_admit - r.t_arrival for r in reqs])
    return {
        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "mean_ms": 1e3 * float(lat.mean()),
        "queue_p50_ms": 1e3 * float(np.percentile(wait, 50)),
        "queue_p99_ms": 1e3 * float(np.percentile(wait, 99)),
    }


# ---------------------------------------------------------------------------
# simulated driver (host only)
# ---------------------------------------------------------------------------
def simulate(trace, backend, budget_bytes, iters_per_step=20, max_slots_per_lane=64):
    """Run the scheduler on a simulated clock.  `backend` provides
    footprint(req), begin(req), step(lane, jobs, iters) -> seconds,
    poll(job) -> (done, stats), end(job).  Lanes are stepped round-robin;
    each lane keeps its own clock (lanes model concurrent streams)."""
    sched = Scheduler(budget_bytes, backend.footprint, max_slots_per_lane)
    pending = deque(sorted(trace, key=lambda r: r.t_arrival))
    lane_clock: dict = {}
    handles = {}
    now = 0.0
    while pending or sched.queue or sched.lanes_busy():
        while pending and pending[0].t_arrival <= now:
            sched.arrive(pending.popleft())
        for r in sched.admit(now):
            lane_clock.setdefault(r.lane, now)
            lane_clock[r.lane] = max(lane_clock[r.lane], now)
        for lane in list(sched.starting):
            for r in sched.take_starting(lane):
                handles[r.id] = backend.begin(r)
                sched.activate(r)
        lanes = [l for l, js in sched.active.items() if js]
        if not lanes:
            if pending:
                now = max(now, pending[0].t_arrival)
                continue
            break
        # advance the lane that is furthest behind
        lane = min(lanes, key=lambda l: lane_clock[l])
        jobs = sched.lane_jobs(lane)
        dt = backend.step(lane, [handles[r.id] for r in jobs], iters_per_step)
        lane_clock[lane] += dt
        now = max(now, min(lane_clock[l] for l in lanes))
        for r in jobs:
            done, stats = backend.poll(handles[r.id])
            if done:
                backend.end(handles.pop(r.id))
                sched.retire(r, lane_clock[lane], stats)
    return sched


# ---------------------------------------------------------------------------
# GPU driver
# ---------------------------------------------------------------------------
class GPUBackend:
    """Resident gauge fields per volume, one context (stream) per lane."""

    def __init__(self, volumes, gauge_eps=0.2, gauge_seeds=None, inner="f32", tol=1e-10,
                 b5=1.5, c5=0.5, M5=1.3, device=0):
        import mdwf_synth as S
        from . import mdwf as M

        self.M = M
        self.inner = inner
        self.tol = tol
        self.b5, self.c5, self.M5 = b5, c5, M5
        self.device = device
        self.ctx0 = M.Context(device, use_torch_stream=False)
        self.gauge = {}
        seeds = gauge_seeds or {}
        for i, V in enumerate(volumes):
            V = tuple(V)
            U = S.gauge_field(V, gauge_eps, seeds.get(V, 11 + i))
            self.gauge[V] = self.ctx0.gauge_load(V, U, precs=("f64", inner))
        self.lane_ctx = {}
        self.lane_streams = {}
        self.lock = threading.Lock()

    @property
    def resident_bytes(self):
        return sum(g.nbytes for g in self.gauge.values())

    def act(self, req):
        return self.M.Action.make(req.volume, req.L5, self.b5, self.c5, self.M5, req.mq)

    def opts(self):
        return self.M.CGOpts.make(tol=self.tol, inner=self.inner)

    def footprint(self, req):
        # job state + the user-layout source and solution tensors
        user = 16 * req.L5 * 12 * req.volume[0] * req.volume[1] * req.volume[2] * req.volume[3] * req.nsrc
        return self.M.job_footprint(self.act(req), self.opts(), req.nsrc) + 2 * user

    def ctx_for(self, lane):
        """The lane's context, on a stream of its own: a torch stream (created
        non-blocking, default priority), so the lane's work never waits for
        torch's default stream or for another lane."""
        import torch

        with self.lock:
            if lane not in self.lane_ctx:
                s = torch.cuda.Stream(device=f"cuda:{self.device}")
                self.lane_streams[lane] = s
                self.lane_ctx[lane] = self.M.Context(self.device, stream=s.cuda_stream)
            return self.lane_ctx[lane]

    def lane_stream(self, lane):
        """The lane's torch stream (the one its context adopted)."""
        self.ctx_for(lane)
        return self.lane_streams[lane]

    def begin(self, req):
        import torch

        ctx = self.ctx_for(req.lane)
        a = self.act(req)
        # torch caches freed blocks per stream, and with one stream per lane
        # its cache can grow to most of the device: when the device's free
        # memory would not hold this request, the cache goes back first
        if torch.cuda.mem_get_info(self.device)[0] < self.footprint(req) + 8e9:
            torch.cuda.empty_cache()
        # the request's tensors are allocated and cleared on the lane's own
        # stream, so the library's kernels that follow on that stream are
        # ordered after the clearing without waiting for any other lane
        with torch.cuda.stream(self.lane_stream(req.lane)):
            eta = torch.zeros((req.nsrc,) + a.spinor_shape(), dtype=torch.complex128, device=f"cuda:{self.device}")
            psi = torch.zeros_like(eta)
        for k in range(req.nsrc):
            ctx.source_z2(a, req.seed, req.src_offset + k, eta[k])
        try:
            job = ctx.job_begin(self.gauge[tuple(req.volume)], a, self.opts(), eta, psi, nrhs=req.nsrc)
        except self.M.MDWFError as e:
            # the admitted footprints fit the budget, but torch's caching
            # allocator may still hold blocks freed by finished requests:
            # return them to the device and try once more
            if e.status != self.M.ENOMEM:
                raise
            torch.cuda.empty_cache()
            job = ctx.job_begin(self.gauge[tuple(req.volume)], a, self.opts(), eta, psi, nrhs=req.nsrc)
        job.req = req
        job.psi = psi
        return job

    def solution(self, lane, job):
        """The finished job's psi on the host (waits for the lane's stream only)."""
        import torch

        s = self.lane_stream(lane)
        s.synchronize()
        with torch.cuda.stream(s):
            return job.psi.cpu().numpy()

    def step(self, lane, jobs, iters):
        ctx = self.ctx_for(lane)
        t = time.perf_counter()
        st = ctx.job_step(jobs, iters)
        if st not in (0, -4, -5, -6):  # per-RHS failures are reported through poll
            raise self.M.MDWFError(st, "mdwf_job_step")
        return time.perf_counter() - t

    def poll(self, job):
        return job.poll()

    def end(self, job):
        job.end()
        job.psi = None  # the request's tensors go with the job, not with the last reference to it

    def idle(self, lane):
        """The lane has no job left: its context releases the FP64 workspace
        it keeps between calls (each job's footprint counts it while the job
        runs, so the budget stays exact across lanes)."""
        if lane in self.lane_ctx:
            self.lane_ctx[lane].trim()

    def close(self):
        for g in self.gauge.values():
            g.free()
        for c in self.lane_ctx.values():
            c.close()
        self.ctx0.close()


def serve_gpu(trace, backend: GPUBackend, budget_bytes, iters_per_step=25, max_slots_per_lane=24,
              keep_solutions=False, progress=None, progress_every=10.0):
    """Serve a trace in real time: arrivals at their t_arrival (seconds from
    start), one worker thread per lane.  progress(done, total, seconds,
    admitted bytes) is called about every `progress_every` seconds."""
    sched = Scheduler(budget_bytes, backend.footprint, max_slots_per_lane)
    pending = deque(sorted(trace, key=lambda r: r.t_arrival))
    handles = {}
    solutions = {}
    stop = threading.Event()
    errors = []
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    workers = {}
    wake = threading.Condition()

    def lane_worker(lane):
        try:
            while not stop.is_set():
                for r in sched.take_starting(lane):
                    handles[r.id] = backend.begin(r)  # this lane's context, this thread only
                    sched.activate(r)
                jobs = sched.lane_jobs(lane)
                if not jobs:
                    with wake:
                        wake.wait(timeout=0.002)
                    continue
                hs = [handles[r.id] for r in jobs]
                backend.step(lane, hs, iters_per_step)
                for r in jobs:
                    done, stats = backend.poll(handles[r.id])
                    if done:
                        h = handles.pop(r.id)
                        if keep_solutions:
                            solutions[r.id] = backend.solution(lane, h)
                        backend.end(h)
                        sched.retire(r, now(), stats)
                        if not sched.lane_jobs(lane) and hasattr(backend, "idle"):
                            backend.idle(lane)
                        with wake:
                            wake.notify_all()
        except Exception as e:  # surface errors from worker threads
            errors.append(e)
            stop.set()

    n_total = len(pending)
    t_report = 0.0
    while len(sched.done) < n_total and not stop.is_set():
        if progress is not None and now() - t_report >= progress_every:
            t_report = now()
            progress(len(sched.done), n_total, t_report, sched.used)
        while pending and pending[0].t_arrival <= now():
            sched.arrive(pending.popleft())
        for r in sched.admit(now()):
            if r.lane not in workers:
                th = threading.Thread(target=lane_worker, args=(r.lane,), daemon=True)
                workers[r.lane] = th
                th.start()
        with wake:
            wake.wait(timeout=0.001)
    stop.set()
    for th in workers.values():
        th.join()
    for h in handles.values():
        backend.end(h)
    if errors:
        raise errors[0]
    return sched, solutions, now()


def serve_fifo(trace, backend: GPUBackend, keep_solutions=False, progress=None):
    """The plain baseline: requests in arrival order, one right-hand side at a
    time, each a complete single-RHS solve in the backend's inner precision
    (FP64 for the baseline) on one context -- no batching, no overlap.  A
    request that arrives while the GPU is busy waits in the queue."""
    import torch

    M = backend.M
    ctx = backend.ctx_for(("fifo", 0))
    stream = backend.lane_stream(("fifo", 0))
    order = sorted(trace, key=lambda r: r.t_arrival)
    solutions = {}
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    done = []
    t_report = 0.0
    for r in order:
        if progress is not None and now() - t_report >= 10.0:
            t_report = now()
            progress(len(done), len(order), t_report)
        while now() < r.t_arrival:
            time.sleep(min(0.001, r.t_arrival - now()))
        r.t_admit = now()
        a = backend.act(r)
        with torch.cuda.stream(stream):
            eta = torch.zeros(a.spinor_shape(), dtype=torch.complex128, device=f"cuda:{backend.device}")
            psi = torch.zeros_like(eta)
        stats, sols = [], []
        for k in range(r.nsrc):
            ctx.source_z2(a, r.seed, r.src_offset + k, eta)
            stats.extend(ctx.solve(backend.gauge[tuple(r.volume)], a, backend.opts(), eta, psi, raise_on_fail=False))
            if keep_solutions:
                stream.synchronize()
                with torch.cuda.stream(stream):
                    sols.append(psi.cpu().numpy())
        stream.synchronize()
        r.t_done = now()
        r.stats = stats
        done.append(r)
        if keep_solutions:
            solutions[r.id] = sols
    return done, solutions, now()
