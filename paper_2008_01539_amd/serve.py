"""Serving loop: timestep-solve requests from many reservoir models, batched
continuously on one GPU.

Each request asks to advance one session (a resident model) by its next
scheduled timestep.  A scheduler tick runs one Newton iteration of every
in-flight request (iteration-level continuous batching): requests that
arrive while others are on the GPU join at the next tick as soon as a slot
and device memory are free, finished requests leave, and members of a tick
with the same block size share one batched Krylov solve.  Sessions stay
resident in HBM between requests; admission checks the device footprint
against a budget and evicts idle sessions (their state goes to host memory
and comes back on re-admission).

The executor is pluggable: ``GpuExecutor`` drives the library;
``FakeExecutor`` is a deterministic CPU stand-in used to test admission,
batching and latency bookkeeping without a GPU.
"""
from __future__ import annotations

import heapq
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    session: int
    arrival: float
    dt: float = 0.0
    step_index: int = 0
    start: float | None = None
    finish: float | None = None
    iterations: int = 0
    status: str = "queued"       # queued / running / done / failed


@dataclass
class SessionSpec:
    """A model a client can advance: its description, solver options and
    timestep schedule (the request for step k uses schedule[k % len])."""
    name: str
    model: object
    options: object
    schedule: np.ndarray
    mode: int = 1                 # FIM_LOCAL


@dataclass
class Session:
    spec: SessionSpec
    footprint: int
    handle: object = None         # executor handle when resident
    saved: object = None          # host copy of the state when evicted
    next_step: int = 0
    busy: bool = False
    last_used: float = 0.0


class FakeExecutor:
    """Deterministic stand-in: every Newton iteration of a tick costs
    `iter_cost` seconds of virtual time plus `per_member` per member, and a
    step converges after `iters_per_step(session, step)` iterations."""

    def __init__(self, iter_cost=1e-3, per_member=1e-4, iters_per_step=lambda s, k: 3):
        self.iter_cost = iter_cost
        self.per_member = per_member
        self.iters_per_step = iters_per_step
        self.clock = 0.0
        self.live = {}
        self.ticks = []

    def now(self):
        return self.clock

    def admit(self, session, saved):
        h = object()
        self.live[id(h)] = saved
        return h

    def evict(self, session):
        self.live.pop(id(session.handle), None)
        return ("state", session.next_step)

    def tick(self, members):
        """members: list of (session, request).  Returns per member
        (converged, failed)."""
        self.ticks.append(len(members))
        self.clock += self.iter_cost + self.per_member * len(members)
        out = []
        for s, r in members:
            r.iterations += 1
            need = self.iters_per_step(s.spec.name, r.step_index)
            out.append((r.iterations >= need, False, 0))
        return out

    def result(self, session):
        return None


class GpuExecutor:
    """Drives libfim: one FimModel per resident session, one FimBatch per
    block size, rebuilt when the membership of a tick changes."""

    def __init__(self, stream=None):
        import paper_2008_01539_amd as P
        self.P = P
        self.stream = stream
        self._batches = {}

    def now(self):
        return time.perf_counter()

    def admit(self, session, saved):
        P = self.P
        fm = P.FimModel(session.spec.model, session.spec.options, stream=self.stream)
        if saved is None:
            fm.set_state(session.spec.model.u0, session.spec.model.status0)
        else:
            fm.set_state(saved[0], saved[1])
        return fm

    def evict(self, session):
        fm = session.handle
        u, st = fm.get_state()
        # a batch that holds the model must not outlive it
        for key in [k for k, b in self._batches.items() if any(m is fm for m in b.models)]:
            self._batches.pop(key).close()
        fm.close()
        return (u, st)

    def tick(self, members):
        groups = {}
        for pos, (s, r) in enumerate(members):
            groups.setdefault(s.handle.b, []).append(pos)
        out = [None] * len(members)
        for b, poss in groups.items():
            models = [members[p][0].handle for p in poss]
            key = b
            bat = self._batches.get(key)
            if bat is None:
                bat = self.P.FimBatch(models, stream=self.stream)
                self._batches[key] = bat
            elif len(bat.models) != len(models) or any(a is not b for a, b in zip(bat.models, models)):
                bat.set_models(models)
            dts = [members[p][1].dt for p in poss]
            modes = [members[p][0].spec.mode for p in poss]
            stats, codes = bat.newton_step(dts, modes)
            for p, st, c in zip(poss, stats, codes):
                members[p][1].iterations += 1
                out[p] = (bool(st["converged"]), int(c) != 0, int(st["n_active"]))
        return out

    def result(self, session):
        return session.handle.get_state()

    def close(self):
        for b in self._batches.values():
            b.close()
        self._batches.clear()


@dataclass
class ServeStats:
    completed: int = 0
    failed: int = 0
    ticks: int = 0
    evictions: int = 0
    admissions: int = 0
    latencies: list = field(default_factory=list)
    by_family: dict = field(default_factory=dict)   # family -> latencies
    cell_updates: float = 0.0
    wall: float = 0.0
    max_batch: int = 0

    def summary(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        fam = {f: dict(n=len(v), p50_ms=float(np.percentile(v, 50) * 1e3),
                       p99_ms=float(np.percentile(v, 99) * 1e3))
               for f, v in sorted(self.by_family.items())}
        return dict(completed=self.completed, failed=self.failed, ticks=self.ticks,
                    evictions=self.evictions, admissions=self.admissions,
                    throughput_rps=self.completed / self.wall if self.wall else 0.0,
                    cell_updates_per_s=self.cell_updates / self.wall if self.wall else 0.0,
                    p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3), wall_s=self.wall,
                    max_batch=self.max_batch, by_family=fam)


class Server:
    """Continuous-batching scheduler.

    budget_bytes: device memory the resident sessions may use;
    max_inflight: requests that may be on the GPU in one tick."""

    def __init__(self, specs, executor, budget_bytes, max_inflight=64, footprint=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        fp = footprint or (lambda spec: 0)
        self.sessions = [Session(spec=s, footprint=int(fp(s))) for s in specs]
        self.resident = OrderedDict()     # session index -> None (LRU order)
        self.used = 0
        self.queue = deque()
        self.inflight = []                # (session index, request)
        self.stats = ServeStats()
        self.done = []

    # ------------------------------------------------------------ memory
    def _fits(self, need):
        return self.used + need <= self.budget

    def _make_room(self, need):
        """Evict idle resident sessions (least recently used first)."""
        for idx in list(self.resident.keys()):
            if self._fits(need):
                return True
            s = self.sessions[idx]
            if s.busy:
                continue
            s.saved = self.ex.evict(s)
            s.handle = None
            del self.resident[idx]
            self.used -= s.footprint
            self.stats.evictions += 1
        return self._fits(need)

    def _admit(self, idx):
        s = self.sessions[idx]
        if s.handle is not None:
            self.resident.move_to_end(idx)
            return True
        if s.footprint > self.budget:
            raise ValueError(f"session {s.spec.name} needs {s.footprint} B, budget {self.budget} B")
        if not self._make_room(s.footprint):
            return False
        s.handle = self.ex.admit(s, s.saved)
        s.saved = None
        self.resident[idx] = None
        self.used += s.footprint
        self.stats.admissions += 1
        return True

    def warm(self, order=None):
        """Admit sessions (in `order`, default all) while they fit the
        budget without evicting; returns how many are resident."""
        for idx in (range(len(self.sessions)) if order is None else order):
            s = self.sessions[idx]
            if s.handle is None and self._fits(s.footprint):
                self._admit(idx)
        return len(self.resident)

    # ----------------------------------------------------------- requests
    def submit(self, req: Request):
        self.queue.append(req)

    def _fill(self):
        """Move queued requests onto the GPU while slots and memory allow;
        a session runs at most one request at a time (FIFO per session)."""
        kept = deque()
        while self.queue:
            r = self.queue.popleft()
            s = self.sessions[r.session]
            if len(self.inflight) >= self.max_inflight or s.busy or not self._admit(r.session):
                kept.append(r)
                continue
            s.busy = True
            r.step_index = s.next_step
            sched = s.spec.schedule
            r.dt = float(sched[s.next_step % len(sched)])
            r.start = self.ex.now()
            r.status = "running"
            self.inflight.append((r.session, r))
        self.queue = kept

    def tick(self):
        self._fill()
        if not self.inflight:
            return False
        members = [(self.sessions[i], r) for i, r in self.inflight]
        res = self.ex.tick(members)
        self.stats.ticks += 1
        self.stats.max_batch = max(self.stats.max_batch, len(members))
        now = self.ex.now()
        still = []
        for (i, r), (conv, failed, n_act) in zip(self.inflight, res):
            s = self.sessions[i]
            s.last_used = now
            self.stats.cell_updates += n_act
            if conv or failed:
                r.finish = now
                r.status = "failed" if failed else "done"
                s.busy = False
                if conv:
                    s.next_step += 1
                    self.stats.completed += 1
                    self.stats.latencies.append(r.finish - r.arrival)
                    fam = s.spec.name.split("-")[0]
                    self.stats.by_family.setdefault(fam, []).append(r.finish - r.arrival)
                else:
                    self.stats.failed += 1
                self.done.append(r)
            else:
                still.append((i, r))
        self.inflight = still
        return True

    def run_poisson(self, rate, duration, mix, seed=5, max_ticks=10 ** 7, progress=None,
                    every=10.0):
        """Poisson arrivals at `rate`/s for `duration` s of the executor's
        clock; `mix[k]` is the probability that a request targets session
        k.  `progress(elapsed, stats)` is called about every `every`
        seconds.  Returns the statistics."""
        rng = np.random.default_rng(seed)
        t0 = self.ex.now()
        t = 0.0
        arrivals = []
        while True:
            t += rng.exponential(1.0 / rate)
            if t > duration:
                break
            arrivals.append((t, int(rng.choice(len(self.sessions), p=mix))))
        heapq.heapify(arrivals)
        rid = 0
        ticks = 0
        next_report = every
        while (arrivals or self.queue or self.inflight) and ticks < max_ticks:
            now = self.ex.now() - t0
            if progress is not None and now >= next_report:
                progress(now, self.stats)
                next_report += every
            while arrivals and arrivals[0][0] <= now:
                ta, sidx = heapq.heappop(arrivals)
                self.submit(Request(rid=rid, session=sidx, arrival=t0 + ta))
                rid += 1
            if not self.tick():
                # idle: jump the executor clock (fake) or wait (real)
                if arrivals:
                    if isinstance(self.ex, FakeExecutor):
                        self.ex.clock = t0 + arrivals[0][0]
                    else:
                        time.sleep(max(0.0, arrivals[0][0] - (self.ex.now() - t0)))
            ticks += 1
        self.stats.wall = self.ex.now() - t0
        return self.stats.summary()
