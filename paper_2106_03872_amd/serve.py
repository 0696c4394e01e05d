"""Continuous-batching request loop for many small Kohn-Sham systems.

Each request is an independent system (grid, cell, atoms, orbitals) that must
be propagated by ``nsteps`` Taylor-4 steps (Section "Real-time propagation";
the states of one system, and whole systems, are independent, which is what
makes them batchable).  The loop

* admits waiting requests in arrival order while their device footprint fits
  the HBM budget.  Admission (system creation in a device memory pool, table
  and orbital uploads, Cholesky orthonormalisation, one step captured into a
  HIP graph) runs on worker threads, each with its own stream, so it never
  holds up the issue loop; launch schedules are tuned per grid and pass-size bucket
  before the trace starts;
* keeps every admitted request's orbitals resident in HBM (packed layout)
  and issues its next step as soon as the previous one completed, on a pool
  of streams, so that the steps of many requests overlap on the device;
* retires finished requests without blocking: the final norms and energy
  are copied to pinned host memory behind an event, and the system is freed
  (back into the pool, waiting for its own work only) once that event has
  completed, which admits more;
* isolates failures: a request whose admission or step fails is reported
  failed and its memory released; the others carry on.

Per-step latency is the time between the completions of consecutive steps of
one request (the first step: from the end of its admission); time-to-first-
step is from arrival.  The scheduler is written against a small backend
interface so that its admission and ordering logic can be tested on the CPU
with a simulated device (``FakeBackend``).
"""
from __future__ import annotations

import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    spec: object              # synth.Spec
    nsteps: int = 50
    # filled in by the server
    footprint: int = 0
    t_submit: float = -1.0    # admission started
    t_admit: float = -1.0     # admission finished: steps may be issued
    t_done: float = -1.0
    step_times: list = field(default_factory=list)
    result: dict = field(default_factory=dict)
    error: str = ""


class _RWLock:
    """Shared/exclusive lock with writer preference: admission workers hold
    it shared while they make HIP calls; the issue loop holds it exclusively
    while it captures a graph, so that no other thread touches the runtime
    during a capture."""

    def __init__(self):
        self._c = threading.Condition()
        self._readers = 0
        self._writer = False
        self._waiting = 0

    def acquire_read(self):
        with self._c:
            while self._writer or self._waiting:
                self._c.wait()
            self._readers += 1

    def release_read(self):
        with self._c:
            self._readers -= 1
            if self._readers == 0:
                self._c.notify_all()

    def acquire_write(self):
        with self._c:
            self._waiting += 1
            while self._writer or self._readers:
                self._c.wait()
            self._waiting -= 1
            self._writer = True

    def release_write(self):
        with self._c:
            self._writer = False
            self._c.notify_all()


def percentile(x, q):
    return float(np.percentile(np.asarray(x, float), q)) if len(x) else float("nan")


class Server:
    """Request loop.  backend: HipBackend or FakeBackend."""

    def __init__(self, backend, hbm_budget, max_active=64, keep_orbitals=False):
        self.be = backend
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.keep_orbitals = keep_orbitals
        self.max_used = 0
        self.max_resident = 0
        self.failed = []

    def run(self, requests):
        be = self.be
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        for r in pending:
            r.footprint = be.footprint(r)
            if r.footprint > self.budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} B, more than the budget {self.budget} B")
        self.failed = []
        self._used = 0
        done = []
        be.start()
        try:
            self._loop(be, pending, done)
        finally:
            be.finish()          # admission workers joined even when the loop raises
        self.elapsed = be.now()
        self.used_at_end = self._used
        return done

    def _fail(self, r, exc):
        """Request r fails alone: error recorded, resources and reservation released."""
        r.error = f"{type(exc).__name__}: {exc}"
        r.t_done = self.be.now()
        self._used -= r.footprint
        try:
            self.be.discard(getattr(r, "handle", None))
        except Exception:
            pass
        r.handle = None
        self.failed.append(r)

    def _loop(self, be, pending, done):
        waiting, admitting, active, retiring = deque(), [], [], []
        self._hold = False         # admissions paused until the next retire (device memory short)
        self.requeued = 0
        while pending or waiting or admitting or active or retiring:
            progressed = False
            now = be.now()
            requeue = []
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
                progressed = True
            while (waiting and not self._hold and len(active) + len(admitting) < self.max_active
                   and self._used + waiting[0].footprint <= self.budget):
                r = waiting.popleft()
                self._used += r.footprint
                self.max_used = max(self.max_used, self._used)
                r.t_submit = be.now()
                r.handle = None
                r.admit_tok = be.admit_submit(r)
                admitting.append(r)
                progressed = True
            still = []
            for r in admitting:
                try:
                    h = be.admit_poll(r.admit_tok)
                except Exception as exc:
                    r.admit_tries = getattr(r, "admit_tries", 0) + 1
                    others = active or retiring or len(admitting) > 1
                    if be.retryable(exc) and (others or r.admit_tries < 3):   # memory short: retry later
                        self._used -= r.footprint
                        requeue.append(r)
                        self._hold = True
                    else:                     # this request fails alone
                        self._fail(r, exc)
                    progressed = True
                    continue
                if h is None:
                    still.append(r)
                    continue
                r.handle = h
                r.t_admit = be.now()
                r.inflight = None
                active.append(r)
                progressed = True
            admitting = still
            for r in reversed(sorted(requeue, key=lambda q: (q.arrival, q.rid))):
                waiting.appendleft(r)      # back at the head, in arrival order
                self.requeued += 1
            if self._hold and not active and not admitting and not retiring:
                self._hold = False         # nothing left to retire: try again
            self.max_resident = max(self.max_resident, len(active))
            for r in active:
                if r.inflight is None and len(r.step_times) < r.nsteps:
                    try:
                        r.inflight = be.issue_step(r.handle)
                    except Exception as exc:
                        r.inflight = exc
                    progressed = True
            for h, exc in be.flush():             # batched launches of the steps asked for
                for q in active:
                    if q.handle is h:
                        q.inflight = exc
            still = []
            for r in active:
                if isinstance(r.inflight, Exception):
                    self._fail(r, r.inflight)
                    continue
                if r.inflight is not None and be.is_done(r.inflight):
                    r.step_times.append(be.done_time(r.inflight))
                    r.inflight = None
                    progressed = True
                if len(r.step_times) == r.nsteps and r.inflight is None:
                    try:
                        r.retire_tok = be.retire_submit(r.handle, self.keep_orbitals)
                    except Exception as exc:
                        self._fail(r, exc)
                        progressed = True
                        continue
                    retiring.append(r)
                    progressed = True
                else:
                    still.append(r)
            active = still
            still = []
            for r in retiring:
                try:
                    res = be.retire_poll(r.retire_tok)
                except Exception as exc:
                    self._fail(r, exc)
                    progressed = True
                    continue
                if res is None:
                    still.append(r)
                    continue
                r.result = res
                r.t_done = be.now()
                r.handle = None
                self._used -= r.footprint
                self._hold = False
                done.append(r)
                progressed = True
            retiring = still
            if not progressed:
                be.idle(pending[0].arrival if pending else None)

    @staticmethod
    def report(done, elapsed, hpsi_per_step):
        """Latency percentiles and aggregate throughput of a finished run."""
        lat, ttfs, adm = [], [], []
        total_hpsi = 0
        for r in done:
            prev = r.t_admit
            for t in r.step_times:
                lat.append(t - prev)
                prev = t
            ttfs.append(r.step_times[0] - r.arrival if r.step_times else float("nan"))
            adm.append(r.t_admit - r.t_submit)
            total_hpsi += hpsi_per_step(r) * len(r.step_times)
        return {
            "requests": len(done),
            "steps": len(lat),
            "step_latency_ms_p50": 1e3 * percentile(lat, 50),
            "step_latency_ms_p99": 1e3 * percentile(lat, 99),
            "time_to_first_step_ms_p50": 1e3 * percentile(ttfs, 50),
            "time_to_first_step_ms_p99": 1e3 * percentile(ttfs, 99),
            "admission_ms_p50": 1e3 * percentile(adm, 50),
            "admission_ms_p99": 1e3 * percentile(adm, 99),
            "makespan_s": elapsed,
            "orbital_hpsi_per_s": total_hpsi / elapsed if elapsed > 0 else float("nan"),
        }


def hpsi_per_step(r):
    return 4 * r.spec.norb


# ------------------------------------------------------------------ backends

class HipBackend:
    """Runs requests on the MI355X through the C ABI: one pooled system +
    resident state per request, steps replayed from a captured graph on a
    stream pool; admissions on worker threads, each with its own stream."""

    def __init__(self, precision=None, nstreams=4, use_graphs=True, dt=0.05, pool_bytes=None, admit_workers=4,
                 chunk=None):
        import torch

        from paper_2106_03872_amd import ks
        self.torch = torch
        self.ks = ks
        self.precision = ks.KS_MIXED if precision is None else precision
        # non-blocking streams: graphs are captured on them while other
        # threads make blocking (legacy-stream) host transfers
        self.streams = [ks.stream_pool(i).torch for i in range(nstreams)]
        self._next_admit_stream = nstreams + 1
        self._stream_lock = threading.Lock()
        self.admit_workers = int(admit_workers)
        self._tls = threading.local()     # one admission stream per worker thread
        self._rw = _RWLock()
        self._capture_stream = ks.stream_pool(nstreams)
        self.use_graphs = use_graphs
        self.dt = dt
        self._next = 0
        self.inputs = {}
        self.pool_bytes = pool_bytes
        self.pool = None
        self.tuning_s = 0.0
        self._exec = None
        # orbitals per pass of a request's system (None: the library default,
        # one pass): a smaller pass shrinks each system's workspace, so more
        # requests fit the budget, at the cost of more passes per step
        self.chunk = chunk

    def _chunk(self, r):
        return 0 if self.chunk is None else min(int(self.chunk), r.spec.norb)

    def prepare(self, requests, pretune=True):
        """Draw every request's inputs on the host (the request payload) and,
        with pretune, tune the launch schedule of every grid and pass-size
        bucket of the trace before it starts (cached by the library)."""
        from paper_2106_03872_amd import synth
        for r in requests:
            sysm = synth.system(r.spec)
            sel, vals = synth.orbital_values(r.spec)
            self.inputs[r.rid] = (sysm, sel, vals)
        if pretune:
            t0 = time.perf_counter()
            seen = set()
            for r in sorted(requests, key=lambda q: -q.spec.norb):
                key = (tuple(r.spec.n), 1 << max(0, (r.spec.norb - 1).bit_length()), self._chunk(r))
                if key in seen:
                    continue
                seen.add(key)
                gs = self.ks.system_from_synth(self.inputs[r.rid][0], precision=self.precision, chunk=self._chunk(r))
                gs.autotune(r.spec.norb)
                gs.close()
            self.torch.cuda.synchronize()
            self.tuning_s = time.perf_counter() - t0

    def footprint(self, r):
        sysm = self.inputs[r.rid][0]
        s = r.spec
        base = self.ks.plan_footprint(s.n, s.L, s.ecut, s.norb, int(sysm.proj.npts.sum()), 4, self.precision,
                                      self._chunk(r))
        npw_stride = len(self.ks.plan_sphere(s.n, s.L, s.ecut)) + 64
        ortho = 2 * s.norb * npw_stride * 16 + 2 * s.norb * s.norb * 16
        return base + ortho + 64 * 256        # pool alignment of the system's buffers

    def start(self):
        self.torch.cuda.synchronize()
        if self.pool is None and self.pool_bytes:
            self.pool = self.ks.Pool(self.pool_bytes)
        self._exec = ThreadPoolExecutor(max_workers=self.admit_workers)
        self.t0 = time.perf_counter()

    def finish(self):
        if self._exec is not None:
            self._exec.shutdown(wait=True)
            self._exec = None

    def now(self):
        return time.perf_counter() - self.t0

    def _admit(self, r, sysm, sel, vals):
        torch, ks = self.torch, self.ks
        if getattr(self._tls, "stream", None) is None:
            with self._stream_lock:
                idx = self._next_admit_stream
                self._next_admit_stream += 1
            self._tls.stream = ks.stream_pool(idx).torch
        stream = self._tls.stream
        h = {"stream": self.streams[r.rid % len(self.streams)]}
        self._rw.acquire_read()
        try:
            with torch.cuda.stream(stream):
                gs = ks.system_from_synth(sysm, precision=self.precision, pool=self.pool, chunk=self._chunk(r))
                h["system"] = gs
                gs.autotune(r.spec.norb)     # cached: tuned before the trace
                c = torch.zeros((r.spec.norb, r.spec.npoints), dtype=torch.complex128, device="cuda")
                c[:, torch.from_numpy(sel).to("cuda", non_blocking=False)] = torch.from_numpy(vals).to("cuda")
                c = c.reshape((r.spec.norb,) + tuple(r.spec.n))
                gs.orthonormalize(c)
                st = ks.State(gs, r.spec.norb)
                h["state"] = st
                st.upload(c, stream)
                occ = torch.full((r.spec.norb,), float(r.spec.occ), dtype=torch.float64, device="cuda")
                h["occ"] = occ
                h["occ_sum"] = float(r.spec.occ) * r.spec.norb
                # pinned read-back buffers of the retire, allocated here so
                # that the issue loop allocates no host memory
                h["pin_norms"] = torch.empty(r.spec.norb, dtype=torch.float64, pin_memory=True)
                h["pin_energy"] = torch.empty(1, dtype=torch.float64, pin_memory=True)
                ready = torch.cuda.Event()
                ready.record(stream)
                del c
            ready.synchronize()              # the worker waits; the issue loop does not
        except Exception:
            self.discard(h)
            raise
        finally:
            self._rw.release_read()
        return h

    def admit_submit(self, r):
        sysm, sel, vals = self.inputs.pop(r.rid)
        return self._exec.submit(self._admit, r, sysm, sel, vals)

    def admit_poll(self, tok):
        if not tok.done():
            return None
        h = tok.result()                     # raises the admission's error
        if self.use_graphs and "graph" not in h:
            # one step captured into a graph, here in the issue loop while
            # no worker makes HIP calls
            self._rw.acquire_write()
            try:
                h["state"].capture(self.dt, stream=self._capture_stream.torch)
                h["graph"] = True
            except Exception:
                self.discard(h)
                raise
            finally:
                self._rw.release_write()
        return h

    def issue_step(self, h):
        with self.torch.cuda.stream(h["stream"]):
            if self.use_graphs:
                h["state"].replay(h["stream"])
            else:
                h["state"].propagate(self.dt, 1, stream=h["stream"])
            ev = self.torch.cuda.Event()
            ev.record(h["stream"])
        return [ev, None]

    def flush(self):
        """Launch what issue_step deferred; returns [(handle, error)] of
        requests whose launch failed."""
        return []

    def retryable(self, exc):
        """Admission errors that mean "not now": the device pool (or device)
        is short of memory, so the request waits for a retire and tries again."""
        return isinstance(exc, self.ks.KSError) and exc.status == self.ks.KS_ENOMEM

    def is_done(self, tok):
        if tok[1] is None and tok[0] is not None and tok[0].query():
            tok[1] = self.now()
        return tok[1] is not None

    def done_time(self, tok):
        return tok[1]

    def retire_submit(self, h, keep_orbitals):
        torch = self.torch
        with torch.cuda.stream(h["stream"]):
            norms, energy = h["state"].reduce(h["occ"], stream=h["stream"])
            h["pin_norms"].copy_(norms, non_blocking=True)
            h["pin_energy"].copy_(energy, non_blocking=True)
            psi = h["state"].download(stream=h["stream"]) if keep_orbitals else None
            ev = torch.cuda.Event()
            ev.record(h["stream"])
        h["retire"] = (ev, psi, (norms, energy))
        return h

    def retire_poll(self, h):
        ev, psi, _ = h["retire"]
        if not ev.query():
            return None
        res = {"norms": h["pin_norms"].numpy().copy(), "energy": float(h["pin_energy"][0]),
               "electrons": float(h["occ_sum"])}
        if psi is not None:
            res["orbitals"] = psi.cpu().numpy()     # complete: its event has passed
        self.discard(h)
        return res

    def discard(self, h):
        """Free a request's state and system (each waits for its own work)."""
        if not h:
            return
        if h.get("state") is not None:
            h["state"].close()
            h["state"] = None
        if h.get("system") is not None:
            h["system"].close()
            h["system"] = None

    def idle(self, next_arrival):
        time.sleep(20e-6)


class BatchedHipBackend(HipBackend):
    """HipBackend whose steps are ragged-batched: the resident requests of
    one grid (one plane-wave sphere) that want a step are stepped together by
    one launch per kernel (ks_batch), on the grid's stream.  A grid issues its
    next batched step once the previous one has completed, so requests that
    became ready meanwhile join it.  Every request's orbitals go through the
    same arithmetic as alone, so results are bit-identical to HipBackend's."""

    def __init__(self, *args, lockstep=False, **kw):
        kw.setdefault("use_graphs", False)
        super().__init__(*args, **kw)
        # lockstep: every grid's next batched step waits until the steps of
        # all grids in flight have completed (global rounds: every resident
        # request advances once per round, whatever its grid)
        self.lockstep = lockstep
        self._want = {}       # grid -> [(handle, token)]
        self._inflight = {}   # grid -> event of the grid's step in flight
        self._batches = {}    # grid -> (composition, ks.Batch)
        self.batched_steps = 0
        self.batch_sizes = []
        self._grid_slot = {}  # grid -> stream index (round-robin on first sight)
        self._grid_lock = threading.Lock()

    def _grid(self, h):
        return h["grid"]

    def _grid_stream(self, grid):
        with self._grid_lock:
            if grid not in self._grid_slot:
                self._grid_slot[grid] = len(self._grid_slot) % len(self.streams)
            return self.streams[self._grid_slot[grid]]

    def _admit(self, r, sysm, sel, vals):
        h = super()._admit(r, sysm, sel, vals)
        h["grid"] = tuple(r.spec.n)
        h["stream"] = self._grid_stream(h["grid"])   # steps and retire on the grid's stream, in order
        return h

    def issue_step(self, h):
        tok = [None, None]
        self._want.setdefault(h["grid"], []).append((h, tok))
        return tok

    def flush(self):
        torch, ks = self.torch, self.ks
        failed = []
        if self.lockstep:
            if any(not ev.query() for ev in self._inflight.values()):
                return failed
            self._inflight.clear()
        for gi, (grid, items) in enumerate(sorted(self._want.items())):
            ev = self._inflight.get(grid)
            if not items or (ev is not None and not ev.query()):
                continue
            hs = [h for h, _ in items]
            comp = tuple(id(h["state"]) for h in hs)
            cur = self._batches.get(grid)
            stream = self._grid_stream(grid)
            try:
                if cur is None or cur[0] != comp:
                    if cur is not None:
                        cur[1].close()
                    cur = (comp, ks.Batch([h["state"] for h in hs]))
                    self._batches[grid] = cur
                with torch.cuda.stream(stream):
                    cur[1].propagate(self.dt, 1, stream=stream)
                    ev = torch.cuda.Event()
                    ev.record(stream)
            except Exception as exc:            # the grid's requests fail; others carry on
                self._batches.pop(grid, None)
                failed.extend((h, exc) for h in hs)
                self._want[grid] = []
                continue
            self._inflight[grid] = ev
            for _, tok in items:
                tok[0] = ev
            self._want[grid] = []
            self.batched_steps += 1
            self.batch_sizes.append(len(hs))
        return failed

    def discard(self, h):
        if h and h.get("grid") in self._batches:
            comp, b = self._batches[h["grid"]]
            if h.get("state") is not None and id(h["state"]) in comp:
                b.close()
                del self._batches[h["grid"]]
        super().discard(h)

    def finish(self):
        for _, b in self._batches.values():
            b.close()
        self._batches.clear()
        super().finish()


class FakeBackend:
    """Simulated device for testing the scheduler on the CPU: a virtual clock,
    per-request step durations from a cost model, and `lanes` steps that can
    run at once (a step waits for the earliest free lane)."""

    def __init__(self, lanes=4, cost_per_hpsi=1e-6, footprint_fn=None, fail_admit=(), fail_step=(), fail_retire=(),
                 short_once=()):
        self.lanes = lanes
        self.cost = cost_per_hpsi
        self.footprint_fn = footprint_fn or (lambda r: r.spec.norb * r.spec.npoints * 16)
        self.t = 0.0
        self.lane_free = [0.0] * lanes
        self.running = []
        self.admitted = []
        self.retired = []
        self.discarded = []
        self.fail_admit = set(fail_admit)
        self.fail_step = set(fail_step)
        self.fail_retire = set(fail_retire)
        self.short_once = set(short_once)       # admission is short of memory the first time

    def footprint(self, r):
        return self.footprint_fn(r)

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def admit_submit(self, r):
        self.admitted.append(r.rid)
        if r.rid in self.fail_admit:
            return RuntimeError(f"admission of request {r.rid} failed")
        if r.rid in self.short_once:
            self.short_once.discard(r.rid)
            return MemoryError(f"no device memory for request {r.rid} now")
        return {"rid": r.rid, "cost": self.cost * 4 * r.spec.norb * (r.spec.npoints / 1e5)}

    def admit_poll(self, tok):
        if isinstance(tok, Exception):
            raise tok
        return tok

    def finish(self):
        pass

    def discard(self, h):
        if h:
            self.discarded.append(h["rid"])

    def issue_step(self, h):
        if h["rid"] in self.fail_step:
            raise RuntimeError(f"step of request {h['rid']} failed")
        i = min(range(self.lanes), key=lambda k: self.lane_free[k])
        end = max(self.t, self.lane_free[i]) + h["cost"]
        self.lane_free[i] = end
        self.running.append(end)
        return end

    def is_done(self, tok):
        return tok <= self.t

    def done_time(self, tok):
        return tok

    def flush(self):
        return []

    def retryable(self, exc):
        return isinstance(exc, MemoryError)

    def retire_submit(self, h, keep_orbitals):
        return h

    def retire_poll(self, h):
        if h["rid"] in self.fail_retire:
            raise RuntimeError(f"read-back of request {h['rid']} failed")
        self.retired.append(h["rid"])
        return {"rid": h["rid"]}

    def idle(self, next_arrival):
        cands = [e for e in self.running if e > self.t]
        if next_arrival is not None and next_arrival > self.t:
            cands.append(next_arrival)
        if cands:
            self.t = min(cands)
        self.running = [e for e in self.running if e > self.t]
