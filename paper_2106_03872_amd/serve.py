"""Continuous-batching request loop for many small Kohn-Sham systems.

Each request is an independent system (grid, cell, atoms, orbitals) that must
be propagated by ``nsteps`` Taylor-4 steps (Section "Real-time propagation";
the states of one system, and whole systems, are independent, which is what
makes them batchable).  The loop

* admits waiting requests in arrival order while their device footprint fits
  the HBM budget (admission = system creation, uploads, the launch schedule
  from the library's autotuner (timed once per grid and pass-size bucket,
  then cached), Cholesky orthonormalisation of the orbitals, one step
  captured into a HIP graph);
* keeps every admitted request's orbitals resident in HBM (packed layout)
  and issues its next step as soon as the previous one completed, on a pool
  of streams, so that the steps of many requests overlap on the device;
* retires finished requests (final energy, norms, orbitals on request) and
  frees their memory, which admits more.

Per-step latency is the time between the completions of consecutive steps of
one request (the first step: from admission); time-to-first-step is from
arrival.  The scheduler is written against a small backend interface so that
its admission and ordering logic can be tested on the CPU with a simulated
device (``FakeBackend``).
"""
from __future__ import annotations

import time
from collections import deque
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
    t_admit: float = -1.0
    t_done: float = -1.0
    step_times: list = field(default_factory=list)
    result: dict = field(default_factory=dict)


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

    def run(self, requests):
        be = self.be
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        for r in pending:
            r.footprint = be.footprint(r)
            if r.footprint > self.budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} B, more than the budget {self.budget} B")
        waiting, active, done = deque(), [], []
        used = 0
        be.start()
        while pending or waiting or active:
            progressed = False
            now = be.now()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
                progressed = True
            while waiting and len(active) < self.max_active and used + waiting[0].footprint <= self.budget:
                r = waiting.popleft()
                used += r.footprint
                self.max_used = max(self.max_used, used)
                r.t_admit = be.now()
                r.handle = be.admit(r)
                r.inflight = None
                active.append(r)
                progressed = True
            for r in active:
                if r.inflight is None and len(r.step_times) < r.nsteps:
                    r.inflight = be.issue_step(r.handle)
                    progressed = True
            still = []
            for r in active:
                if r.inflight is not None and be.is_done(r.inflight):
                    r.step_times.append(be.done_time(r.inflight))
                    r.inflight = None
                    progressed = True
                if len(r.step_times) == r.nsteps and r.inflight is None:
                    r.result = be.retire(r.handle, self.keep_orbitals)
                    r.t_done = be.now()
                    r.handle = None
                    used -= r.footprint
                    done.append(r)
                else:
                    still.append(r)
            active = still
            if not progressed:
                be.idle(pending[0].arrival if pending else None)
        self.elapsed = be.now()
        return done

    @staticmethod
    def report(done, elapsed, hpsi_per_step):
        """Latency percentiles and aggregate throughput of a finished run."""
        lat, ttfs = [], []
        total_hpsi = 0
        for r in done:
            prev = r.t_admit
            for t in r.step_times:
                lat.append(t - prev)
                prev = t
            ttfs.append(r.step_times[0] - r.arrival if r.step_times else float("nan"))
            total_hpsi += hpsi_per_step(r) * len(r.step_times)
        return {
            "requests": len(done),
            "steps": len(lat),
            "step_latency_ms_p50": 1e3 * percentile(lat, 50),
            "step_latency_ms_p99": 1e3 * percentile(lat, 99),
            "time_to_first_step_ms_p50": 1e3 * percentile(ttfs, 50),
            "time_to_first_step_ms_p99": 1e3 * percentile(ttfs, 99),
            "makespan_s": elapsed,
            "orbital_hpsi_per_s": total_hpsi / elapsed if elapsed > 0 else float("nan"),
        }


def hpsi_per_step(r):
    return 4 * r.spec.norb


# ------------------------------------------------------------------ backends

class HipBackend:
    """Runs requests on the MI355X through the C ABI (one system + resident
    state per request, steps replayed from a captured graph on a stream pool)."""

    def __init__(self, precision=None, nstreams=4, use_graphs=True, dt=0.05):
        import torch

        from paper_2106_03872_amd import ks
        self.torch = torch
        self.ks = ks
        self.precision = ks.KS_MIXED if precision is None else precision
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.use_graphs = use_graphs
        self.dt = dt
        self._next = 0
        self.inputs = {}

    def prepare(self, requests):
        """Draw every request's inputs on the host (the request payload)."""
        from paper_2106_03872_amd import synth
        for r in requests:
            sysm = synth.system(r.spec)
            sel, vals = synth.orbital_values(r.spec)
            self.inputs[r.rid] = (sysm, sel, vals)

    def footprint(self, r):
        sysm = self.inputs[r.rid][0]
        s = r.spec
        base = self.ks.plan_footprint(s.n, s.L, s.ecut, s.norb, int(sysm.proj.npts.sum()), 4, self.precision)
        npw_stride = len(self.ks.plan_sphere(s.n, s.L, s.ecut)) + 64
        box = s.norb * s.npoints * 16                       # transient box copy at admission
        ortho = 2 * s.norb * npw_stride * 16 + 2 * s.norb * s.norb * 16 + 256
        return base + box + ortho

    def start(self):
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def admit(self, r):
        torch, ks = self.torch, self.ks
        sysm, sel, vals = self.inputs.pop(r.rid)
        stream = self.streams[self._next % len(self.streams)]
        self._next += 1
        with torch.cuda.stream(stream):
            gs = ks.system_from_synth(sysm, precision=self.precision)
            gs.autotune(r.spec.norb)     # launch schedule; cached per grid and pass-size bucket
            c = torch.zeros((r.spec.norb, r.spec.npoints), dtype=torch.complex128, device="cuda")
            c[:, torch.from_numpy(sel).to("cuda")] = torch.from_numpy(vals).to("cuda")
            c = c.reshape((r.spec.norb,) + tuple(r.spec.n))
            gs.orthonormalize(c)
            st = ks.State(gs, r.spec.norb)
            st.upload(c, stream)
            occ = torch.full((r.spec.norb,), float(r.spec.occ), dtype=torch.float64, device="cuda")
            if self.use_graphs:
                st.capture(self.dt, stream=stream)
            del c
        return {"system": gs, "state": st, "stream": stream, "occ": occ}

    def issue_step(self, h):
        with self.torch.cuda.stream(h["stream"]):
            if self.use_graphs:
                h["state"].replay(h["stream"])
            else:
                h["state"].propagate(self.dt, 1, stream=h["stream"])
            ev = self.torch.cuda.Event()
            ev.record(h["stream"])
        return [ev, None]

    def is_done(self, tok):
        if tok[1] is None and tok[0].query():
            tok[1] = self.now()
        return tok[1] is not None

    def done_time(self, tok):
        return tok[1]

    def retire(self, h, keep_orbitals):
        torch = self.torch
        with torch.cuda.stream(h["stream"]):
            norms, energy = h["state"].reduce(h["occ"], stream=h["stream"])
            out = {"norms": norms.cpu().numpy(), "energy": energy.item(),
                   "electrons": float(h["occ"].sum().item())}
            if keep_orbitals:
                out["orbitals"] = h["state"].download(stream=h["stream"]).cpu().numpy()
        h["state"].close()
        h["system"].close()
        return out

    def idle(self, next_arrival):
        time.sleep(20e-6)


class FakeBackend:
    """Simulated device for testing the scheduler on the CPU: a virtual clock,
    per-request step durations from a cost model, and `lanes` steps that can
    run at once (a step waits for the earliest free lane)."""

    def __init__(self, lanes=4, cost_per_hpsi=1e-6, footprint_fn=None):
        self.lanes = lanes
        self.cost = cost_per_hpsi
        self.footprint_fn = footprint_fn or (lambda r: r.spec.norb * r.spec.npoints * 16)
        self.t = 0.0
        self.lane_free = [0.0] * lanes
        self.running = []
        self.admitted = []
        self.retired = []

    def footprint(self, r):
        return self.footprint_fn(r)

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def admit(self, r):
        self.admitted.append(r.rid)
        return {"rid": r.rid, "cost": self.cost * 4 * r.spec.norb * (r.spec.npoints / 1e5)}

    def issue_step(self, h):
        i = min(range(self.lanes), key=lambda k: self.lane_free[k])
        end = max(self.t, self.lane_free[i]) + h["cost"]
        self.lane_free[i] = end
        self.running.append(end)
        return end

    def is_done(self, tok):
        return tok <= self.t

    def done_time(self, tok):
        return tok

    def retire(self, h, keep_orbitals):
        self.retired.append(h["rid"])
        return {"rid": h["rid"]}

    def idle(self, next_arrival):
        cands = [e for e in self.running if e > self.t]
        if next_arrival is not None and next_arrival > self.t:
            cands.append(next_arrival)
        if cands:
            self.t = min(cands)
        self.running = [e for e in self.running if e > self.t]
