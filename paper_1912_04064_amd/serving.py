"""Request loop for parameter-scan runs: continuous batching on one GPU.

Requests (runs of different sizes and step counts) arrive over time.  A
request is admitted as soon as a run slot is free and its device footprint
(``pic_mem_bytes``) fits in what is left of the HBM budget; until then it
waits in FIFO order.  Admitted runs share the GPU: every ``pic_step`` call
advances all active runs together, and each run stops by itself on its last
step (its step budget lives on the device), so a run admitted mid-way never
waits for the others to finish.  A finished run's results are read and its
slot and memory released, which may admit the next waiting request.

Latency of a request = time its results are read - its arrival time.

The backend is the thin interface below; :class:`GpuBackend` drives the HIP
library through the binding, :class:`FakeBackend` is a CPU stand-in (step
time proportional to the particles it advances) used to test the scheduler
without a GPU.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class RunRecord:
    rid: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    steps: int = 0
    particles: int = 0
    bytes: int = 0
    result: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class GpuBackend:
    """Runs admitted into one live context of the HIP library."""

    def __init__(self, max_runs: int, hbm_budget: int, track_ids: bool = False, capture=()):
        from . import binding
        self.B = binding
        # requests whose final fields (E, Bm, J) are kept at finish, e.g. to
        # compare precision forms
        self.capture = set(capture)
        self.captured = {}
        # the library holds the context to hbm_budget device bytes in total
        # (runs, their set-up and read-out scratch, the context's own tables)
        self.ctx = binding.Context([], max_runs=max_runs, hbm_budget=hbm_budget, track_ids=track_ids)
        self.start = time.perf_counter()
        self.admit_s = 0.0      # host time spent admitting runs (upload, binning, patch choice)
        self.admits = 0
        self.peak_bytes = 0     # the library's high-water mark of device bytes

    def clock(self) -> float:
        return time.perf_counter() - self.start

    def wait_until(self, t: float):
        d = t - self.clock()
        if d > 0:
            time.sleep(d)

    def mem_bytes(self, wl) -> int:
        return self.B.mem_bytes(wl)

    def admit(self, wl, steps: int) -> Optional[int]:
        """The new run's id, or None when the library refuses it for memory
        (the context's own tables take a little beyond the runs' footprints):
        the request then waits for a run to finish."""
        t0 = time.perf_counter()
        try:
            run = self.ctx.admit(wl, max_steps=steps)
        except self.B.PicError as e:
            if e.code != self.B.PIC_E_NOMEM:
                raise
            return None
        self.admit_s += time.perf_counter() - t0
        self.admits += 1
        return run

    def step(self, k: int):
        self.ctx.step(k)

    def steps_done(self, run: int) -> int:
        return self.ctx.run_steps(run)

    def finish(self, run: int, rid=None) -> dict:
        d = self.ctx.diag(run)              # synchronises
        self.peak_bytes = max(self.peak_bytes, d["device_bytes_peak"])
        if rid in self.capture:
            B = self.B
            self.captured[rid] = self.ctx.fields(run, B.F_E | B.F_B | B.F_J)
        return {"n_particles": d["n_particles"], "U_E": d["U_E"], "U_B": d["U_B"], "K": d["K"],
                "step": d["step"]}

    def retire(self, run: int):
        self.ctx.retire(run)

    def close(self):
        self.ctx.close()


class FakeBackend:
    """CPU stand-in: a step of all active runs costs (sum of their particles)
    / rate seconds of simulated time; memory is what ``mem_fn`` says."""

    def __init__(self, rate: float, mem_fn: Callable, max_runs: int, launch_s: float = 0.0):
        self.rate = rate
        self.mem_fn = mem_fn
        self.max_runs = max_runs
        self.launch_s = launch_s
        self.t = 0.0
        self.runs: Dict[int, dict] = {}
        self.next_id = 0

    def clock(self) -> float:
        return self.t

    def wait_until(self, t: float):
        self.t = max(self.t, t)

    def mem_bytes(self, wl) -> int:
        return int(self.mem_fn(wl))

    def admit(self, wl, steps: int) -> int:
        if len(self.runs) >= self.max_runs:
            raise RuntimeError("no free slot")
        rid = self.next_id
        self.next_id += 1
        self.runs[rid] = {"n": wl.n_particles, "target": steps, "done": 0}
        return rid

    def step(self, k: int):
        for _ in range(k):
            active = [r for r in self.runs.values() if r["done"] < r["target"]]
            if not active:
                break
            self.t += self.launch_s + sum(r["n"] for r in active) / self.rate
            for r in active:
                r["done"] += 1

    def steps_done(self, run: int) -> int:
        return self.runs[run]["done"]

    def finish(self, run: int, rid=None) -> dict:
        return {"n_particles": self.runs[run]["n"], "step": self.runs[run]["done"]}

    def retire(self, run: int):
        del self.runs[run]

    def close(self):
        pass


class Server:
    """Continuous-batching request loop over a backend."""

    def __init__(self, backend, hbm_budget: int, max_runs: int, steps_per_call: int = 20):
        self.be = backend
        self.budget = hbm_budget
        self.max_runs = max_runs
        self.k = steps_per_call
        self.used = 0
        self.max_active = 0
        self.trace: List[tuple] = []   # (time, event, rid)

    def serve(self, requests, make_workload: Callable) -> List[RunRecord]:
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending: List = []           # arrived, waiting for a slot / memory
        active: Dict[int, tuple] = {}  # backend run id -> (request, record, bytes)
        records: Dict[int, RunRecord] = {}
        i = 0
        while i < len(reqs) or pending or active:
            now = self.be.clock()
            while i < len(reqs) and reqs[i].arrival <= now:
                pending.append(reqs[i])
                records[reqs[i].rid] = RunRecord(reqs[i].rid, reqs[i].arrival)
                i += 1
            # admission, FIFO: a request that does not fit blocks the ones behind it
            while pending and len(active) < self.max_runs:
                req = pending[0]
                wl = make_workload(req)
                need = self.be.mem_bytes(wl)
                if need > self.budget:
                    raise ValueError(f"request {req.rid} needs {need} bytes, more than the whole budget")
                if self.used + need > self.budget:
                    break
                run = self.be.admit(wl, req.steps)
                if run is None:
                    if not active:
                        raise ValueError(f"request {req.rid} does not fit in the budget even alone")
                    break
                pending.pop(0)
                rec = records[req.rid]
                rec.admitted = self.be.clock()
                rec.particles = wl.n_particles
                rec.steps = req.steps
                rec.bytes = need
                self.used += need
                active[run] = (req, rec, need)
                self.trace.append((rec.admitted, "admit", req.rid))
            self.max_active = max(self.max_active, len(active))
            if not active:
                if i < len(reqs):
                    self.be.wait_until(reqs[i].arrival)
                continue
            self.be.step(self.k)
            for run in [r for r, (req, rec, need) in active.items() if self.be.steps_done(r) >= req.steps]:
                req, rec, need = active.pop(run)
                rec.result = self.be.finish(run, req.rid)
                rec.finished = self.be.clock()
                self.be.retire(run)
                self.used -= need
                self.trace.append((rec.finished, "finish", req.rid))
        return [records[k] for k in sorted(records)]


def summarize(records: List[RunRecord], elapsed: Optional[float] = None) -> dict:
    lat = np.array([r.latency for r in records])
    t0 = min(r.arrival for r in records)
    t1 = max(r.finished for r in records)
    span = elapsed if elapsed is not None else (t1 - t0)
    pushes = float(sum(r.particles * r.steps for r in records))
    return {"runs": len(records), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "runs_per_s": len(records) / span,
            "particle_pushes_per_s": pushes / span, "span_s": span}
