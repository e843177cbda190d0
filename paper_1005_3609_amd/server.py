"""Continuous-batching server for rectangle jobs.

Jobs (lattice, m, n_max, q points, primes) arrive over time.  Each job keeps
its state vectors, read-out vector and constants resident in HBM between
ticks.  A tick advances every active job by ``rows_per_tick`` rows
(``chromatic_server_step``): step k of every active job runs in one grouped
launch, so jobs of different lattices, widths and instance counts share each
launch.  Between ticks finished jobs
are retired and their memory freed, and queued jobs are admitted in arrival
order while the resident footprint stays within the byte budget (factor
maps are counted once per (lattice, m) in use).  A job that arrives while a
tick runs joins at the next tick.

The scheduler logic is independent of the device: ``Server`` drives a
backend object; ``GpuBackend`` is the native one.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from .api import _u32, check, lattice_id, lib


@dataclass
class Job:
    id: int
    lattice: str
    m: int
    n_max: int
    q_points: list
    primes: list
    arrival: float = 0.0
    # filled by the server
    state: str = "queued"          # queued -> active -> done | failed
    rows_done: int = 0
    t_admit: float = float("nan")
    t_done: float = float("nan")
    error: str = ""
    handle: object = None          # backend-owned resources
    result: np.ndarray | None = None

    @property
    def instances(self) -> int:
        return len(self.q_points) * len(self.primes)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class GpuBackend:
    """Native backend: device buffers from torch, grouped launches on a
    dedicated stream."""

    def __init__(self, device="cuda", tuning=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.tuning = _lib.tuning(tuning)
        self._map_bytes = {}

    def footprint(self, job: Job) -> int:
        t = self.tuning
        n = lib().chromatic_slot_state_bytes(lattice_id(job.lattice), job.m, len(job.q_points), len(job.primes),
                                             C.byref(t) if t else None)
        if n == 0:
            check(-1)
        return int(n) + 4 * job.n_max * job.instances

    def map_bytes(self, lattice, m) -> int:
        key = (lattice, m)
        if key not in self._map_bytes:
            from .api import maps_info
            info = maps_info(lattice, m)
            # entry words + row pointers (one per row of every factor; bounded by the entries' rows)
            self._map_bytes[key] = 4 * info["total_nnz"] + 8 * m * info["max_states"]
        return self._map_bytes[key]

    def prepare(self, lattice, m):
        check(lib().chromatic_prepare(lattice_id(lattice), m))

    def start(self, job: Job):
        torch = self.torch
        nbytes = self.footprint(job) - 4 * job.n_max * job.instances
        with torch.cuda.stream(self.stream):
            state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            out = torch.zeros((job.n_max, len(job.q_points), len(job.primes)), dtype=torch.int32, device=self.device)
        q = _u32(job.q_points)
        p = _u32(job.primes)
        job.handle = dict(state=state, out=out, q=q, p=p)

    def step(self, jobs, rows: int):
        arr = (_lib.Slot * len(jobs))()
        for k, jb in enumerate(jobs):
            h = jb.handle
            s = arr[k]
            s.lattice = lattice_id(jb.lattice)
            s.m = jb.m
            s.n_max = jb.n_max
            s.rows_done = jb.rows_done
            s.nq = len(jb.q_points)
            s.np = len(jb.primes)
            s.q_points = h["q"].ctypes.data_as(C.POINTER(C.c_uint32))
            s.primes = h["p"].ctypes.data_as(C.POINTER(C.c_uint32))
            s.d_state = C.c_void_p(h["state"].data_ptr())
            s.state_bytes = h["state"].numel()
            s.d_out = C.c_void_p(h["out"].data_ptr())
        t = self.tuning
        check(lib().chromatic_server_step(arr, len(jobs), rows, C.byref(t) if t else None,
                                          C.c_void_p(self.stream.cuda_stream)))
        for k, jb in enumerate(jobs):
            jb.rows_done = arr[k].rows_done
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, ev):
        ev.synchronize()
        check(lib().chromatic_device_status(C.c_void_p(self.stream.cuda_stream)))

    def finish(self, job: Job):
        job.result = job.handle["out"].cpu().numpy().view(np.uint32)

    def release(self, job: Job):
        job.handle = None


@dataclass
class Report:
    jobs: list = field(default_factory=list)
    makespan: float = 0.0
    ticks: int = 0
    peak_bytes: int = 0

    def summary(self) -> dict:
        lat = np.array([j.latency for j in self.jobs if j.state == "done"])
        done = len(lat)
        return dict(jobs=len(self.jobs), done=done, failed=sum(j.state == "failed" for j in self.jobs),
                    p50_s=float(np.percentile(lat, 50)) if done else None,
                    p99_s=float(np.percentile(lat, 99)) if done else None,
                    mean_s=float(lat.mean()) if done else None,
                    jobs_per_s=done / self.makespan if self.makespan > 0 else None,
                    makespan_s=self.makespan, ticks=self.ticks, peak_bytes=self.peak_bytes)


class Server:
    """Admission by footprint, one fused launch per tick, FIFO queue."""

    def __init__(self, backend, budget_bytes: int, rows_per_tick: int = 1, clock=time.perf_counter,
                 sleep=time.sleep):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.rows_per_tick = rows_per_tick
        self.clock = clock
        self.sleep = sleep
        self.resident = 0
        self.maps_in_use: dict = {}

    def _cost(self, job: Job) -> int:
        key = (job.lattice, job.m)
        extra = 0 if self.maps_in_use.get(key, 0) > 0 else self.backend.map_bytes(*key)
        return self.backend.footprint(job) + extra

    def _admit(self, job: Job, now: float):
        key = (job.lattice, job.m)
        self.resident += self._cost(job)
        self.maps_in_use[key] = self.maps_in_use.get(key, 0) + 1
        self.backend.start(job)
        job.state = "active"
        job.t_admit = now

    def _retire(self, job: Job, now: float, failed: str = ""):
        key = (job.lattice, job.m)
        self.resident -= self.backend.footprint(job)
        self.maps_in_use[key] -= 1
        if self.maps_in_use[key] == 0:
            self.resident -= self.backend.map_bytes(*key)
        if failed:
            job.state, job.error = "failed", failed
        else:
            self.backend.finish(job)
            job.state = "done"
        job.t_done = now
        self.backend.release(job)

    def run(self, jobs: list[Job]) -> Report:
        """Serves jobs whose ``arrival`` times are seconds from now."""
        pending = sorted(jobs, key=lambda j: (j.arrival, j.id))
        for j in pending:
            if self._cost(j) > self.budget:
                j.state, j.error = "failed", "footprint exceeds the budget"
        queue: list[Job] = []
        rep = Report(jobs=list(jobs))
        t0 = self.clock()
        k = 0
        while True:
            now = self.clock() - t0
            while k < len(pending) and pending[k].arrival <= now:
                if pending[k].state == "queued":
                    queue.append(pending[k])
                k += 1
            # admission, FIFO while the footprint fits
            while queue and self.resident + self._cost(queue[0]) <= self.budget:
                self._admit(queue.pop(0), now)
            rep.peak_bytes = max(rep.peak_bytes, self.resident)
            active = [j for j in pending if j.state == "active"]
            if not active and not queue and k >= len(pending):
                break
            if not active:
                if k < len(pending):
                    self.sleep(max(0.0, min(pending[k].arrival - now, 0.01)))
                continue
            try:
                ev = self.backend.step(active, self.rows_per_tick)
                self.backend.wait(ev)
            except Exception as exc:  # a failed tick fails its jobs only
                now = self.clock() - t0
                for j in active:
                    self._retire(j, now, failed=str(exc))
                continue
            rep.ticks += 1
            now = self.clock() - t0
            for j in active:
                if j.rows_done >= j.n_max:
                    self._retire(j, now)
        rep.makespan = self.clock() - t0
        return rep


def fifo_baseline(backend_run, jobs: list[Job], clock=time.perf_counter, sleep=time.sleep) -> Report:
    """The same arrival stream served one job at a time in arrival order by
    ``backend_run(job)`` (e.g. the plain per-instance path)."""
    rep = Report(jobs=list(jobs))
    t0 = clock()
    for j in sorted(jobs, key=lambda x: (x.arrival, x.id)):
        now = clock() - t0
        if j.arrival > now:
            sleep(j.arrival - now)
        j.t_admit = clock() - t0
        backend_run(j)
        j.t_done = clock() - t0
        j.state = "done"
    rep.makespan = clock() - t0
    return rep
