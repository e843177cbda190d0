"""Scheduler logic of the continuous-batching server on the CPU: a fake
backend advances a simulated clock, so admission, budgets, retirement,
failure isolation and latency accounting are checked without a GPU."""
import numpy as np
import pytest

from paper_1005_3609_amd import workloads as W
from paper_1005_3609_amd.server import Job, Server


class Clock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeBackend:
    """Footprint ~ instances x 2^m; a tick costs time ~ the largest job."""

    def __init__(self, clock, fail_tick=None):
        self.clock = clock
        self.ticks = 0
        self.fail_tick = fail_tick
        self.resident_log = []
        self.server = None
        self.started = []

    def footprint(self, job):
        return job.instances * (2 ** job.m) * 8

    def map_bytes(self, lattice, m):
        return (2 ** m) * 40

    def start(self, job):
        self.started.append(job.id)
        job.handle = object()

    def step(self, jobs, rows):
        self.ticks += 1
        if self.server is not None:
            self.resident_log.append(self.server.resident)
        if self.fail_tick is not None and self.ticks == self.fail_tick:
            raise RuntimeError("simulated device error")
        for j in jobs:
            j.rows_done = min(j.n_max, j.rows_done + rows)
        return max(j.instances * 2 ** j.m for j in jobs) * 1e-9

    def wait(self, dt):
        self.clock.t += dt

    def finish(self, job):
        job.result = np.zeros(1)

    def release(self, job):
        job.handle = None


def _jobs(n, rate=20.0, seed=1):
    return [Job(id=j["id"], lattice=j["lattice"], m=j["m"], n_max=j["n_max"], q_points=j["q_points"],
                primes=j["primes"], arrival=j["arrival"]) for j in W.serving_stream(n, rate, seed)]


def _server(backend, clock, budget, rows=1):
    s = Server(backend, budget, rows_per_tick=rows, clock=clock.now, sleep=clock.sleep)
    backend.server = s
    return s


def test_all_jobs_complete_within_budget():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(60)
    budget = 4 * max(be.footprint(j) + be.map_bytes(j.lattice, j.m) for j in jobs)
    rep = _server(be, clock, budget).run(jobs)
    s = rep.summary()
    assert s["done"] == 60 and s["failed"] == 0
    assert max(be.resident_log) <= budget and rep.peak_bytes <= budget
    for j in jobs:
        assert j.rows_done == j.n_max and j.t_admit >= j.arrival - 1e-12 and j.latency > 0
    assert s["p50_s"] <= s["p99_s"]
    lat = np.array([j.latency for j in jobs])
    assert s["p99_s"] == pytest.approx(np.percentile(lat, 99))


def test_continuous_batching_overlaps_jobs():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(40, rate=200.0)
    budget = 10 ** 12
    rep = _server(be, clock, budget).run(jobs)
    # with room for everyone, ticks are shared: fewer ticks than total rows
    assert rep.ticks < sum(j.n_max for j in jobs)


def test_oversized_job_is_rejected_and_others_run():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(10)
    big = Job(id=99, lattice="square", m=16, n_max=17, q_points=list(range(1, 81)), primes=[7, 11, 13, 17],
              arrival=0.01)
    budget = 2 * max(be.footprint(j) + be.map_bytes(j.lattice, j.m) for j in jobs)
    assert be.footprint(big) > budget
    rep = _server(be, clock, budget).run(jobs + [big])
    assert big.state == "failed" and "budget" in big.error
    assert all(j.state == "done" for j in jobs)
    assert 99 not in be.started


def test_admission_is_fifo():
    clock = Clock()
    be = FakeBackend(clock)
    jobs = _jobs(30)
    budget = max(be.footprint(j) + be.map_bytes(j.lattice, j.m) for j in jobs)   # one at a time
    _server(be, clock, budget).run(jobs)
    order = sorted(jobs, key=lambda j: (j.arrival, j.id))
    assert be.started == [j.id for j in order]
    assert max(be.resident_log) <= budget


def test_failed_tick_fails_only_its_jobs():
    clock = Clock()
    be = FakeBackend(clock, fail_tick=3)
    jobs = _jobs(25)
    budget = 3 * max(be.footprint(j) + be.map_bytes(j.lattice, j.m) for j in jobs)
    _server(be, clock, budget).run(jobs)
    failed = [j for j in jobs if j.state == "failed"]
    assert failed and all("simulated" in j.error for j in failed)
    assert any(j.state == "done" for j in jobs)
    assert all(j.state in ("done", "failed") for j in jobs)


def test_maps_counted_once_per_width():
    clock = Clock()
    be = FakeBackend(clock)
    a = Job(id=0, lattice="square", m=8, n_max=9, q_points=[1, 2], primes=[7], arrival=0.0)
    b = Job(id=1, lattice="square", m=8, n_max=9, q_points=[1, 2], primes=[7], arrival=0.0)
    s = _server(be, clock, 10 ** 9)
    s.run([a, b])
    assert be.resident_log[0] == 2 * be.footprint(a) + be.map_bytes("square", 8)
    assert s.resident == 0 and s.maps_in_use[("square", 8)] == 0


def test_serving_stream_is_seeded():
    a = W.serving_stream(50)
    b = W.serving_stream(50)
    assert a == b
    assert all(6 <= j["m"] <= 16 and j["n_max"] == j["m"] + 1 for j in a)
    assert all(16 <= len(j["q_points"]) <= 80 and 1 <= len(j["primes"]) <= 4 for j in a)
    gaps = np.diff([0.0] + [j["arrival"] for j in a])
    assert 0.02 < gaps.mean() < 0.09          # mean 1/20 s
