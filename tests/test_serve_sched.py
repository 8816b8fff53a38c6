"""Serving-loop logic on the CPU: a fake engine (footprint accounting, a fixed
number of passes per job, a launch that advances a fake clock) drives the real
Server and Scheduler.  Checks the admission rules, the bookkeeping of
latencies and failures, and that no request starves."""
import math

import pytest

from paper_2409_14697_amd.serve import Job, Scheduler, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


class FakeEngine:
    """Each launch takes `launch_s`; a finished job's result is seen one launch
    later (as if copied back asynchronously)."""
    elem_bytes = 8

    def __init__(self, clock, sched_ref, launch_s=1.0, fail_prepare=(), fail_start=()):
        self.clock = clock
        self.sched_ref = sched_ref
        self.launch_s = launch_s
        self.fail_prepare = set(fail_prepare)
        self.fail_start = set(fail_start)
        self.launch = 0
        self.log = []          # (launch number, sorted rids) per launch
        self.admitted = []     # rids in admission order
        self.used_seen = []

    def prepare(self, job):
        if job.rid in self.fail_prepare:
            raise RuntimeError("bad circuit")
        job.footprint = job.gates["bytes"]
        job.n_passes = job.gates["passes"]
        return job

    def start(self, job):
        if job.rid in self.fail_start:
            raise RuntimeError("device error")
        self.admitted.append(job.rid)
        s = self.sched_ref[0]
        self.used_seen.append((s.used, s.active))
        job.handle = {}

    def step(self, active):
        self.launch += 1
        self.clock.t += self.launch_s
        self.log.append((self.launch, sorted(j.rid for j in active)))

    def finish(self, job):
        job.handle["seen_at"] = self.launch + 1

    def poll(self, job):
        return self.launch >= job.handle["seen_at"]

    def wait_any(self, jobs):
        self.launch += 1
        self.clock.t += self.launch_s

    def release(self, job):
        job.handle = None


def make(rid, arrival, nbytes, passes, n=10):
    return Job(rid=rid, n=n, arrival=arrival, gates={"bytes": nbytes, "passes": passes})


def serve(jobs, budget, max_active=64, max_bypass=8, **kw):
    clock = FakeClock()
    ref = [None]
    eng = FakeEngine(clock, ref, **kw)
    srv = Server(eng, budget, max_active=max_active, max_bypass=max_bypass, plan_workers=0, clock=clock)
    ref[0] = srv.sched
    res = srv.run(jobs)
    return res, eng


def test_scheduler_unit_rules():
    s = Scheduler(100, 2, max_bypass=1)
    a, b, c, d = make(0, 0, 60, 1), make(1, 0, 50, 1), make(2, 0, 30, 1), make(3, 0, 101, 1)
    for j in (a, b, c, d):
        j.footprint = j.gates["bytes"]
    assert not s.offer(d) and d.status == "rejected" and "exceeds" in d.error
    for j in (a, b, c):
        assert s.offer(j)
    got = s.admit()
    assert [j.rid for j in got] == [0, 2]          # b does not fit; c passes it
    assert b.bypassed == 1 and s.used == 90 and s.active == 2
    s.release(a)
    assert [j.rid for j in s.admit()] == [1]
    with pytest.raises(ValueError):
        Scheduler(0, 1)


def test_admission_never_exceeds_budget_or_slots():
    jobs = [make(i, 0.5 * i, 10 + 27 * (i % 7), 1 + i % 5) for i in range(60)]  # at most 172 B each
    res, eng = serve(jobs, budget=200, max_active=4)
    assert all(j.status == "done" for j in jobs)
    assert res.peak_used <= 200 and res.peak_active <= 4
    for used, active in eng.used_seen:
        assert used <= 200 and active <= 4


def test_fifo_order_when_everything_fits():
    jobs = [make(i, 0.0, 10, 3) for i in range(20)]
    res, eng = serve(jobs, budget=10_000)
    assert eng.admitted == list(range(20))
    # all admitted at once: one launch per pass, run together
    assert res.launches == 3 and eng.log[0][1] == list(range(20))


def test_fifo_with_fit_lets_small_jobs_pass():
    # job 0 holds 80 of 100 bytes for 5 launches; job 1 (50) waits; 2 and 3 (10 each) pass it
    jobs = [make(0, 0.0, 80, 5), make(1, 0.1, 50, 1), make(2, 0.2, 10, 1), make(3, 0.3, 10, 1)]
    res, eng = serve(jobs, budget=100)
    assert eng.admitted.index(2) < eng.admitted.index(1)
    assert eng.admitted.index(3) < eng.admitted.index(1)
    assert all(j.status == "done" for j in jobs)


def test_oversized_request_is_rejected_cleanly():
    jobs = [make(0, 0.0, 10, 2), make(1, 0.0, 10_000, 2), make(2, 0.0, 10, 2)]
    res, eng = serve(jobs, budget=100)
    assert jobs[1].status == "rejected" and "exceeds" in jobs[1].error
    assert jobs[0].status == jobs[2].status == "done"
    s = res.summary()
    assert s["rejected"] == 1 and s["completed"] == 2


def test_failures_are_retired_alone():
    jobs = [make(i, 0.0, 10, 2) for i in range(5)]
    res, eng = serve(jobs, budget=100, fail_prepare={1}, fail_start={3})
    assert jobs[1].status == "error" and "planning" in jobs[1].error
    assert jobs[3].status == "error" and "start" in jobs[3].error
    assert all(jobs[i].status == "done" for i in (0, 2, 4))
    assert res.summary()["errors"] == 2
    # the failed start released its reservation: the budget is whole again at the end
    assert res.peak_used <= 100


def test_latency_bookkeeping_with_fake_clock():
    # one job, 3 passes, each launch 1 s: arrival 2.0, launches end at 3, 4, 5; seen one launch later (6)
    jobs = [make(0, 2.0, 10, 3)]
    res, eng = serve(jobs, budget=100)
    j = jobs[0]
    assert j.t_admit == pytest.approx(2.0)
    assert j.t_done == pytest.approx(6.0)
    assert j.latency == pytest.approx(4.0)
    assert res.makespan == pytest.approx(4.0)
    s = res.summary()
    assert s["p50_ms"] == pytest.approx(4000.0) and s["circuits_per_s"] == pytest.approx(0.25)
    assert res.bytes_moved == pytest.approx(3 * 2 * (1 << 10) * 8)


def test_empty_circuit_completes():
    jobs = [make(0, 0.0, 10, 0), make(1, 0.0, 10, 2)]
    res, eng = serve(jobs, budget=100)
    assert all(j.status == "done" for j in jobs)
    assert all(0 not in rids for _, rids in eng.log)


def test_no_starvation_under_a_stream_of_small_jobs():
    # a large job arrives behind a busy server; small jobs keep arriving and would fit
    jobs = [make(0, 0.0, 60, 4)]
    jobs.append(make(1, 0.05, 80, 1))
    jobs += [make(2 + i, 0.1 + 0.5 * i, 20, 2) for i in range(60)]
    res, eng = serve(jobs, budget=100, max_bypass=3)
    big = jobs[1]
    assert big.status == "done"
    assert big.bypassed <= 3
    # admitted well before the small-job stream ends
    assert eng.admitted.index(1) <= 6
    assert all(j.status == "done" for j in jobs)


def test_jobs_progress_together_continuous_batching():
    # a long job and short jobs arriving later share launches
    jobs = [make(0, 0.0, 10, 10), make(1, 2.5, 10, 2), make(2, 4.5, 10, 1)]
    res, eng = serve(jobs, budget=100)
    together = [rids for _, rids in eng.log if 0 in rids and len(rids) > 1]
    assert together, eng.log
    assert jobs[1].t_done < jobs[0].t_done and jobs[2].t_done < jobs[0].t_done
    assert not math.isnan(jobs[0].t_done)
