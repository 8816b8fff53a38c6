"""Continuous-batching serving loop for many circuit requests on one GPU.

Requests arrive over time (each a gate list of its own size N and depth).  A
request is planned on the host (in-cache tile passes, one plan per request,
built by worker threads: sv_fuse releases the Python lock), admitted when its
device footprint fits a memory budget and a slot is free, and then advanced
by one tile pass per launch together with every other active request: one
sv_batcher_run call per loop iteration runs the next pass of all of them.
Requests with N at or below the tile size have a single pass that holds the
whole circuit, so one workgroup runs the entire circuit from LDS.  A finished
request's marginal probabilities over its lowest min(N, 16) qubits are
reduced on the device and copied to the host; its latency is the host time at
which that copy is seen complete minus its scheduled arrival.

The scheduling policy (class Scheduler) is plain Python and independent of the
device, so it is tested on the CPU with a fake engine and clock:
  * a request whose footprint exceeds the whole budget is rejected at once;
  * admission is first-in-first-out with fit: a waiting request that does not
    fit may be passed by later ones that do, but at most `max_bypass` times,
    after which nothing passes it until it fits (no starvation);
  * the admitted footprint never exceeds the budget, nor the slot count.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

ELEM_BYTES = {"c64": 8, "c128": 16}


@dataclass
class Job:
    """A request inside the server."""
    rid: int
    n: int
    arrival: float                 # scheduled arrival time (s, server clock)
    gates: object = None           # marshalled gate array (client format)
    n_gates: int = 0
    footprint: int = 0             # bytes held on the device while active
    n_passes: int = 0
    next_pass: int = 0
    status: str = "waiting"        # waiting/planning/ready/active/draining/done/rejected/error
    error: str = ""
    bypassed: int = 0
    t_admit: float = math.nan
    t_done: float = math.nan
    probs: Optional[np.ndarray] = None
    handle: object = None          # engine-private resources

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Scheduler:
    """Admission policy: memory budget + slot cap, FIFO with bounded bypass."""

    def __init__(self, budget_bytes: int, max_active: int, max_bypass: int = 8):
        if budget_bytes <= 0 or max_active <= 0:
            raise ValueError("budget and slot count must be positive")
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.max_bypass = int(max_bypass)
        self.used = 0
        self.active = 0
        self.queue: collections.deque = collections.deque()

    def offer(self, job: Job) -> bool:
        """Queue a planned job; False (job rejected) if it can never fit."""
        if job.footprint > self.budget:
            job.status = "rejected"
            job.error = f"footprint {job.footprint} B exceeds the budget of {self.budget} B"
            return False
        job.status = "ready"
        self.queue.append(job)
        return True

    def admit(self) -> List[Job]:
        out = []
        blocked = False  # a starving job holds the line: nothing passes it
        keep = collections.deque()
        while self.queue:
            job = self.queue.popleft()
            fits = self.used + job.footprint <= self.budget and self.active < self.max_active
            if fits and not blocked:
                self.used += job.footprint
                self.active += 1
                job.status = "active"
                out.append(job)
                for w in keep:      # every waiting job ahead of it is passed once more
                    w.bypassed += 1
                    blocked = blocked or w.bypassed >= self.max_bypass
                continue
            keep.append(job)
            if job.bypassed >= self.max_bypass:
                blocked = True
        self.queue = keep
        return out

    def release(self, job: Job) -> None:
        self.used -= job.footprint
        self.active -= 1
        assert self.used >= 0 and self.active >= 0


@dataclass
class ServeResult:
    jobs: List[Job]
    makespan: float
    launches: int
    bytes_moved: float             # sum over passes of read + write of the state
    budget: int
    peak_used: int
    peak_active: int

    def completed(self) -> List[Job]:
        return [j for j in self.jobs if j.status == "done"]

    def summary(self) -> Dict:
        done = self.completed()
        lat = np.array([j.latency for j in done]) if done else np.zeros(1)
        return {
            "requests": len(self.jobs),
            "completed": len(done),
            "rejected": sum(j.status == "rejected" for j in self.jobs),
            "errors": sum(j.status == "error" for j in self.jobs),
            "makespan_s": self.makespan,
            "circuits_per_s": len(done) / self.makespan if self.makespan > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "gbps": self.bytes_moved / self.makespan / 1e9 if self.makespan > 0 else 0.0,
            "launches": self.launches,
            "budget_bytes": self.budget,
            "peak_used_bytes": self.peak_used,
            "peak_active": self.peak_active,
        }


class WallClock:
    """Host time in seconds."""

    def __call__(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float) -> None:
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(min(dt, 0.002))


class Server:
    """The serving loop; `engine` supplies planning and device work, `clock`
    the time (a callable returning seconds, with sleep_until(t))."""

    def __init__(self, engine, budget_bytes: int, max_active: int = 512, max_bypass: int = 8,
                 plan_workers: int = 8, clock=None):
        self.engine = engine
        self.sched = Scheduler(budget_bytes, max_active, max_bypass)
        self.plan_workers = plan_workers
        self.clock = clock if clock is not None else WallClock()

    def run(self, jobs: Sequence[Job]) -> ServeResult:
        eng, sched = self.engine, self.sched
        order = sorted(jobs, key=lambda j: (j.arrival, j.rid))
        pending = collections.deque(order)
        planning: collections.deque = collections.deque()   # (job, future) in arrival order
        active: List[Job] = []
        draining: List[Job] = []
        launches = 0
        moved = 0.0
        peak_used = peak_active = 0
        pool = cf.ThreadPoolExecutor(self.plan_workers) if self.plan_workers > 0 else None
        t0 = self.clock()
        try:
            while pending or planning or sched.queue or active or draining:
                now = self.clock() - t0
                # arrivals go to the planners
                while pending and pending[0].arrival <= now:
                    job = pending.popleft()
                    job.status = "planning"
                    fut = pool.submit(eng.prepare, job) if pool else _done_future(eng.prepare, job)
                    planning.append((job, fut))
                # planned jobs join the admission queue in arrival order
                while planning and planning[0][1].done():
                    job, fut = planning.popleft()
                    err = fut.exception()
                    if err is not None:
                        job.status, job.error = "error", f"planning failed: {err}"
                        job.t_done = self.clock() - t0
                        continue
                    sched.offer(job)
                # admission
                for job in sched.admit():
                    job.t_admit = self.clock() - t0
                    try:
                        eng.start(job)
                    except Exception as e:  # a request that fails to start is retired alone
                        sched.release(job)
                        job.status, job.error = "error", f"start failed: {e}"
                        job.t_done = self.clock() - t0
                        continue
                    job.next_pass = 0
                    if job.n_passes == 0:  # empty circuit: nothing to launch
                        eng.finish(job)
                        job.status = "draining"
                        draining.append(job)
                    else:
                        active.append(job)
                peak_used = max(peak_used, sched.used)
                peak_active = max(peak_active, sched.active)
                # one launch: the next pass of every active request
                if active:
                    eng.step(active)
                    launches += 1
                    for job in active:
                        moved += 2.0 * (1 << job.n) * eng.elem_bytes
                        job.next_pass += 1
                    finished = [j for j in active if j.next_pass >= j.n_passes]
                    if finished:
                        active = [j for j in active if j.next_pass < j.n_passes]
                        for job in finished:
                            eng.finish(job)
                            job.status = "draining"
                            draining.append(job)
                # retire what the device has completed
                if draining:
                    still = []
                    for job in draining:
                        if eng.poll(job):
                            job.t_done = self.clock() - t0
                            job.status = "done"
                            eng.release(job)
                            sched.release(job)
                        else:
                            still.append(job)
                    draining = still
                if not active:
                    if draining:
                        eng.wait_any(draining)
                    elif planning:
                        cf.wait([f for _, f in planning], timeout=0.001, return_when=cf.FIRST_COMPLETED)
                    elif pending and not sched.queue:
                        self.clock.sleep_until(t0 + pending[0].arrival)
        finally:
            if pool:
                pool.shutdown(wait=True)
        ends = [j.t_done for j in order if not math.isnan(j.t_done)]
        makespan = (max(ends) - min(j.arrival for j in order)) if ends else 0.0
        return ServeResult(list(jobs), makespan, launches, moved, sched.budget, peak_used, peak_active)



def _done_future(fn, *args):
    f: cf.Future = cf.Future()
    try:
        f.set_result(fn(*args))
    except Exception as e:  # noqa: BLE001 - delivered through the future
        f.set_exception(e)
    return f


# ----------------------------------------------------------------- device engine
class DeviceEngine:
    """Runs jobs on the GPU through the library: plans (sv_fuse), device-resident
    programs, the batched pass step and the batched marginal reduction.  All
    device work goes to one stream."""

    def __init__(self, dtype: str = "c64", probs_qubits: int = 16, inflight: int = 3, keep_states: bool = False,
                 lds_qubits: int = 0, max_pass_ops: int = 64, time_launches: bool = False,
                 matrix_qubits: int = 24):
        import torch
        from . import binding as B
        if dtype not in ELEM_BYTES:
            raise ValueError(f"dtype {dtype}")
        self.B = B
        self.torch = torch
        self.dtype = dtype
        self.elem_bytes = ELEM_BYTES[dtype]
        self.probs_qubits = probs_qubits
        self.inflight = max(1, inflight)
        self.keep_states = keep_states
        # states larger than one LDS tile run passes of at most max_pass_ops
        # ops (one pass per launch, like every other request); a state that
        # fits one tile (n <= tile qubits) runs its whole circuit as one pass
        # whose tile stays in LDS from the first gate to the last, so it
        # completes in a single launch
        self.opts = {"mode": "pass", "lds_qubits": lds_qubits, "max_pass_ops": max_pass_ops}
        self.tile_qubits = lds_qubits or (13 if dtype == "c64" else 12)
        # states of at least matrix_qubits qubits are planned in mode AUTO:
        # fused dense ops in matrix passes where the cost model prefers them
        # (each such pass is a launch of its own within the batched step; at
        # these sizes one state fills the device by itself)
        self.matrix_qubits = matrix_qubits
        self.stream = torch.cuda.current_stream()
        self.batcher = B.Batcher(self.stream)
        self.launch_events: collections.deque = collections.deque()
        self.time_launches = time_launches
        self.timed: list = []

    # worker thread: host planning only
    def prepare(self, job: Job) -> Job:
        B = self.B
        if job.n <= self.tile_qubits:
            opts = dict(self.opts, max_pass_ops=0)
        elif self.matrix_qubits and job.n >= self.matrix_qubits:
            opts = dict(self.opts, mode="auto")
        else:
            opts = self.opts
        plan = B.Plan.from_array(job.n, self.dtype, job.gates, job.n_gates, opts)
        flops = None
        if self.time_launches:
            flops = plan.pass_flops()
            if opts["mode"] != "pass":
                # count the gates' flops (one-qubit runs merged, as tile passes
                # apply them) spread over the passes, not the products of the
                # fused blocks, so that plan forms compare on one basis
                ref = B.Plan.from_array(job.n, self.dtype, job.gates, job.n_gates,
                                        {"mode": "sweep", "max_fuse_qubits": 1})
                total = sum(ref.pass_flops())
                ref.close()
                flops = [total / len(flops)] * len(flops)
        job.handle = {"plan": plan, "flops": flops}
        job.n_passes = plan.info()[1]
        job.footprint = (1 << job.n) * self.elem_bytes + _round_up(plan.program_bytes(), 512) \
            + (8 << min(job.n, self.probs_qubits))
        return job

    def start(self, job: Job) -> None:
        torch, B = self.torch, self.B
        h = job.handle
        tdt = torch.complex64 if self.dtype == "c64" else torch.complex128
        with torch.cuda.stream(self.stream):  # allocations belong to the serving stream
            h["tensor"] = torch.empty(1 << job.n, dtype=tdt, device="cuda")
        h["state"] = B.StateVector(job.n, self.dtype, tensor=h["tensor"], stream=self.stream, init=True)
        h["program"] = B.Program(h["plan"], stream=self.stream)
        h["plan"].close()
        h["plan"] = None

    def step(self, active: List[Job]) -> None:
        t0 = None
        if self.time_launches:
            t0 = self.torch.cuda.Event(enable_timing=True)
            t0.record(self.stream)
        self.batcher.run([j.handle["state"] for j in active], [j.handle["program"] for j in active],
                         [j.next_pass for j in active])
        ev = self.torch.cuda.Event(enable_timing=self.time_launches)
        ev.record(self.stream)
        if t0 is not None:
            nbytes = sum(2 * (1 << j.n) * self.elem_bytes for j in active)
            flops = sum(j.handle["flops"][j.next_pass] * (1 << j.n) for j in active)
            self.timed.append((t0, ev, nbytes, len(active), flops))
        self.launch_events.append(ev)
        while len(self.launch_events) > self.inflight:
            self.launch_events.popleft().synchronize()

    def launch_stats(self) -> Dict:
        """Batched-pass launches timed with HIP events on the serving stream:
        count, mean duration, algorithmic bytes (read + write of every state in
        the launch) and algorithmic flops (sv_plan_pass_flops x amplitudes)
        per second of launch time."""
        self.torch.cuda.synchronize()
        if not self.timed:
            return {"launches": 0}
        secs = [rec[0].elapsed_time(rec[1]) * 1e-3 for rec in self.timed]
        nbytes = sum(rec[2] for rec in self.timed)
        items = sum(rec[3] for rec in self.timed)
        flops = sum(rec[4] for rec in self.timed)
        return {"launches": len(secs), "mean_launch_us": 1e6 * sum(secs) / len(secs),
                "busy_s": sum(secs), "bytes": nbytes, "GBs": nbytes / sum(secs) / 1e9,
                "flops": flops, "TFLOPs": flops / sum(secs) / 1e12,
                "mean_states_per_launch": items / len(secs)}

    def finish(self, job: Job) -> None:
        torch = self.torch
        h = job.handle
        k = min(job.n, self.probs_qubits)
        with torch.cuda.stream(self.stream):
            dev = torch.empty(1 << k, dtype=torch.float64, device="cuda")
        self.batcher.probs(h["state"], list(range(k - 1, -1, -1)), dev)
        host = torch.empty(1 << k, dtype=torch.float64, pin_memory=True)
        with torch.cuda.stream(self.stream):  # ordered after the reduction
            host.copy_(dev, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        h["probs_dev"], h["probs_host"], h["done"] = dev, host, ev

    def poll(self, job: Job) -> bool:
        if not job.handle["done"].query():
            return False
        job.probs = job.handle["probs_host"].numpy().copy()
        return True

    def wait_any(self, jobs: List[Job]) -> None:
        jobs[0].handle["done"].synchronize()

    def release(self, job: Job) -> None:
        h = job.handle
        h["program"].close()
        h["state"].close()
        if self.keep_states:
            job.handle = {"tensor": h["tensor"]}
        else:
            job.handle = None

    def close(self):
        self.batcher.close()


def _round_up(x: int, a: int) -> int:
    return (x + a - 1) // a * a


def make_jobs(requests, rate: Optional[float], marshal: Callable) -> List[Job]:
    """Jobs from svgen serving requests: arrival = arrival_unit / rate (all at
    t=0 when rate is None: the closed-loop calibration).  Circuits are built
    and marshalled here, before serving starts: they are the clients' input."""
    jobs = []
    for r in requests:
        gates = r.circuit()
        arr = marshal(gates)
        jobs.append(Job(rid=r.rid, n=r.n, arrival=0.0 if rate is None else r.arrival_unit / rate,
                        gates=arr, n_gates=len(gates)))
    return jobs


def _marshal_one(req):
    from .binding import make_gates
    gates = req.circuit()
    arr, keep = make_gates(gates)
    if keep:
        raise ValueError("explicit-matrix gates cannot be marshalled across processes")
    return len(gates), bytes(arr)


def marshal_requests(requests, workers: int = 8) -> List[tuple]:
    """Build and marshal every request's circuit, in `workers` forked
    processes.  Call before the GPU is first used (a forked child must not
    inherit an initialised device).  Returns (n_gates, (array, keepalive))."""
    from .binding import SvGate
    if workers > 1 and len(requests) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            raw = pool.map(_marshal_one, requests, chunksize=8)
    else:
        raw = [_marshal_one(r) for r in requests]
    out = []
    for count, blob in raw:
        arr = (SvGate * max(1, count)).from_buffer_copy(blob)
        out.append((count, (arr, [])))
    return out


def jobs_from_marshalled(requests, marshalled, rate: Optional[float]) -> List[Job]:
    """Jobs with arrival = arrival_unit / rate (all at t=0 for rate None)."""
    return [Job(rid=r.rid, n=r.n, arrival=0.0 if rate is None else r.arrival_unit / rate, gates=g, n_gates=c)
            for r, (c, g) in zip(requests, marshalled)]


def free_budget(fraction: float = 0.8) -> int:
    import torch
    free, _ = torch.cuda.mem_get_info()
    return int(fraction * free)
