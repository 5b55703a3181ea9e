"""Serving loop for FCT jobs with continuous batching on one GPU.

Requests (approximation jobs of any dimension, degree and grid set) arrive
over time.  The dispatcher admits a waiting job as soon as a slot is free
and its device-memory footprint fits the budget; every slot runs its job on
its own HIP stream, so the kernels of all admitted jobs overlap on the
device, and a job that arrives while others are running starts without
waiting for them.  Plans (alias structure, DCT pass tables) stay resident in
a cache keyed by (support, grids) and are reused by later jobs; workspaces
(DCT scratch and CG state) are pooled per plan.  Each job is solved by the
same kernels, on its own data, whether it runs alone or among others, so its
result is bitwise the same.

The scheduler only talks to an executor (``footprint``, ``run``), so its
admission and ordering logic is tested on the CPU with a fake executor.
"""
from __future__ import annotations

import hashlib
import threading
import time
from collections import OrderedDict
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

__all__ = ["Job", "JobResult", "Engine", "GpuExecutor", "latency_summary"]


@dataclass
class Job:
    id: int
    problem: object             # workloads.Problem: support, grids, family, params, coeffs
    arrival: float              # seconds after the start of the run
    dct_mode: int = 0           # fct_dct_mode
    solve_mode: int = 0         # fct_solve_mode


@dataclass
class JobResult:
    id: int
    c: np.ndarray | None         # None when the job failed
    iterations: int
    converged: bool
    arrival: float
    admitted: float
    done: float
    slot: int
    error: str | None = None

    @property
    def latency(self):
        return self.done - self.arrival


@dataclass
class _Stats:
    admitted: int = 0
    max_queue: int = 0
    max_running: int = 0
    max_bytes: int = 0
    waits_for_memory: int = 0
    failed: int = 0


class Engine:
    """Dispatcher: FIFO admission under a slot limit and a device-byte budget.

    ``executor.footprint(job)`` gives the bytes a job holds while it runs (and
    may evict cached state to make room); ``executor.run(job, slot)`` runs it
    to completion on that slot and returns (c, iterations, converged).
    """

    def __init__(self, executor, slots: int = 4, budget_bytes: int = 64 << 30):
        if slots < 1:
            raise ValueError("need at least one slot")
        self.executor = executor
        self.slots = slots
        self.budget = int(budget_bytes)
        self.stats = _Stats()

    def run(self, jobs, clock=time.perf_counter, cancel=None, fail_fast=False):
        """Serve ``jobs`` (arrival times relative to the start); returns the
        results in completion order.  ``cancel`` is an optional set of job
        ids to drop if they have not been admitted yet.  A job whose executor
        call raises frees its slot and memory and is reported with
        ``error`` set; the other jobs run on (``fail_fast`` instead stops
        admitting and raises once the running jobs have finished)."""
        cancel = cancel if cancel is not None else set()
        order = sorted(jobs, key=lambda j: (j.arrival, j.id))
        t0 = clock()
        lock = threading.Condition()
        free_slots = list(range(self.slots))[::-1]
        in_use = [0]
        results = []
        done_events = []
        queue = []
        nxt = 0
        running = 0

        errors = []

        def finished(job, slot, nbytes, t_adm, fut):
            nonlocal running
            err = None
            try:
                c, iters, conv = fut.result()
            except BaseException as exc:        # noqa: BLE001 - reported per job
                c, iters, conv = None, 0, False
                err = f"{type(exc).__name__}: {exc}"
                errors.append((job.id, exc))
            with lock:
                results.append(JobResult(job.id, c, iters, conv, job.arrival, t_adm,
                                         clock() - t0, slot, err))
                free_slots.append(slot)
                in_use[0] -= nbytes
                running -= 1
                done_events.append(job.id)
                lock.notify_all()

        with ThreadPoolExecutor(max_workers=self.slots) as pool:
            while True:
                with lock:
                    now = clock() - t0
                    while nxt < len(order) and order[nxt].arrival <= now:
                        if order[nxt].id not in cancel:
                            queue.append(order[nxt])
                        nxt += 1
                    queue = [j for j in queue if j.id not in cancel]
                    self.stats.max_queue = max(self.stats.max_queue, len(queue))
                    # admit in arrival order while a slot and the memory allow
                    while queue and free_slots:
                        job = queue[0]
                        need = self.executor.footprint(job)
                        if need > self.budget:
                            raise MemoryError(f"job {job.id} needs {need} bytes, budget "
                                              f"{self.budget}")
                        if in_use[0] + need > self.budget:
                            self.stats.waits_for_memory += 1
                            break
                        queue.pop(0)
                        slot = free_slots.pop()
                        in_use[0] += need
                        running += 1
                        self.stats.admitted += 1
                        self.stats.max_running = max(self.stats.max_running, running)
                        self.stats.max_bytes = max(self.stats.max_bytes, in_use[0])
                        t_adm = now
                        fut = pool.submit(self.executor.run, job, slot)
                        fut.add_done_callback(
                            lambda f, job=job, slot=slot, need=need, t_adm=t_adm:
                            finished(job, slot, need, t_adm, f))
                    if (fail_fast and errors) or (nxt >= len(order) and not queue
                                                  and running == 0):
                        break
                    # sleep until the next arrival or a completion
                    wait = None
                    if nxt < len(order):
                        wait = max(0.0, order[nxt].arrival - (clock() - t0))
                    if not done_events:
                        lock.wait(timeout=wait if wait is not None else 0.05)
                    done_events.clear()
        self.stats.failed = len(errors)
        if fail_fast and errors:
            jid, exc = errors[0]
            raise RuntimeError(f"job {jid} failed") from exc
        return results


def latency_summary(results, skip_before: float = 0.0):
    """p50 / p99 latency (ms) of jobs that arrived at or after skip_before."""
    lat = np.array([r.latency for r in results if r.arrival >= skip_before])
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "jobs": 0}
    return {"p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "jobs": int(lat.size)}


def _key(problem):
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(problem.support, dtype=np.int32).tobytes())
    h.update(b"|")
    h.update(np.ascontiguousarray(problem.grids, dtype=np.int32).tobytes())
    return h.hexdigest()


class GpuExecutor:
    """Runs jobs through libfct, one HIP stream per slot.

    Device-resident state: a cache of plans (LRU, evicted only when idle and
    the budget needs the room) and, per plan, a pool of workspaces.  The
    footprint of a job is its plan (when not cached yet), one workspace and
    its sample, right-hand-side and coefficient buffers.
    """

    def __init__(self, fct, torch, device=0, cache_bytes: int = 32 << 30):
        self.fct, self.torch = fct, torch
        self.device = device
        self.cache_bytes = cache_bytes
        self._plans = OrderedDict()      # key -> [plan, bytes, active users]
        self._ws = {}                    # key -> list of free workspace handles
        self._streams = {}
        self._lock = threading.Lock()
        self._cached = 0

    @staticmethod
    def _estimate(problem):
        n, D, K = problem.n, problem.D, problem.K
        P = int(sum(int(np.prod(np.asarray(g, dtype=np.int64) + 1)) for g in problem.grids))
        E = K * n
        plan = 4 * n * D + 44 * E + 64 * K * D + (1 << 20)
        ws = 8 * P + 24 * E + 80 * n + (1 << 20)
        bufs = 8 * P + 8 * E + 8 * n
        return plan, ws + bufs

    def footprint(self, job):
        plan_b, run_b = self._estimate(job.problem)
        with self._lock:
            cached = _key(job.problem) in self._plans
            # make room in the plan cache by dropping idle plans (LRU)
            while not cached and self._cached + plan_b > self.cache_bytes:
                victim = next((k for k, v in self._plans.items() if v[2] == 0), None)
                if victim is None:
                    break
                self._drop(victim)
        return run_b + (0 if cached else plan_b)

    def _drop(self, key):
        plan, nbytes, _ = self._plans.pop(key)
        for w in self._ws.pop(key, []):
            w.close()
        plan.close()
        self._cached -= nbytes

    def _stream(self, slot):
        s = self._streams.get(slot)
        if s is None:
            s = self._streams[slot] = self.torch.cuda.Stream(device=self.device)
        return s

    def _acquire(self, problem, stream):
        key = _key(problem)
        with self._lock:
            ent = self._plans.get(key)
            if ent is not None:
                ent[2] += 1
                self._plans.move_to_end(key)
                pool = self._ws.setdefault(key, [])
                ws = pool.pop() if pool else None
                plan = ent[0]
        if ent is None:
            plan = self.fct.Plan(problem.support, problem.grids, stream=stream)
            with self._lock:
                if key in self._plans:             # another slot built it meanwhile
                    plan.close()
                    ent = self._plans[key]
                    ent[2] += 1
                    plan = ent[0]
                else:
                    self._plans[key] = [plan, plan.info.device_bytes, 1]
                    self._cached += plan.info.device_bytes
                pool = self._ws.setdefault(key, [])
                ws = pool.pop() if pool else None
        if ws is None:
            ws = plan.new_workspace()
        return key, plan, ws

    def _release(self, key, ws):
        with self._lock:
            self._ws.setdefault(key, []).append(ws)
            self._plans[key][2] -= 1

    def run(self, job, slot):
        torch, fct = self.torch, self.fct
        torch.cuda.set_device(self.device)
        stream = self._stream(slot)
        p = job.problem
        with torch.cuda.stream(stream):
            key, plan, ws = self._acquire(p, stream)
            try:
                dev = torch.device("cuda", self.device)
                samples = torch.empty(plan.P, dtype=torch.float64, device=dev)
                coeffs = None
                if p.family == fct.FAMILY_PLANTED:
                    coeffs = torch.as_tensor(p.coeffs, dtype=torch.float64).to(dev, non_blocking=False)
                plan.sample(p.family, p.params, coeffs=coeffs, out=samples, ws=ws)
                b = plan.dct(samples, mode=job.dct_mode, ws=ws)
                c, info = plan.solve(b, mode=job.solve_mode, raise_on_noconv=False, ws=ws)
                host = c.cpu().numpy()
            finally:
                self._release(key, ws)
        return host, info.iterations, info.converged

    def close(self):
        with self._lock:
            for key in list(self._plans):
                self._drop(key)
