"""Serving dispatcher logic on the CPU, with a fake executor standing in for
the GPU: admission order, the memory budget, overlap of admitted jobs,
continuous admission of late arrivals, error propagation, latency summary."""
import threading
import time

import numpy as np
import pytest

from paper_2309_14584_amd.serve import Engine, Job, latency_summary


class FakeExecutor:
    """Each job 'runs' for job.problem['t'] seconds and needs
    job.problem['bytes'] bytes; records the overlap it saw."""

    def __init__(self, fail=()):
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.fail = set(fail)
        self.started = {}

    def footprint(self, job):
        return job.problem["bytes"]

    def run(self, job, slot):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.started[job.id] = time.perf_counter()
        try:
            time.sleep(job.problem["t"])
            if job.id in self.fail:
                raise ValueError("planted failure")
            return np.full(3, float(job.id)), job.id + 1, True
        finally:
            with self.lock:
                self.active -= 1


def _jobs(arrivals, t=0.02, nbytes=1):
    return [Job(i, {"t": t, "bytes": nbytes}, a) for i, a in enumerate(arrivals)]


def test_results_and_fifo_with_one_slot():
    jobs = _jobs([0.0, 0.001, 0.002, 0.003], t=0.01)
    eng = Engine(FakeExecutor(), slots=1)
    res = eng.run(jobs)
    assert [r.id for r in res] == [0, 1, 2, 3]
    for r in res:
        assert np.array_equal(r.c, np.full(3, float(r.id)))
        assert r.iterations == r.id + 1 and r.converged
        assert r.admitted >= r.arrival and r.done >= r.admitted
    # one slot: every job starts after the previous one finished
    for a, b in zip(res, res[1:]):
        assert b.admitted >= a.done - 1e-3


def test_slots_overlap_jobs():
    ex = FakeExecutor()
    jobs = _jobs([0.0] * 8, t=0.05)
    t0 = time.perf_counter()
    res = Engine(ex, slots=4).run(jobs)
    wall = time.perf_counter() - t0
    assert len(res) == 8 and ex.max_active == 4
    assert wall < 8 * 0.05 * 0.75          # well under the serial time
    assert len({r.slot for r in res}) == 4


def test_memory_budget_limits_concurrency():
    ex = FakeExecutor()
    jobs = _jobs([0.0] * 6, t=0.03, nbytes=40)
    eng = Engine(ex, slots=4, budget_bytes=100)
    res = eng.run(jobs)
    assert len(res) == 6
    assert ex.max_active == 2 and eng.stats.max_bytes <= 100
    assert eng.stats.waits_for_memory > 0


def test_job_larger_than_budget_is_refused():
    jobs = _jobs([0.0], nbytes=200)
    with pytest.raises(MemoryError):
        Engine(FakeExecutor(), slots=2, budget_bytes=100).run(jobs)


def test_late_arrival_admitted_while_others_run():
    ex = FakeExecutor()
    jobs = [Job(0, {"t": 0.2, "bytes": 1}, 0.0), Job(1, {"t": 0.01, "bytes": 1}, 0.05)]
    res = {r.id: r for r in Engine(ex, slots=2).run(jobs)}
    # continuous batching: the short late job finishes before the long one
    assert res[1].done < res[0].done
    assert res[1].admitted < res[0].done
    assert res[1].admitted >= 0.05


def test_fifo_head_blocks_under_memory_pressure():
    """A big job at the head of the queue is not overtaken by small ones
    (no starvation of large jobs)."""
    ex = FakeExecutor()
    jobs = [Job(0, {"t": 0.05, "bytes": 60}, 0.0),
            Job(1, {"t": 0.01, "bytes": 60}, 0.001),
            Job(2, {"t": 0.01, "bytes": 10}, 0.002)]
    res = {r.id: r for r in Engine(ex, slots=3, budget_bytes=100).run(jobs)}
    assert res[2].admitted >= res[1].admitted


def test_failed_job_frees_its_slot_and_others_run_on():
    ex = FakeExecutor(fail={2})
    eng = Engine(ex, slots=1, budget_bytes=10)
    res = {r.id: r for r in eng.run(_jobs([0.0, 0.0, 0.0, 0.01, 0.02], t=0.01, nbytes=10))}
    assert sorted(res) == [0, 1, 2, 3, 4]
    assert res[2].c is None and "planted failure" in res[2].error
    for j in (0, 1, 3, 4):                 # unchanged by the failure
        assert res[j].error is None and np.array_equal(res[j].c, np.full(3, float(j)))
    assert eng.stats.failed == 1 and eng.stats.max_bytes <= 10


def test_fail_fast_raises():
    ex = FakeExecutor(fail={2})
    with pytest.raises(RuntimeError, match="job 2"):
        Engine(ex, slots=2).run(_jobs([0.0, 0.0, 0.0, 0.01], t=0.01), fail_fast=True)


class OracleExecutor:
    """The same executor interface, backed by the oracle (small jobs)."""

    def footprint(self, job):
        return 1

    def run(self, job, slot):
        import oracle as O
        p = job.problem
        c, _, _ = O.fct_solve(p.support, p.grids, O.sample_problem(p), "qr")
        return c, 0, True


def test_oracle_executor_mix_matches_alone():
    import oracle as O
    import workloads as W
    probs = [W.config1(), W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_PLANTED),
             W.small_problem(5, 3, 5, 2, 7, 3, W.FAMILY_EXPCOS)]
    alone = [OracleExecutor().run(Job(i, p, 0.0), 0)[0] for i, p in enumerate(probs)]
    jobs = [Job(i, probs[i % 3], 0.001 * i) for i in range(9)]
    res = Engine(OracleExecutor(), slots=3).run(jobs)
    assert len(res) == 9
    for r in res:
        assert np.array_equal(r.c, alone[r.id % 3])
    assert O.max_rel_err(alone[0], probs[0].coeffs) < 1e-12


def test_cancel_drops_waiting_jobs():
    jobs = _jobs([0.0, 0.0, 0.0], t=0.01)
    res = Engine(FakeExecutor(), slots=1).run(jobs, cancel={1})
    assert sorted(r.id for r in res) == [0, 2]


def test_latency_summary():
    jobs = _jobs([0.0, 0.01, 0.02, 0.03], t=0.01)
    res = Engine(FakeExecutor(), slots=2).run(jobs)
    s = latency_summary(res)
    lat = sorted(r.latency for r in res)
    assert s["jobs"] == 4
    assert s["p50_ms"] == pytest.approx(1e3 * np.percentile(lat, 50))
    assert s["p99_ms"] >= s["p50_ms"] >= 10.0 * 0.9
    assert latency_summary(res, skip_before=1.0)["jobs"] == 0


def test_poisson_arrivals_shape():
    import workloads as W
    t = W.poisson_arrivals(3, 200.0, 2.0)
    assert np.all(np.diff(t) > 0) and t[0] >= 0 and t[-1] < 2.0
    assert 300 < len(t) < 500              # 400 expected
    assert np.array_equal(t, W.poisson_arrivals(3, 200.0, 2.0))
