"""Serving form on the GPU: jobs of the four serving kinds arrive as a
Poisson stream and run on several HIP streams at once.  Every job must give,
bit for bit, the coefficients it gives when run alone, and be correct
(planted jobs: recovered to 1e-10 max-relative; exp-cos jobs: the oracle's
least-squares solution to 1e-10)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(
    not os.path.exists(os.path.join(os.path.dirname(__file__), "golden", "serving_extra_grids.json")),
    reason="oracle reference data not generated yet")]

torch = pytest.importorskip("torch")


def serving_pool_selected():
    path = os.path.join(os.path.dirname(__file__), "golden", "serving_extra_grids.json")
    with open(path) as fh:
        fx = json.load(fh)
    return W.serving_pool(fx["seed"], extra_grids=fx["extra_grids"])


@pytest.fixture(scope="module")
def executor():
    from paper_2309_14584_amd import fct
    from paper_2309_14584_amd.serve import GpuExecutor
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    ex = GpuExecutor(fct, torch)
    yield ex
    ex.close()


def test_serving_mix_matches_alone(executor):
    from paper_2309_14584_amd.serve import Engine, Job
    pool = serving_pool_selected()
    picks = list(range(12))                     # three jobs of each kind
    alone = {}
    for j in picks:
        c, its, conv = executor.run(Job(j, pool[j], 0.0), slot=0)
        assert conv, f"job {j} ({pool[j].name}) did not converge alone"
        alone[j] = c
    # the same jobs, twice each, arriving at 200/s and served on 4 streams
    arr = W.poisson_arrivals(9, 200.0, 10.0)[: 2 * len(picks)]
    jobs = [Job(i, pool[picks[i % len(picks)]], float(t)) for i, t in enumerate(arr)]
    eng = Engine(executor, slots=4, budget_bytes=64 << 30)
    res = eng.run(jobs)
    assert len(res) == len(jobs)
    assert eng.stats.max_running > 1
    for r in res:
        j = picks[r.id % len(picks)]
        assert r.converged
        assert np.array_equal(r.c, alone[j]), f"job {j} differs from its alone run"
    for j in picks:
        p = pool[j]
        if p.family == W.FAMILY_PLANTED:
            assert O.max_rel_err(alone[j], p.coeffs) < 1e-10, p.name
        else:
            c_ref, _, _ = O.fct_solve(p.support, p.grids, O.sample_problem(p), "normal")
            assert O.max_rel_err(alone[j], c_ref) < 1e-10, p.name


def test_plan_cache_and_workspace_reuse(executor):
    from paper_2309_14584_amd.serve import Job
    pool = serving_pool_selected()
    p = pool[0]
    n0 = len(executor._plans)
    c1, _, _ = executor.run(Job(0, p, 0.0), slot=1)
    c2, _, _ = executor.run(Job(1, p, 0.0), slot=2)
    assert np.array_equal(c1, c2)
    assert len(executor._plans) <= n0 + 1
    assert executor.footprint(Job(2, p, 0.0)) < sum(executor._estimate(p))
