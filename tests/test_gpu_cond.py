"""Condition of A on the GPU (Lanczos on A^T A with full reorthogonalisation)
and Alg. 2's grid-count loop, against the oracle's exact eigenvalues."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fct():
    from paper_2309_14584_amd import fct as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    return mod


def _v0(n, seed=0):
    return torch.as_tensor(np.random.default_rng(seed).standard_normal(n), dtype=torch.float64,
                           device="cuda")


def _exact(plan):
    G = O.gram_matrix(plan)
    ev = np.linalg.eigvalsh(G)
    return ev[0], ev[-1]


SMALL = [W.config1(), W.small_problem(3, 3, 5, 2, 6, 4), W.small_problem(6, 4, 5, 3, 7, 4)]


@pytest.mark.parametrize("prob", SMALL, ids=[p.name for p in SMALL])
def test_condition_matches_exact_eigenvalues(fct, prob):
    """Run to the invariant subspace (at most n steps): the extreme Ritz
    values are the extreme eigenvalues of the integer Gram matrix."""
    plan = fct.Plan(prob.support, prob.grids)
    est = plan.condition(_v0(plan.n), max_steps=plan.n, tol=0.0)
    lmin, lmax = _exact(O.build_plan(prob.support, prob.grids))
    print(prob.name, est, lmin, lmax)
    assert est["full_rank"]
    assert abs(est["lambda_max"] - lmax) <= 1e-9 * lmax
    assert abs(est["lambda_min"] - lmin) <= 1e-9 * lmax
    assert abs(est["kappa"] / np.sqrt(lmax / lmin) - 1.0) < 1e-6
    again = plan.condition(_v0(plan.n), max_steps=plan.n, tol=0.0)
    assert again == est                       # fixed-order sums: reproducible
    plan.close()


def test_rank_deficient_is_detected(fct):
    S = W.total_degree_support(3, 5)
    grids = np.array([[2, 3, 4]], dtype=np.int32)   # 60 points for 56 columns, but aliases collide
    oplan = O.build_plan(S, grids)
    assert not O.rank_check(oplan)[0]
    plan = fct.Plan(S, grids, allow_rank_deficient=True)
    est = plan.condition(_v0(plan.n, 3), max_steps=plan.n, tol=0.0)
    assert not est["full_rank"] and est["kappa"] == float("inf")
    plan.close()


def test_condition_of_the_d6_workload(fct):
    """D=6, 18,564 columns: the tolerance stop reaches the oracle's kappa."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "cfg2_meta.json")) as fh:
        meta = json.load(fh)
    prob = W.config2()
    plan = fct.Plan(prob.support, prob.grids)
    est = plan.condition(_v0(plan.n, 5), max_steps=400, tol=1e-12)
    print("cfg2", est, meta["kappa_A"])
    assert est["full_rank"] and est["steps"] < 400
    assert abs(est["kappa"] / meta["kappa_A"] - 1.0) < 1e-6
    plan.close()


SELECT = [("D3_d5", W.total_degree_support(3, 5), 59, 1, 6),
          ("D4_d6", W.total_degree_support(4, 6), 61, 1, 7),
          ("D2_d16", W.total_degree_support(2, 16), 63, 6, 20),
          ("euclid_D4_r5", W.euclidean_degree_support(4, 5.0), 17, 2, 5)]


@pytest.mark.parametrize("name,S,seed,lo,hi", SELECT, ids=[c[0] for c in SELECT])
def test_select_grids_matches_oracle(fct, name, S, seed, lo, hi):
    """Alg. 2 with kappa_0 = 1e4 over the same seeded candidates (Alg.-1
    draws are inputs): the GPU stops at the oracle's L.  The cases are clear
    cut (the prefixes before L are rank deficient or far above kappa_0)."""
    cands = np.random.default_rng(seed).integers(lo, hi + 1, size=(16, S.shape[1])).astype(np.int32)
    L_ref, k_ref = O.select_grid_count(S, cands, 1e4)
    assert L_ref > 0 and k_ref < 1e2
    L, est = fct.select_grids(S, cands, 1e4, _v0(S.shape[0], 7), max_steps=S.shape[0], tol=0.0)
    assert L == L_ref
    assert abs(est["kappa"] / k_ref - 1.0) < 1e-6


def test_select_grids_reports_no_prefix(fct):
    S = W.total_degree_support(3, 5)
    cands = np.array([[1, 1, 1], [2, 1, 1]], dtype=np.int32)      # cannot resolve degree 5
    L, est = fct.select_grids(S, cands, 1e4, _v0(S.shape[0]), max_steps=S.shape[0], tol=0.0)
    assert L == 0 and not est["full_rank"]
