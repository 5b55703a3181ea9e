"""The paper's f3 family on the GPU: D = 100, random sparse supports of
S^inf_{8,100}, 20 Alg.-1 grids (mostly single-node dimensions), planted
coefficients in [-1, 1] -- plan, inverse-DCT sampling, DCT and CGLS."""
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


def _run(fct, p):
    plan = fct.Plan(p.support, p.grids, allow_rank_deficient=True)
    c_true = torch.as_tensor(p.coeffs, dtype=torch.float64, device="cuda")
    b = plan.dct(plan.sample(fct.FAMILY_PLANTED, coeffs=c_true))
    c, info = plan.solve(b)
    return plan, b.cpu().numpy(), c.cpu().numpy(), info


def test_f3_small_against_oracle(fct):
    p = W.f3_problem(2000)
    plan, b, c, info = _run(fct, p)
    c_ref, oplan, b_ref = O.fct_solve(p.support, p.grids, O.sample_problem(p), "auto")
    assert plan.M == oplan.M
    assert np.max(np.abs(b - b_ref)) <= 1e-12 * np.max(np.abs(b_ref))
    assert info.converged and O.max_rel_err(c, c_ref) < 1e-10
    assert O.max_rel_err(c, p.coeffs) < 1e-10
    plan.close()


@pytest.mark.parametrize("N", [200_000])
def test_f3_large_recovers_planted(fct, N):
    """Exact recovery of the planted coefficients (the unique least-squares
    solution when A has full column rank)."""
    p = W.f3_problem(N)
    plan, b, c, info = _run(fct, p)
    err = O.max_rel_err(c, p.coeffs)
    print(f"f3 N={N}: rows {plan.M}, points {plan.P}, {info.iterations} iterations, err {err:.2e}")
    assert info.converged and err < 1e-10
    plan.close()
