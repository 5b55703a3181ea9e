"""FP64 row kernel on rows of hundreds of entries (summed by the whole wave).

D = 20, |n|_1 <= 3 (1,771 coefficients) on a cover of every 3-set of
dimensions by 48 grids of degree 3 on eight dimensions (single nodes
elsewhere): in each grid the columns supported on unresolved dimensions
share one bin, so rows reach 455 entries.  The planted polynomial is
recovered exactly (kappa(A) = 1.3e3 by the oracle's SVD), and the problem
gives the same bits alone, in a batch and in the single-kernel iteration.
"""
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


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _problem():
    S = W.total_degree_support(20, 3)
    G = W.d20_grids(4, 3, 8)
    c = W.planted_coefficients(np.random.default_rng([4, 23]), S)
    return S, G, c


def test_long_rows_solve_and_identity(fct):
    S, G, c = _problem()
    plan = fct.Plan(S, G)
    lens = np.diff(_host(plan.export()["seg_off"]))
    assert lens.max() > 96 and int((lens > 96).sum()) >= G.shape[0]
    b = plan.dct(plan.sample(fct.FAMILY_PLANTED, coeffs=torch.tensor(c, device="cuda")))
    x, info = plan.solve(b, tol=1e-15, maxit=20000)
    x = _host(x).copy()
    print(f"D20 d3: M={plan.M} max row {lens.max()} iterations={info.iterations} "
          f"max_rel={O.max_rel_err(x, c):.2e}")
    assert info.converged and O.max_rel_err(x, c) < 1e-10
    # the single-kernel iteration runs the same row code
    xf, infof = plan.solve(b, tol=1e-15, maxit=20000, single_kernel=True)
    assert infof.iterations == info.iterations and np.array_equal(_host(xf), x)
    # and so does a batch
    small = W.config1()
    other = fct.Plan(small.support, small.grids)
    batch = fct.Plan.batch([other, plan])
    b_other = other.dct(other.sample(fct.FAMILY_PLANTED,
                                     coeffs=torch.tensor(small.coeffs, device="cuda")))
    bb = torch.cat([b_other, b])
    xb, _ = batch.solve(bb, tol=1e-15, maxit=20000)
    n0 = other.n
    assert np.array_equal(_host(xb)[n0:n0 + plan.n], x)
    for p in (batch, other, plan):
        p.close()
