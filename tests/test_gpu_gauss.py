"""Parity of Gauss-grid / DCT-II plans (FCT_PLAN_GAUSS) with the Gauss
oracle, through the C ABI.

Bars: integer maps and entry weights bit for bit; samples and transforms
1e-12 of the largest magnitude; A c and A^T r on integer-valued vectors
exactly (small integer sums); coefficients 1e-10 max-relative against the
oracle's QR minimiser, and exact recovery of planted polynomials.
"""
import numpy as np
import pytest

import oracle as O
from oracle import gauss_oracle as G
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fct():
    from paper_2309_14584_amd import fct as mod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    return mod


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x), dtype=dtype, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    b = np.asarray(b)
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


# Full rank on their Gauss grids (checked against the oracle's SVD): D = 2..5,
# single-node axes (N_i = 0, node x = 0), extents up to 64, analytic families.
CASES = [W.small_problem(22, 2, 10, 6, 12, 5),
         W.small_problem(3, 3, 6, 2, 8, 6),
         W.small_problem(4, 4, 5, 2, 7, 7),
         W.small_problem(5, 2, 16, 9, 24, 4),
         W.small_problem(23, 2, 12, 5, 14, 5, W.FAMILY_EXPCOS),
         W.small_problem(2, 3, 9, 0, 7, 9),
         W.small_problem(9, 2, 30, 40, 63, 3, W.FAMILY_OSC),
         W.small_problem(10, 5, 4, 1, 6, 8, W.FAMILY_GAUSS)]
IDS = [p.name for p in CASES]


def _plan(fct, prob):
    return fct.Plan(prob.support, prob.grids, gauss=True)


def _offsets(prob):
    pts = [int(np.prod(g.astype(np.int64) + 1)) for g in prob.grids]
    return np.concatenate([[0], np.cumsum(pts)])


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_gauss_maps_and_weights(fct, prob):
    plan = _plan(fct, prob)
    ex = plan.export()
    alias = _host(ex["alias"])
    w = _host(plan.weights())
    rowmap = _host(ex["rowmap"])
    bin_id = _host(ex["bin_id"])
    for l in range(prob.K):
        bins, wr = G.signed_alias(prob.support, prob.grids[l])
        assert np.array_equal(w[l], wr)
        nz = wr != 0
        assert np.array_equal(alias[l][nz], bins[nz])
        # every entry sits in the row of its bin
        assert np.array_equal(bin_id[rowmap[l]], alias[l])
    plan.close()


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_gauss_nodes_and_sampler(fct, prob):
    plan = _plan(fct, prob)
    for l in range(prob.K):
        for i in range(prob.D):
            ref = G.gauss_nodes(int(prob.grids[l, i]))
            assert np.max(np.abs(plan.nodes(l, i) - ref)) < 1e-15
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    out = _host(plan.sample(prob.family, prob.params, coeffs=coeffs))
    ref = np.concatenate(G.sample_problem_gauss(prob))
    assert _rel(out, ref) < 1e-12
    plan.close()


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_gauss_dct(fct, prob):
    rng = np.random.default_rng(31)
    plan = _plan(fct, prob)
    offs = _offsets(prob)
    x = rng.standard_normal(plan.P)
    ref_full = [G.dct2_grid(x[offs[l]:offs[l + 1]], prob.grids[l]) for l in range(prob.K)]
    xd = _dev(x)
    assert _rel(_host(plan.dct_full(xd)), np.concatenate(ref_full)) < 1e-12
    b = _host(plan.dct(xd))
    bin_id = _host(plan.export()["bin_id"])
    ref_b = np.concatenate([ref_full[l][bin_id[plan.grid(l)[3]:plan.grid(l)[3] + plan.grid(l)[1]]]
                            for l in range(prob.K)])
    assert _rel(b, ref_b) < 1e-12
    # the matrix engine in FP64 gives the same transform within the bar
    # (it takes degrees up to 31)
    if int(prob.grids.max()) <= 31:
        plan.set_dct_engine(fct.DCT_F64, fct.ENGINE_MATRIX)
        assert _rel(_host(plan.dct_full(xd)), np.concatenate(ref_full)) < 1e-12
    plan.close()


@pytest.mark.parametrize("prob", CASES[:6], ids=IDS[:6])
def test_gauss_operator_exact(fct, prob):
    rng = np.random.default_rng(32)
    plan = _plan(fct, prob)
    A = G.dense_A_gauss(prob.support, prob.grids)          # rows: every bin of every grid
    offs = _offsets(prob)
    ex = plan.export()
    bin_id = _host(ex["bin_id"])
    rows = []
    for l in range(prob.K):
        _, nrows, _, roff = plan.grid(l)
        rows.append(offs[l] + bin_id[roff:roff + nrows])
    rows = np.concatenate(rows)
    c = rng.integers(-50, 51, size=plan.n).astype(np.float64)
    assert np.array_equal(_host(plan.apply_A(_dev(c))), A[rows] @ c)
    r = rng.integers(-50, 51, size=plan.M).astype(np.float64)
    assert np.array_equal(_host(plan.apply_AT(_dev(r))), A[rows].T @ r)
    plan.close()


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_gauss_solve_against_oracle(fct, prob):
    samples = G.sample_problem_gauss(prob)
    c_ref, _ = G.solve_gauss(prob.support, prob.grids, samples)
    plan = _plan(fct, prob)
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    b = plan.dct(plan.sample(prob.family, prob.params, coeffs=coeffs))
    c, info = plan.solve(b)
    c = _host(c)
    print(f"{prob.name}: iterations={info.iterations} max_rel={O.max_rel_err(c, c_ref):.2e}")
    assert info.converged
    assert O.max_rel_err(c, c_ref) < 1e-10
    if prob.coeffs is not None:
        assert O.max_rel_err(c, prob.coeffs) < 1e-10
    plan.close()


def test_gauss_solve_deterministic_warm_and_limits(fct):
    prob = CASES[2]
    plan = _plan(fct, prob)
    b = plan.dct(plan.sample(prob.family, coeffs=_dev(prob.coeffs)))
    outs = []
    for use_graph, chunk in ((True, 32), (False, 32), (True, 7)):
        c, info = plan.solve(b, use_graph=use_graph, check_every=chunk)
        outs.append((_host(c).copy(), info.iterations))
    for c, it in outs[1:]:
        assert it == outs[0][1] and np.array_equal(c, outs[0][0])
    c, info = plan.solve(b, maxit=3, raise_on_noconv=False)
    assert info.status == fct.FCT_ENOCONV and info.iterations == 3
    c2, info2 = plan.solve(b, out=c, warm_start=True)
    assert info2.converged and O.max_rel_err(_host(c2), prob.coeffs) < 1e-10
    plan.close()


def test_gauss_condition(fct):
    prob = CASES[1]
    plan = _plan(fct, prob)
    A = G.dense_A_gauss(prob.support, prob.grids)
    sv = np.linalg.svd(A, compute_uv=False)
    v0 = _dev(np.random.default_rng(4).standard_normal(plan.n))
    cond = plan.condition(v0, max_steps=plan.n)
    assert cond["full_rank"]
    assert abs(cond["kappa"] - sv[0] / sv[-1]) < 1e-6 * sv[0] / sv[-1]
    plan.close()


def test_gauss_planted_d6_at_scale(fct):
    """D=6, |n|_1 <= 12 (18,564 coefficients) on eight Gauss grids
    N_i ~ U{4..8}: a planted polynomial is recovered exactly (the oracle's
    QR does not fit; exact recovery is the known answer)."""
    prob = W.small_problem(41, 6, 12, 4, 8, 8)
    plan = _plan(fct, prob)
    b = plan.dct(plan.sample(prob.family, coeffs=_dev(prob.coeffs)))
    c, info = plan.solve(b)
    err = O.max_rel_err(_host(c), prob.coeffs)
    print(f"gauss D6 planted: n={plan.n} M={plan.M} iterations={info.iterations} max_rel={err:.2e}")
    assert info.converged and err < 1e-10
    plan.close()


def test_gauss_rejections(fct):
    prob = CASES[0]
    plan = _plan(fct, prob)
    b = plan.dct(plan.sample(prob.family, coeffs=_dev(prob.coeffs)))
    for kw in ({"mode": fct.SOLVE_F32_REFINE}, {"mode": fct.SOLVE_F32}, {"single_kernel": True}):
        with pytest.raises(fct.FctError) as ei:
            plan.solve(b, **kw)
        assert ei.value.status == fct.FCT_EINVAL and "Gauss" in str(ei.value)
    other = _plan(fct, CASES[1])
    with pytest.raises(fct.FctError) as ei:
        fct.Plan.batch([plan, other])
    assert ei.value.status == fct.FCT_EINVAL
    other.close()
    plan.close()
