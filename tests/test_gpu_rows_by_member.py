"""Plans whose rows are ordered by first member (FCT_PLAN_ROWS_BY_MEMBER)
against the oracle and against the same plan in (grid, bin) order.

The row set, each row's run and its bin are the oracle's, bit for bit,
under the row permutation the plan reports; b, A c and A^T r equal the
(grid, bin)-order plan's values permuted, bit for bit (same sums in the
same order); solves meet the 1e-10 bar against the oracle's QR.
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


def _dev(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x), dtype=dtype, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [W.config1(),
         W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS),
         W.small_problem(2, 3, 9, 0, 7, 9),
         W.small_problem(7, 2, 12, 17, 30, 3, W.FAMILY_EXPCOS)]
IDS = [p.name for p in CASES]


def _old_rows(ref, bin_id, row_off):
    """(grid, bin)-order index of every row, from its grid and bin."""
    out = np.empty(len(bin_id), dtype=np.int64)
    for l in range(len(row_off) - 1):
        a, b = int(row_off[l]), int(row_off[l + 1])
        r0, r1 = ref.rows_of_grid(l)
        out[a:b] = r0 + np.searchsorted(ref.bin_id[r0:r1], bin_id[a:b])
    return out


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_rows_by_member_structure(fct, prob):
    ref = O.build_plan(prob.support, prob.grids)
    plan = fct.Plan(prob.support, prob.grids, rows_by_member=True)
    assert plan.M == ref.M
    ex = plan.export()
    perm = _host(ex["perm"]).ravel()
    seg = _host(ex["seg_off"])
    bins = _host(ex["bin_id"])
    rowmap = _host(ex["rowmap"])
    row_off = np.array([plan.grid(l)[3] for l in range(prob.K)] + [plan.M])
    assert np.array_equal(row_off, ref.row_off)
    old = _old_rows(ref, bins, row_off)
    assert np.array_equal(ref.bin_id[old], bins)            # every bin found
    assert len(set(old.tolist())) == plan.M                  # a permutation
    rperm = ref.perm.ravel()
    for r in range(plan.M):
        ro = old[r]
        assert np.array_equal(perm[seg[r]:seg[r + 1]], rperm[ref.seg_off[ro]:ref.seg_off[ro + 1]])
    first = perm[seg[:-1]]
    for l in range(prob.K):
        assert np.all(np.diff(first[row_off[l]:row_off[l + 1]]) > 0)
    for l in range(prob.K):
        assert np.array_equal(bins[rowmap[l]], ref.alias[l])
    plan.close()


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_rows_by_member_values_are_permuted(fct, prob):
    rng = np.random.default_rng(41)
    base = fct.Plan(prob.support, prob.grids)
    plan = fct.Plan(prob.support, prob.grids, rows_by_member=True)
    ref = O.build_plan(prob.support, prob.grids)
    row_off = np.array([plan.grid(l)[3] for l in range(prob.K)] + [plan.M])
    old = _old_rows(ref, _host(plan.export()["bin_id"]), row_off)
    x = _dev(rng.standard_normal(plan.P))
    assert np.array_equal(_host(plan.dct(x)), _host(base.dct(x))[old])
    c = _dev(rng.standard_normal(plan.n))
    assert np.array_equal(_host(plan.apply_A(c)), _host(base.apply_A(c))[old])
    r_old = rng.standard_normal(plan.M)
    assert np.array_equal(_host(plan.apply_AT(_dev(r_old[old]))), _host(base.apply_AT(_dev(r_old))))
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    assert np.array_equal(_host(plan.sample(prob.family, prob.params, coeffs=coeffs)),
                          _host(base.sample(prob.family, prob.params, coeffs=coeffs)))
    base.close()
    plan.close()


FULL_RANK = [p for p in CASES if O.rank_check(O.build_plan(p.support, p.grids))[0]]


@pytest.mark.parametrize("prob", FULL_RANK, ids=[p.name for p in FULL_RANK])
def test_rows_by_member_solve(fct, prob):
    samples = O.sample_problem(prob)
    c_ref, _, _ = O.fct_solve(prob.support, prob.grids, samples, "qr")
    plan = fct.Plan(prob.support, prob.grids, rows_by_member=True)
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    b = plan.dct(plan.sample(prob.family, prob.params, coeffs=coeffs))
    for kw in ({}, {"mode": fct.SOLVE_F32_REFINE}, {"one_reduction": True}):
        c, info = plan.solve(b, **kw)
        assert info.converged and O.max_rel_err(_host(c), c_ref) < 1e-10, kw
    plan.close()


def test_rows_by_member_sparse_d100(fct):
    """The f3 family (D = 100, random sparse support): exact recovery."""
    p = W.f3_problem(3000)
    plan = fct.Plan(p.support, p.grids, allow_rank_deficient=True, rows_by_member=True)
    b = plan.dct(plan.sample(fct.FAMILY_PLANTED, coeffs=_dev(p.coeffs)))
    c, info = plan.solve(b)
    assert info.converged and O.max_rel_err(_host(c), p.coeffs) < 1e-10
    plan.close()


def test_rows_by_member_in_a_batch(fct):
    """A batch of reordered and plain plans: every problem's b and
    coefficients are the bits it gives alone (FP64 and mixed solves)."""
    probs = [CASES[1], CASES[0], W.small_problem(4, 5, 5, 2, 9, 7, W.FAMILY_GAUSS)]
    flags = [True, False, True]
    plans = [fct.Plan(p.support, p.grids, rows_by_member=f) for p, f in zip(probs, flags)]
    batch = fct.Plan.batch(plans)
    rng = np.random.default_rng(43)
    x = rng.standard_normal(batch.P)
    bb = _host(batch.dct(_dev(x)))
    alone_b, poff, roff = [], 0, 0
    for pl in plans:
        alone_b.append(_host(pl.dct(_dev(x[poff:poff + pl.P]))))
        assert np.array_equal(bb[roff:roff + pl.M], alone_b[-1])
        poff += pl.P
        roff += pl.M
    for mode in (fct.SOLVE_F64, fct.SOLVE_F32_REFINE):
        cb, _ = batch.solve(_dev(bb), mode=mode, raise_on_noconv=False)
        cb = _host(cb)
        coff = 0
        for pl, b in zip(plans, alone_b):
            ca, _ = pl.solve(_dev(b), mode=mode, raise_on_noconv=False)
            assert np.array_equal(cb[coff:coff + pl.n], _host(ca)), mode
            coff += pl.n
    batch.close()
    for pl in plans:
        pl.close()


def test_rows_by_member_rejections(fct):
    prob = CASES[0]
    with pytest.raises(fct.FctError) as ei:
        fct.Plan(prob.support, prob.grids, rows_by_member=True, gauss=True)
    assert ei.value.status == fct.FCT_EINVAL
