"""Batched form: many independent problems in one plan (through the C ABI).

Every problem of a batch must give exactly the bits it gives alone (same
kernels, same per-problem blocking and reduction order), and match the
oracle within the FP64 tolerance (1e-10 max-relative).
"""
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


def _dev(x):
    return torch.as_tensor(np.asarray(x), dtype=torch.float64, device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def config3_selected():
    """The 256-problem workload with the grid counts chosen by the oracle's
    run of Alg. 2 (tests/golden/cfg3_extra_grids.json)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "cfg3_extra_grids.json")
    with open(path) as fh:
        return W.config3(extra_grids=json.load(fh)["extra_grids"])


def _mixed_batch():
    return [W.config1(),
            W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_PLANTED),
            W.small_problem(12, 5, 5, 0, 5, 12, W.FAMILY_PLANTED),
            W.small_problem(7, 2, 12, 17, 30, 3, W.FAMILY_PLANTED),
            W.small_problem(11, 3, 8, 2, 7, 6, W.FAMILY_PLANTED)]


def test_batch_layout_and_operator(fct):
    probs = _mixed_batch()
    plans = [fct.Plan(p.support, p.grids) for p in probs]
    batch = fct.Plan.batch(plans)
    assert batch.problems == len(probs)
    assert batch.n == sum(p.n for p in plans) and batch.M == sum(p.M for p in plans)
    rng = np.random.default_rng(5)
    c = rng.standard_normal(batch.n)
    r = rng.standard_normal(batch.M)
    q_b = _host(batch.apply_A(_dev(c)))
    s_b = _host(batch.apply_AT(_dev(r)))
    for i, (pl, pr) in enumerate(zip(plans, probs)):
        n, rows, coff, roff, poff, pts = batch.problem(i)
        assert (n, rows, pts) == (pl.n, pl.M, pl.P)
        q1 = _host(pl.apply_A(_dev(c[coff:coff + n])))
        s1 = _host(pl.apply_AT(_dev(r[roff:roff + rows])))
        assert np.array_equal(q_b[roff:roff + rows], q1)
        assert np.array_equal(s_b[coff:coff + n], s1)
        A = O.dense_A(O.build_plan(pr.support, pr.grids))
        assert np.allclose(q1, A @ c[coff:coff + n], atol=1e-13)


def test_batch_sample_dct_solve_match_alone(fct):
    probs = _mixed_batch()
    plans = [fct.Plan(p.support, p.grids) for p in probs]
    batch = fct.Plan.batch(plans)
    coeffs = np.concatenate([p.coeffs for p in probs])
    samples_b = batch.sample(fct.FAMILY_PLANTED, coeffs=_dev(coeffs))
    full_b = _host(batch.dct_full(samples_b))
    b_b = batch.dct(samples_b)
    c_b, info_b = batch.solve(b_b)
    c_b = _host(c_b)
    s_host = _host(samples_b)
    b_host = _host(b_b)
    assert info_b.converged and info_b.problems_converged == len(probs)
    for i, (pl, pr) in enumerate(zip(plans, probs)):
        n, rows, coff, roff, poff, pts = batch.problem(i)
        s1 = pl.sample(fct.FAMILY_PLANTED, coeffs=_dev(pr.coeffs))
        assert np.array_equal(s_host[poff:poff + pts], _host(s1))
        assert np.array_equal(full_b[poff:poff + pts], _host(pl.dct_full(s1)))
        b1 = pl.dct(s1)
        assert np.array_equal(b_host[roff:roff + rows], _host(b1))
        c1, info1 = pl.solve(b1)
        res = batch.problem_result(i)
        assert res.iterations == info1.iterations
        assert np.array_equal(c_b[coff:coff + n], _host(c1))      # bit for bit
        c_ref, _, _ = O.fct_solve(pr.support, pr.grids, O.sample_problem(pr), "qr")
        assert O.max_rel_err(c_b[coff:coff + n], c_ref) < 1e-10
        assert O.max_rel_err(c_b[coff:coff + n], pr.coeffs) < 1e-10


def test_batched_workload_256(fct):
    """256 problems, D in 3..8, total degree 6..16 capped at 50k coefficients,
    Alg.-1 grids (>= 6D of them, counts from the oracle's Alg.-2 run),
    planted polynomials: every problem is recovered to 1e-10; small ones also
    against the oracle's QR, and a few alone against the batch, bit for bit."""
    probs = config3_selected()
    plans = [fct.Plan(p.support, p.grids) for p in probs]
    batch = fct.Plan.batch(plans)
    coeffs = _dev(np.concatenate([p.coeffs for p in probs]))
    samples = batch.sample(fct.FAMILY_PLANTED, coeffs=coeffs)
    b = batch.dct(samples)
    c, info = batch.solve(b)
    c = _host(c)
    print(f"batch: n={batch.n} M={batch.M} P={batch.P} iterations={info.iterations} "
          f"converged={info.problems_converged}/{len(probs)}")
    assert info.converged
    errs = []
    for i, p in enumerate(probs):
        n, rows, coff, roff, poff, pts = batch.problem(i)
        errs.append(O.max_rel_err(c[coff:coff + n], p.coeffs))
    worst = int(np.argmax(errs))
    print(f"worst problem {worst} ({probs[worst].name}, n={probs[worst].n}, "
          f"K={probs[worst].K}, iterations={batch.problem_result(worst).iterations}): "
          f"max_rel {errs[worst]:.2e}; {sum(e < 1e-10 for e in errs)}/256 at 1e-10")
    assert errs[worst] < 1e-10
    small = [i for i, p in enumerate(probs) if p.n <= 600][:4]
    for i in small:
        p = probs[i]
        n, rows, coff, roff, poff, pts = batch.problem(i)
        c_ref, _, _ = O.fct_solve(p.support, p.grids, O.sample_problem(p), "qr")
        assert O.max_rel_err(c[coff:coff + n], c_ref) < 1e-10
    b_host = _host(b)
    for i in [0, 17, 255]:
        n, rows, coff, roff, poff, pts = batch.problem(i)
        c1, _ = plans[i].solve(_dev(b_host[roff:roff + rows]))
        assert np.array_equal(c[coff:coff + n], _host(c1))


def test_batch_mixed_precision_matches_alone(fct):
    probs = _mixed_batch()
    plans = [fct.Plan(p.support, p.grids) for p in probs]
    batch = fct.Plan.batch(plans)
    coeffs = np.concatenate([p.coeffs for p in probs])
    b = batch.dct(batch.sample(fct.FAMILY_PLANTED, coeffs=_dev(coeffs)))
    c_b, info = batch.solve(b, mode=fct.SOLVE_F32_REFINE)
    c_b = _host(c_b)
    b_host = _host(b)
    assert info.converged
    for i, (pl, pr) in enumerate(zip(plans, probs)):
        n, rows, coff, roff, poff, pts = batch.problem(i)
        c1, _ = pl.solve(_dev(b_host[roff:roff + rows]), mode=fct.SOLVE_F32_REFINE)
        assert np.array_equal(c_b[coff:coff + n], _host(c1))
        assert O.max_rel_err(c_b[coff:coff + n], pr.coeffs) < 1e-10


def test_tuning_changes_no_result(fct):
    """The autotuner picks the DCT tile, the DCT engine and the LDS unit size
    by timing.  With the vector engine the DCT gives the same bits before
    and after tuning, whatever the tile; the FP64 and mixed-precision solves
    of a fixed right-hand side give the same bits whatever the unit size."""
    probs = _mixed_batch()
    plans = [fct.Plan(p.support, p.grids) for p in probs]
    batch = fct.Plan.batch(plans)
    coeffs = np.concatenate([p.coeffs for p in probs])
    samples = batch.sample(fct.FAMILY_PLANTED, coeffs=_dev(coeffs))
    before = {}
    for mode in (fct.DCT_F64, fct.DCT_F32):
        before[mode] = _host(batch.dct(samples, mode=mode))
    b = batch.dct(samples)
    c64 = _host(batch.solve(b)[0])
    c32 = _host(batch.solve(b, mode=fct.SOLVE_F32_REFINE)[0])
    info = batch.tune()
    print(info)
    assert info["dct_tile"] in (1024, 2048, 4096)
    assert info["unit_rows"] in (0, 4096, 8192, 16384, 32768)
    assert info["dct_engine"] in (fct.ENGINE_VECTOR, fct.ENGINE_MATRIX)
    # the tuned engine rounds differently at most; the tile alone changes no bit
    tuned = _host(batch.dct(samples))
    ref = before[fct.DCT_F64]
    assert np.max(np.abs(tuned - ref)) <= 1e-13 * np.max(np.abs(ref))
    batch.set_dct_engine(fct.DCT_F64, fct.ENGINE_VECTOR)
    for mode in (fct.DCT_F64, fct.DCT_F32):
        assert np.array_equal(_host(batch.dct(samples, mode=mode)), before[mode])
    assert np.array_equal(_host(batch.solve(b)[0]), c64)
    assert np.array_equal(_host(batch.solve(b, mode=fct.SOLVE_F32_REFINE)[0]), c32)
    # every tile size gives the same transform on a single plan too
    single = plans[1]
    ref = _host(single.dct(single.sample(fct.FAMILY_PLANTED, coeffs=_dev(probs[1].coeffs))))
    single.tune()
    single.set_dct_engine(fct.DCT_F64, fct.ENGINE_VECTOR)
    assert np.array_equal(_host(single.dct(single.sample(fct.FAMILY_PLANTED,
                                                         coeffs=_dev(probs[1].coeffs)))), ref)
