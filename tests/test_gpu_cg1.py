"""The one-reduction conjugate-gradient solve (fct_solve_opts.one_reduction)
against the oracle's least-squares minimiser, and its host contract.

It runs CG on A^T A c = A^T b with Chronopoulos-Gear recurrences: the CGLS
iterates in exact arithmetic, rounded differently, so it is held to the
tolerance of the FP64 solve (max-relative 1e-10 against the oracle's QR),
not to the bits of the CGLS kernels.  Runs of it are compared with each
other bit for bit (graph and eager, chunk sizes, repeats).
"""
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


CASES = [W.config1(),
         W.small_problem(1, 1, 40, 3, 30, 3),
         W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS),
         W.small_problem(4, 5, 5, 2, 9, 7, W.FAMILY_GAUSS),
         W.small_problem(6, 2, 20, 40, 63, 2, W.FAMILY_OSC),
         W.small_problem(7, 2, 12, 17, 30, 3, W.FAMILY_EXPCOS)]


def _rhs(fct, plan, prob):
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    return plan.dct(plan.sample(prob.family, prob.params, coeffs=coeffs))


@pytest.mark.parametrize("prob", [p for p in CASES if O.rank_check(
    O.build_plan(p.support, p.grids))[0]], ids=lambda p: p.name)
def test_one_reduction_small(fct, prob):
    samples = O.sample_problem(prob)
    c_ref, _, _ = O.fct_solve(prob.support, prob.grids, samples, "qr")
    plan = fct.Plan(prob.support, prob.grids)
    b = _rhs(fct, plan, prob)
    c, info = plan.solve(b, one_reduction=True)
    c = _host(c)
    print(f"{prob.name}: iterations={info.iterations} max_rel={O.max_rel_err(c, c_ref):.2e}")
    assert info.converged
    assert O.max_rel_err(c, c_ref) < 1e-10
    if prob.coeffs is not None:
        assert O.max_rel_err(c, prob.coeffs) < 1e-10
    plan.close()


def test_one_reduction_config2(fct):
    """D=6, |n|_1<=12, 18,564 coefficients: against the committed QR
    minimiser, with about the iterations of CGLS."""
    prob = W.config2()
    c_ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "cfg2_coeffs_qr.npy"))
    plan = fct.Plan(prob.support, prob.grids)
    b = _rhs(fct, plan, prob)
    c, info = plan.solve(b, one_reduction=True)
    c = _host(c).copy()
    _, info_ls = plan.solve(b)
    print(f"cfg2 one-reduction iterations={info.iterations} (CGLS {info_ls.iterations}) "
          f"max_rel={O.max_rel_err(c, c_ref):.2e}")
    assert info.converged and O.max_rel_err(c, c_ref) < 1e-10
    assert abs(info.iterations - info_ls.iterations) <= max(3, info_ls.iterations // 20)
    plan.close()


def test_one_reduction_deterministic(fct):
    """Graph and eager launches, chunk sizes and repeats give the same bits."""
    prob = W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS)
    plan = fct.Plan(prob.support, prob.grids)
    b = _rhs(fct, plan, prob)
    outs = []
    for use_graph, chunk in ((True, 32), (True, 32), (False, 32), (True, 7), (False, 5)):
        c, info = plan.solve(b, one_reduction=True, use_graph=use_graph, check_every=chunk)
        outs.append((_host(c).copy(), info.iterations))
    for c, it in outs[1:]:
        assert it == outs[0][1]
        assert np.array_equal(c, outs[0][0])
    plan.close()


def test_one_reduction_limits_and_warm_start(fct):
    prob = W.config1()
    plan = fct.Plan(prob.support, prob.grids)
    b = _rhs(fct, plan, prob)
    c, info = plan.solve(b, maxit=3, one_reduction=True, raise_on_noconv=False)
    assert info.status == fct.FCT_ENOCONV and info.iterations == 3 and not info.converged
    assert np.isfinite(info.rel_normal_residual) and info.rel_normal_residual > 0
    c2, info2 = plan.solve(b, out=c, warm_start=True, one_reduction=True)
    assert info2.converged and O.max_rel_err(_host(c2), prob.coeffs) < 1e-12
    bad = b.clone()
    bad[0] = float("nan")
    with pytest.raises(fct.FctError) as ei:
        plan.solve(bad, one_reduction=True)
    assert ei.value.status == fct.FCT_ENONFINITE
    plan.close()


def test_one_reduction_timing(fct):
    prob = W.config2()
    plan = fct.Plan(prob.support, prob.grids)
    b = _rhs(fct, plan, prob)
    _, info = plan.solve(b, one_reduction=True, timing=True)
    assert info.rows_kernel_us > 0.0 and info.cols_kernel_us == 0.0
    plan.close()


def test_one_reduction_rejections(fct):
    """FP32 modes, the single-kernel form and batches are refused on the host."""
    prob = W.config1()
    plan = fct.Plan(prob.support, prob.grids)
    b = _rhs(fct, plan, prob)
    for kw in ({"mode": fct.SOLVE_F32_REFINE}, {"mode": fct.SOLVE_F32}, {"single_kernel": True}):
        with pytest.raises(fct.FctError) as ei:
            plan.solve(b, one_reduction=True, **kw)
        assert ei.value.status == fct.FCT_EINVAL and "one_reduction" in str(ei.value)
    other = W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS)
    plan2 = fct.Plan(other.support, other.grids)
    batch = fct.Plan.batch([plan, plan2])
    bb = torch.zeros(batch.M, dtype=torch.float64, device="cuda")
    with pytest.raises(fct.FctError) as ei:
        batch.solve(bb, one_reduction=True)
    assert ei.value.status == fct.FCT_EINVAL
    for p in (batch, plan2, plan):
        p.close()
