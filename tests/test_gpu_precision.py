"""Precision sweep at full size (D=12, |n|_1 <= 10, 646,646 coefficients,
Gaussian bump on the workload's Alg.-1 grids): the DCT in FP64, FP32 and
split-BF16x3 on the matrix cores, each followed by the FP64 solve and by the
mixed-precision solve (FP32 rounds, FP64 refinement); every result is
compared with the oracle's least-squares minimiser
(tests/golden/cfg4_coeffs_lsqr.npy).

Bounds: the FP64 paths must reach 1e-10 max-relative.  A reduced-precision
DCT perturbs b itself, which no refinement of the solve can undo, so those
modes are held to the floor their rounding allows: the per-axis transforms
of a grid are at most 12 passes of length <= 7 with FP32 accumulation, so
each entry of b carries a relative error of about 12 * sqrt(7) * 2^-24 ~ 2e-6
(FP32) or the same with the split-BF16x3 products, which drop terms of
order 2^-16 * 2^-16 relative; through the solve this is amplified by at
most kappa(A) (the oracle's LSQR estimate, stored with the reference).
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(
    not os.path.exists(os.path.join(os.path.dirname(__file__), "golden", "cfg4_meta.json")),
    reason="oracle reference data not generated yet")]

torch = pytest.importorskip("torch")

HERE = os.path.dirname(__file__)


def _meta():
    with open(os.path.join(HERE, "golden", "cfg4_meta.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def setup():
    from paper_2309_14584_amd import fct
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    meta = _meta()
    prob = W.config4(min_grids=meta["K"])
    c_ref = np.load(os.path.join(HERE, "golden", "cfg4_coeffs_lsqr.npy"))
    plan = fct.Plan(prob.support, prob.grids)
    assert (plan.K, plan.P, plan.M) == (meta["K"], meta["total_points"], meta["rows"])
    samples = plan.sample(prob.family, prob.params)
    yield fct, plan, samples, c_ref, meta
    plan.close()


def _err(c, c_ref):
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    return float(np.max(np.abs(c - c_ref)) / np.max(np.abs(c_ref)))


def test_precision_sweep_f64_dct(setup):
    fct, plan, samples, c_ref, meta = setup
    b = plan.dct(samples, mode=fct.DCT_F64)
    c, info = plan.solve(b)
    e64 = _err(c, c_ref)
    c2, info2 = plan.solve(b, mode=fct.SOLVE_F32_REFINE)
    e_mixed = _err(c2, c_ref)
    print(f"F64 DCT: FP64 solve {e64:.2e} ({info.iterations} it), "
          f"mixed {e_mixed:.2e} ({info2.iterations} it, {info2.refinements} rounds)")
    assert info.converged and info2.converged
    assert e64 < 1e-10
    assert e_mixed < 1e-10


@pytest.mark.parametrize("mode_name", ["DCT_F32", "DCT_BF16X3"])
def test_precision_sweep_reduced_dct(setup, mode_name):
    fct, plan, samples, c_ref, meta = setup
    b = plan.dct(samples, mode=getattr(fct, mode_name))
    c, info = plan.solve(b)
    e = _err(c, c_ref)
    c2, _ = plan.solve(b, mode=fct.SOLVE_F32_REFINE)
    e2 = _err(c2, c_ref)
    bound = max(1.0, meta["lsqr_condition_estimate"]) * 2e-6
    print(f"{mode_name}: FP64 solve {e:.2e}, mixed {e2:.2e} (bound {bound:.1e})")
    assert info.converged
    assert e < bound and e2 < bound
