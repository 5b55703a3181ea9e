"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer maps must match bit for bit; floating-point results within the
stated tolerances:
  * samples and transforms: 1e-12 of the largest magnitude (a few FP64
    roundings per axis; the DCT sums at most 64 terms per axis);
  * coefficients of the FP64 path: max-relative error 1e-10 against the
    oracle's least-squares minimiser (the tolerance the method is held to).
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


def _rel(a, b):
    b = np.asarray(b)
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


# Problems spanning: D = 1 .. 8, single-node axes (N_i = 0), ragged sizes
# (n not a multiple of the 256-thread workgroup, K*n above one 1024-entry
# sort tile so that global merge levels run), grids needing one, two and
# three DCT passes, and extents up to 64 (all register-tile variants).
def _cases():
    yield W.config1()
    yield W.small_problem(1, 1, 40, 3, 30, 3)                   # D=1
    yield W.small_problem(2, 3, 9, 0, 7, 9)                     # N_i = 0 axes
    yield W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS)
    yield W.small_problem(4, 5, 5, 2, 9, 7, W.FAMILY_GAUSS)
    yield W.small_problem(5, 8, 3, 1, 4, 6, W.FAMILY_RUNGE)
    yield W.small_problem(6, 2, 20, 40, 63, 2, W.FAMILY_OSC)     # extents 41..64
    yield W.small_problem(7, 2, 12, 17, 30, 3, W.FAMILY_EXPCOS)  # extents 18..31


CASES = list(_cases())
IDS = [p.name for p in CASES]


def _plan(fct, prob):
    return fct.Plan(prob.support, prob.grids, allow_rank_deficient=True)


@pytest.mark.parametrize("prob", CASES + [W.config2()], ids=IDS + ["cfg2"])
def test_plan_maps_bit_exact(fct, prob):
    ref = O.build_plan(prob.support, prob.grids)
    plan = _plan(fct, prob)
    assert plan.M == ref.M
    ex = plan.export()
    assert np.array_equal(_host(ex["alias"]), ref.alias)
    assert np.array_equal(_host(ex["perm"]), ref.perm)
    assert np.array_equal(_host(ex["seg_off"]), ref.seg_off)
    assert np.array_equal(_host(ex["bin_id"]), ref.bin_id)
    assert np.array_equal(_host(ex["rowmap"]), ref.rowmap)
    for l in range(prob.K):
        pts, rows, poff, roff = plan.grid(l)
        assert pts == ref.points[l] and roff == ref.row_off[l]
        assert rows == ref.row_off[l + 1] - ref.row_off[l]
    plan.close()


def test_plan_rank_error(fct):
    S = W.total_degree_support(2, 6)
    with pytest.raises(fct.FctError) as ei:
        fct.Plan(S, [[3, 3], [3, 3]])
    assert ei.value.status == fct.FCT_ERANK


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_nodes(fct, prob):
    plan = _plan(fct, prob)
    for l in range(prob.K):
        for i in range(prob.D):
            ref = O.lobatto_nodes(int(prob.grids[l, i]))
            # the oracle rounds pi*k/N before its cosine; a few ulp apart
            assert np.max(np.abs(plan.nodes(l, i) - ref)) < 1e-15
    plan.close()


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_sampler(fct, prob):
    plan = _plan(fct, prob)
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    out = _host(plan.sample(prob.family, prob.params, coeffs=coeffs))
    ref = np.concatenate(O.sample_problem(prob))
    assert _rel(out, ref) < 1e-12
    plan.close()


@pytest.mark.parametrize("prob", CASES + [W.config2()], ids=IDS + ["cfg2"])
def test_dct(fct, prob):
    rng = np.random.default_rng(11)
    plan = _plan(fct, prob)
    ref_plan = O.build_plan(prob.support, prob.grids)
    x = rng.standard_normal(plan.P)
    offs = np.concatenate([[0], np.cumsum(prob.points)])
    ref_full = [O.dct_grid(x[offs[l]:offs[l + 1]], prob.grids[l]) for l in range(prob.K)]
    xd = _dev(x)
    full = _host(plan.dct_full(xd))
    assert _rel(full, np.concatenate(ref_full)) < 1e-12
    b = _host(plan.dct(xd))
    assert _rel(b, O.rhs_from_transforms(ref_plan, ref_full)) < 1e-12
    plan.close()


@pytest.mark.parametrize("prob", CASES, ids=IDS)
def test_operator(fct, prob):
    rng = np.random.default_rng(12)
    plan = _plan(fct, prob)
    A = O.dense_A(O.build_plan(prob.support, prob.grids))
    c = rng.standard_normal(plan.n)
    r = rng.standard_normal(plan.M)
    assert _rel(_host(plan.apply_A(_dev(c))), A @ c) < 1e-14
    assert _rel(_host(plan.apply_AT(_dev(r))), A.T @ r) < 1e-14
    plan.close()


def _solve_case(fct, prob, **kw):
    plan = fct.Plan(prob.support, prob.grids)
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    s = plan.sample(prob.family, prob.params, coeffs=coeffs)
    b = plan.dct(s)
    c, info = plan.solve(b, **kw)
    return plan, b, _host(c), info


@pytest.mark.parametrize("prob", [p for p in CASES if O.rank_check(
    O.build_plan(p.support, p.grids))[0]], ids=lambda p: p.name)
def test_solve_small(fct, prob):
    samples = O.sample_problem(prob)
    c_ref, _, _ = O.fct_solve(prob.support, prob.grids, samples, "qr")
    plan, b, c, info = _solve_case(fct, prob)
    assert info.converged
    assert O.max_rel_err(c, c_ref) < 1e-10
    if prob.coeffs is not None:   # planted: exact recovery
        assert O.max_rel_err(c, prob.coeffs) < 1e-10
    plan.close()


def test_solve_config1_exact(fct):
    prob = W.config1()
    plan, b, c, info = _solve_case(fct, prob)
    assert info.converged and O.max_rel_err(c, prob.coeffs) < 1e-12
    plan.close()


def test_solve_config2_against_oracle(fct):
    """D=6, |n|_1<=12, 18,564 coefficients, exp-cos: oracle by dense QR."""
    import os
    prob = W.config2()
    golden = os.path.join(os.path.dirname(__file__), "golden", "cfg2_coeffs_qr.npy")
    c_ref = np.load(golden)
    plan, b, c, info = _solve_case(fct, prob)
    print(f"cfg2 iterations={info.iterations} rel_normal_residual={info.rel_normal_residual:.2e} "
          f"max_rel={O.max_rel_err(c, c_ref):.2e}")
    assert info.converged
    assert O.max_rel_err(c, c_ref) < 1e-10
    plan.close()


def test_solve_deterministic_and_graph_matches_eager(fct):
    prob = W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS)
    plan = fct.Plan(prob.support, prob.grids)
    b = plan.dct(plan.sample(prob.family, prob.params))
    outs = []
    for use_graph in (True, True, False, True):
        c, info = plan.solve(b, use_graph=use_graph, check_every=8)
        outs.append((_host(c).copy(), info.iterations))
    for c, it in outs[1:]:
        assert it == outs[0][1]
        assert np.array_equal(c, outs[0][0])      # bit for bit
    plan.close()


@pytest.mark.parametrize("prob", [W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS),
                                  W.config1(), W.config2()], ids=["expcos_D4", "cfg1", "cfg2"])
def test_single_kernel_iteration_matches_two_kernels(fct, prob):
    """A single problem runs each chunk of CGLS iterations as one cooperative
    kernel with grid barriers; it gives the bits of two kernels per
    iteration, in FP64 and in the mixed-precision rounds."""
    plan = fct.Plan(prob.support, prob.grids)
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    b = plan.dct(plan.sample(prob.family, prob.params, coeffs=coeffs))
    for mode in (fct.SOLVE_F64, fct.SOLVE_F32_REFINE):
        for chunk in (7, 32):
            c1, i1 = plan.solve(b, mode=mode, check_every=chunk, single_kernel=True)
            c1 = _host(c1).copy()
            c2, i2 = plan.solve(b, mode=mode, check_every=chunk, single_kernel=False)
            assert i1.iterations == i2.iterations
            assert np.array_equal(c1, _host(c2))
    plan.close()


def test_solve_warm_start_and_limits(fct):
    prob = W.config1()
    plan = fct.Plan(prob.support, prob.grids)
    b = plan.dct(plan.sample(fct.FAMILY_PLANTED, coeffs=_dev(prob.coeffs)))
    c, info = plan.solve(b, maxit=3, raise_on_noconv=False)
    assert info.status == fct.FCT_ENOCONV and info.iterations == 3 and not info.converged
    with pytest.raises(fct.FctError):
        plan.solve(b, maxit=3)
    c2, info2 = plan.solve(b, out=c, warm_start=True)     # resume from the stopped iterate
    assert info2.converged and O.max_rel_err(_host(c2), prob.coeffs) < 1e-12
    bad = b.clone()
    bad[0] = float("nan")
    with pytest.raises(fct.FctError) as ei:
        plan.solve(bad)
    assert ei.value.status == fct.FCT_ENONFINITE
    plan.close()


# Reduced-precision DCT modes: error bound per axis ~ e * unit roundoff of
# the mode (FP32: 2^-24 per product and sum; split-BF16x3: the dropped
# C_lo x_lo term and the bf16 rounding of the low parts, ~2^-16 relative per
# product, plus FP32 sums); summed over the D axes, relative to the largest
# magnitude.
MODE_EPS = {1: 2.0 ** -24, 2: 2.0 ** -15}


@pytest.mark.parametrize("mode", [1, 2], ids=["f32", "bf16x3"])
@pytest.mark.parametrize("prob", [p for p in CASES if int(p.grids.max()) <= 31] + [W.config2()],
                         ids=[p.name for p in CASES if int(p.grids.max()) <= 31] + ["cfg2"])
def test_dct_reduced_precision(fct, prob, mode):
    rng = np.random.default_rng(13)
    plan = _plan(fct, prob)
    ref_plan = O.build_plan(prob.support, prob.grids)
    x = rng.standard_normal(plan.P)
    offs = np.concatenate([[0], np.cumsum(prob.points)])
    ref_full = [O.dct_grid(x[offs[l]:offs[l + 1]], prob.grids[l]) for l in range(prob.K)]
    ref_b = O.rhs_from_transforms(ref_plan, ref_full)
    b = _host(plan.dct(_dev(x), mode=mode))
    emax = int(prob.grids.max()) + 1
    bound = 4.0 * prob.D * emax * MODE_EPS[mode] * np.max(np.abs(x)) / max(np.max(np.abs(ref_b)), 1e-300)
    err = _rel(b, ref_b)
    print(f"mode {mode}: rel err {err:.2e} (bound {bound:.2e})")
    assert err < bound
    # and the same bits through the full-tensor entry point at the kept bins
    full = _host(plan.dct_full(_dev(x), mode=mode))
    assert _rel(full, np.concatenate(ref_full)) < bound
    plan.close()


_MATRIX_CASES = [p for p in CASES if int(p.grids.max()) <= 31] + [W.config2()]


@pytest.mark.parametrize("mode", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("prob", _MATRIX_CASES, ids=[p.name for p in _MATRIX_CASES[:-1]] + ["cfg2"])
def test_dct_matrix_engine(fct, prob, mode):
    """The FP64 and FP32 contractions on the matrix cores (16x16x4 MFMA):
    FP64 to the same 1e-12 as the vector engine, FP32 to its rounding bound;
    both engines agree to rounding."""
    rng = np.random.default_rng(14)
    plan = _plan(fct, prob)
    ref_plan = O.build_plan(prob.support, prob.grids)
    x = rng.standard_normal(plan.P)
    offs = np.concatenate([[0], np.cumsum(prob.points)])
    ref_full = [O.dct_grid(x[offs[l]:offs[l + 1]], prob.grids[l]) for l in range(prob.K)]
    ref_b = O.rhs_from_transforms(ref_plan, ref_full)
    xd = _dev(x)
    vec = _host(plan.dct(xd, mode=mode))
    plan.set_dct_engine(mode, fct.ENGINE_MATRIX)
    b = _host(plan.dct(xd, mode=mode))
    full = _host(plan.dct_full(xd, mode=mode))
    if mode == 0:
        bound = 1e-12
    else:
        emax = int(prob.grids.max()) + 1
        bound = (4.0 * prob.D * emax * MODE_EPS[mode] * np.max(np.abs(x))
                 / max(np.max(np.abs(ref_b)), 1e-300))
    assert _rel(b, ref_b) < bound
    assert _rel(full, np.concatenate(ref_full)) < bound
    assert _rel(b, vec) < 2 * bound
    plan.close()


def test_dct_engine_errors(fct):
    prob = W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS)
    plan = _plan(fct, prob)
    with pytest.raises(fct.FctError):
        plan.set_dct_engine(fct.DCT_BF16X3, fct.ENGINE_VECTOR)
    with pytest.raises(fct.FctError):
        plan.set_dct_engine(7, fct.ENGINE_VECTOR)
    with pytest.raises(fct.FctError):
        plan.set_dct_engine(fct.DCT_F64, 2)
    plan.set_dct_engine(fct.DCT_F64, fct.ENGINE_MATRIX)
    plan.close()
    long_axes = W.small_problem(6, 2, 20, 40, 63, 2, W.FAMILY_OSC)     # extents 41..64
    plan = _plan(fct, long_axes)
    with pytest.raises(fct.FctError):
        plan.set_dct_engine(fct.DCT_F64, fct.ENGINE_MATRIX)
    plan.close()


# Mixed precision: FP32 CGLS rounds refined in FP64 reach the FP64 bar
# (1e-10 max-relative); a single FP32 round (pure FP32 vectors) is held to
# 1e-5.
@pytest.mark.parametrize("prob", [W.config1(), W.small_problem(3, 4, 6, 1, 6, 6, W.FAMILY_EXPCOS),
                                  W.small_problem(12, 5, 5, 0, 5, 12, W.FAMILY_PLANTED)],
                         ids=["cfg1", "expcos_D4", "planted_D5"])
def test_solve_mixed_precision_small(fct, prob):
    c_ref, _, _ = O.fct_solve(prob.support, prob.grids, O.sample_problem(prob), "qr")
    plan = fct.Plan(prob.support, prob.grids)
    coeffs = _dev(prob.coeffs) if prob.coeffs is not None else None
    b = plan.dct(plan.sample(prob.family, prob.params, coeffs=coeffs))
    c, info = plan.solve(b, mode=fct.SOLVE_F32_REFINE)
    err = O.max_rel_err(_host(c), c_ref)
    print(f"refined: iterations={info.iterations} rounds={info.refinements} err={err:.2e}")
    assert info.converged and err < 1e-10
    c32, info32 = plan.solve(b, mode=fct.SOLVE_F32)
    assert O.max_rel_err(_host(c32), c_ref) < 1e-5
    plan.close()


def test_solve_mixed_precision_config2(fct):
    import os
    prob = W.config2()
    c_ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "cfg2_coeffs_qr.npy"))
    plan = fct.Plan(prob.support, prob.grids)
    b = plan.dct(plan.sample(prob.family, prob.params))
    c, info = plan.solve(b, mode=fct.SOLVE_F32_REFINE)
    err = O.max_rel_err(_host(c), c_ref)
    print(f"cfg2 refined: iterations={info.iterations} rounds={info.refinements} err={err:.2e}")
    assert info.converged and err < 1e-10
    c32, _ = plan.solve(b, mode=fct.SOLVE_F32)
    err32 = O.max_rel_err(_host(c32), c_ref)
    print(f"cfg2 fp32: err={err32:.2e}")
    assert err32 < 1e-5
    # FP32 and split-BF16x3 transforms feed the FP64 solve: error floors of
    # the right-hand side (refinement cannot repair b)
    for mode, bound in [(fct.DCT_F32, 1e-5), (fct.DCT_BF16X3, 1e-3)]:
        bm = plan.dct(plan.sample(prob.family, prob.params), mode=mode)
        cm, _ = plan.solve(bm)
        e = O.max_rel_err(_host(cm), c_ref)
        print(f"cfg2 dct mode {mode}: err={e:.2e}")
        assert e < bound
    plan.close()
