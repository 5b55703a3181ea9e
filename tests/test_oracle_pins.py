"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties an oracle function to something other than itself: an integer
identity checked exhaustively, a library routine that computes the same
quantity another way (scipy's DCT, numpy's Chebyshev module, numpy/LAPACK
least squares), a closed form, a special case with a textbook answer, or
brute force on tiny inputs.  None of these tests touches the GPU.
"""
import itertools
import json
import math
import os

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest
import scipy.fft

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Aliasing fold: Lobatto analogue of Lemma 3.1 (Sec. 3.1)
# --------------------------------------------------------------------------

def test_fold_integer_identity_exhaustive():
    """cos(n k pi/N) = cos(m k pi/N) for every node k, as integers mod 2N.

    For each N <= 39 and n < 6N, the folded m lies in 0..N, satisfies
    n k = +-m k (mod 2N) for every k, and is the only index in 0..N that
    does (so the alias is unique and the block of A has one 1 per column).
    """
    bad = 0
    for N in range(1, 40):
        ks = range(N + 1)
        for n in range(6 * N):
            m = O.fold(n, N)
            assert 0 <= m <= N
            ok = all((n * k - m * k) % (2 * N) == 0 or (n * k + m * k) % (2 * N) == 0
                     for k in ks)
            if not ok:
                bad += 1
            others = [mm for mm in range(N + 1) if mm != m and all(
                (n * k - mm * k) % (2 * N) == 0 or (n * k + mm * k) % (2 * N) == 0
                for k in ks)]
            assert not others, (n, N, m, others)
    assert bad == 0


def test_fold_single_node():
    # one node at x = 1: every T_n(1) = 1 = T_0(1)
    assert all(O.fold(n, 0) == 0 for n in range(50))


def test_fold_numeric_against_numpy_chebval():
    """T_n at the Lobatto nodes equals T_fold(n) there (numpy's Chebyshev
    evaluation, independent of the oracle's recurrence)."""
    for N in [1, 2, 3, 5, 8, 13]:
        x = O.lobatto_nodes(N)
        for n in range(5 * N + 3):
            en = np.zeros(n + 1); en[n] = 1
            m = O.fold(n, N)
            em = np.zeros(m + 1); em[m] = 1
            assert np.allclose(npc.chebval(x, en), npc.chebval(x, em), atol=1e-12)


def test_chebyshev_evaluations_agree():
    x = np.linspace(-1, 1, 37)
    tab = O.cheb_T_recurrence(20, x)
    for n in range(21):
        e = np.zeros(n + 1); e[n] = 1
        ref = npc.chebval(x, e)
        assert np.allclose(tab[n], ref, atol=1e-12)
        assert np.allclose(O.cheb_T(n, x), ref, atol=1e-12)


def test_fold_by_hand_D1():
    """D = 1, degrees 0..7 on N = 3 and N = 4 (P6): fold tables by hand.
    N=3: period 6, n -> 0 1 2 3 2 1 0 1;  N=4: period 8, n -> 0 1 2 3 4 3 2 1."""
    assert [O.fold(n, 3) for n in range(8)] == [0, 1, 2, 3, 2, 1, 0, 1]
    assert [O.fold(n, 4) for n in range(8)] == [0, 1, 2, 3, 4, 3, 2, 1]
    S = np.arange(8, dtype=np.int32)[:, None]
    plan = O.build_plan(S, np.array([[3], [4]], dtype=np.int32))
    assert plan.alias.tolist() == [[0, 1, 2, 3, 2, 1, 0, 1], [0, 1, 2, 3, 4, 3, 2, 1]]
    # grid 0 bins 0..3 hold {0,6}, {1,5,7}, {2,4}, {3}; grid 1 bins 0..4
    assert plan.perm[0].tolist() == [0, 6, 1, 5, 7, 2, 4, 3]
    assert plan.perm[1].tolist() == [0, 1, 7, 2, 6, 3, 5, 4]
    assert plan.seg_off.tolist() == [0, 2, 5, 7, 8, 9, 11, 13, 15, 16]
    assert plan.M == 9
    # degrees 1 and 7 alias together on both N=3 and N=4, so that stack
    # cannot separate them; N=3 with N=5 separates every degree 0..7
    assert not O.fold_injective(S, [[3], [4]])
    assert O.fold_injective(S, [[3], [5]])
    assert not O.fold_injective(S, [[3], [3]])


# --------------------------------------------------------------------------
# DCT-I (interpolation normalisation)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N", list(range(1, 31)) + [47, 63])
def test_dct1_matches_scipy(N):
    rng = np.random.default_rng(N)
    v = rng.standard_normal(N + 1)
    g = np.ones(N + 1); g[0] = g[N] = 0.5
    ref = g * scipy.fft.dct(v, type=1) / N
    assert np.allclose(O.dct1_matrix(N) @ v, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", [1, 2, 4, 7, 9, 16, 24])
def test_dct1_closed_form_chebyshev_samples(N):
    """Samples of T_n (numpy chebval) transform to e_fold(n) exactly."""
    x = O.lobatto_nodes(N)
    C = O.dct1_matrix(N)
    for n in range(4 * N + 2):
        e = np.zeros(n + 1); e[n] = 1
        a = C @ npc.chebval(x, e)
        want = np.zeros(N + 1); want[O.fold(n, N)] = 1
        assert np.allclose(a, want, atol=1e-13), (N, n)


@pytest.mark.parametrize("N", [0, 1, 3, 8, 24])
def test_dct1_round_trip(N):
    rng = np.random.default_rng(7 + N)
    v = rng.standard_normal(N + 1)
    C, E = O.dct1_matrix(N), O.dct1_eval_matrix(N)
    assert np.allclose(E @ (C @ v), v, atol=1e-13)
    assert np.allclose(C @ (E @ v), v, atol=1e-13)


@pytest.mark.parametrize("grid", [(3, 5), (6, 2), (4, 1, 3), (0, 4), (2, 0, 5)])
def test_dct_grid_full_resolution(grid):
    """P5: a coefficient tensor of matching size evaluated on its tensor grid
    (numpy chebgrid) is recovered exactly by the separable transform.
    Unequal extents catch a transposed or misordered axis."""
    rng = np.random.default_rng(sum(grid))
    shape = tuple(g + 1 for g in grid)
    Ct = rng.standard_normal(shape)
    xs = [O.lobatto_nodes(g) for g in grid]
    if len(grid) == 2:
        vals = npc.chebgrid2d(xs[0], xs[1], Ct)
    else:
        vals = npc.chebgrid3d(xs[0], xs[1], xs[2], Ct)
    got = O.dct_grid(vals.reshape(-1), grid).reshape(shape)
    assert np.allclose(got, Ct, atol=1e-12)
    back = O.idct_grid(Ct.reshape(-1), grid).reshape(shape)
    assert np.allclose(back, vals, atol=1e-12)


# --------------------------------------------------------------------------
# Supports (Sec. 2 cardinalities)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("D,d,count", [(2, 16, 153), (6, 12, 18564), (12, 10, 646646),
                                       (20, 4, 10626), (3, 5, 56)])
def test_total_degree_counts(D, d, count):
    S = W.total_degree_support(D, d)
    assert len(S) == count == math.comb(d + D, d)


def test_total_degree_support_is_the_set_in_order():
    for D, d in [(1, 5), (2, 4), (3, 3), (4, 2)]:
        S = W.total_degree_support(D, d)
        brute = [t for t in itertools.product(range(d + 1), repeat=D) if sum(t) <= d]
        assert [tuple(r) for r in S.tolist()] == brute   # product() is lexicographic


def test_euclidean_support():
    for D, d in [(2, 5.0), (3, 4.5)]:
        S = W.euclidean_degree_support(D, d)
        brute = [t for t in itertools.product(range(int(d) + 1), repeat=D)
                 if sum(v * v for v in t) <= d * d]
        assert [tuple(r) for r in S.tolist()] == brute


# --------------------------------------------------------------------------
# The operator A and the plan
# --------------------------------------------------------------------------

def _chebval_nd(support, coeffs, grid):
    """Samples of sum_n c_n T_n on a tensor grid via numpy's chebval."""
    xs = [O.lobatto_nodes(int(g)) for g in grid]
    mesh = np.meshgrid(*xs, indexing="ij")
    out = np.zeros(mesh[0].shape)
    for j, n in enumerate(np.asarray(support)):
        term = np.full(mesh[0].shape, float(coeffs[j]))
        for i, ni in enumerate(n):
            e = np.zeros(int(ni) + 1); e[int(ni)] = 1
            term = term * npc.chebval(mesh[i], e)
        out += term
    return out.reshape(-1)


def test_A_columns_from_definition():
    """Each column of A^(l) is the DCT of T_n's samples (Sec. 3.1, b = A c = F p):
    transform the samples of one basis polynomial and read where the 1 lands."""
    S = W.total_degree_support(3, 6)
    grids = np.array([[2, 3, 1], [4, 0, 2], [3, 5, 4]], dtype=np.int32)
    plan = O.build_plan(S, grids)
    for l, g in enumerate(grids):
        for j in range(len(S)):
            e = np.zeros(len(S)); e[j] = 1
            t = O.dct_grid(_chebval_nd(S, e, g), g)
            nz = np.flatnonzero(np.abs(t) > 1e-9)
            assert nz.tolist() == [plan.alias[l, j]]
            assert abs(t[nz[0]] - 1) < 1e-12


def test_operator_identity_planted():
    """P3: A c = F f for f = sum c_n T_n sampled by brute force."""
    for prob in [W.config1(), W.small_problem(3, 3, 7, 1, 6, 5),
                 W.small_problem(4, 4, 5, 0, 4, 6)]:
        plan = O.build_plan(prob.support, prob.grids)
        samples = O.sample_problem(prob)
        trans = [O.dct_grid(samples[l], prob.grids[l]) for l in range(prob.K)]
        b = O.rhs_from_transforms(plan, trans)
        A = O.dense_A(plan)
        assert np.allclose(A @ prob.coeffs, b, atol=1e-12)
        # empty bins carry nothing
        for l in range(prob.K):
            empty = np.setdiff1d(np.arange(plan.points[l]), plan.alias[l])
            assert np.allclose(trans[l][empty], 0, atol=1e-12)


def test_planted_sampler_matches_numpy():
    prob = W.small_problem(5, 3, 5, 1, 5, 2)
    for g in prob.grids:
        assert np.allclose(O.sample_planted(prob.support, prob.coeffs, g),
                           _chebval_nd(prob.support, prob.coeffs, g), atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_invariants(seed):
    """P10: one 1 per column per grid; rows sorted by (bin, position);
    segment lengths sum to n per grid; M_l <= min(P_l, n)."""
    prob = W.small_problem(seed, 4, 6, 0, 5, 5)
    plan = O.build_plan(prob.support, prob.grids)
    A = O.dense_A(plan)
    assert np.all(A.sum(axis=0) == plan.K)
    n = plan.n
    flat = plan.perm.reshape(-1)
    for l in range(plan.K):
        r0, r1 = plan.rows_of_grid(l)
        assert r1 - r0 <= min(plan.points[l], n)
        keys = [(plan.alias[l, j], j) for j in plan.perm[l]]
        assert all(keys[i] < keys[i + 1] for i in range(n - 1))
        assert plan.seg_off[r0] == l * n
        assert np.all(np.diff(plan.bin_id[r0:r1]) > 0)
        for r in range(r0, r1):
            js = flat[plan.seg_off[r]:plan.seg_off[r + 1]]
            assert len(js) > 0
            assert np.all(plan.alias[l, js] == plan.bin_id[r])
            assert np.all(plan.rowmap[l, js] == r)
    assert plan.seg_off[-1] == plan.K * n
    assert np.all(A[plan.rowmap[0], np.arange(n)] == 1)


# --------------------------------------------------------------------------
# Least squares and recovery (Sec. 3.4, Alg. 3)
# --------------------------------------------------------------------------

def test_exact_recovery_config1():
    """P4: a planted polynomial on the support is recovered exactly."""
    prob = W.config1()
    c, plan, _ = O.fct_solve(prob.support, prob.grids, O.sample_problem(prob), "qr")
    assert O.max_rel_err(c, prob.coeffs) < 1e-13
    full, kappa = O.rank_check(plan)
    assert full and kappa < 1e4


@pytest.mark.parametrize("args", [(11, 3, 8, 2, 7, 6), (12, 5, 5, 0, 5, 12)])
def test_exact_recovery_small(args):
    prob = W.small_problem(*args)
    plan = O.build_plan(prob.support, prob.grids)
    assert O.rank_check(plan)[0]
    for method in ("qr", "normal"):
        c, _, _ = O.fct_solve(prob.support, prob.grids, O.sample_problem(prob), method)
        assert O.max_rel_err(c, prob.coeffs) < 1e-12


def test_sample_space_least_squares_agrees():
    """P7: least squares on B_ij = T_n_j(x_i) (no DCT, no aliasing) gives the
    same coefficients for a polynomial on the support."""
    prob = W.config1()
    Bs, fs = [], []
    for g in prob.grids:
        xs = [O.lobatto_nodes(int(v)) for v in g]
        X = np.stack([m.reshape(-1) for m in np.meshgrid(*xs, indexing="ij")], axis=1)
        V0 = npc.chebvander(X[:, 0], 16)
        V1 = npc.chebvander(X[:, 1], 16)
        Bs.append(V0[:, prob.support[:, 0]] * V1[:, prob.support[:, 1]])
        fs.append(_chebval_nd(prob.support, prob.coeffs, g))
    B, f = np.vstack(Bs), np.concatenate(fs)
    cB = np.linalg.lstsq(B, f, rcond=None)[0]
    c, _, _ = O.fct_solve(prob.support, prob.grids, O.sample_problem(prob), "qr")
    assert np.allclose(cB, prob.coeffs, atol=1e-12)
    assert np.allclose(c, cB, atol=1e-12)


def test_least_squares_methods_agree_inconsistent():
    """For f outside the span (exp-cos), QR, normal equations and LAPACK's
    SVD-based lstsq on the explicit A give one minimiser, and the normal
    residual A^T(b - A c) vanishes there."""
    prob = W.small_problem(21, 3, 7, 2, 6, 6, W.FAMILY_EXPCOS)
    samples = O.sample_problem(prob)
    c_qr, plan, b = O.fct_solve(prob.support, prob.grids, samples, "qr")
    c_ne, _, _ = O.fct_solve(prob.support, prob.grids, samples, "normal")
    c_sv = np.linalg.lstsq(O.dense_A(plan), b, rcond=None)[0]
    assert O.max_rel_err(c_qr, c_sv) < 1e-12
    assert O.max_rel_err(c_ne, c_sv) < 1e-12
    c_ls, _, _ = O.lstsq_lsqr(plan, b)
    assert O.max_rel_err(c_ls, c_sv) < 1e-10
    assert np.abs(O.normal_residual(plan, b, c_qr)).max() < 1e-13 * np.abs(b).max()
    # the system is inconsistent: the residual itself is not zero
    assert np.linalg.norm(b - O.dense_A(plan) @ c_qr) > 1e-8


def test_certificate_bound():
    """P8: ||c - c*||_2 <= ||A^T(b - A c)||_2 / sigma_min(A)^2 for any c, and
    A^T A is the integer collision-count matrix with diagonal K."""
    prob = W.small_problem(22, 3, 6, 2, 6, 6, W.FAMILY_EXPCOS)
    assert O.rank_check(O.build_plan(prob.support, prob.grids))[0]
    c_star, plan, b = O.fct_solve(prob.support, prob.grids, O.sample_problem(prob), "qr")
    G = O.gram_matrix(plan)
    assert np.all(G == np.round(G)) and np.all(np.diag(G) == plan.K)
    smin2 = np.linalg.eigvalsh(G)[0]
    rng = np.random.default_rng(3)
    for scale in [1e-2, 1e-6]:
        c = c_star + scale * rng.standard_normal(plan.n)
        bound = np.linalg.norm(O.normal_residual(plan, b, c)) / smin2
        assert np.linalg.norm(c - c_star) <= bound * (1 + 1e-9)


def test_rank_deficient_detected():
    """Two copies of one grid alias degrees 0 and 2N together: rank deficient."""
    S = W.total_degree_support(2, 6)
    plan = O.build_plan(S, np.array([[3, 3], [3, 3]], dtype=np.int32))
    assert not O.rank_check(plan)[0]
    assert not O.fold_injective(S, [[3, 3], [3, 3]])


def test_config2_instance_full_rank():
    prob = W.config2()
    assert prob.n == 18564 and prob.K == W.CFG2_MIN_GRIDS
    assert prob.total_points >= 2 * prob.n
    plan = O.build_plan(prob.support, prob.grids)
    assert O.fold_injective(prob.support, prob.grids)
    full, kappa = O.rank_check(plan)
    assert full and kappa < 1e4


@pytest.mark.slow
def test_config2_normal_equations_match_qr_golden():
    """The normal-equation route reproduces the stored QR minimiser."""
    path = os.path.join(GOLDEN, "cfg2_coeffs_qr.npy")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    c_qr = np.load(path)
    prob = W.config2()
    c_ne, plan, b = O.fct_solve(prob.support, prob.grids, O.sample_problem(prob), "normal")
    assert O.max_rel_err(c_ne, c_qr) < 1e-11
    with open(os.path.join(GOLDEN, "cfg2_meta.json")) as fh:
        meta = json.load(fh)
    assert meta["grids"] == prob.grids.tolist() and meta["M"] == plan.M


def test_error_measures():
    assert O.max_rel_err([1.0, 2.0], [1.0, 2.0]) == 0.0
    assert abs(O.max_rel_err([1.0, 2.5], [1.0, 2.0]) - 0.25) < 1e-15
    assert abs(O.mean_l2_err([3.0, 4.0], [0.0, 0.0]) - 2.5) < 1e-15


def test_analytic_families_special_points():
    """Values at the grid corner x = (1,..,1) and, for odd degrees, x = 0."""
    D = 3
    a = np.array([0.3, 0.5, 0.7]); w = np.array([0.6, 1.1, 1.9])
    f1 = O.sample_function(1, np.concatenate([a, w]), [2, 2, 2])
    # node (0,0,0) is x = (1,1,1); node (1,1,1) is x = (0,0,0)
    assert abs(f1[0] - math.exp(-a.sum()) * math.cos(w.sum())) < 1e-15
    assert abs(f1[1 * 9 + 1 * 3 + 1] - 1.0) < 1e-15
    f3 = O.sample_function(3, [10.0], [2, 2, 2])
    assert abs(f3[0] - 1 / 31) < 1e-15 and abs(f3[13] - 1.0) < 1e-15
    f2 = O.sample_function(2, np.concatenate([[0.8], [0.1, 0.2, 0.3]]), [2, 2, 2])
    assert abs(f2[13] - math.exp(-0.14 / 1.28)) < 1e-15
    f4 = O.sample_function(4, [], [2, 2, 2])
    assert abs(f4[13] - (math.sin(3 * math.cos(3.0)) + 1.0)) < 1e-14


def test_batched_workload_instances():
    """The 256-problem batch: sizes within the cap, every problem passes the
    rank pre-check, and a sample of the small ones is full rank with
    kappa(A) <= 1e4 (Alg. 2's stopping rule)."""
    with open(os.path.join(GOLDEN, "cfg3_extra_grids.json")) as fh:
        extra = json.load(fh)["extra_grids"]
    probs = W.config3(extra_grids=extra)
    assert len(probs) == 256
    assert all(p.n <= 50_000 and 3 <= p.D <= 8 for p in probs)
    assert all(p.K >= 6 * p.D and p.total_points >= 2 * p.n for p in probs)
    assert all(O.fold_injective(p.support, p.grids) for p in probs)
    small = [p for p in probs if p.n <= 1000][:8]
    assert small
    for p in small:
        full, kappa = O.rank_check(O.build_plan(p.support, p.grids))
        assert full and kappa <= 1e4


@pytest.mark.slow
def test_batched_workload_selected_grids_recover():
    """Alg. 2 as run by tests/golden/make_cfg3_grids.py: the problem that
    needed extra grids, and one that did not, are recovered exactly by the
    oracle's LSQR (consistent system, full column rank)."""
    with open(os.path.join(GOLDEN, "cfg3_extra_grids.json")) as fh:
        extra = json.load(fh)["extra_grids"]
    probs = W.config3(extra_grids=extra)
    for i in [int(k) for k in extra][:1] + [0]:
        p = probs[i]
        plan = O.build_plan(p.support, p.grids)
        c, its, _ = O.lstsq_lsqr(plan, O.sparse_A(plan) @ p.coeffs)
        assert O.max_rel_err(c, p.coeffs) < 1e-10


def test_single_node_dimensions_null_vector():
    """prod_{i in I} (T_0 - T_1)(x_i) lies in the null space of every grid
    with a single node (degree 0) in some dimension of I: the reason the
    workloads let the oracle choose their grid counts.  Checked against A
    built from its definition; adding a grid that resolves all of I removes
    that null vector."""
    S = W.total_degree_support(4, 3)
    I = (0, 2)
    c = np.zeros(len(S))
    index = {tuple(r): j for j, r in enumerate(S.tolist())}
    for a in (0, 1):
        for b in (0, 1):
            n = [0, 0, 0, 0]
            n[I[0]], n[I[1]] = a, b
            c[index[tuple(n)]] = (-1.0) ** (a + b)        # (T_0 - T_1) x (T_0 - T_1)
    grids = np.array([[0, 5, 4, 3], [6, 2, 0, 4], [0, 3, 0, 5]], dtype=np.int32)
    A = O.dense_A(O.build_plan(S, grids))
    assert np.abs(A @ c).max() == 0.0
    # the polynomial really vanishes on those grids (brute-force samples)
    for g in grids:
        assert np.abs(O.sample_planted(S, c, g)).max() < 1e-12
    more = np.vstack([grids, [[2, 1, 3, 2]]]).astype(np.int32)
    assert np.abs(O.dense_A(O.build_plan(S, more)) @ c).max() > 0.5


def test_sampling_in_slabs_is_pointwise_identical():
    g = [3, 4, 2, 5]
    for fam, prm in [(W.FAMILY_GAUSS, np.concatenate([[0.8], np.linspace(-.3, .3, 4)])),
                     (W.FAMILY_EXPCOS, np.linspace(0.2, 1.0, 8))]:
        full = O.sample_function(fam, prm, g)
        assert np.array_equal(full, O.sample_function(fam, prm, g, chunk=7))


def test_serving_pool_small_jobs_recover():
    """The serving pool's D=2 and D=20 jobs, with the grid counts the
    oracle's Alg.-2 run stored, recover their planted coefficients (QR)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "serving_extra_grids.json")) as fh:
        fx = json.load(fh)
    pool = W.serving_pool(fx["seed"], extra_grids=fx["extra_grids"])
    for p in pool[0:8]:
        if p.family != W.FAMILY_PLANTED or p.n > 2000:
            continue
        c, _, _ = O.fct_solve(p.support, p.grids, O.sample_problem(p), "qr")
        assert O.max_rel_err(c, p.coeffs) < 1e-10, p.name
    # the D=20 L-grid covers every pair of dimensions at degree 2
    g = W.d20_grids(fx["seed"])
    assert g.shape[1] == 20 and set(np.unique(g)) <= {0, 2}
    res = [set(np.nonzero(r)[0]) for r in g]
    for a in range(20):
        for b in range(a + 1, 20):
            assert any(a in r and b in r for r in res)


# --------------------------------------------------------------------------
# Evaluation of an expansion at arbitrary points (Sec. 2 definition)
# --------------------------------------------------------------------------

def _dense_tensor(support, coeffs, D):
    S = np.asarray(support)
    shape = tuple(int(S[:, i].max()) + 1 for i in range(D))
    t = np.zeros(shape)
    for row, c in zip(S, coeffs):
        t[tuple(row)] += c
    return t


@pytest.mark.parametrize("D,d", [(1, 9), (2, 7), (3, 5)])
def test_evaluate_expansion_against_numpy_chebval(D, d):
    """numpy's Chebyshev module (Clenshaw recurrences) on the dense tensor."""
    rng = np.random.default_rng(41 + D)
    S = W.total_degree_support(D, d)
    c = rng.standard_normal(S.shape[0])
    X = rng.uniform(-1, 1, size=(37, D))
    t = _dense_tensor(S, c, D)
    ref = {1: lambda: npc.chebval(X[:, 0], t),
           2: lambda: npc.chebval2d(X[:, 0], X[:, 1], t),
           3: lambda: npc.chebval3d(X[:, 0], X[:, 1], X[:, 2], t)}[D]()
    got = O.evaluate_expansion(S, c, X, chunk=8)
    assert O.linf_error(got, ref) < 1e-13 * np.sum(np.abs(c))


def test_evaluate_expansion_cosine_closed_form():
    """T_n(cos theta) = cos(n theta): one term per coefficient, D = 6."""
    rng = np.random.default_rng(47)
    S = W.euclidean_degree_support(6, 4.5)
    theta = rng.uniform(0, np.pi, size=(11, 6))
    X = np.cos(theta)
    for j in rng.choice(S.shape[0], size=12, replace=False):
        c = np.zeros(S.shape[0])
        c[j] = 1.0
        ref = np.prod(np.cos(S[j][None, :] * theta), axis=1)
        assert O.linf_error(O.evaluate_expansion(S, c, X), ref) < 1e-13


def test_evaluate_expansion_at_nodes_obeys_aliasing():
    """Values at the nodes of a grid, transformed by the DCT-I, are A c at
    the grid's bins (the aliasing identity, eq. aliasing_matrix_nd_diff)."""
    prob = W.small_problem(49, 3, 6, 2, 5, 3)
    plan = O.build_plan(prob.support, prob.grids)
    A = O.dense_A(plan)
    transforms = []
    for g in prob.grids:
        X = np.stack(np.meshgrid(*[O.lobatto_nodes(int(N)) for N in g], indexing="ij"),
                     axis=-1).reshape(-1, 3)
        transforms.append(O.dct_grid(O.evaluate_expansion(prob.support, prob.coeffs, X), g))
    b = O.rhs_from_transforms(plan, transforms)
    assert np.max(np.abs(b - A @ prob.coeffs)) < 1e-13 * np.sum(np.abs(prob.coeffs))


def test_euclidean_support_is_the_ball():
    """S^2_{d,D} by brute force over the cube (Sec. 2)."""
    for D, d in [(2, 5.0), (3, 4.2), (5, 3.0)]:
        S = W.euclidean_degree_support(D, d)
        cube = np.array(list(itertools.product(range(int(d) + 1), repeat=D)))
        ref = cube[np.sum(cube ** 2, axis=1) <= d * d + 1e-9]
        assert np.array_equal(S, ref)       # both lexicographic


def test_workload_family_values_match_the_oracle():
    """The workloads' analytic test functions equal the oracle's (two
    independent codings of the same definitions)."""
    rng = np.random.default_rng(53)
    X = rng.uniform(-1, 1, size=(50, 4))
    for fam, prm in [(W.FAMILY_EXPCOS, rng.uniform(0.2, 2, 8)),
                     (W.FAMILY_GAUSS, np.concatenate([[0.8], rng.uniform(-.5, .5, 4)])),
                     (W.FAMILY_RUNGE, [10.0]), (W.FAMILY_OSC, [])]:
        assert np.allclose(W.family_values(fam, prm, X), O.function_values(fam, prm, X),
                           rtol=1e-14, atol=1e-15)


def test_euclidean_workload_recovers_planted():
    """The Euclidean-degree workload's grid count makes A full rank (Alg. 2's
    stopping rule) and the oracle recovers a planted expansion exactly."""
    prob = W.euclidean_problem()
    plan = O.build_plan(prob.support, prob.grids)
    full, kappa = O.rank_check(plan)
    assert full and kappa < 1e2
    c, _, _ = O.fct_solve(prob.support, prob.grids, O.sample_problem(prob), "qr")
    assert O.max_rel_err(c, prob.coeffs) < 1e-12


def test_rank_check_kappa_is_the_svd_condition_number():
    """kappa(A) from the Gram matrix's eigenvalues equals LAPACK's SVD
    condition number of the dense A (numpy.linalg.cond)."""
    for prob in [W.config1(), W.small_problem(3, 3, 5, 2, 6, 4), W.euclidean_problem()]:
        plan = O.build_plan(prob.support, prob.grids)
        full, kappa = O.rank_check(plan)
        assert full
        assert abs(kappa / np.linalg.cond(O.dense_A(plan)) - 1.0) < 1e-8


def test_select_grid_count_is_the_first_qualifying_prefix():
    """Alg. 2 on explicit candidates: the returned L qualifies and L - 1 does
    not, checked with SVD ranks and condition numbers of the dense A."""
    S = W.total_degree_support(3, 5)
    cands = np.random.default_rng(59).integers(1, 6, size=(12, 3)).astype(np.int32)
    L, kappa = O.select_grid_count(S, cands, 1e4)
    assert L >= 2

    def svd_ok(k):
        A = O.dense_A(O.build_plan(S, cands[:k]))
        sv = np.linalg.svd(A, compute_uv=False)
        return sv[-1] > 1e-5 * sv[0] and sv[0] / sv[-1] <= 1e4
    assert svd_ok(L) and not svd_ok(L - 1)


def test_dct_entries_equal_the_full_transform():
    """Single DCT-I entries by slab-wise contraction equal the entries of the
    whole transform (dct_grid, itself pinned to scipy's DCT-I)."""
    grid = [3, 4, 2, 5]
    prm = np.concatenate([[0.8], np.random.default_rng(61).uniform(-.5, .5, 4)])
    full = O.dct_grid(O.sample_function(W.FAMILY_GAUSS, prm, grid), grid).reshape(
        [N + 1 for N in grid])
    ms = np.array([[0, 0, 0, 0], [3, 4, 2, 5], [1, 2, 0, 3], [2, 0, 1, 4]])
    vals, abss = O.dct_entries(W.FAMILY_GAUSS, prm, grid, ms, slab_points=64)
    for v, a, m in zip(vals, abss, ms):
        assert abs(v - full[tuple(m)]) <= 1e-14 * a
        assert a >= abs(v)
    whole, _ = O.dct_entries(W.FAMILY_GAUSS, prm, grid, ms)        # one slab
    assert np.allclose(whole, vals, rtol=0, atol=1e-14 * np.max(abss))


def test_single_node_axes_dropped_from_tensors():
    """Samples and transforms on a grid with single-node axes (N = 0, the
    node x = 1) equal the expansion evaluated at the nodes and the DCT taken
    over every axis of the full-rank tensor."""
    rng = np.random.default_rng(67)
    S = W.total_degree_support(5, 3)
    c = rng.standard_normal(S.shape[0])
    grid = [3, 0, 2, 0, 1]
    X = np.stack(np.meshgrid(*[O.lobatto_nodes(N) for N in grid], indexing="ij"),
                 axis=-1).reshape(-1, 5)
    smp = O.sample_planted(S, c, grid)
    assert np.max(np.abs(smp - O.evaluate_expansion(S, c, X))) < 1e-13 * np.abs(c).sum()
    t = smp.reshape([N + 1 for N in grid])
    for axis, N in enumerate(grid):
        t = O.dct_axis(t, axis, O.dct1_matrix(N))
    assert np.allclose(O.dct_grid(smp, grid), t.reshape(-1), rtol=0, atol=1e-15)


@pytest.mark.slow
def test_f3_sparse_support_recovers_exactly():
    """The paper's f3 family in D = 100 (N = 2000 random multi-indices of
    S^inf_{8,100}, 20 Alg.-1 grids): the oracle recovers the planted
    coefficients (so A has full column rank)."""
    p = W.f3_problem(2000)
    assert p.D == 100 and len(np.unique(p.support, axis=0)) == p.n
    c, plan, _ = O.fct_solve(p.support, p.grids, O.sample_problem(p), "auto")
    assert O.max_rel_err(c, p.coeffs) < 1e-12


@pytest.mark.parametrize("d", [2, 3, 4])
def test_d20_cover_resolves_every_d_set(d):
    """The D=20 grid covers used by the serving and long-row workloads
    resolve every set of d dimensions in some grid (degree d there)."""
    from itertools import combinations
    G = W.d20_grids(4, d, 8)
    resolved = [frozenset(np.nonzero(g)[0].tolist()) for g in G]
    assert all(int(v) in (0, d) for v in np.unique(G))
    for c in combinations(range(20), d):
        assert any(set(c) <= r for r in resolved)
