"""Pins of the Gauss-grid / DCT-II oracle against what the paper and the
mathematics fix (no GPU):

* Lemma 3.1 by brute-force quadrature sums (pins Delta_N and its period);
* the transform against scipy's DCT-II (library routine);
* interpolation: samples of T_j, j <= N, map to e_j (closed form);
* b = F p = A c (Sec. 3.1): the transform of the samples of every T_n,
  n up to several periods, equals column n of the row-scaled aliasing
  matrix; the vanishing T_{N+1} gives a zero column;
* hand-derived sign and fold values for a few degrees;
* a planted polynomial is recovered exactly by the stacked least squares.
"""
import numpy as np
import pytest
import scipy.fft

from oracle import gauss_oracle as G
from oracle import fct_oracle as O
import workloads as W


@pytest.mark.parametrize("N", range(0, 8))
def test_lemma_3_1_by_brute_force(N):
    th = (np.arange(N + 1) + 0.5) * np.pi / (N + 1)
    for n in range(6 * (N + 1)):
        for m in range(6 * (N + 1)):
            q = np.mean(np.cos(n * th) * np.cos(m * th))
            assert abs(q - (0.5 * G.delta(m + n, N) + 0.5 * G.delta(m - n, N))) < 1e-13


def test_delta_values():
    # N = 2: period 12, +1 at 0, -1 at 6
    assert [G.delta(l, 2) for l in (0, 6, 12, 18, -6, 3, 1)] == [1, -1, 1, -1, -1, 0, 0]


@pytest.mark.parametrize("N", [0, 1, 2, 5, 9, 24])
def test_transform_against_scipy_dct2(N):
    v = np.random.default_rng(N).standard_normal(N + 1)
    y = scipy.fft.dct(v, type=2)          # y_m = 2 sum_k v_k cos(pi m (2k+1) / (2(N+1)))
    ref = y / (N + 1)
    ref[0] /= 2.0
    assert np.max(np.abs(G.dct2_matrix(N) @ v - ref)) < 1e-13


@pytest.mark.parametrize("N", [0, 1, 3, 8, 17])
def test_interpolation_closed_form(N):
    x = G.gauss_nodes(N)
    T = O.cheb_T_recurrence(N, x)
    assert np.max(np.abs(G.dct2_matrix(N) @ T.T - np.eye(N + 1))) < 1e-13
    assert np.max(np.abs(G.dct2_eval_matrix(N) - T.T)) < 1e-13


@pytest.mark.parametrize("N", [0, 1, 2, 4, 7])
def test_b_equals_Ac_equals_Fp(N):
    nmax = 5 * (N + 1)
    x = G.gauss_nodes(N)
    T = O.cheb_T_recurrence(nmax, x)
    A = G.row_scale(N)[:, None] * G.aliasing_matrix_1d(N, nmax)
    F = G.dct2_matrix(N)
    assert np.max(np.abs(F @ T.T - A)) < 1e-12
    # the vanishing T_{N+1} (and T_{3(N+1)}): zero samples, zero column
    for n in (N + 1, 3 * (N + 1)):
        assert np.max(np.abs(T[n])) < 1e-12 and not np.any(A[:, n])
    # entries in {-1, 0, 1}, at most one per column
    assert set(np.unique(A)) <= {-1.0, 0.0, 1.0}
    assert np.all(np.count_nonzero(A, axis=0) <= 1)


def test_hand_derived_aliases():
    # N = 2 (3 nodes, period 6 up to sign): T_5 = -T_1, T_4 = -T_2, T_6 = -T_0,
    # T_7 = -T_1, T_3 = 0, T_8 = -T_2 ... n = 6j + r: sign (-1)^j for r <= 3,
    # (-1)^(j+1) and m = 6 - r for r > 3
    S = np.array([[0], [1], [3], [4], [5], [6], [7], [12], [13]])
    bins, w = G.signed_alias(S, [2])
    assert bins.tolist() == [0, 1, -1, 2, 1, 0, 1, 0, 1]
    assert w.tolist() == [1, 1, 0, -1, -1, -1, -1, 1, 1]


def test_multidim_entries_are_products():
    rng = np.random.default_rng(3)
    S = W.total_degree_support(3, 7)
    grid = [2, 3, 1]
    bins, w = G.signed_alias(S, grid)
    for j in rng.choice(S.shape[0], size=25, replace=False):
        c = np.zeros(S.shape[0])
        c[j] = 1.0
        t = G.dct2_grid(G.sample_planted_gauss(S, c, grid), grid)
        ref = np.zeros_like(t)
        if w[j] != 0:
            ref[bins[j]] = w[j]
        assert np.max(np.abs(t - ref)) < 1e-12


@pytest.mark.parametrize("args", [(22, 2, 10, 6, 12, 5), (3, 3, 6, 2, 8, 6)])
def test_planted_recovery_exact(args):
    prob = W.small_problem(*args)
    assert G.rank_precheck_gauss(prob.support, prob.grids)
    samples = G.sample_problem_gauss(prob)
    c, _ = G.solve_gauss(prob.support, prob.grids, samples)
    assert O.max_rel_err(c, prob.coeffs) < 1e-12


def test_rank_deficient_instance_passes_precheck():
    # the per-dimension pre-check is necessary only: this D=2 instance
    # passes it and still has a rank-65 A for 66 coefficients
    prob = W.small_problem(21, 2, 10, 4, 9, 4)
    assert G.rank_precheck_gauss(prob.support, prob.grids)
    assert np.linalg.matrix_rank(G.dense_A_gauss(prob.support, prob.grids)) == 65


def test_rank_precheck_detects_dependent_columns():
    S = np.arange(4)[:, None]
    # N = 1 on every grid: T_2 vanishes and T_3 = -T_1
    assert not G.rank_precheck_gauss(S, [[1], [1]])
    # T_{N+1} vanishes on every grid -> zero column
    assert not G.rank_precheck_gauss(np.array([[0], [3]]), [[2], [2]])
    assert G.rank_precheck_gauss(S, [[3]])


@pytest.mark.parametrize("N", [0, 1, 2, 3, 6, 11])
def test_signed_fold_rule_matches_lemma(N):
    """The closed fold-and-sign rule (r = a mod 2(N+1), m = min(r, 2(N+1) - r),
    sign (-1)^(a div 2(N+1)) for r < N+1, its negation for r > N+1, zero at
    r = N+1) against the Delta-based aliasing matrix of Lemma 3.1."""
    g = N + 1
    S = np.arange(0, 9 * g + 3)[:, None]
    bins, w = G.signed_alias(S, [N])
    for a in range(S.shape[0]):
        r = a % (2 * g)
        odd = (a // (2 * g)) % 2
        if r == g:
            assert w[a] == 0
            continue
        m = r if r < g else 2 * g - r
        s = (-1 if odd else 1) if r < g else (1 if odd else -1)
        assert bins[a] == m and w[a] == s
