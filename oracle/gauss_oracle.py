"""CPU FP64 oracle for the paper's literal operator: Chebyshev-Gauss grids
and the DCT-II.

TEST INFRASTRUCTURE.  Like the Lobatto oracle beside it, this module is a
plain, slow reference that the GPU path is checked against; only the test
suite, the package smoke check and the benchmark's CPU-baseline leg may
import it, and it imports nothing from the library.

It follows Sec. 2 ("Problem setup") and Sec. 3.1 of arXiv 2309.14584 as
printed:

* nodes x_k = cos(theta_k), theta_k = (k + 1/2) pi / (N + 1), k = 0..N
  (eq. chebyshev_grid);
* the 1-D transform is the quadrature b_n = (1/(N+1)) sum_k cos(n theta_k)
  p(x_k), n = 0..N (eq. quad_1D), i.e. a DCT-II;
* Lemma 3.1: the quadrature of cos(n theta) cos(m theta) equals
  Delta_N(m + n)/2 + Delta_N(m - n)/2 with Delta_N(l) = 1 when
  l = 0 mod 4(N+1), -1 when l = 2(N+1) mod 4(N+1), and 0 otherwise
  (eq. aliasing_delta), so the 1-D aliasing matrix has entries
  A_{n,m} = Delta_N(m+n)/2 + Delta_N(m-n)/2 (eq. aliasing_matrix_1d);
* multi-dimensional entries are products of 1-D entries over the axes
  (eq. aliasing_matrix_nd_diff), and the L grids stack (eq.
  main_linear_system); the result is argmin_c ||F f - A c||_2 (Alg. 3).

One reading is taken (the same as for the Lobatto form): rows are
interpolation-normalised, i.e. row n >= 1 of the 1-D quadrature and of the
1-D aliasing matrix is multiplied by 2, so that the samples of T_m, m <= N,
map to the unit vector e_m and every entry of A lies in {-1, 0, 1}.  The
scaling multiplies b and A by the same diagonal, so it changes the
least-squares weighting only when f is not in the span of the support.

Every function is written from these definitions; numpy's tensordot and
LAPACK's QR (numpy.linalg) are the only library steps.
"""
from __future__ import annotations

import numpy as np

from .fct_oracle import cheb_T_recurrence, _function_at

__all__ = [
    "gauss_nodes", "delta", "quadrature_matrix", "aliasing_matrix_1d", "row_scale",
    "dct2_matrix", "dct2_eval_matrix", "dct2_grid", "signed_alias", "dense_A_gauss",
    "grid_coordinates_gauss", "sample_planted_gauss", "sample_function_gauss",
    "sample_problem_gauss", "solve_gauss", "rank_precheck_gauss",
]


def gauss_nodes(N: int) -> np.ndarray:
    """x_k = cos((k + 1/2) pi / (N + 1)), k = 0..N (eq. chebyshev_grid)."""
    k = np.arange(N + 1)
    return np.cos((k + 0.5) * np.pi / (N + 1))


def delta(l: int, N: int) -> int:
    """Delta_N(l) of Lemma 3.1 (eq. aliasing_delta), plain integers."""
    r = l % (4 * (N + 1))
    if r == 0:
        return 1
    if r == 2 * (N + 1):
        return -1
    return 0


def quadrature_matrix(N: int) -> np.ndarray:
    """The paper's 1-D transform (eq. quad_1D): F[n, k] = cos(n theta_k)/(N+1)."""
    n = np.arange(N + 1)[:, None]
    k = np.arange(N + 1)[None, :]
    return np.cos(n * (k + 0.5) * np.pi / (N + 1)) / (N + 1)


def aliasing_matrix_1d(N: int, nmax: int) -> np.ndarray:
    """The paper's 1-D aliasing matrix (eq. aliasing_matrix_1d), rows n = 0..N,
    columns m = 0..nmax: A[n, m] = Delta_N(m + n)/2 + Delta_N(m - n)/2."""
    A = np.zeros((N + 1, nmax + 1))
    for n in range(N + 1):
        for m in range(nmax + 1):
            A[n, m] = 0.5 * delta(m + n, N) + 0.5 * delta(m - n, N)
    return A


def row_scale(N: int) -> np.ndarray:
    """Interpolation normalisation of the 1-D rows: 1 for n = 0, 2 otherwise."""
    s = np.full(N + 1, 2.0)
    s[0] = 1.0
    return s


def dct2_matrix(N: int) -> np.ndarray:
    """Interpolation-normalised DCT-II: row-scaled quadrature matrix."""
    return row_scale(N)[:, None] * quadrature_matrix(N)


def dct2_eval_matrix(N: int) -> np.ndarray:
    """E[k, m] = T_m(x_k) = cos(m theta_k), m, k = 0..N."""
    k = np.arange(N + 1)[:, None]
    m = np.arange(N + 1)[None, :]
    return np.cos(m * (k + 0.5) * np.pi / (N + 1))


def dct2_grid(samples: np.ndarray, grid) -> np.ndarray:
    """Separable D-dim transform of one grid's flat row-major samples.
    A single-node axis (N = 0) has the 1x1 matrix [1] and is skipped."""
    axes = [int(v) for v in grid if int(v) > 0]
    t = np.asarray(samples, dtype=np.float64).reshape(tuple(v + 1 for v in axes))
    for axis, N in enumerate(axes):
        t = np.moveaxis(np.tensordot(dct2_matrix(N), t, axes=([1], [axis])), 0, axis)
    return t.reshape(-1)


def _strides(grid) -> list[int]:
    ext = [int(v) + 1 for v in grid]
    st = [1] * len(ext)
    for i in range(len(ext) - 2, -1, -1):
        st[i] = st[i + 1] * ext[i + 1]
    return st


def signed_alias(support, grid):
    """Flat bin and weight of every support multi-index on one grid.

    Column n_i of the row-scaled 1-D aliasing matrix holds at most one
    nonzero, +-1, at row m_i (or is zero: the vanishing T_{N+1}); the
    D-dim entry is the product over the axes.  Returns (bins int64 [n],
    weights int8 [n]) with bin -1 where the weight is 0.
    """
    S = np.asarray(support, dtype=np.int64)
    grid = [int(v) for v in grid]
    st = _strides(grid)
    nmax = int(S.max()) if S.size else 0
    cols = []
    for N in grid:
        A1 = row_scale(N)[:, None] * aliasing_matrix_1d(N, nmax)
        row = np.full(nmax + 1, -1, dtype=np.int64)
        sgn = np.zeros(nmax + 1, dtype=np.int64)
        for m in range(nmax + 1):
            nz = np.nonzero(A1[:, m])[0]
            assert nz.size <= 1 and np.all(np.abs(A1[nz, m]) == 1.0)
            if nz.size == 1:
                row[m], sgn[m] = nz[0], int(A1[nz[0], m])
        cols.append((row, sgn))
    bins = np.zeros(S.shape[0], dtype=np.int64)
    w = np.ones(S.shape[0], dtype=np.int64)
    for i, (row, sgn) in enumerate(cols):
        bins += np.where(row[S[:, i]] >= 0, row[S[:, i]], 0) * st[i]
        w *= sgn[S[:, i]]
    bins[w == 0] = -1
    return bins, w.astype(np.int8)


def dense_A_gauss(support, grids) -> np.ndarray:
    """Stacked A over every bin of every grid (sum of P_l rows; rows whose
    bins hold no support entry are zero and do not change the minimiser)."""
    S = np.asarray(support, dtype=np.int64)
    blocks = []
    for g in np.asarray(grids, dtype=np.int64):
        P = int(np.prod(g + 1))
        bins, w = signed_alias(S, g)
        A = np.zeros((P, S.shape[0]))
        j = np.nonzero(w)[0]
        A[bins[j], j] = w[j]
        blocks.append(A)
    return np.vstack(blocks)


def grid_coordinates_gauss(grid) -> np.ndarray:
    """Coordinates [P, D] of one Gauss grid's points, row-major."""
    axes = [gauss_nodes(int(N)) for N in grid]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def sample_planted_gauss(support, coeffs, grid) -> np.ndarray:
    """Brute-force samples of sum_n c_n prod_i T_{n_i}(x_i) at the Gauss
    nodes (three-term recurrence; no transform, no aliasing).  A single-node
    axis has the node x = 0, where T_n(0) = cos(n pi / 2) is not constant."""
    S = np.asarray(support, dtype=np.int64)
    grid = [int(v) for v in grid]
    nmax = int(S.max()) if S.size else 0
    tables = [cheb_T_recurrence(nmax, gauss_nodes(N)) for N in grid]
    out = np.zeros(tuple(N + 1 for N in grid))
    for j in range(S.shape[0]):
        term = np.asarray(coeffs[j], dtype=np.float64)
        for i in range(len(grid)):
            term = np.multiply.outer(term, tables[i][S[j, i]])
        out += term
    return out.reshape(-1)


def sample_function_gauss(family: int, params, grid) -> np.ndarray:
    """Samples of an analytic test family (the Lobatto oracle's formulas)
    at the Gauss grid's points."""
    return _function_at(family, params, grid_coordinates_gauss(grid))


def sample_problem_gauss(prob) -> list[np.ndarray]:
    out = []
    for g in prob.grids:
        if prob.family == 0:
            out.append(sample_planted_gauss(prob.support, prob.coeffs, g))
        else:
            out.append(sample_function_gauss(prob.family, prob.params, g))
    return out


def solve_gauss(support, grids, samples):
    """argmin_c ||F f - A c||_2 over the stacked grids by Householder QR.
    Returns (c, b) with b the stacked full transforms."""
    b = np.concatenate([dct2_grid(s, g) for s, g in zip(samples, grids)])
    A = dense_A_gauss(support, grids)
    Q, R = np.linalg.qr(A)
    c = np.linalg.solve(R, Q.T @ b)
    return c, b


def rank_precheck_gauss(support, grids) -> bool:
    """Necessary condition for full column rank: per dimension, the columns
    a e_i (a = 0..max degree) restricted to that axis, i.e. the vectors of
    signed 1-D rows over the grids, are nonzero and pairwise independent
    (no two equal up to sign)."""
    S = np.asarray(support, dtype=np.int64)
    G = np.asarray(grids, dtype=np.int64)
    for i in range(S.shape[1]):
        amax = int(S[:, i].max())
        seen = set()
        for a in range(amax + 1):
            key = []
            for l in range(G.shape[0]):
                N = int(G[l, i])
                col = row_scale(N) * aliasing_matrix_1d(N, a)[:, a]
                nz = np.nonzero(col)[0]
                key.append(0 if nz.size == 0 else int(col[nz[0]]) * (int(nz[0]) + 1))
            if all(v == 0 for v in key):
                return False
            first = next(v for v in key if v != 0)
            key = tuple(v if first > 0 else -v for v in key)
            if key in seen:
                return False
            seen.add(key)
    return True
