"""CPU FP64 oracle for the sparse Fast Chebyshev Transform hot path.

TEST INFRASTRUCTURE.  This module is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only the test suite, the
package smoke check and the benchmark's CPU-baseline leg may import it; the
library itself never does, and this module imports nothing from the library.

It follows "A (Sparse) Fast Chebyshev Transform for High-Dimensional
(Smooth Function) Approximation" (Jones, Letourneau, Morse, Langston,
arXiv 2309.14584) in the Chebyshev-Lobatto form:

* grid nodes x_k = cos(pi k / N), k = 0..N, on each dimension (the
  second-kind analogue of the grid of Sec. 2, "Problem setup");
* the per-axis transform is the interpolation-normalised DCT-I, under which
  the samples of T_n map to the unit vector of the aliased index (the
  Lobatto analogue of Lemma 3.1 and of the 1-D relation b = A c = F p of
  Sec. 3.1);
* the aliasing fold is r = n mod 2N, m = min(r, 2N - r) (N = 0: m = 0), so
  each block A^(l) of the stacked system (eq. main_linear_system, Sec. 3) is
  0/1 with exactly one 1 per column, and the multi-dimensional entry is the
  product of 1-D entries (eq. aliasing_matrix_nd_diff, Sec. 3.1);
* the result is c* = argmin_c || F f - A c ||_2 (Sec. 3.4, Alg. 3), computed
  by dense Householder QR (or, for large supports, the normal equations with
  the exact integer Gram matrix and a Cholesky factorisation).

Readings of the paper taken here (Gauss grid -> Lobatto grid, the
normalisation, empty rows, row order, flattening order, the error measure)
are listed in the design notes of the repository.

Every function is written from the definitions; library primitives used as
steps are numpy's matmul/tensordot, numpy/LAPACK QR, triangular and
Cholesky solves, and scipy.sparse products.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "fold", "fold_array", "lobatto_nodes", "cheb_T", "cheb_T_recurrence",
    "dct1_matrix", "dct1_eval_matrix", "dct_axis", "dct_grid",
    "idct_grid", "alias_bins", "build_plan", "Plan", "sample_planted",
    "sample_function", "sample_problem", "rhs_from_transforms",
    "dense_A", "sparse_A", "lstsq_qr", "lstsq_normal", "rank_check",
    "gram_matrix", "normal_residual", "fct_solve", "max_rel_err", "lstsq_lsqr",
    "mean_l2_err", "fold_injective", "evaluate_expansion", "linf_error",
    "function_values", "select_grid_count", "dct_entries", "grid_coordinates",
]


# ---------------------------------------------------------------------------
# Aliasing (Sec. 3.1, Lemma 3.1; Lobatto analogue)
# ---------------------------------------------------------------------------

def fold(n: int, N: int) -> int:
    """Aliased index of T_n on the (N+1)-node Lobatto grid.

    cos(n pi k / N) depends on n only through n mod 2N and is unchanged by
    n -> 2N - n, so T_n equals T_m on the grid with m = min(r, 2N - r),
    r = n mod 2N.  A single node (N = 0, x = 1) sees every T_n as T_0.
    Plain Python integers.
    """
    if N < 0 or n < 0:
        raise ValueError("fold needs n >= 0 and N >= 0")
    if N == 0:
        return 0
    r = n % (2 * N)
    return min(r, 2 * N - r)


def fold_array(n, N: int) -> np.ndarray:
    """Vectorised fold over an int64 array of degrees (same rule as fold)."""
    n = np.asarray(n, dtype=np.int64)
    if N == 0:
        return np.zeros_like(n)
    r = np.mod(n, 2 * N)
    return np.minimum(r, 2 * N - r)


def fold_injective(support, grids) -> bool:
    """Necessary condition for full column rank on a downward-closed support.

    For each dimension i, the map a -> (fold(a, N_i^(l)))_l over the degrees
    a = 0..max_n n_i must be one-to-one; otherwise two coefficients differing
    only in entry i alias together on every grid.
    """
    S = np.asarray(support, dtype=np.int64)
    G = np.asarray(grids, dtype=np.int64)
    for i in range(S.shape[1]):
        seen = set()
        for a in range(int(S[:, i].max()) + 1):
            key = tuple(fold(a, int(G[l, i])) for l in range(G.shape[0]))
            if key in seen:
                return False
            seen.add(key)
    return True


# ---------------------------------------------------------------------------
# Chebyshev polynomials and nodes (Sec. 2)
# ---------------------------------------------------------------------------

def lobatto_nodes(N: int) -> np.ndarray:
    """x_k = cos(pi k / N), k = 0..N; the single node x = 1 when N = 0."""
    if N == 0:
        return np.ones(1)
    return np.cos(np.pi * np.arange(N + 1) / N)


def cheb_T(n: int, x) -> np.ndarray:
    """T_n(x) = cos(n arccos x) (Sec. 2, definition)."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    return np.cos(n * np.arccos(x))


def cheb_T_recurrence(nmax: int, x) -> np.ndarray:
    """[T_0(x), ..., T_nmax(x)] from T_{n+1} = 2x T_n - T_{n-1} (Sec. 2)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((nmax + 1,) + x.shape)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = x
    for n in range(1, nmax):
        out[n + 1] = 2.0 * x * out[n] - out[n - 1]
    return out


# ---------------------------------------------------------------------------
# DCT-I (Sec. 2 change of variables; Sec. 3.1 b = A c = F p)
# ---------------------------------------------------------------------------

def _cos_pi_ratio(num: np.ndarray, N: int) -> np.ndarray:
    """cos(pi * num / N) with num reduced modulo 2N in integers first."""
    return np.cos(np.pi * (np.mod(num, 2 * N)) / N)


def dct1_matrix(N: int) -> np.ndarray:
    """Interpolation-normalised DCT-I matrix C (size (N+1) x (N+1)).

    a_m = (g_m / N) [v_0 + (-1)^m v_N + 2 sum_{k=1}^{N-1} v_k cos(pi m k / N)],
    g_0 = g_N = 1/2, g_m = 1 otherwise.  With v_k = T_j(x_k) this gives
    a_m = delta_{mj} for 0 <= j <= N (discrete orthogonality of cosines on
    the Lobatto grid), so C maps grid samples to interpolation coefficients.
    N = 0 is the 1x1 identity.
    """
    if N == 0:
        return np.ones((1, 1))
    m = np.arange(N + 1)[:, None]
    k = np.arange(N + 1)[None, :]
    w = np.full(N + 1, 2.0)
    w[0] = w[N] = 1.0
    g = np.ones(N + 1)
    g[0] = g[N] = 0.5
    return (g[:, None] / N) * w[None, :] * _cos_pi_ratio(m * k, N)


def dct1_eval_matrix(N: int) -> np.ndarray:
    """Evaluation matrix E[k, m] = T_m(x_k) = cos(pi m k / N): inverse of C."""
    if N == 0:
        return np.ones((1, 1))
    k = np.arange(N + 1)[:, None]
    m = np.arange(N + 1)[None, :]
    return _cos_pi_ratio(m * k, N)


def dct_axis(t: np.ndarray, axis: int, Mat: np.ndarray) -> np.ndarray:
    """Apply a square matrix along one axis of a tensor (direct sums)."""
    out = np.tensordot(Mat, t, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def dct_grid(samples: np.ndarray, grid) -> np.ndarray:
    """Separable D-dim DCT-I of one grid's samples (Sec. 3.1, eq. multi_dim_dct).

    ``samples`` is the flat row-major tensor (last dimension fastest) of
    shape (N_1+1, ..., N_D+1); the result has the same layout.
    """
    # single-node axes (N = 0) carry the 1x1 identity and do not change the
    # flat row-major layout, so the tensor is formed over the other axes only
    grid = [int(v) for v in grid if int(v) > 0]
    shape = tuple(v + 1 for v in grid)
    t = np.asarray(samples, dtype=np.float64).reshape(shape)
    for axis, N in enumerate(grid):
        t = dct_axis(t, axis, dct1_matrix(N))
    return t.reshape(-1)


def dct_entries(family: int, params, grid, multis, slab_points: int = 1 << 21):
    """Selected entries of the D-dimensional DCT-I of f sampled on one grid
    (eq. multi_dim_dct), each by its definition
        a_m = sum_k f(x_k) prod_i C_{N_i}[m_i, k_i],
    without forming the transformed tensor.  The leading axes 0..s-1 (s the
    fewest such that a slab of the trailing axes holds at most slab_points
    points) index slabs; every slab is sampled, contracted with the rows
    C_{N_i}[m_i] of the trailing axes, and weighted by the product of
    C_{N_i}[m_i, k_i] over the leading axes.  Also returns the same sums of
    absolute values (|f|, |C|), the scale of the rounding error of any
    evaluation order.  multis: int [r][D].  Returns (values [r], abs_sums [r])."""
    grid = [int(v) for v in grid]
    D = len(grid)
    ext = [N + 1 for N in grid]
    mats = [dct1_matrix(N) for N in grid]
    multis = np.asarray(multis, dtype=np.int64)
    s = 0
    while s < D and int(np.prod(ext[s:], dtype=np.int64)) > slab_points:
        s += 1
    rest = int(np.prod(ext[s:], dtype=np.int64))
    vals = np.zeros(len(multis))
    abss = np.zeros(len(multis))
    for lead in itertools.product(*[range(e) for e in ext[:s]]):
        flat = 0
        for i in range(s):
            flat = flat * ext[i] + lead[i]
        X = grid_coordinates(grid, flat * rest, (flat + 1) * rest)
        f = _function_at(family, params, X).reshape(ext[s:])
        for r, m in enumerate(multis):
            w = 1.0
            for i in range(s):
                w *= mats[i][m[i], lead[i]]
            if w == 0.0:
                continue
            t, ta = f, np.abs(f)
            for i in range(s, D):                 # contract the trailing axes in order
                row = mats[i][m[i]]
                t = np.tensordot(t, row, axes=([0], [0]))
                ta = np.tensordot(ta, np.abs(row), axes=([0], [0]))
            vals[r] += w * float(t)
            abss[r] += abs(w) * float(ta)
    return vals, abss


def idct_grid(coef: np.ndarray, grid) -> np.ndarray:
    """Evaluate a coefficient tensor on the grid (inverse of dct_grid)."""
    grid = [int(v) for v in grid if int(v) > 0]    # single-node axes: identity
    shape = tuple(v + 1 for v in grid)
    t = np.asarray(coef, dtype=np.float64).reshape(shape)
    for axis, N in enumerate(grid):
        t = dct_axis(t, axis, dct1_eval_matrix(N))
    return t.reshape(-1)


# ---------------------------------------------------------------------------
# Alias maps and the stacked operator A (Sec. 3.1-3.3)
# ---------------------------------------------------------------------------

def grid_strides(grid) -> list[int]:
    """Row-major strides of the (N_i+1)-extent tensor, last dimension 1."""
    ext = [int(v) + 1 for v in grid]
    st = [1] * len(ext)
    for i in range(len(ext) - 2, -1, -1):
        st[i] = st[i + 1] * ext[i + 1]
    return st


def alias_bins(support, grid) -> np.ndarray:
    """Flat bin of each support multi-index on one grid (int64 [n]).

    The multi-dimensional alias of n is (fold(n_1, N_1), ..., fold(n_D, N_D))
    because A_{m,n} = prod_i A^(i)_{m_i,n_i} (eq. aliasing_matrix_nd_diff);
    its position in the row-major transform tensor is the flat bin.
    """
    S = np.asarray(support, dtype=np.int64)
    st = grid_strides(grid)
    out = np.zeros(S.shape[0], dtype=np.int64)
    for i, N in enumerate(grid):
        out += fold_array(S[:, i], int(N)) * st[i]
    return out


class Plan:
    """Alias structure of a support on an L-grid (the A of Alg. 2).

    Attributes (K grids, n support entries):
      alias   int64 [K, n]  flat bin of support j on grid l
      perm    int32 [K, n]  support positions sorted by (bin, position)
      seg_off int64 [M+1]   global offsets into perm.ravel() of each row
      bin_id  int64 [M]     flat bin of each row (rows = non-empty bins)
      rowmap  int64 [K, n]  global row of support j on grid l
      row_off int64 [K+1]   first global row of each grid
      points  int64 [K]     nodes per grid
    Rows are ordered by (grid ascending, bin ascending); empty bins carry a
    zero row of A and are dropped, which does not change the minimiser.
    """

    def __init__(self, support, grids):
        S = np.asarray(support, dtype=np.int64)
        G = np.asarray(grids, dtype=np.int64)
        self.support, self.grids = S, G
        self.K, self.n = G.shape[0], S.shape[0]
        self.points = np.array([int(np.prod(g + 1)) for g in G], dtype=np.int64)
        self.alias = np.stack([alias_bins(S, g) for g in G])
        perms, seg, bins, rowmap, row_off = [], [], [], [], [0]
        for l in range(self.K):
            a = self.alias[l]
            # stable sort: ties keep ascending support position
            order = np.argsort(a, kind="stable")
            sa = a[order]
            head = np.ones(self.n, dtype=bool)
            head[1:] = sa[1:] != sa[:-1]
            local = np.cumsum(head) - 1
            rm = np.empty(self.n, dtype=np.int64)
            rm[order] = row_off[-1] + local
            perms.append(order)
            seg.extend((l * self.n + np.nonzero(head)[0]).tolist())
            bins.extend(sa[head].tolist())
            rowmap.append(rm)
            row_off.append(row_off[-1] + int(head.sum()))
        seg.append(self.K * self.n)
        self.perm = np.array(perms, dtype=np.int32).reshape(self.K, self.n)
        self.seg_off = np.array(seg, dtype=np.int64)
        self.bin_id = np.array(bins, dtype=np.int64)
        self.rowmap = np.stack(rowmap)
        self.row_off = np.array(row_off, dtype=np.int64)
        self.M = int(self.row_off[-1])

    def rows_of_grid(self, l):
        return self.row_off[l], self.row_off[l + 1]


def build_plan(support, grids) -> Plan:
    return Plan(support, grids)


def dense_A(plan: Plan) -> np.ndarray:
    """Explicit stacked A (M x n), A[row_l(bin_l(n)), n] = 1."""
    A = np.zeros((plan.M, plan.n))
    for l in range(plan.K):
        A[plan.rowmap[l], np.arange(plan.n)] = 1.0
    return A


def sparse_A(plan: Plan):
    import scipy.sparse as sp
    rows = plan.rowmap.reshape(-1)
    cols = np.tile(np.arange(plan.n), plan.K)
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(plan.M, plan.n))


def gram_matrix(plan: Plan) -> np.ndarray:
    """A^T A as a dense float64 matrix of exact integers (collision counts)."""
    As = sparse_A(plan)
    return (As.T @ As).toarray()


# ---------------------------------------------------------------------------
# Sampling (Alg. 3, sample f on the L-grid)
# ---------------------------------------------------------------------------

def grid_coordinates(grid, start: int = 0, stop: int | None = None):
    """Node coordinates of the points start..stop-1 (flat row-major index)
    of one grid, [stop - start, D]; by default every point."""
    axes = [lobatto_nodes(int(N)) for N in grid]
    shape = tuple(int(N) + 1 for N in grid)
    if start == 0 and stop is None:
        mesh = np.meshgrid(*axes, indexing="ij")
        return np.stack([m.reshape(-1) for m in mesh], axis=1)
    idx = np.unravel_index(np.arange(start, stop, dtype=np.int64), shape)
    return np.stack([axes[i][idx[i]] for i in range(len(shape))], axis=1)


def sample_planted(support, coeffs, grid) -> np.ndarray:
    """Brute-force samples of p(x) = sum_n c_n prod_i T_{n_i}(x_i) (Sec. 2).

    Each T_{n_i} is evaluated at the 1-D nodes with the three-term recurrence,
    then the tensor products are summed coefficient by coefficient.  No DCT
    and no aliasing is involved, so this checks the transform independently.
    """
    S = np.asarray(support, dtype=np.int64)
    grid = [int(v) for v in grid]
    nmax = int(S.max()) if S.size else 0
    # a single-node axis (N = 0, node x = 1) contributes T_n(1) = 1 to every
    # term and no axis to the flat layout; the tensor spans the other axes
    axes = [i for i, N in enumerate(grid) if N > 0]
    tables = {i: cheb_T_recurrence(nmax, lobatto_nodes(grid[i])) for i in axes}
    shape = tuple(grid[i] + 1 for i in axes)
    out = np.zeros(shape)
    for j in range(S.shape[0]):
        term = np.asarray(coeffs[j], dtype=np.float64)
        for i in axes:
            vec = tables[i][S[j, i]]
            term = np.multiply.outer(term, vec)
        out += term
    return out.reshape(-1)


def sample_function(family: int, params, grid, chunk: int = 1 << 22) -> np.ndarray:
    """Samples of an analytic test function on one grid, FP64, pointwise.

    family 1: exp(-sum a_i x_i^2) cos(sum w_i x_i), params = [a_1..a_D, w_1..w_D]
    family 2: exp(-|x - x0|^2 / (2 s^2)),           params = [s, x0_1..x0_D]
    family 3: 1 / (1 + alpha |x|^2)   (f1, Sec. 4.3.1), params = [alpha]
    family 4: sin(3 cos(3 exp|x|^2)) + exp(sin(3 sum x))  (f2, Sec. 4.3.2)
    """
    P = int(np.prod([int(N) + 1 for N in grid]))
    if P > chunk:                      # large grids: the same pointwise formula in slabs
        out = np.empty(P)
        for a in range(0, P, chunk):
            b = min(P, a + chunk)
            out[a:b] = _function_at(family, params, grid_coordinates(grid, a, b))
        return out
    return _function_at(family, params, grid_coordinates(grid))


def _function_at(family: int, params, X) -> np.ndarray:
    D = X.shape[1]
    p = np.asarray(params, dtype=np.float64)
    if family == 1:
        a, w = p[:D], p[D:2 * D]
        return np.exp(-(X * X) @ a) * np.cos(X @ w)
    if family == 2:
        s, x0 = p[0], p[1:1 + D]
        r2 = ((X - x0) ** 2).sum(axis=1)
        return np.exp(-r2 / (2.0 * s * s))
    if family == 3:
        return 1.0 / (1.0 + p[0] * (X * X).sum(axis=1))
    if family == 4:
        r2 = (X * X).sum(axis=1)
        return np.sin(3.0 * np.cos(3.0 * np.exp(r2))) + np.exp(np.sin(3.0 * X.sum(axis=1)))
    raise ValueError(f"unknown family {family}")


def sample_problem(prob) -> list[np.ndarray]:
    """Samples of a workloads.Problem on each of its grids."""
    out = []
    for g in prob.grids:
        if prob.family == 0:
            out.append(sample_planted(prob.support, prob.coeffs, g))
        else:
            out.append(sample_function(prob.family, prob.params, g))
    return out


# ---------------------------------------------------------------------------
# Right-hand side and least squares (Sec. 3.4, Alg. 3)
# ---------------------------------------------------------------------------

def rhs_from_transforms(plan: Plan, transforms) -> np.ndarray:
    """Stacked F f restricted to the non-empty bins, in row order."""
    b = np.empty(plan.M)
    for l in range(plan.K):
        r0, r1 = plan.rows_of_grid(l)
        b[r0:r1] = np.asarray(transforms[l])[plan.bin_id[r0:r1]]
    return b


def lstsq_qr(plan: Plan, b: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """argmin ||b - A c||_2 by Householder QR of the augmented matrix [A | b].

    The grid blocks are folded in one at a time, R <- qr([R; A_l b_l]), which
    gives the same triangular factor as one QR of the full stack while only
    ever holding n+1 plus one block of rows.  Returns (c, diag(R)).
    """
    n = plan.n
    Raug = np.zeros((0, n + 1))
    for l in range(plan.K):
        r0, r1 = plan.rows_of_grid(l)
        blk = np.zeros((r1 - r0, n + 1))
        blk[plan.rowmap[l] - r0, np.arange(n)] = 1.0
        blk[:, n] = b[r0:r1]
        Raug = np.linalg.qr(np.vstack([Raug, blk]), mode="r")
        Raug = Raug[: min(Raug.shape[0], n + 1)]
    if Raug.shape[0] < n:
        raise np.linalg.LinAlgError("fewer rows than unknowns: rank deficient")
    R = Raug[:n, :n]
    z = Raug[:n, n]
    import scipy.linalg as sla
    c = sla.solve_triangular(R, z, lower=False)
    return c, np.diag(R).copy()


def lstsq_normal(plan: Plan, b: np.ndarray) -> np.ndarray:
    """argmin ||b - A c||_2 from the normal equations A^T A c = A^T b.

    A^T A holds exact integers (collision counts), so forming it adds no
    rounding; it is factorised by Cholesky.  Used for supports too large for
    the dense QR route.
    """
    import scipy.linalg as sla
    As = sparse_A(plan)
    Gm = (As.T @ As).toarray()
    h = As.T @ b
    cf = sla.cho_factor(Gm, lower=False, overwrite_a=True, check_finite=False)
    return sla.cho_solve(cf, h, check_finite=False)


def lstsq_lsqr(plan: Plan, b: np.ndarray, tol: float = 1e-15, iter_lim: int = 20000):
    """argmin ||b - A c||_2 by LSQR on the explicit sparse A (scipy's
    Golub-Kahan bidiagonalisation); for supports too large for dense QR.
    Returns (c, iterations, LSQR's condition estimate)."""
    import scipy.sparse.linalg as spl
    res = spl.lsqr(sparse_A(plan), b, atol=tol, btol=tol, conlim=1e12, iter_lim=iter_lim)
    return res[0], int(res[2]), float(res[6])


def rank_check(plan: Plan, kappa_max: float = 1e4):
    """(full_rank, kappa(A)) from the extreme eigenvalues of A^T A.

    Uses the dense eigenvalues for small supports and Lanczos on the sparse
    Gram matrix otherwise.  kappa(A) = sqrt(lmax / lmin).
    """
    As = sparse_A(plan)
    Gs = (As.T @ As).tocsc()
    if plan.n <= 2500:
        ev = np.linalg.eigvalsh(Gs.toarray())
        lmin, lmax = ev[0], ev[-1]
    else:
        import scipy.sparse.linalg as spl
        lmax = spl.eigsh(Gs, k=1, which="LA", return_eigenvectors=False)[0]
        # smallest eigenvalue by shift-invert around 0 (Gram is PSD)
        try:
            lmin = spl.eigsh(Gs, k=1, sigma=-1e-3, which="LM",
                             return_eigenvectors=False)[0]
        except Exception:
            lmin = 0.0
    full = lmin > 1e-10 * lmax
    kappa = math.sqrt(lmax / lmin) if lmin > 0 else math.inf
    return bool(full and kappa <= kappa_max), kappa


def select_grid_count(support, candidates, kappa_max: float = 1e4):
    """Alg. 2: append the candidate grids (drawn by Alg. 1) one at a time and
    stop at the first L whose stacked A is full rank with kappa(A) <=
    kappa_max.  Returns (L, kappa), or (0, kappa of all candidates)."""
    kappa = math.inf
    for L in range(1, len(candidates) + 1):
        ok, kappa = rank_check(build_plan(support, np.asarray(candidates)[:L]), kappa_max)
        if ok:
            return L, kappa
    return 0, kappa


def normal_residual(plan: Plan, b: np.ndarray, c: np.ndarray) -> np.ndarray:
    """A^T (b - A c): zero at the least-squares minimiser."""
    As = sparse_A(plan)
    return As.T @ (b - As @ c)


def fct_solve(support, grids, samples, method: str = "auto"):
    """End-to-end Alg. 3: DCT each grid, stack, least squares.

    Returns (c, plan, b).  ``method``: 'qr', 'normal' or 'auto' (QR up to
    4000 unknowns, normal equations above).
    """
    plan = build_plan(support, grids)
    trans = [dct_grid(samples[l], plan.grids[l]) for l in range(plan.K)]
    b = rhs_from_transforms(plan, trans)
    if method == "auto":
        method = "qr" if plan.n <= 4000 else "normal"
    if method == "qr":
        c, _ = lstsq_qr(plan, b)
    elif method == "normal":
        c = lstsq_normal(plan, b)
    else:
        raise ValueError(method)
    return c, plan, b


# ---------------------------------------------------------------------------
# Error measures
# ---------------------------------------------------------------------------

def max_rel_err(c, c_ref) -> float:
    """Normwise relative error ||c - c_ref||_inf / ||c_ref||_inf."""
    c = np.asarray(c, dtype=np.float64)
    c_ref = np.asarray(c_ref, dtype=np.float64)
    return float(np.max(np.abs(c - c_ref)) / np.max(np.abs(c_ref)))


def mean_l2_err(c, c_ref) -> float:
    """||c - c_ref||_2 / N, the paper's mean l2 coefficient error (Sec. 4.5.1)."""
    c = np.asarray(c, dtype=np.float64)
    return float(np.linalg.norm(c - np.asarray(c_ref)) / c.size)


# ---------------------------------------------------------------------------
# Evaluation of a recovered expansion (Sec. 2, definition of the Chebyshev
# expansion on the support; Sec. 4 measures accuracy at random points)
# ---------------------------------------------------------------------------

def evaluate_expansion(support, coeffs, X, chunk: int = 256) -> np.ndarray:
    """p(x) = sum_j c_j prod_i T_{n_ji}(x_i) at every row x of X ([m][D]).

    Per point and dimension the values T_0..T_nmax come from the three-term
    recurrence; each term is the product over the dimensions, and the terms
    are summed in support order.  Points are taken `chunk` at a time.
    """
    S = np.asarray(support, dtype=np.int64)
    c = np.asarray(coeffs, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    m, D = X.shape
    if S.shape[1] != D:
        raise ValueError("support and points differ in dimension")
    nmax = int(S.max()) if S.size else 0
    out = np.empty(m)
    for a in range(0, m, chunk):
        xb = X[a:a + chunk]
        # T[i][k][point]
        T = [cheb_T_recurrence(nmax, xb[:, i]) for i in range(D)]
        terms = np.ones((S.shape[0], xb.shape[0]))
        for i in range(D):
            terms *= T[i][S[:, i]]
        out[a:a + chunk] = c @ terms
    return out


def function_values(family: int, params, X) -> np.ndarray:
    """The test function of `family` at the rows of X ([m][D])."""
    return _function_at(family, params, np.asarray(X, dtype=np.float64))


def linf_error(values, reference) -> float:
    """max |values - reference| (the sup-norm error at sample points)."""
    return float(np.max(np.abs(np.asarray(values) - np.asarray(reference))))
