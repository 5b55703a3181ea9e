"""Seeded synthetic inputs for the sparse Fast Chebyshev Transform.

This module is shared by the CPU oracle and by the GPU tests and benchmark.
It produces *inputs only*: multi-index supports, grid resolutions, planted
coefficient vectors and the parameters of analytic test functions.  It holds
none of the transform's arithmetic (no Chebyshev evaluation, no aliasing, no
DCT, no least squares), so that neither side can inherit a mistake from the
other through it.

Conventions (paper notation in brackets):

* A support [the index set of nonzero coefficients, Sec. 2 and Sec. 4.5.3]
  is an int32 array ``[n_support, D]`` in lexicographic ascending order.
* A grid [one member of an L-grid, Sec. 3.2] is a row of D non-negative
  ints ``N_i``: the Chebyshev-Lobatto *degree* along dimension i, i.e. the
  grid has ``N_i + 1`` nodes ``cos(pi k / N_i)``; ``N_i = 0`` is the single
  node ``x = 1``.  A stack of K grids is int32 ``[K, D]``.
* Grid-point counts ``P = prod(N_i + 1)`` are plain counting, used only for
  the oversampling stop rules of the workload recipes.

Every generator takes an integer seed and derives independent streams with
``numpy.random.SeedSequence(seed).spawn(3)`` -> (grid stream,
coefficient/parameter stream, arrival stream).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "total_degree_support", "euclidean_degree_support", "grid_points",
    "draw_grids_uniform", "draw_grid_capped", "planted_coefficients",
    "Problem", "config1", "config2", "config3", "config3_problem", "small_problem", "streams",
    "config4", "CFG4_MIN_GRIDS", "FAMILY_PLANTED", "FAMILY_EXPCOS", "FAMILY_GAUSS", "FAMILY_RUNGE",
    "FAMILY_OSC", "SERVING_TYPES", "serving_problem", "serving_pool", "poisson_arrivals",
    "d20_grids", "d20_d4_problem",
]

# Function-family identifiers (same integers as the C ABI's fct_family).
FAMILY_PLANTED = 0   # f = sum_n c_n T_n(x) on the support (Sec. 4.5.1 recovery runs)
FAMILY_EXPCOS = 1    # f = exp(-sum a_i x_i^2) cos(sum w_i x_i)
FAMILY_GAUSS = 2     # f = exp(-|x - x0|^2 / (2 sigma^2))
FAMILY_RUNGE = 3     # f1 of Sec. 4.3.1: 1 / (1 + alpha |x|^2)
FAMILY_OSC = 4       # f2 of Sec. 4.3.2: sin(3 cos(3 exp|x|^2)) + exp(sin(3 sum x))


def streams(seed: int):
    """Three independent generators (grid, coefficient/parameter, arrival)."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3)]


def total_degree_support(D: int, d: int) -> np.ndarray:
    """All n in N^D with |n|_1 <= d, lexicographic ascending (Sec. 2, S^1_{d,D}).

    Built dimension by dimension: every partial row of the first i entries is
    extended by each admissible value of entry i in increasing order, which
    keeps the rows sorted lexicographically.
    """
    if D < 1 or d < 0:
        raise ValueError("need D >= 1 and d >= 0")
    rows = np.zeros((1, 0), dtype=np.int64)
    used = np.zeros(1, dtype=np.int64)
    for _ in range(D):
        counts = d - used + 1
        rep = np.repeat(np.arange(rows.shape[0]), counts)
        starts = np.repeat(np.cumsum(counts) - counts, counts)
        vals = np.arange(rep.size) - starts
        rows = np.concatenate([rows[rep], vals[:, None]], axis=1)
        used = used[rep] + vals
    return np.ascontiguousarray(rows.astype(np.int32))


def euclidean_degree_support(D: int, d: float) -> np.ndarray:
    """All n in N^D with |n|_2 <= d, lexicographic ascending (Sec. 2, S^2_{d,D})."""
    dmax = int(math.floor(d))
    rows = np.zeros((1, 0), dtype=np.int64)
    sq = np.zeros(1, dtype=np.int64)
    lim = d * d + 1e-9
    for _ in range(D):
        rem = np.floor(np.sqrt(np.maximum(lim - sq, 0.0))).astype(np.int64)
        rem = np.minimum(rem, dmax)
        counts = rem + 1
        rep = np.repeat(np.arange(rows.shape[0]), counts)
        starts = np.repeat(np.cumsum(counts) - counts, counts)
        vals = np.arange(rep.size) - starts
        rows = np.concatenate([rows[rep], vals[:, None]], axis=1)
        sq = sq[rep] + vals * vals
        keep = sq <= lim
        rows, sq = rows[keep], sq[keep]
    return np.ascontiguousarray(rows.astype(np.int32))


def grid_points(grid) -> int:
    """Number of nodes of one tensor grid: prod(N_i + 1) (plain counting)."""
    return int(np.prod(np.asarray(grid, dtype=np.int64) + 1))


def draw_grids_uniform(rng, D, lo, hi, n_support, oversample, min_grids=1,
                       max_grids=4096):
    """i.i.d. ``N_i ~ U{lo..hi}`` grids, appended until the stacked point
    count reaches ``oversample * n_support`` and at least ``min_grids`` grids
    exist (the workload's floor that keeps the stacked system full rank)."""
    grids, total = [], 0
    while (total < oversample * n_support or len(grids) < min_grids):
        g = rng.integers(lo, hi + 1, size=D)
        grids.append(g)
        total += grid_points(g)
        if len(grids) >= max_grids:
            break
    return np.ascontiguousarray(np.array(grids, dtype=np.int32))


def draw_grid_capped(rng, D, lo, hi, cap, rest=0):
    """One grid drawn the way the sampling-rate selection (Alg. 1) draws it.

    Dimensions are visited in a random order; each gets a degree drawn from
    ``U{lo..hi}``; once the running point count exceeds ``cap`` every
    remaining dimension gets degree ``rest`` (0: a single node, as in the
    algorithm).  Degrees here are Lobatto degrees, so the algorithm's draw of
    1..d+1 *points* is a draw of 0..d here.
    """
    order = rng.permutation(D)
    g = np.full(D, rest, dtype=np.int64)
    prod = 1
    for i in order:
        g[i] = rng.integers(lo, hi + 1)
        prod *= int(g[i]) + 1
        if prod > cap:
            break
    return g


def draw_grids_capped(rng, D, lo, hi, n_support, oversample, min_grids=1,
                      max_grids=4096, rest=0):
    grids, total = [], 0
    while (total < oversample * n_support or len(grids) < min_grids):
        g = draw_grid_capped(rng, D, lo, hi, n_support, rest)
        grids.append(g)
        total += grid_points(g)
        if len(grids) >= max_grids:
            break
    return np.ascontiguousarray(np.array(grids, dtype=np.int32))


def planted_coefficients(rng, support) -> np.ndarray:
    """c_n = z_n * 2^(-|n|_1/4), z ~ N(0,1): the planted-polynomial recipe."""
    s = np.asarray(support, dtype=np.int64).sum(axis=1)
    z = rng.standard_normal(len(support))
    return z * np.exp2(-s / 4.0)


@dataclass
class Problem:
    """One approximation job: support, grids and the function to sample."""
    name: str
    support: np.ndarray            # int32 [n, D]
    grids: np.ndarray              # int32 [K, D]
    family: int
    params: np.ndarray = field(default_factory=lambda: np.zeros(0))
    coeffs: np.ndarray | None = None   # planted coefficients (FAMILY_PLANTED)
    seed: int = 0

    @property
    def D(self):
        return int(self.support.shape[1])

    @property
    def n(self):
        return int(self.support.shape[0])

    @property
    def K(self):
        return int(self.grids.shape[0])

    @property
    def points(self):
        return [grid_points(g) for g in self.grids]

    @property
    def total_points(self):
        return int(sum(self.points))


def config1(seed: int = 0) -> Problem:
    """D=2, |n|_1 <= 16 (153 coefficients), K=4 grids with N_i ~ U{9..24},
    planted polynomial c_n ~ N(0,1) 2^(-|n|_1/4)."""
    g_grid, g_coef, _ = streams(seed)
    S = total_degree_support(2, 16)
    grids = np.ascontiguousarray(g_grid.integers(9, 25, size=(4, 2)).astype(np.int32))
    c = planted_coefficients(g_coef, S)
    return Problem("cfg1_D2_d16_K4", S, grids, FAMILY_PLANTED, np.zeros(0), c, seed)


# Grid floor for the D=6 workload: the 2x point-count stop rule alone stops
# after one grid, which can never give a full-rank system.  Four grids is the
# smallest count for which the seeded instance is full rank with
# kappa(A) <= 1e4 (the stopping rule of Alg. 2), as the oracle's rank test
# checks.
CFG2_MIN_GRIDS = 4


def config2(seed: int = 1, min_grids: int = CFG2_MIN_GRIDS) -> Problem:
    """D=6, |n|_1 <= 12 (18,564 coefficients), grids N_i ~ U{4..8} appended
    until the stacked points reach 2x the support size (and the grid floor),
    f = exp(-sum a_i x_i^2) cos(sum w_i x_i), a_i ~ U(0.2,1), w_i ~ U(0.5,2)."""
    g_grid, g_par, _ = streams(seed)
    S = total_degree_support(6, 12)
    grids = draw_grids_uniform(g_grid, 6, 4, 8, len(S), 2.0, min_grids)
    a = g_par.uniform(0.2, 1.0, size=6)
    w = g_par.uniform(0.5, 2.0, size=6)
    return Problem("cfg2_D6_d12_expcos", S, grids, FAMILY_EXPCOS,
                   np.concatenate([a, w]), None, seed)


CFG4_MIN_GRIDS = 17


def config4(seed: int = 3, min_grids: int = CFG4_MIN_GRIDS, d: int = 10) -> Problem:
    """The precision-sweep workload: D=12, |n|_1 <= d (646,646 coefficients at
    d = 10), grids with N_i ~ U{2..6} i.i.d. appended until the stacked points
    reach 3x the support size and the grid floor, f = exp(-|x - x0|^2 /
    (2 0.8^2)) with x0 ~ U(-0.5, 0.5)^12.  A single such grid already holds
    ~10^8 points, far beyond 3x; the floor is the grid count at which the
    oracle finds the stacked system full rank (every dimension's degrees
    0..d separated by the folds, and exact recovery).  ``d`` < 10 gives a
    small twin drawn by the same rule."""
    g_grid, g_par, _ = streams(seed)
    S = total_degree_support(12, d)
    grids = draw_grids_uniform(g_grid, 12, 2, 6, len(S), 3.0, min_grids)
    x0 = g_par.uniform(-0.5, 0.5, size=12)
    return Problem(f"cfg4_D12_d{d}_gauss", S, grids, FAMILY_GAUSS,
                   np.concatenate([[0.8], x0]), None, seed)


def small_problem(seed: int, D: int, d: int, lo: int, hi: int, K: int,
                  family: int = FAMILY_PLANTED) -> Problem:
    """A small total-degree problem with K i.i.d. U{lo..hi} grids."""
    g_grid, g_coef, _ = streams(seed)
    S = total_degree_support(D, d)
    grids = np.ascontiguousarray(g_grid.integers(lo, hi + 1, size=(K, D)).astype(np.int32))
    c = None
    params = np.zeros(0)
    if family == FAMILY_PLANTED:
        c = planted_coefficients(g_coef, S)
    elif family == FAMILY_EXPCOS:
        params = np.concatenate([g_coef.uniform(0.2, 1.0, size=D),
                                 g_coef.uniform(0.5, 2.0, size=D)])
    elif family == FAMILY_GAUSS:
        params = np.concatenate([[0.8], g_coef.uniform(-0.5, 0.5, size=D)])
    elif family == FAMILY_RUNGE:
        params = np.array([10.0])
    return Problem(f"small_D{D}_d{d}_K{K}_s{seed}", S, grids, family, params, c, seed)


# Euclidean-degree workload: S^2 of radius 6 in D = 5 (2,673 coefficients),
# i.i.d. U{2..6} grids; 9 grids is where the oracle's rank test (the stopping
# rule of Alg. 2) first finds A full rank for seed 11 (kappa ~ 9).
EUCLID_GRIDS = 9


def euclidean_problem(seed: int = 11, family: int = FAMILY_PLANTED) -> Problem:
    """D = 5, |n|_2 <= 6 (Sec. 2, S^2_{d,D}) on EUCLID_GRIDS grids."""
    g_grid = np.random.default_rng(seed)
    S = euclidean_degree_support(5, 6.0)
    grids = np.ascontiguousarray(g_grid.integers(2, 7, size=(EUCLID_GRIDS, 5)).astype(np.int32))
    _, g_coef, _ = streams(seed)
    c = None
    params = np.zeros(0)
    if family == FAMILY_PLANTED:
        c = planted_coefficients(g_coef, S)
    elif family == FAMILY_EXPCOS:
        params = np.concatenate([g_coef.uniform(0.2, 1.0, size=5), g_coef.uniform(0.5, 2.0, size=5)])
    else:
        raise ValueError("euclidean_problem: planted or exp-cos")
    return Problem(f"euclid_D5_r6_s{seed}_f{family}", S, grids, family, params, c, seed)


def sparse_support(rng, D: int, d: int, N: int) -> np.ndarray:
    """N random multi-indices of S^inf_{d,D} (every coordinate uniform in
    0..d), the sparse supports of the paper's f3 family (Sec. 4).  Rows are
    drawn independently; a repeated row (probability about N^2 / (2 (d+1)^D),
    zero in practice for D = 100) is replaced by a fresh draw."""
    S = rng.integers(0, d + 1, size=(N, D), dtype=np.int32)
    if N * N < 2 * float(d + 1) ** D * 1e-6:
        return np.ascontiguousarray(S)
    while True:
        _, first = np.unique(S, axis=0, return_index=True)
        if len(first) == N:
            return np.ascontiguousarray(S)
        dup = np.setdiff1d(np.arange(N), first)
        S[dup] = rng.integers(0, d + 1, size=(len(dup), D), dtype=np.int32)


def f3_problem(N: int, seed: int = 5, D: int = 100, d: int = 8, K: int = 20) -> Problem:
    """The paper's f3 family (Sec. 4): N random multi-indices of S^inf_{d,D},
    coefficients uniform in [-1, 1], on K grids drawn by Alg. 1 (dimensions in
    random order, degrees U{0..d} -- 1..d+1 nodes --, single nodes once the
    running point count exceeds N).  K = 20 recovers the planted
    coefficients exactly at every N tried (the oracle's LSQR check on the
    small instance; the GPU's exact recovery on the large ones)."""
    g_grid, g_coef, _ = streams(seed)
    S = sparse_support(g_coef, D, d, N)
    c = g_coef.uniform(-1.0, 1.0, size=N)
    grids = np.ascontiguousarray(np.array([draw_grid_capped(g_grid, D, 0, d, N, 0)
                                           for _ in range(K)], dtype=np.int32))
    return Problem(f"f3_D{D}_d{d}_N{N}_K{K}", S, grids, FAMILY_PLANTED, np.zeros(0), c, seed)


def config3_problem(rng_grid, rng_coef, cap=50_000):
    """One problem of the batched workload: D ~ U{3..8}, d ~ U{6..16}, d
    lowered until C(D+d, d) <= cap; grids drawn as in Alg. 1 (dimensions in
    random order, degrees U{1..d}, once the running point count exceeds |S|
    the remaining dimensions get degree 1) until the points reach 2|S| and
    there are at least 6D grids; planted polynomial.

    Two departures from Alg. 1 keep the seeded problems well posed: a
    dimension beyond the cap gets two Lobatto nodes instead of one (a single
    node leaves it entirely unresolved, which made a share of the problems
    rank deficient), and 6D grids instead of the paper's 3D."""
    D = int(rng_grid.integers(3, 9))
    d = int(rng_grid.integers(6, 17))
    while math.comb(D + d, d) > cap:
        d -= 1
    S = total_degree_support(D, d)
    grids = draw_grids_capped(rng_grid, D, 1, d, len(S), 2.0, min_grids=6 * D, rest=1)
    c = planted_coefficients(rng_coef, S)
    return Problem(f"cfg3_D{D}_d{d}", S, grids, FAMILY_PLANTED, np.zeros(0), c)


def config3(seed: int = 2, count: int = 256, extra_grids=None):
    """The batched workload: `count` independent problems (config3_problem).

    ``extra_grids`` maps a problem index to a number of further grids to
    append (drawn by the same rule from a stream of their own): the output of
    the grid-count selection (Alg. 2) that the oracle runs once and stores
    under tests/golden/."""
    g_grid, g_coef, _ = streams(seed)
    g_more = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[3])
    out = []
    for i in range(count):
        p = config3_problem(g_grid, g_coef)
        p.name = f"{p.name}_{i}"
        p.seed = seed
        out.append(p)
    for i in sorted(int(k) for k in (extra_grids or {})):
        p = out[i]
        d = int(p.support.max())
        more = [draw_grid_capped(g_more, p.D, 1, d, p.n, 1)
                for _ in range(int(extra_grids[str(i)] if str(i) in extra_grids else extra_grids[i]))]
        p.grids = np.ascontiguousarray(np.concatenate([p.grids, np.array(more, dtype=np.int32)]))
    return out


SERVING_TYPES = ("cfg1_shape", "cfg2_shape", "cfg3_style", "D20_d2")

# D=20 jobs.  Alg.-1 grids (a few resolved dimensions, single nodes
# elsewhere) leave total-degree supports rank deficient or badly conditioned
# unless very many are stacked: a coefficient whose multi-index touches the
# dimensions I is only told apart from its aliases by a grid that resolves
# all of I.  The D=20 L-grids here therefore resolve `k` dimensions per grid
# at degree `d` (the fold is one-to-one on 0..d) and cover every set of d
# dimensions: grids are added greedily, each the best of 256 seeded random
# choices by the number of still-uncovered d-sets it covers.  At |n|_1 <= 4
# (10,626 coefficients) even the full 4-set cover (173 grids, 6.8e7 samples)
# stays ill-conditioned (about 1.2e4 FP64 CGLS iterations), so the serving
# mix uses D=20 at |n|_1 <= 2 (231 coefficients, a 13-grid pair cover) and
# the |n|_1 <= 4 job is measured on its own (d20_d4_problem).
D20_CANDIDATES = 256


def d20_grids(seed: int, d: int = 2, k: int = 8) -> np.ndarray:
    """A D=20 L-grid of degree-d grids on k dimensions (single nodes
    elsewhere) covering every set of d dimensions."""
    from itertools import combinations
    rng = np.random.default_rng([seed, 20])
    sets = np.array([sum(1 << i for i in c) for c in combinations(range(20), d)], dtype=np.int64)
    uncovered = np.ones(len(sets), dtype=bool)
    grids = []
    while uncovered.any():
        best, best_n = None, -1
        for _ in range(D20_CANDIDATES):
            dims = rng.choice(20, size=k, replace=False)
            mask = int(sum(1 << int(i) for i in dims))
            n_cov = int(np.count_nonzero(uncovered & ((sets & ~mask) == 0)))
            if n_cov > best_n:
                best, best_n = (dims, mask), n_cov
        dims, mask = best
        uncovered &= ~((sets & ~mask) == 0)
        g = np.zeros(20, dtype=np.int32)
        g[dims] = d
        grids.append(g)
    return np.array(grids, dtype=np.int32)


def d20_d4_problem(seed: int = 4) -> Problem:
    """D=20, |n|_1 <= 4 (10,626 coefficients) on the 4-set cover with eight
    resolved dimensions per grid, planted polynomial."""
    S = total_degree_support(20, 4)
    c = planted_coefficients(np.random.default_rng([seed, 21]), S)
    return Problem("D20_d4", S, d20_grids(seed, 4, 8), FAMILY_PLANTED, np.zeros(0), c, seed)


def serving_problem(kind: str, rng_grid, rng_coef) -> Problem:
    """One request of the serving mix.

    cfg1_shape: D=2, |n|_1<=16, K=4 grids N_i ~ U{9..24}, planted polynomial.
    cfg2_shape: D=6, |n|_1<=12, grids N_i ~ U{4..8} until 2|S| points and
                K >= 4, exp-cos with a_i ~ U(0.2,1), w_i ~ U(0.5,2).
    cfg3_style: one problem drawn like the batched workload.
    D20_d2:     D=20, |n|_1<=2 (231 coefficients) on the shared L-grid
                (d20_grids), planted.
    """
    if kind == "cfg1_shape":
        S = total_degree_support(2, 16)
        grids = np.ascontiguousarray(rng_grid.integers(9, 25, size=(4, 2)).astype(np.int32))
        return Problem(kind, S, grids, FAMILY_PLANTED, np.zeros(0),
                       planted_coefficients(rng_coef, S))
    if kind == "cfg2_shape":
        S = total_degree_support(6, 12)
        grids = draw_grids_uniform(rng_grid, 6, 4, 8, len(S), 2.0, 4)
        params = np.concatenate([rng_coef.uniform(0.2, 1.0, size=6),
                                 rng_coef.uniform(0.5, 2.0, size=6)])
        return Problem(kind, S, grids, FAMILY_EXPCOS, params, None)
    if kind == "cfg3_style":
        p = config3_problem(rng_grid, rng_coef)
        p.name = kind
        return p
    if kind == "D20_d2":
        S = total_degree_support(20, 2)
        return Problem(kind, S, None, FAMILY_PLANTED, np.zeros(0),
                       planted_coefficients(rng_coef, S))
    raise ValueError(kind)


def serving_extra_grid(p: Problem, rng):
    """One more grid for a serving job, drawn by the job's own rule."""
    d = int(p.support.max())
    kind = p.name.rsplit("_", 1)[0]
    if kind == "cfg1_shape":
        return rng.integers(9, 25, size=2)
    if kind == "cfg2_shape":
        return rng.integers(4, 9, size=6)
    return draw_grid_capped(rng, p.D, 1, d, p.n, 1)


def serving_pool(seed: int = 4, per_type: int = 16, extra_grids=None):
    """The serving workload's pool of seeded jobs: per_type jobs of each of
    the four kinds, interleaved (job i has kind SERVING_TYPES[i % 4]).

    ``extra_grids`` maps a job index to a number of further grids appended
    to it, drawn by the job's own rule from a stream of its own (job i:
    default_rng([seed, 1000 + i])): the oracle's Alg.-2 selection stored
    under tests/golden/.  The D=20 jobs share d20_grids(seed)."""
    g_grid, g_coef, _ = streams(seed)
    shared = d20_grids(seed)
    jobs = []
    for i in range(per_type * len(SERVING_TYPES)):
        kind = SERVING_TYPES[i % len(SERVING_TYPES)]
        p = serving_problem(kind, g_grid, g_coef)
        if kind == "D20_d2":
            p.grids = shared
        p.name = f"{kind}_{i}"
        p.seed = seed
        jobs.append(p)
    for key, cnt in (extra_grids or {}).items():
        i = int(key)
        p = jobs[i]
        rng = np.random.default_rng([seed, 1000 + i])
        more = [serving_extra_grid(p, rng) for _ in range(int(cnt))]
        if more:
            p.grids = np.ascontiguousarray(
                np.concatenate([p.grids, np.array(more, dtype=np.int32)]))
    return jobs


def family_values(family: int, params, X) -> np.ndarray:
    """The analytic test functions (the inputs the workloads sample) at the
    rows of X ([m][D]), for measuring the accuracy of a recovered expansion."""
    X = np.asarray(X, dtype=np.float64)
    D = X.shape[1]
    p = np.asarray(params, dtype=np.float64)
    if family == FAMILY_EXPCOS:
        return np.exp(-(X * X) @ p[:D]) * np.cos(X @ p[D:2 * D])
    if family == FAMILY_GAUSS:
        return np.exp(-((X - p[1:1 + D]) ** 2).sum(axis=1) / (2.0 * p[0] * p[0]))
    if family == FAMILY_RUNGE:
        return 1.0 / (1.0 + p[0] * (X * X).sum(axis=1))
    if family == FAMILY_OSC:
        r2 = (X * X).sum(axis=1)
        return np.sin(3.0 * np.cos(3.0 * np.exp(r2))) + np.exp(np.sin(3.0 * X.sum(axis=1)))
    raise ValueError(f"no analytic values for family {family}")


def poisson_arrivals(seed: int, rate: float, duration: float):
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    _, _, g_arr = streams(seed)
    t, out = 0.0, []
    while True:
        t += g_arr.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)
