/*
 * libfct: sparse Fast Chebyshev Transform on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the transform's hot path, after "A (Sparse) Fast Chebyshev
 * Transform for High-Dimensional (Smooth Function) Approximation" (Jones,
 * Letourneau, Morse, Langston; arXiv 2309.14584).  Given the known support
 * of a function's Chebyshev expansion (the multi-indices of its nonzero
 * coefficients, Sec. 4.5.3) and an L-grid of tensor Chebyshev grids
 * (Sec. 3.2), the library
 *
 *   1. builds the alias structure of the stacked operator A (Sec. 3.1,
 *      eq. aliasing_matrix_nd_diff; Alg. 2 without its conditioning loop),
 *   2. samples f on every grid (Alg. 3, sampling step),
 *   3. applies a separable D-dimensional DCT-I to every grid (Alg. 3,
 *      transform step) and keeps the non-empty aliasing bins,
 *   4. solves min_c || F f - A c ||_2 by CGLS (Alg. 3, least-squares step).
 *
 * Grids are Chebyshev-Lobatto grids: a grid is given by D Lobatto degrees
 * N_i >= 0, with nodes x_k = cos(pi k / N_i), k = 0..N_i (N_i = 0 is the
 * single node x = 1).  On such a grid T_n coincides with T_m,
 * m = fold(n, N) = min(r, 2N - r), r = n mod 2N (the Lobatto analogue of
 * Lemma 3.1), so every block A^(l) is 0/1 with exactly one 1 per column.
 * The transform is the interpolation-normalised DCT-I
 *   a_m = (g_m / N) [v_0 + (-1)^m v_N + 2 sum_{k=1}^{N-1} v_k cos(pi m k / N)],
 *   g_0 = g_N = 1/2, g_m = 1 otherwise,
 * which maps the samples of T_n to the unit vector of fold(n).
 *
 * Layouts (all row-major, "last dimension fastest"):
 *   support   int32 [n_support][D], entries >= 0, no duplicate rows;
 *   grids     int32 [K][D], Lobatto degrees 0 <= N_i <= FCT_MAX_DEGREE;
 *   samples   double [P_total]: grid l's tensor of shape (N_1+1,...,N_D+1)
 *             at offset point_offset(l), grids concatenated in order;
 *   b         double [M]: the transform of grid l at its non-empty bins,
 *             rows ordered by (grid ascending, flat bin ascending);
 *   c         double [n_support] in support order.
 *
 * Conventions: every function returns an fct_status; on failure a message
 * is available from fct_last_error() (per thread).  No call aborts the
 * process.  Functions that take a stream enqueue their GPU work on it and
 * return without waiting, except where stated.  Device pointers ("d_")
 * are caller-owned device memory on the plan's device; the library never
 * frees them.  A plan is immutable after creation (fct_plan_tune aside) and
 * may be used from several streams at once; a workspace belongs to one
 * stream at a time.
 */
#ifndef LIBFCT_FCT_H
#define LIBFCT_FCT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FCT_ABI_VERSION 3
#define FCT_MAX_DIM 128      /* largest D accepted */
#define FCT_MAX_DEGREE 63    /* largest Lobatto degree N_i (64 nodes) */

typedef enum fct_status {
  FCT_OK = 0,
  FCT_EINVAL = 1,      /* invalid argument or unsupported size */
  FCT_ENOMEM = 2,      /* device or host allocation failed */
  FCT_EDEVICE = 3,     /* a HIP runtime call failed */
  FCT_ERANK = 4,       /* the grids cannot separate the support (rank pre-check) */
  FCT_ENOCONV = 5,     /* the solve stopped at its iteration limit */
  FCT_ENONFINITE = 6   /* NaN or Inf met in the right-hand side */
} fct_status;

/* Function families understood by fct_sample. */
typedef enum fct_family {
  FCT_F_PLANTED = 0, /* p(x) = sum_j c_j T_{n_j}(x) on the support; params unused,
                        d_coeffs = device double [n_support] */
  FCT_F_EXPCOS = 1,  /* exp(-sum_i a_i x_i^2) cos(sum_i w_i x_i); params = a[D], w[D] */
  FCT_F_GAUSS = 2,   /* exp(-|x - x0|^2 / (2 s^2)); params = s, x0[D] */
  FCT_F_RUNGE = 3,   /* 1 / (1 + alpha |x|^2) (Sec. 4.3.1, f1); params = alpha */
  FCT_F_OSC = 4      /* sin(3 cos(3 exp|x|^2)) + exp(sin(3 sum_i x_i)) (Sec. 4.3.2, f2) */
} fct_family;

/* Arithmetic of the DCT contractions.  FCT_DCT_F32 and FCT_DCT_BF16X3 need
 * every extent <= 32 (degrees <= 31); FCT_DCT_F64 takes extents up to 64. */
typedef enum fct_dct_mode {
  FCT_DCT_F64 = 0,    /* FP64 products and sums, FP64 intermediate tensors */
  FCT_DCT_F32 = 1,    /* FP32 products and sums, FP32 intermediate tensors */
  FCT_DCT_BF16X3 = 2  /* operands split into bf16 high/low parts (round to nearest
                         even); C_hi x_hi + C_hi x_lo + C_lo x_hi with FP32
                         accumulation; FP32 intermediate tensors */
} fct_dct_mode;

/* Units that run the FP64 and FP32 DCT contractions of a plan (set with
 * fct_plan_set_dct_engine or chosen by fct_plan_tune).  The two engines
 * accumulate in different orders, so their results differ by rounding
 * within the mode's precision; each is deterministic. */
typedef enum fct_dct_engine {
  FCT_ENGINE_VECTOR = 0,  /* E*E multiply-adds per fibre of E points on the
                             vector units (default for FP64 and FP32) */
  FCT_ENGINE_MATRIX = 1   /* 16x16x4 MFMA tiles on the matrix cores, 16 fibres
                             per wave (extents <= 32; the only engine of
                             FCT_DCT_BF16X3) */
} fct_dct_engine;

/* Arithmetic of the least-squares solve. */
typedef enum fct_solve_mode {
  FCT_SOLVE_F64 = 0,        /* CGLS in FP64 throughout */
  FCT_SOLVE_F32_REFINE = 1, /* rounds of conjugate gradients on the normal equations
                               with FP32 vectors (q, p, s) and FP64 inner products,
                               each started from s = A^T (b - A c) computed in FP64
                               for the FP64 iterate c (iterative refinement, which
                               converges for inconsistent systems too), continuing the
                               previous round's search direction unless
                               restart_rounds is set; stops on the FP64 normal
                               residual */
  FCT_SOLVE_F32 = 2         /* a single such round, to tol (default 2e-7) on its own
                               FP32 normal residual; rel_normal_residual reports the
                               FP64 one */
} fct_solve_mode;

/* Plan creation flags. */
#define FCT_PLAN_ALLOW_RANK_DEFICIENT 1u /* skip the per-dimension rank pre-check */
/* The paper's literal operator (Sec. 2 "Problem setup", Sec. 3.1, Lemma 3.1):
 * Chebyshev-Gauss grids x_k = cos(pi (k + 1/2) / (N + 1)), k = 0..N, and the
 * DCT-II a_m = (g_m 2 / (N + 1)) sum_k v_k cos(pi m (2k + 1) / (2 (N + 1))),
 * g_0 = 1/2 else 1 (the quadrature of eq. quad_1D with rows m >= 1 doubled,
 * so that samples of T_m, m <= N, map to e_m).  T_a then equals s T_m on
 * the nodes with r = a mod 2(N+1), m = min(r, 2(N+1) - r) and the sign
 * s = (-1)^(a div 2(N+1)) for r < N + 1, its negation for r > N + 1; at
 * r = N + 1 (T_{N+1}) it vanishes.  A's entries are the products of the 1-D
 * signs over the axes, in {-1, 0, 1}; a zero entry stays in the structure
 * (bin with m_i = N_i) with weight 0.  A Gauss plan: single problem (not
 * batched), FP64 solves only, solved by the one-reduction CG (see
 * fct_solve_opts.one_reduction, implied); sampling, transforms, apply,
 * condition estimate and evaluation as for Lobatto plans.  N_i = 0 is the
 * single node x = 0. */
#define FCT_PLAN_GAUSS 2u
/* Row order for sparse supports: each grid's rows ordered by their first
 * (smallest) support column instead of by bin, runs unchanged.  When most
 * rows hold one entry (random high-dimensional supports) the matvecs then
 * read p and r nearly in order instead of at random.  perm, seg_off, bin_id
 * and rowmap (fct_plan_export) follow this order; b from fct_dct is in it
 * (the transform writes the bins in bin order to the workspace, then gathers
 * them), so fct_dct needs the workspace.  Such plans may be batched (each
 * problem keeps its own order); not with FCT_PLAN_GAUSS. */
#define FCT_PLAN_ROWS_BY_MEMBER 4u

typedef struct fct_plan fct_plan;
typedef struct fct_ws fct_ws;

typedef struct fct_plan_info {
  int32_t D;              /* dimension */
  int32_t K;              /* number of grids */
  int64_t n_support;      /* number of unknown coefficients */
  int64_t total_points;   /* P_total = sum_l prod_i (N_i^(l) + 1) */
  int64_t total_rows;     /* M = number of non-empty bins over all grids */
  int64_t max_points;     /* largest single-grid point count */
  int32_t max_degree;     /* largest N_i over all grids */
  int32_t dct_levels;     /* kernel launches per DCT (axis-group passes) */
  int64_t device_bytes;   /* device memory held by the plan */
  int32_t problems;       /* 1, or the number of problems of a batch plan */
  int32_t reserved;
  int64_t entries;        /* nonzeros of A: sum over problems of K * n_support */
} fct_plan_info;

typedef struct fct_solve_opts {
  int32_t mode;         /* fct_solve_mode */
  int32_t maxit;        /* iteration limit; 0 selects 4000 */
  int32_t check_every;  /* iterations between host convergence checks; 0 selects 32 */
  int32_t warm_start;   /* nonzero: d_c holds the starting guess, else start from 0 */
  int32_t use_graph;    /* nonzero: replay the iteration chunk as a HIP graph */
  int32_t timing;       /* nonzero: after the solve, time 200 back-to-back launches of
                           the row kernel and of the column kernel with HIP events on
                           `stream` and report the means in fct_solve_info (d_c is
                           left as solved) */
  double tol;           /* stop when ||A^T r||_2 <= tol ||A^T r_0||_2; 0 selects 1e-14
                           (2e-7 for FCT_SOLVE_F32) */
  int32_t max_refine;   /* FCT_SOLVE_F32_REFINE: most rounds; 0 selects 12 */
  int32_t restart_rounds; /* FCT_SOLVE_F32_REFINE: nonzero restarts conjugate gradients
                           (p = 0) at every round; 0 (default) continues each problem's
                           last search direction with the recomputed FP64 residual
                           (a reliable update) */
  double inner_tol;     /* FCT_SOLVE_F32_REFINE: per-round reduction of the FP32
                           normal residual; 0 selects 1e-5 */
  int32_t single_kernel; /* 1: for one problem whose row and column blocks each
                           get a workgroup of their own, run each chunk of
                           iterations as one cooperative kernel with grid
                           barriers (same bits as two kernels per iteration;
                           on MI355X about 6x slower, since every barrier's
                           agent-scope fences write back and invalidate L2);
                           0 (default): two kernels per iteration */
  int32_t one_reduction; /* 1: FP64 solve of a single-problem plan as conjugate
                           gradients on A^T A c = A^T b with one reduction per
                           iteration (Chronopoulos-Gear recurrences; the CGLS
                           iterates in exact arithmetic, rounded differently):
                           one kernel per iteration that forms A^T A r from
                           each column's neighbour list (built on first use
                           with this workspace), instead of the row and
                           column kernels; about a quarter of their memory
                           traffic, faster on small problems, not on the D=6
                           workload, where both are bound by launch and gather
                           latency.  Implied for FCT_PLAN_GAUSS plans.  Timing
                           mode then reports that kernel in rows_kernel_us
                           (cols_kernel_us 0).
                           FCT_EINVAL with a batch, FP32 modes or
                           single_kernel.  0 (default): CGLS */
} fct_solve_opts;

typedef struct fct_solve_info {
  int32_t iterations;   /* CGLS iterations taken (largest over the plan's problems) */
  int32_t converged;    /* 1 if the tolerance was met (by every problem) */
  double rel_normal_residual; /* ||A^T r_k||_2 / ||A^T r_0||_2 at exit (largest) */
  double normal_residual0;    /* ||A^T r_0||_2 (largest) */
  double rows_kernel_us;      /* timing mode: mean time of one row-kernel launch (q = A p) */
  double cols_kernel_us;      /* timing mode: mean time of one column-kernel launch (A^T r) */
  int32_t problems;           /* problems solved */
  int32_t problems_converged; /* problems that met the tolerance */
  int32_t refinements;        /* FP32 rounds (largest over problems; 0 in FP64 mode) */
  int32_t reserved;
} fct_solve_info;

/* ---- errors ------------------------------------------------------------ */

/* Message of the last failing call on this thread ("" if none). */
const char* fct_last_error(void);
/* Static name of a status code. */
const char* fct_status_string(fct_status s);
/* FCT_ABI_VERSION of the loaded library. */
int32_t fct_abi_version(void);

/* ---- plans (alias structure of A; Sec. 3.1-3.3, Alg. 2) ------------------
 *
 * fct_plan_create: copies the support and the grids to the current HIP
 * device and builds, on the GPU, the alias structure of the stacked 0/1
 * operator A = [A^(1); ...; A^(K)]:
 *   alias[l][j]  flat bin of support row j on grid l:
 *                sum_i fold(n_ji, N_i^(l)) * stride_i^(l), strides row-major;
 *   perm[l][.]   support rows of grid l sorted by (bin, row) (stable);
 *   seg_off[r]   start of row r's run in perm (flattened, K*n entries);
 *   bin_id[r]    flat bin of row r;  rowmap[l][j] = global row of j on l.
 * support and grids are host arrays read during the call only.  Unless
 * flags has FCT_PLAN_ALLOW_RANK_DEFICIENT, the call fails with FCT_ERANK
 * when some dimension i has two degrees a != a' <= max_j n_ji with
 * fold(a, N_i^(l)) = fold(a', N_i^(l)) on every grid (two coefficients that
 * differ only in entry i would then be indistinguishable).
 * With FCT_PLAN_GAUSS the pre-check asks, per dimension, that every degree's
 * signed 1-D rows over the K grids be nonzero (T_a does not vanish on every
 * grid) and that no two degrees have the same rows up to sign.
 * Limits (else FCT_EINVAL): 1 <= D <= FCT_MAX_DIM, n_support >= 1,
 * 1 <= K < 2^19, K * n_support < 2^31, each grid's point count < 2^44,
 * 0 <= N_i <= FCT_MAX_DEGREE, duplicate support rows rejected.
 * Synchronous: waits for its work on `stream` before returning.
 */
fct_status fct_plan_create(int32_t D, int64_t n_support, const int32_t* support,
                           int32_t K, const int32_t* grids, uint32_t flags,
                           hipStream_t stream, fct_plan** out);
void fct_plan_destroy(fct_plan* plan);
fct_status fct_plan_get_info(const fct_plan* plan, fct_plan_info* out);
/* Host query of grid l: point count, non-empty rows, offset of its tensor in
 * the sample buffer and of its first row in b.  Any pointer may be NULL. */
fct_status fct_plan_grid(const fct_plan* plan, int32_t grid, int64_t* points,
                         int64_t* rows, int64_t* point_offset, int64_t* row_offset);
/* Copy the alias structure into caller device buffers (any may be NULL):
 * d_alias int64 [K*n], d_perm int32 [K*n], d_seg_off int32 [M+1],
 * d_bin_id int64 [M], d_rowmap int32 [K*n].  Asynchronous on `stream`. */
fct_status fct_plan_export(const fct_plan* plan, int64_t* d_alias, int32_t* d_perm,
                           int32_t* d_seg_off, int64_t* d_bin_id, int32_t* d_rowmap,
                           hipStream_t stream);
/* Entry weights of A (Gauss plans: the sign in {-1, 0, 1} of support row j on
 * grid l; Lobatto plans: all 1) into d_w int8 [K*n], layout of alias.
 * Single-problem plans.  Asynchronous on `stream`. */
fct_status fct_plan_weights(const fct_plan* plan, int8_t* d_w, hipStream_t stream);
/* Node coordinates of grid `grid` along dimension `dim` as used by the
 * sampler: host_out[k] = cos(pi k / N), k = 0..N, or for a Gauss plan
 * cos(pi (k + 1/2) / (N + 1)) (synchronous). */
fct_status fct_grid_nodes(const fct_plan* plan, int32_t grid, int32_t dim,
                          double* host_out);

/* ---- batches of independent problems ------------------------------------
 *
 * fct_batch_create: packs `count` single-problem plans (same device) into
 * one batch plan whose buffers are the concatenation of the problems'
 * buffers in order: samples (problem p's grids at point_offset(p)), b (its
 * rows at row_offset(p)) and c (its coefficients at col_offset(p)).  A
 * batch plan is accepted by fct_dct, fct_dct_full, fct_apply_A, fct_apply_AT,
 * fct_solve and by fct_sample with FCT_F_PLANTED (d_coeffs concatenated);
 * every DCT level and every CGLS half-iteration of all problems is one kernel
 * launch.  The solve keeps separate CG scalars, convergence tests and
 * reduction orders per problem, so each problem's result is bitwise the same
 * as when it is solved alone.  The source plans are only read during the
 * call and may be destroyed afterwards.  Synchronous.
 * Limits: sum of K*n_support < 2^31, sum of rows < 2^31.
 */
fct_status fct_batch_create(int32_t count, const fct_plan* const* plans,
                            hipStream_t stream, fct_plan** out);
/* Layout of problem p of a plan (any pointer may be NULL). */
fct_status fct_plan_problem(const fct_plan* plan, int32_t p, int64_t* n_support,
                            int64_t* rows, int64_t* col_offset, int64_t* row_offset,
                            int64_t* point_offset, int64_t* points);

/* ---- workspaces ---------------------------------------------------------
 * Device scratch for one stream: the DCT intermediate tensor (P_total
 * doubles) and the CGLS vectors and scalars.  Allocated on the plan's device.
 */
fct_status fct_ws_create(const fct_plan* plan, fct_ws** out);
void fct_ws_destroy(fct_ws* ws);

/* ---- sampling (Alg. 3: sample f on the L-grid) ---------------------------
 * Writes f at every node of every grid into d_samples (double [P_total]).
 * params: host array of n_params doubles as listed for fct_family.
 * FCT_F_PLANTED evaluates p = sum_j c_j T_{n_j} by aliasing c onto each
 * grid (q = A c) and applying the inverse DCT-I (evaluation at the nodes);
 * it needs d_coeffs and a workspace.  Other families ignore d_coeffs and ws.
 */
fct_status fct_sample(const fct_plan* plan, int32_t family, const double* params,
                      int32_t n_params, const double* d_coeffs, double* d_samples,
                      fct_ws* ws, hipStream_t stream);

/* ---- transform (Alg. 3: DCTs of every grid; eq. multi_dim_dct) ----------
 * fct_dct: d_b[r] = (F^(l) f^(l))[bin_id[r]] for every non-empty row r,
 * i.e. the separable interpolation-normalised DCT-I of each grid restricted
 * to the bins that some support row aliases to.  d_samples double [P_total],
 * d_b double [M].  mode: fct_dct_mode.
 * fct_dct_full: the whole transformed tensors, d_out double [P_total].
 */
fct_status fct_dct(const fct_plan* plan, const double* d_samples, double* d_b,
                   int32_t mode, fct_ws* ws, hipStream_t stream);
fct_status fct_dct_full(const fct_plan* plan, const double* d_samples, double* d_out,
                        int32_t mode, fct_ws* ws, hipStream_t stream);

/* ---- condition of A and the grid count (Sec. 3.3, Alg. 2) ---------------
 * fct_plan_condition: extreme eigenvalues of A^T A by Lanczos from the start
 * vector d_v0 (double [n], nonzero; the caller draws it, e.g. Gaussian) with
 * full reorthogonalisation, on a single-problem plan.  Runs until
 * max_steps steps (at most n), an invariant subspace (exact), or, with
 * tol > 0, until both extreme Ritz values moved by at most tol * lambda_max
 * over the last 8 steps (checked from step 16).  The Ritz values bound the
 * spectrum from inside (lambda_min from above), so a short run can only
 * under-state kappa.  full_rank = lambda_min > rank_tol * lambda_max;
 * kappa = sqrt(lambda_max / lambda_min), HUGE_VAL when not full rank.
 * Allocates (max_steps + 1) vectors of n doubles (FCT_EINVAL above 32 GiB);
 * synchronous on `stream`.  Sums are in fixed order (reproducible).
 * fct_select_grids: Alg. 2's loop.  For L = 1, 2, ... builds the plan of the
 * first L candidate grids (host int32 [n_cand][D], drawn by the caller with
 * Alg. 1; plan flag FCT_PLAN_ALLOW_RANK_DEFICIENT) and stops at the first L
 * whose estimate is full rank with kappa <= kappa0: *out_L = L, out = its
 * estimate.  FCT_ENOCONV with *out_L = 0 if no prefix qualifies. */
typedef struct fct_cond_info {
  double lambda_min;    /* smallest Ritz value of A^T A */
  double lambda_max;    /* largest Ritz value of A^T A */
  double kappa;         /* sqrt(lambda_max / lambda_min); HUGE_VAL if not full rank */
  int32_t steps;        /* Lanczos steps taken */
  int32_t full_rank;    /* lambda_min > rank_tol * lambda_max */
} fct_cond_info;

fct_status fct_plan_condition(const fct_plan* plan, const double* d_v0, int32_t max_steps,
                              double tol, double rank_tol, hipStream_t stream,
                              fct_cond_info* out);
fct_status fct_select_grids(int32_t D, int64_t n_support, const int32_t* support,
                            int32_t n_cand, const int32_t* candidates, double kappa0,
                            const double* d_v0, int32_t max_steps, double tol, double rank_tol,
                            hipStream_t stream, int32_t* out_L, fct_cond_info* out);

/* ---- evaluation (Sec. 2: p(x) = sum over the support of c_n T_n(x)) ------
 * d_f[q] = sum_j d_c[j] prod_i T_{S[j][i]}(d_x[q * D + i]) for 0 <= q < m:
 * the expansion with coefficients d_c (double [n], the plan's support
 * order) at m arbitrary points d_x (double, row-major [m][D]; any real
 * coordinates, T_k from T_{k+1} = 2 x T_k - T_{k-1}).  d_f double [m].
 * ws (optional, the plan's workspace) lets few points with a long support
 * run on the whole device: the support is cut into slices whose partial sums
 * go to the workspace's scratch tensor and are added in slice order.  Each
 * point's terms are summed in a fixed order for given (m, ws present), so
 * results are reproducible.  Single-problem plans only; FCT_EINVAL for a
 * batch plan, m < 0, NULL pointers, a workspace of another plan, or a
 * per-point table D * (max support entry + 1) above the LDS capacity (about
 * 290 values).  m = 0 does nothing.  Asynchronous on `stream`.
 */
fct_status fct_eval(const fct_plan* plan, const double* d_c, int64_t m, const double* d_x,
                    double* d_f, fct_ws* ws, hipStream_t stream);

/* ---- operator (eq. main_linear_system) ----------------------------------
 * fct_apply_A:  d_q[r] = sum over support rows j aliased to row r of d_c[j]
 *               (double [n] -> double [M]); summed in perm order.
 * fct_apply_AT: d_s[j] = sum_l d_r[rowmap[l][j]] (double [M] -> double [n]),
 *               summed in grid order.  No atomics: results are reproducible.
 * For a Gauss plan every term carries its entry weight (fct_plan_weights).
 */
fct_status fct_apply_A(const fct_plan* plan, const double* d_c, double* d_q,
                       hipStream_t stream);
fct_status fct_apply_AT(const fct_plan* plan, const double* d_r, double* d_s,
                        hipStream_t stream);

/* DCT engine of one mode of a plan (fct_dct_engine).  FCT_EINVAL for an
 * unknown mode or engine, the vector engine with FCT_DCT_BF16X3, or the
 * matrix engine on a plan with an extent above 32.  Not to be called while
 * other calls use the plan. */
fct_status fct_plan_set_dct_engine(fct_plan* plan, int32_t dct_mode, int32_t engine);

/* Autotuner (the batched form's tile shapes): times the forward DCT
 * (dct_mode) with LDS tiles of 1024, 2048 and 4096 elements on each engine
 * the mode allows and, for a batch plan, the FP32 row kernels with LDS units
 * of 4096 ... 32768 rows, on the plan's own shapes, and keeps the fastest of
 * each in the plan.  The tile and unit choices leave every result unchanged
 * (only the work decomposition changes); a change of DCT engine changes the
 * DCT's rounding (fct_dct_engine).  Uses `ws` (its solver state is
 * overwritten) and allocates temporary device buffers; synchronous on
 * `stream`.  Not to be called while other calls use the plan or its
 * workspaces.  `out` (optional) receives the choices and the timings. */
typedef struct fct_tune_info {
  int32_t dct_tile;     /* chosen LDS tile of the DCT passes (elements) */
  int32_t unit_rows;    /* chosen rows per LDS unit of the FP32 rounds (0: none) */
  double dct_us[3];     /* forward DCT, vector engine, per tile 1024, 2048, 4096
                           (0: not run) */
  double rows_us[4];    /* FP32 row kernels per unit candidate 4096 ... 32768 (0: not run) */
  int32_t dct_engine;   /* chosen engine of dct_mode (fct_dct_engine) */
  int32_t reserved;
  double dct_matrix_us[3];  /* forward DCT, matrix engine, per tile (0: not run) */
} fct_tune_info;

fct_status fct_plan_tune(fct_plan* plan, fct_ws* ws, int32_t dct_mode, hipStream_t stream,
                         fct_tune_info* out);

/* ---- least squares (Sec. 3.4, Alg. 3: c* = argmin ||F f - A c||_2) -------
 * CGLS on A c ~ b from c_0 = 0 (or the warm start in d_c).  Writes the
 * iterate into d_c (double [n]).  Synchronous: iterations are enqueued in
 * chunks of at most opts->check_every, two chunks deep; the host reads the
 * convergence state of each chunk while the next one runs, and returns
 * after the stream has drained.
 * opts may be NULL (defaults), info may be NULL.  Returns FCT_ENOCONV if
 * maxit is reached first (d_c still holds the last iterate) and
 * FCT_ENONFINITE if ||A^T b|| is not finite.
 */
fct_status fct_solve(const fct_plan* plan, const double* d_b, double* d_c,
                     const fct_solve_opts* opts, fct_solve_info* info,
                     fct_ws* ws, hipStream_t stream);
/* Result of problem p in the workspace's last fct_solve (host copy). */
fct_status fct_ws_problem_info(const fct_ws* ws, int32_t p, fct_solve_info* out);

#ifdef __cplusplus
}
#endif

#endif /* LIBFCT_FCT_H */
