// The stacked operator A and the CGLS least-squares iteration (Sec. 3.4,
// Alg. 3: c* = argmin_c || F f - A c ||_2, solved by conjugate gradients on
// the normal equations).
//
// A is applied without atomics.  q = A c sums, for each row (non-empty bin),
// the support entries that alias to it; the plan stores those entries
// contiguously (sorted by target bin), so each row is one segmented sum in a
// fixed order.  s = A^T r gathers, for each support entry, the K rows it
// aliases to.  Dot products are reduced per workgroup in a fixed tree and the
// partials are summed in a fixed order by every consumer, so every run gives
// the same bits.
//
// Layout: the row vectors r and q are interleaved as (r, q) pairs and the
// column vectors p and s as (p, s) pairs, so each gather is one 16-byte load.
// The row kernel reads a row's first entries from a 4-wide padded copy of
// perm ("ell"), which saves the dependent load of the row's offset; longer
// rows continue in perm.
//
// One CGLS iteration is two kernels.  With k the iteration number:
//   rows_k: gamma_k = ||s_k||^2 (from the column partials), convergence test,
//           beta_{k-1} = gamma_k / gamma_{k-1},
//           r_k = r_{k-1} - alpha_{k-1} q_{k-1},
//           q_k = A p_k with p_k = s_k + beta_{k-1} p_{k-1} formed on the fly,
//           partials of ||q_k||^2;
//   cols_k: alpha_k = gamma_k / ||q_k||^2,
//           p_k = s_k + beta_{k-1} p_{k-1} (stored), c_{k+1} = c_k + alpha_k p_k,
//           s_{k+1} = A^T (r_k - alpha_k q_k), partials of ||s_{k+1}||^2.
// Scalars live in per-iteration history arrays written by workgroup 0 and
// read by the next kernel, so no value is overwritten while another
// workgroup of the same launch may still read it.  The iteration number is
// a device-side base plus a launch-time offset, which lets a fixed chunk of
// iterations be captured once in a HIP graph and replayed.
#include "fct_internal.h"

namespace fct {
namespace {

// Sum over the workgroup; every thread gets the same value.  Wave sums use a
// xor butterfly (each lane adds the same two operands as its partner, so all
// lanes agree bit for bit), then wave 0 adds the wave sums in order.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    sh[8] = r;
  }
  __syncthreads();
  const double r = sh[8];
  __syncthreads();
  return r;
}

// Fixed-order sum of per-workgroup partials (same value in every workgroup).
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int64_t np,
                                               double* sh) {
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
  return block_sum(v, sh);
}

__global__ __launch_bounds__(kBlock) void apply_A_kernel(const int32_t* __restrict__ seg_off,
                                                         const int32_t* __restrict__ perm,
                                                         int64_t M, const double* __restrict__ c,
                                                         double* __restrict__ q) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= M) return;
  double acc = 0.0;
  const int32_t t1 = seg_off[row + 1];
  for (int32_t t = seg_off[row]; t < t1; ++t) acc += c[perm[t]];
  q[row] = acc;
}

__global__ __launch_bounds__(kBlock) void apply_AT_kernel(const int32_t* __restrict__ rowmap,
                                                          int K, int64_t n,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ s) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  for (int l = 0; l < K; ++l) acc += r[rowmap[(int64_t)l * n + j]];
  s[j] = acc;
}

// r_0 = b - A c_0 (c_0 = 0 unless warm), q = 0, iteration state reset.
__global__ __launch_bounds__(kBlock) void cgls_init_rows_kernel(CglsArgs a,
                                                                const double* __restrict__ b,
                                                                int warm) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row == 0) { a.state[0] = 0; a.state[1] = 0; a.state[2] = 0; }
  if (row >= a.M) return;
  double acc = 0.0;
  if (warm) {
    const int32_t t1 = a.seg_off[row + 1];
    for (int32_t t = a.seg_off[row]; t < t1; ++t) acc += a.c[a.perm[t]];
  }
  a.rq[row] = make_double2(b[row] - acc, 0.0);
}

// s_0 = A^T r_0, p = 0, c = 0 unless warm, partials of ||s_0||^2.
__global__ __launch_bounds__(kBlock) void cgls_init_cols_kernel(CglsArgs a, int warm) {
  __shared__ double sh[16];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sv = 0.0;
  if (j < a.n) {
    for (int l = 0; l < a.K; ++l) sv += a.rq[a.rowmap[(int64_t)l * a.n + j]].x;
    a.ps[j] = make_double2(0.0, sv);
    if (!warm) a.c[j] = 0.0;
  }
  const double part = block_sum(sv * sv, sh);
  if (threadIdx.x == 0) a.part_s[blockIdx.x] = part;
}

// Registers that prefetch a column's K aliases before the iteration scalars
// are known; further grids continue in a loop.
constexpr int kPrefetch = 4;

// This thread's share of the other kernel's per-workgroup sums (loaded
// before the state check so the loads overlap).
__device__ __forceinline__ double load_partials(const double* __restrict__ part, int64_t np) {
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
  return v;
}

__global__ __launch_bounds__(kBlock) void cgls_rows_kernel(CglsArgs a, int rel,
                                                           int64_t ncolblocks) {
  __shared__ double sh[16];
  __shared__ int s_state[2];
  // one read per workgroup, so every wave of it takes the same branch
  if (threadIdx.x == 0) { s_state[0] = a.state[0]; s_state[1] = a.state[1]; }
  const double gpart = load_partials(a.part_s, ncolblocks);
  // operands that do not depend on this iteration's scalars
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = row < a.M;
  double2 rq_old = make_double2(0.0, 0.0);
  int4 e = make_int4(-1, -1, -1, -1);
  if (active) {
    rq_old = a.rq[row];
    e = a.ell[row];
  }
  const double2 z = make_double2(0.0, 0.0);
  const double2 v0 = e.x >= 0 ? a.ps[e.x] : z;
  const double2 v1 = e.y >= 0 ? a.ps[e.y] : z;
  const double2 v2 = e.z >= 0 ? a.ps[e.z] : z;
  const double2 v3 = e.w >= 0 ? a.ps[e.w] : z;
  __syncthreads();
  if (s_state[0] != 0) return;                       // converged or stopped earlier
  const int k = s_state[1] + rel;
  double gprev = 1.0, g0 = 0.0, alpha_prev = 0.0;
  if (k > 0) { gprev = a.hist_gamma[k - 1]; g0 = a.hist_gamma[0]; alpha_prev = a.hist_alpha[k - 1]; }
  const double gamma = block_sum(gpart, sh);
  double beta = 0.0;
  bool stop;
  if (k == 0) {
    stop = !(gamma > 0.0);                           // zero (or non-finite) A^T b
  } else {
    beta = gamma / gprev;
    stop = !(gamma > a.tol2 * g0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.hist_gamma[k] = gamma;
    if (stop) a.state[0] = k + 1;
  }
  if (stop) return;
  double qv = 0.0;
  if (active) {
    // terms in perm order: p_k = s_k + beta p_{k-1} for each aliased column
    if (e.x >= 0) qv += fma(beta, v0.x, v0.y);
    if (e.y >= 0) qv += fma(beta, v1.x, v1.y);
    if (e.z >= 0) qv += fma(beta, v2.x, v2.y);
    if (e.w >= 0) qv += fma(beta, v3.x, v3.y);
    if (e.w < -1) {                                  // long row: rest of its run in perm
      const int32_t t1 = a.seg_off[row + 1];
      for (int32_t t = -(e.w + 2); t < t1; ++t) {
        const double2 v = a.ps[a.perm[t]];
        qv += fma(beta, v.x, v.y);
      }
    }
    a.rq[row] = make_double2(fma(-alpha_prev, rq_old.y, rq_old.x), qv);
  }
  const double part = block_sum(qv * qv, sh);
  if (threadIdx.x == 0) a.part_q[blockIdx.x] = part;
}

__global__ __launch_bounds__(kBlock) void cgls_cols_kernel(CglsArgs a, int rel,
                                                           int64_t nrowblocks) {
  __shared__ double sh[16];
  __shared__ int s_state[2];
  if (threadIdx.x == 0) { s_state[0] = a.state[0]; s_state[1] = a.state[1]; }
  const double dpart = load_partials(a.part_q, nrowblocks);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = j < a.n;
  double2 ps_old = make_double2(0.0, 0.0);
  double c_old = 0.0;
  double2 g[kPrefetch];
  if (active) {
    ps_old = a.ps[j];
    c_old = a.c[j];
  }
#pragma unroll
  for (int l = 0; l < kPrefetch; ++l) {
    g[l] = make_double2(0.0, 0.0);
    if (active && l < a.K) g[l] = a.rq[a.rowmap[(int64_t)l * a.n + j]];
  }
  __syncthreads();
  if (s_state[0] != 0) return;
  const int k = s_state[1] + rel;
  const double gamma = a.hist_gamma[k];
  const double gprev = (k > 0) ? a.hist_gamma[k - 1] : 1.0;
  const double delta = block_sum(dpart, sh);
  const double beta = (k > 0) ? gamma / gprev : 0.0;
  if (!(delta > 0.0)) {                              // A p = 0: breakdown
    if (blockIdx.x == 0 && threadIdx.x == 0) { a.state[2] = 1; a.state[0] = k + 1; }
    return;
  }
  const double alpha = gamma / delta;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.hist_alpha[k] = alpha;
  double sv = 0.0;
  if (active) {
    const double pv = fma(beta, ps_old.x, ps_old.y);
    a.c[j] = fma(alpha, pv, c_old);
#pragma unroll
    for (int l = 0; l < kPrefetch; ++l)
      if (l < a.K) sv += fma(-alpha, g[l].y, g[l].x);
    for (int l = kPrefetch; l < a.K; ++l) {
      const double2 v = a.rq[a.rowmap[(int64_t)l * a.n + j]];
      sv += fma(-alpha, v.y, v.x);
    }
    a.ps[j] = make_double2(pv, sv);
  }
  const double part = block_sum(sv * sv, sh);
  if (threadIdx.x == 0) a.part_s[blockIdx.x] = part;
}

__global__ __launch_bounds__(kBlock) void cgls_gamma_kernel(CglsArgs a, int k,
                                                            int64_t ncolblocks) {
  __shared__ double sh[16];
  const double gamma = sum_partials(a.part_s, ncolblocks, sh);
  if (threadIdx.x == 0) a.hist_gamma[k] = gamma;
}

__global__ void cgls_set_state_kernel(int32_t* state, int s0, int s1, int s2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { state[0] = s0; state[1] = s1; state[2] = s2; }
}

__global__ void cgls_advance_kernel(int32_t* state, int chunk) {
  if (threadIdx.x == 0 && blockIdx.x == 0) state[1] += chunk;
}

}  // namespace

int64_t cgls_row_blocks(int64_t M) { return ceil_div(M, kBlock); }
int64_t cgls_col_blocks(int64_t n) { return ceil_div(n, kBlock); }

hipError_t launch_apply_A(const int32_t* seg_off, const int32_t* perm, int64_t M, const double* c,
                          double* q, hipStream_t s) {
  hipLaunchKernelGGL(apply_A_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0, s,
                     seg_off, perm, M, c, q);
  return hipGetLastError();
}

hipError_t launch_apply_AT(const int32_t* rowmap, int K, int64_t n, const double* r, double* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(apply_AT_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s,
                     rowmap, K, n, r, out);
  return hipGetLastError();
}

hipError_t launch_cgls_init(const CglsArgs& a, const double* b, bool warm, hipStream_t s) {
  hipLaunchKernelGGL(cgls_init_rows_kernel, dim3((unsigned)cgls_row_blocks(a.M)), dim3(kBlock), 0,
                     s, a, b, warm ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cgls_init_cols_kernel, dim3((unsigned)cgls_col_blocks(a.n)), dim3(kBlock), 0,
                     s, a, warm ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_cgls_rows(const CglsArgs& a, int rel, hipStream_t s) {
  hipLaunchKernelGGL(cgls_rows_kernel, dim3((unsigned)cgls_row_blocks(a.M)), dim3(kBlock), 0, s,
                     a, rel, cgls_col_blocks(a.n));
  return hipGetLastError();
}

hipError_t launch_cgls_cols(const CglsArgs& a, int rel, hipStream_t s) {
  hipLaunchKernelGGL(cgls_cols_kernel, dim3((unsigned)cgls_col_blocks(a.n)), dim3(kBlock), 0, s,
                     a, rel, cgls_row_blocks(a.M));
  return hipGetLastError();
}

hipError_t launch_cgls_iter(const CglsArgs& a, int rel, hipStream_t s) {
  hipError_t e = launch_cgls_rows(a, rel, s);
  if (e != hipSuccess) return e;
  return launch_cgls_cols(a, rel, s);
}

hipError_t launch_cgls_gamma(const CglsArgs& a, int k, hipStream_t s) {
  hipLaunchKernelGGL(cgls_gamma_kernel, dim3(1), dim3(kBlock), 0, s, a, k, cgls_col_blocks(a.n));
  return hipGetLastError();
}

hipError_t launch_cgls_timing_state(int32_t* state, int k, hipStream_t s) {
  hipLaunchKernelGGL(cgls_set_state_kernel, dim3(1), dim3(64), 0, s, state, 0, k, 0);
  return hipGetLastError();
}

hipError_t launch_cgls_timing_state_restore(int32_t* state, int stop, int breakdown,
                                            hipStream_t s) {
  hipLaunchKernelGGL(cgls_set_state_kernel, dim3(1), dim3(64), 0, s, state, stop, 0, breakdown);
  return hipGetLastError();
}

hipError_t launch_cgls_advance(int32_t* state, int chunk, hipStream_t s) {
  hipLaunchKernelGGL(cgls_advance_kernel, dim3(1), dim3(64), 0, s, state, chunk);
  return hipGetLastError();
}

}  // namespace fct
