// Vector kernels of the condition estimate of A (Alg. 2's test kappa(A) <=
// kappa_0): Lanczos on A^T A with full reorthogonalisation.  Every sum is
// formed in a fixed order (per-workgroup partials, then one ordered sum), so
// the estimate is reproducible.
#include <algorithm>

#include "fct_internal.h"

namespace fct {
namespace {

// Sum over the workgroup in wave order (thread 0 holds the result).
__device__ __forceinline__ double cond_block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// part[b * ldp + i] = sum over workgroup b's slice of elements of
// X[i][e] * w[e], for rows i < cnt (row stride ld).  Workgroup b owns the
// contiguous slice [b * len, (b + 1) * len); wave w takes rows i = w (mod 4)
// and reduces each row with a butterfly (no barriers).
__global__ __launch_bounds__(kBlock) void multi_dot_kernel(const double* __restrict__ X,
                                                           int64_t ld, int cnt,
                                                           const double* __restrict__ w,
                                                           int64_t n, double* __restrict__ part,
                                                           int64_t ldp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t len = (n + gridDim.x - 1) / gridDim.x;
  const int64_t e0 = (int64_t)blockIdx.x * len;
  const int64_t e1 = min(n, e0 + len);
  for (int i = wave; i < cnt; i += kBlock / 64) {
    const double* xi = X + (int64_t)i * ld;
    double acc = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += 64) acc = fma(xi[e], w[e], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) part[(int64_t)blockIdx.x * ldp + i] = acc;
  }
}

// out[i] = sum over b < nb of part[b * ldp + i], one workgroup per row i:
// thread t adds b = t, t + kBlock, ... in order, then the workgroup sum.
__global__ __launch_bounds__(kBlock) void reduce_rows_kernel(const double* __restrict__ part,
                                                             int nb, int64_t ldp,
                                                             double* __restrict__ out) {
  __shared__ double sh[kBlock / 64];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) acc += part[(int64_t)b * ldp + i];
  const double s = cond_block_sum(acc, sh);
  if (threadIdx.x == 0) out[i] = s;
}

// w[e] -= sum_{i < cnt} X[i][e] * h[i], terms in row order.
__global__ __launch_bounds__(kBlock) void orth_update_kernel(const double* __restrict__ X,
                                                             int64_t ld, int cnt,
                                                             const double* __restrict__ h,
                                                             double* __restrict__ w, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int i = 0; i < cnt; ++i) acc = fma(X[(int64_t)i * ld + e], h[i], acc);
  w[e] -= acc;
}

__global__ __launch_bounds__(kBlock) void scale_kernel(const double* __restrict__ x, double a,
                                                       double* __restrict__ y, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) y[e] = a * x[e];
}

}  // namespace

int cond_dot_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 4 * kBlock), 1024));
}

hipError_t launch_multi_dot(const double* X, int64_t ld, int cnt, const double* w, int64_t n,
                            double* part, int64_t ldp, double* out, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  const int nb = cond_dot_blocks(n);
  hipLaunchKernelGGL(multi_dot_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, X, ld, cnt, w, n,
                     part, ldp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((unsigned)cnt), dim3(kBlock), 0, s, part, nb, ldp,
                     out);
  return hipGetLastError();
}

hipError_t launch_orth_update(const double* X, int64_t ld, int cnt, const double* h, double* w,
                              int64_t n, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(orth_update_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s,
                     X, ld, cnt, h, w, n);
  return hipGetLastError();
}

hipError_t launch_scale(const double* x, double a, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s, x, a,
                     y, n);
  return hipGetLastError();
}

}  // namespace fct
