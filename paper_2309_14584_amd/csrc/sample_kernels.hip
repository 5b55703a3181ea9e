// Sampling of analytic test functions on every grid of a plan (Alg. 3,
// sampling step).  One thread per grid point: the point's multi-index is
// decoded from its row-major position, each coordinate is read from the
// per-degree node table, and f is evaluated in FP64 with the device math
// library.  Coordinates are consumed as they are decoded, so D is not
// bounded by a register array.
#include "fct_internal.h"

namespace fct {
namespace {

__global__ __launch_bounds__(kBlock) void sample_kernel(
    int family, const SampleParams prm_in, int D, int K,
    const int32_t* __restrict__ grids, const int64_t* __restrict__ point_off,
    int64_t total, const double* __restrict__ nodes, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const double* prm = prm_in.v;
  int lo = 0, hi = K - 1;               // grid of point t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (point_off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int l = lo;
  int64_t p = t - point_off[l];
  const int32_t* g = grids + (int64_t)l * D;

  double acc0 = 0.0, acc1 = 0.0;
  // dimensions from last (fastest) to first
  for (int i = D - 1; i >= 0; --i) {
    const int N = g[i];
    const int64_t e = N + 1;
    const int k = (int)(p % e);
    p /= e;
    const double x = nodes[N * 64 + k];
    switch (family) {
      case FCT_F_EXPCOS:
        acc0 = fma(prm[i] * x, x, acc0);          // sum a_i x_i^2
        acc1 = fma(prm[D + i], x, acc1);          // sum w_i x_i
        break;
      case FCT_F_GAUSS: {
        const double dx = x - prm[1 + i];
        acc0 = fma(dx, dx, acc0);                 // |x - x0|^2
        break;
      }
      case FCT_F_RUNGE:
      case FCT_F_OSC:
        acc0 = fma(x, x, acc0);                   // |x|^2
        acc1 += x;                                // sum x_i
        break;
      default:
        break;
    }
  }
  double f = 0.0;
  switch (family) {
    case FCT_F_EXPCOS: f = exp(-acc0) * cos(acc1); break;
    case FCT_F_GAUSS: f = exp(-acc0 / (2.0 * prm[0] * prm[0])); break;
    case FCT_F_RUNGE: f = 1.0 / fma(prm[0], acc0, 1.0); break;
    case FCT_F_OSC: f = sin(3.0 * cos(3.0 * exp(acc0))) + exp(sin(3.0 * acc1)); break;
    default: break;
  }
  out[t] = f;
}

}  // namespace

hipError_t launch_sample(int family, const SampleParams& prm, int D, int K,
                         const int32_t* grids, const int64_t* point_off, int64_t total_points,
                         const double* nodes, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)ceil_div(total_points, kBlock)), dim3(kBlock),
                     0, s, family, prm, D, K, grids, point_off, total_points, nodes, out);
  return hipGetLastError();
}

}  // namespace fct
