// Sampling of analytic test functions on every grid of a plan (Alg. 3,
// sampling step).  One thread per grid point: the point's multi-index is
// decoded from its row-major position, each coordinate is read from the
// per-degree node table, and f is evaluated in FP64 with the device math
// library.  Coordinates are consumed as they are decoded, so D is not
// bounded by a register array.
#include <algorithm>

#include "fct_internal.h"

namespace fct {
namespace {

// f at the point with row-major index p inside grid g (D degrees).  IDX is
// the index type of the mixed-radix decode: 32-bit whenever the grid has
// fewer than 2^32 points (64-bit division is several times slower).
template <typename IDX>
__device__ __forceinline__ double eval_point(int family, const double* prm, int D,
                                             const int32_t* g, IDX p,
                                             const double* __restrict__ nodes) {
  double acc0 = 0.0, acc1 = 0.0;
  // dimensions from last (fastest) to first
  for (int i = D - 1; i >= 0; --i) {
    const int N = g[i];
    const IDX e = (IDX)(N + 1);
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
  switch (family) {
    case FCT_F_EXPCOS: return exp(-acc0) * cos(acc1);
    case FCT_F_GAUSS: return exp(-acc0 / (2.0 * prm[0] * prm[0]));
    case FCT_F_RUNGE: return 1.0 / fma(prm[0], acc0, 1.0);
    case FCT_F_OSC: return sin(3.0 * cos(3.0 * exp(acc0))) + exp(sin(3.0 * acc1));
    default: return 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void sample_kernel(
    int family, const SampleParams prm_in, int D, int K,
    const int32_t* __restrict__ grids, const int64_t* __restrict__ point_off,
    int64_t total, const double* __restrict__ nodes, double* __restrict__ out) {
  const double* prm = prm_in.v;
  // grid-stride loop: a launch has at most kMaxSampleBlocks workgroups
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = K - 1;             // grid of point t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (point_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int64_t p = t - point_off[lo];
    const int32_t* g = grids + (int64_t)lo * D;
    out[t] = (p >> 32) == 0 ? eval_point<uint32_t>(family, prm, D, g, (uint32_t)p, nodes)
                            : eval_point<uint64_t>(family, prm, D, g, (uint64_t)p, nodes);
  }
}

}  // namespace

hipError_t launch_sample(int family, const SampleParams& prm, int D, int K,
                         const int32_t* grids, const int64_t* point_off, int64_t total_points,
                         const double* nodes, double* out, hipStream_t s) {
  constexpr int64_t kMaxSampleBlocks = int64_t(1) << 22;
  const int64_t blocks = std::max<int64_t>(1, std::min(ceil_div(total_points, kBlock),
                                                       kMaxSampleBlocks));
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(kBlock),
                     0, s, family, prm, D, K, grids, point_off, total_points, nodes, out);
  return hipGetLastError();
}

}  // namespace fct
