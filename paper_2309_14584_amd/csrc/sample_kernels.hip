// Sampling of analytic test functions on every grid of a plan (Alg. 3,
// sampling step).  Each grid's tensor is viewed as rows (outer axes) x
// inner positions (trailing axes); a point's coordinates come from the
// per-degree node table through its decoded multi-index, and f is evaluated
// in FP64 with the device math library.  The test families are functions of
// sums over the axes (a weighted sum of squares and a weighted sum), which
// the kernel accumulates per row and per inner position separately.
#include <algorithm>
#include <cstring>

#include "fct_internal.h"

namespace fct {
namespace {

// Index of the last descriptor whose tile_begin is <= b (non-decreasing
// tile_begin, descs[0].tile_begin == 0): a 64-way search by one wave.
__device__ __forceinline__ int find_sdesc(const SampleDesc* __restrict__ descs, int ndesc,
                                          int64_t b) {
  const int lane = threadIdx.x & 63;
  int lo = 0, len = ndesc;
  while (len > 1) {
    const int step = (len + 63) >> 6;
    const int off = lane * step;
    const bool ok = off < len && descs[lo + off].tile_begin <= b;
    const unsigned long long m = __ballot(ok);
    const int last = 63 - __clzll((long long)m);
    lo += last * step;
    len = min(step, len - last * step);
  }
  return lo;
}

// The families' exponent sums are sums of one term per axis, so they split
// into the terms of the outer axes (one pair per row) and of the inner axes
// (one pair per inner position).  acc.x, acc.y: the two sums of a family.
template <int FAM>
__device__ __forceinline__ void add_axis(const double* prm, int D, int i, double x, double& a0,
                                         double& a1) {
  if constexpr (FAM == FCT_F_EXPCOS) {
    a0 = fma(prm[i] * x, x, a0);          // sum a_i x_i^2
    a1 = fma(prm[D + i], x, a1);          // sum w_i x_i
  } else if constexpr (FAM == FCT_F_GAUSS) {
    const double dx = x - prm[1 + i];
    a0 = fma(dx, dx, a0);                 // |x - x0|^2
  } else {                                // Runge, oscillatory
    a0 = fma(x, x, a0);                   // |x|^2
    a1 += x;                              // sum x_i
  }
}

template <int FAM>
__device__ __forceinline__ double finish(const double* prm, double a0, double a1) {
  if constexpr (FAM == FCT_F_EXPCOS) return exp(-a0) * cos(a1);
  else if constexpr (FAM == FCT_F_GAUSS) return exp(-a0 / (2.0 * prm[0] * prm[0]));
  else if constexpr (FAM == FCT_F_RUNGE) return 1.0 / fma(prm[0], a0, 1.0);
  else return sin(3.0 * cos(3.0 * exp(a0))) + exp(sin(3.0 * a1));
}

// q / e for q < 2^24 (float quotient, then one exact correction).
__device__ __forceinline__ uint32_t div_small(uint32_t q, uint32_t e, float inv) {
  uint32_t g = (uint32_t)((float)q * inv);
  if (g * e > q) --g;
  else if ((g + 1) * e <= q) ++g;
  return g;
}

// One workgroup: rows [o0, o0 + R) of one grid, i.e. the contiguous points
// [o0 I, (o0 + R) I) of its tensor viewed as (O rows) x (I inner positions).
// The inner axes' partial sums are tabulated once per workgroup in LDS and
// each row's outer partial sums once per row, so a point costs one LDS read,
// two additions and the family's final function.
template <int FAM>
__global__ __launch_bounds__(kBlock) void sample_kernel(
    const SampleDesc* __restrict__ descs, int ndesc, const SampleParams prm_in, int D,
    const int32_t* __restrict__ grids, const double* __restrict__ nodes,
    double* __restrict__ out) {
  __shared__ SampleDesc d;
  __shared__ double2 inner[kSampleInnerMax];
  __shared__ double2 outer[kSampleRowsMax];
  const double* prm = prm_in.v;
  if (threadIdx.x < 64) {
    const int k = find_sdesc(descs, ndesc, (int64_t)blockIdx.x);
    constexpr int kWords = (int)(sizeof(SampleDesc) / sizeof(int32_t));
    if (threadIdx.x < kWords)
      reinterpret_cast<int32_t*>(&d)[threadIdx.x] =
          reinterpret_cast<const int32_t*>(descs + k)[threadIdx.x];
  }
  __syncthreads();
  const int32_t* g = grids + (int64_t)d.grid * D;
  const int split = d.split;
  const int I = d.I;
  const int64_t o0 = ((int64_t)blockIdx.x - d.tile_begin) * d.R;
  const int Re = (int)min((int64_t)d.R, d.O - o0);

  // inner table: axes split .. D-1, position i < I <= kSampleInnerMax
  for (int i = threadIdx.x; i < I; i += blockDim.x) {
    double a0 = 0.0, a1 = 0.0;
    uint32_t q = (uint32_t)i;
    for (int ax = D - 1; ax >= split; --ax) {
      const int N = g[ax];
      const uint32_t e = (uint32_t)(N + 1);
      const uint32_t qq = div_small(q, e, 1.0f / (float)e);
      const int k = (int)(q - qq * e);
      q = qq;
      add_axis<FAM>(prm, D, ax, nodes[N * 64 + k], a0, a1);
    }
    inner[i] = make_double2(a0, a1);
  }
  // outer partial sums: axes 0 .. split-1 of rows o0 .. o0 + Re - 1
  for (int r = threadIdx.x; r < Re; r += blockDim.x) {
    double a0 = 0.0, a1 = 0.0;
    uint64_t q = (uint64_t)(o0 + r);
    for (int ax = split - 1; ax >= 0; --ax) {
      const int N = g[ax];
      const uint64_t e = (uint64_t)(N + 1);
      int k;
      if ((q >> 32) == 0) {
        const uint32_t q32 = (uint32_t)q;
        k = (int)(q32 % (uint32_t)e);
        q = q32 / (uint32_t)e;
      } else {
        k = (int)(q % e);
        q /= e;
      }
      add_axis<FAM>(prm, D, ax, nodes[N * 64 + k], a0, a1);
    }
    outer[r] = make_double2(a0, a1);
  }
  __syncthreads();

  double* base = out + d.point_off + o0 * I;
  const int npts = Re * I;                  // <= kSamplePoints
  const float invI = 1.0f / (float)I;
  for (int j = threadIdx.x; j < npts; j += blockDim.x) {
    const int r = (int)div_small((uint32_t)j, (uint32_t)I, invI);
    const int i = j - r * I;
    const double2 a = outer[r], b = inner[i];
    base[j] = finish<FAM>(prm, a.x + b.x, a.y + b.y);
  }
}

}  // namespace

// Split every grid into rows x inner positions for the sampler: the inner
// block is the longest run of trailing axes with at most kSampleInnerMax
// positions (at least one axis), and a workgroup takes
// R = clamp(kSamplePoints / I, 1, kSampleRowsMax) rows.
void make_sample_descs(const std::vector<int32_t>& grids, int D, int K,
                       const std::vector<int64_t>& point_off, std::vector<SampleDesc>* out,
                       int64_t* tiles) {
  out->clear();
  int64_t tb = 0;
  for (int l = 0; l < K; ++l) {
    const int32_t* g = &grids[(size_t)l * D];
    int split = D;
    int64_t I = 1;
    while (split > 0 && (split == D || I * (g[split - 1] + 1) <= kSampleInnerMax)) {
      I *= g[split - 1] + 1;
      --split;
    }
    const int64_t O = (point_off[l + 1] - point_off[l]) / I;
    SampleDesc sd;
    std::memset(&sd, 0, sizeof(sd));
    sd.point_off = point_off[l];
    sd.O = O;
    sd.tile_begin = tb;
    sd.grid = l;
    sd.split = split;
    sd.I = (int32_t)I;
    sd.R = (int32_t)std::max<int64_t>(1, std::min<int64_t>(kSamplePoints / I, kSampleRowsMax));
    tb += ceil_div(O, sd.R);
    out->push_back(sd);
  }
  *tiles = tb;
}

hipError_t launch_sample(int family, const SampleParams& prm, int D, const SampleDesc* descs,
                         int ndesc, int64_t tiles, const int32_t* grids, const double* nodes,
                         double* out, hipStream_t s) {
  if (tiles == 0) return hipSuccess;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles), block(kBlock);
  switch (family) {
    case FCT_F_EXPCOS:
      hipLaunchKernelGGL(sample_kernel<FCT_F_EXPCOS>, grid, block, 0, s, descs, ndesc, prm, D,
                         grids, nodes, out);
      break;
    case FCT_F_GAUSS:
      hipLaunchKernelGGL(sample_kernel<FCT_F_GAUSS>, grid, block, 0, s, descs, ndesc, prm, D,
                         grids, nodes, out);
      break;
    case FCT_F_RUNGE:
      hipLaunchKernelGGL(sample_kernel<FCT_F_RUNGE>, grid, block, 0, s, descs, ndesc, prm, D,
                         grids, nodes, out);
      break;
    case FCT_F_OSC:
      hipLaunchKernelGGL(sample_kernel<FCT_F_OSC>, grid, block, 0, s, descs, ndesc, prm, D,
                         grids, nodes, out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fct
