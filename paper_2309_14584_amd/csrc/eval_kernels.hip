// Evaluation of a Chebyshev expansion on the plan's support at arbitrary
// points: p(x) = sum_j c_j prod_i T_{n_ji}(x_i) (Sec. 2, the expansion that
// the transform recovers; Sec. 4 measures accuracy at random points).
//
// A workgroup takes 64 points (one per lane) and 16 waves.  It first
// tabulates T_0..T_dmax of every coordinate of its points in LDS with the
// three-term recurrence (layout [dimension][degree][point], so the lanes of
// a wave read consecutive words), then streams the support through LDS in
// chunks: the row offsets (dimension * (dmax+1) + n_ji) and coefficients of
// a chunk are staged once and read by every wave as broadcasts.  Wave w sums
// the terms j = w (mod 16) of the chunk, four terms interleaved; the 16 wave
// partials of a point are added in wave order.  With few points and a long
// support the support is also cut into slices (grid dimension y), each
// slice's sums are written apart and a second kernel adds the slices in
// order, so results are reproducible for a given slicing.
#include <algorithm>

#include "fct_internal.h"

namespace fct {
namespace {

constexpr int kEvalPoints = 64;            // points per workgroup (lanes)
constexpr int kEvalWaves = 16;             // waves per workgroup
constexpr int kEvalThreads = kEvalPoints * kEvalWaves;
constexpr int kEvalIlp = 4;                // terms a wave interleaves
constexpr int64_t kEvalTargetGroups = 1024; // workgroups that fill the device (4 per CU)

__global__ __launch_bounds__(kEvalThreads) void eval_kernel(
    const int32_t* __restrict__ support, const double* __restrict__ c, int64_t n, int D, int nk,
    int chunk, int64_t per_slice, int64_t m, const double* __restrict__ X,
    double* __restrict__ f) {
  extern __shared__ __align__(16) unsigned char eval_smem[];
  double* T = reinterpret_cast<double*>(eval_smem);                 // [D * nk][64]
  double* part = T + (size_t)D * nk * kEvalPoints;                  // [kEvalWaves][64]
  double* coef = part + kEvalThreads;                               // [chunk]
  uint16_t* off = reinterpret_cast<uint16_t*>(coef + chunk);        // [chunk][D]

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t pt = (int64_t)blockIdx.x * kEvalPoints + lane;
  const bool live = pt < m;

  // Chebyshev values of every coordinate of the workgroup's points
  for (int i = wave; i < D; i += kEvalWaves) {
    const double x = live ? X[pt * D + i] : 0.0;
    double* Ti = T + (size_t)i * nk * kEvalPoints + lane;
    double t0 = 1.0, t1 = x;
    Ti[0] = t0;
    if (nk > 1) Ti[kEvalPoints] = t1;
    for (int k = 2; k < nk; ++k) {
      const double t2 = 2.0 * x * t1 - t0;
      Ti[(size_t)k * kEvalPoints] = t2;
      t0 = t1;
      t1 = t2;
    }
  }

  // this workgroup's support slice [j_lo, j_hi); per_slice is a multiple of chunk
  const int64_t j_lo = (int64_t)blockIdx.y * per_slice;
  const int64_t j_hi = min(n, j_lo + per_slice);
  double acc = 0.0;
  for (int64_t j0 = j_lo; j0 < j_hi; j0 += chunk) {
    const int cnt = (int)min((int64_t)chunk, j_hi - j0);
    __syncthreads();                       // table written / previous chunk consumed
    for (int e = threadIdx.x; e < cnt * D; e += kEvalThreads) {
      const int jj = e / D, i = e - jj * D;
      off[e] = (uint16_t)(i * nk + support[(j0 + jj) * D + i]);
    }
    for (int e = threadIdx.x; e < cnt; e += kEvalThreads) coef[e] = c[j0 + e];
    __syncthreads();
    int jj = wave;
    for (; jj + (kEvalIlp - 1) * kEvalWaves < cnt; jj += kEvalIlp * kEvalWaves) {
      double pr[kEvalIlp];
#pragma unroll
      for (int u = 0; u < kEvalIlp; ++u) pr[u] = coef[jj + u * kEvalWaves];
      for (int i = 0; i < D; ++i) {
#pragma unroll
        for (int u = 0; u < kEvalIlp; ++u)
          pr[u] *= T[(size_t)off[(jj + u * kEvalWaves) * D + i] * kEvalPoints + lane];
      }
#pragma unroll
      for (int u = 0; u < kEvalIlp; ++u) acc += pr[u];
    }
    for (; jj < cnt; jj += kEvalWaves) {
      double pr = coef[jj];
      for (int i = 0; i < D; ++i) pr *= T[(size_t)off[jj * D + i] * kEvalPoints + lane];
      acc += pr;
    }
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (wave == 0 && live) {
    double s = part[lane];
    for (int w = 1; w < kEvalWaves; ++w) s += part[w * kEvalPoints + lane];
    f[(int64_t)blockIdx.y * m + pt] = s;
  }
}

// f[q] = sum over slices s of part[s * m + q], in slice order.
__global__ __launch_bounds__(kBlock) void eval_combine_kernel(const double* __restrict__ part,
                                                              int slices, int64_t m,
                                                              double* __restrict__ f) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  double s = part[q];
  for (int k = 1; k < slices; ++k) s += part[(int64_t)k * m + q];
  f[q] = s;
}

}  // namespace

// Support rows staged per chunk: as many as fit next to the table (at most
// 1024, a multiple of 16); 0 if the table leaves no room for 16.
int eval_chunk(int D, int nk) {
  const int64_t fixed = (int64_t)sizeof(double) * ((int64_t)D * nk * kEvalPoints + kEvalThreads);
  const int64_t room = (int64_t)kEvalLdsMax - fixed;
  if (room <= 0) return 0;
  int64_t chunk = room / (int64_t)(sizeof(double) + sizeof(uint16_t) * D);
  chunk = std::min<int64_t>(chunk, 1024) & ~int64_t(15);
  return chunk >= 16 ? (int)chunk : 0;
}

size_t eval_lds_bytes(int D, int nk, int chunk) {
  return sizeof(double) * ((size_t)D * nk * kEvalPoints + kEvalThreads + chunk) +
         sizeof(uint16_t) * (size_t)chunk * D;
}

int eval_slices(int64_t n, int D, int nk, int64_t m, int64_t scratch_elems) {
  const int chunk = eval_chunk(D, nk);
  if (chunk == 0 || m == 0) return 1;
  const int64_t blocks = ceil_div(m, kEvalPoints);
  int64_t want = ceil_div(kEvalTargetGroups, blocks);          // fill the device
  want = std::min<int64_t>(want, ceil_div(n, (int64_t)chunk));  // at least a chunk each
  want = std::min<int64_t>(want, scratch_elems / m);            // partials must fit
  want = std::min<int64_t>(want, 65535);
  return (int)std::max<int64_t>(want, 1);
}

hipError_t launch_eval(const int32_t* support, const double* c, int64_t n, int D, int nk,
                       int64_t m, const double* X, double* f, int slices, double* scratch,
                       hipStream_t s) {
  if (m == 0) return hipSuccess;
  const int64_t blocks = ceil_div(m, kEvalPoints);
  const int chunk = eval_chunk(D, nk);
  if (blocks > 0x7fffffffLL || chunk == 0 || D * nk > 65535 || slices < 1 || slices > 65535 ||
      (slices > 1 && !scratch))
    return hipErrorInvalidValue;
  // slices of whole chunks; the last slice may be shorter
  const int64_t per_slice = ceil_div(ceil_div(n, (int64_t)chunk), (int64_t)slices) * chunk;
  slices = (int)ceil_div(n, per_slice);
  const size_t lds = eval_lds_bytes(D, nk, chunk);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&eval_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  double* out = slices > 1 ? scratch : f;
  hipLaunchKernelGGL(eval_kernel, dim3((unsigned)blocks, (unsigned)slices), dim3(kEvalThreads),
                     lds, s, support, c, n, D, nk, chunk, per_slice, m, X, out);
  if (slices > 1) {
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(eval_combine_kernel, dim3((unsigned)ceil_div(m, kBlock)), dim3(kBlock), 0,
                       s, scratch, slices, m, f);
  }
  return hipGetLastError();
}

}  // namespace fct
