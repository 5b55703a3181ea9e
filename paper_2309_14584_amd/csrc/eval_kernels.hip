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
// partials of a point are added in wave order, so results are reproducible.
#include <algorithm>

#include "fct_internal.h"

namespace fct {
namespace {

constexpr int kEvalPoints = 64;            // points per workgroup (lanes)
constexpr int kEvalWaves = 16;             // waves per workgroup
constexpr int kEvalThreads = kEvalPoints * kEvalWaves;
constexpr int kEvalIlp = 4;                // terms a wave interleaves

__global__ __launch_bounds__(kEvalThreads) void eval_kernel(
    const int32_t* __restrict__ support, const double* __restrict__ c, int64_t n, int D, int nk,
    int chunk, int64_t m, const double* __restrict__ X, double* __restrict__ f) {
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

  double acc = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += chunk) {
    const int cnt = (int)min((int64_t)chunk, n - j0);
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
    f[pt] = s;
  }
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

hipError_t launch_eval(const int32_t* support, const double* c, int64_t n, int D, int nk,
                       int64_t m, const double* X, double* f, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const int64_t blocks = ceil_div(m, kEvalPoints);
  const int chunk = eval_chunk(D, nk);
  if (blocks > 0x7fffffffLL || chunk == 0 || D * nk > 65535) return hipErrorInvalidValue;
  const size_t lds = eval_lds_bytes(D, nk, chunk);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&eval_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eval_kernel, dim3((unsigned)blocks), dim3(kEvalThreads), lds, s, support, c,
                     n, D, nk, chunk, m, X, f);
  return hipGetLastError();
}

}  // namespace fct
