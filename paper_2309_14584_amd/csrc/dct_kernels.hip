// Separable DCT-I passes over the grids of a plan (Alg. 3, transform step;
// Sec. 3.1, eq. multi_dim_dct).
//
// Each grid's tensor is split into groups of consecutive axes.  A pass
// transforms every axis of one group: a workgroup stages a tile
// (TO outer positions x the whole group x TI inner positions) in LDS, applies
// the group's (N+1)x(N+1) matrices one axis at a time (each thread owns whole
// fibres held in registers, so the update is in place), and writes the tile
// back.  Passes of the outer groups run first; the innermost group's pass
// runs last and, for the forward transform, writes only the non-empty bins
// (rows) of its contiguous tile directly into b.  The inverse transform
// (evaluation at the nodes, used to synthesise planted polynomials) runs the
// groups in the opposite order and its first pass scatters the row values
// into a zero tile.
//
// One launch covers the same pass level of every grid: workgroups are
// assigned to (grid, tile) through a small descriptor table.
#include "fct_internal.h"

namespace fct {
namespace {

__device__ __forceinline__ int64_t lower_bound_i64(const int64_t* __restrict__ a, int64_t lo,
                                                   int64_t hi, int64_t key) {
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (a[m] < key) lo = m + 1; else hi = m;
  }
  return lo;
}

constexpr int kUnroll = kTileMax / kBlock;   // tile elements per thread
constexpr int kRowBatch = 8;                 // rows gathered / scattered per round

// e / TI for 0 <= e < 2^24 (float quotient, then one exact correction).
__device__ __forceinline__ int div_small(int e, int TI, float inv) {
  int g = (int)((float)e * inv);
  if (g * TI > e) --g;
  else if ((g + 1) * TI <= e) ++g;
  return g;
}

template <int EMAX>
__global__ __launch_bounds__(kBlock) void dct_pass_kernel(
    const PassDesc* __restrict__ descs, int ndesc, const double* __restrict__ in,
    double* scratch, double* out, const double* __restrict__ mats,
    const int64_t* __restrict__ bin_id) {
  extern __shared__ double smem[];
  double* tile = smem;                  // [kTileMax]
  double* mat = smem + kTileMax;        // [EMAX * EMAX] when EMAX <= 32
  __shared__ PassDesc d;
  __shared__ int64_t s_rows[2];

  if (threadIdx.x == 0) {
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {                   // last descriptor with tile_begin <= blockIdx.x
      const int mid = (lo + hi + 1) >> 1;
      if (descs[mid].tile_begin <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    d = descs[lo];
  }
  __syncthreads();

  const int64_t t = (int64_t)blockIdx.x - d.tile_begin;
  int64_t o0, i0;
  if (d.I == 1) { o0 = t * d.TO; i0 = 0; }
  else { o0 = t / d.tiles_i; i0 = (t % d.tiles_i) * d.TI; }
  const int TO = d.TO, TI = d.TI;
  const int64_t G = d.G, I = d.I;
  const int TOe = (int)((d.O - o0) < TO ? (d.O - o0) : TO);
  const int TIe = (int)((I - i0) < TI ? (I - i0) : TI);
  const int nel = TO * (int)G * TI;
  // flat range covered by a contiguous (I == 1) tile
  const int64_t flat_lo = o0 * G;
  const int64_t flat_hi = (o0 + TOe) * G;

  // ---- load ----
  // Every thread issues all of its global loads before it writes any of
  // them to LDS, so their latencies overlap.
  const float invTI = 1.0f / (float)TI;
  if (d.src == kSrcRows) {
    for (int e = threadIdx.x; e < nel; e += blockDim.x) tile[e] = 0.0;
    if (threadIdx.x == 0) {
      s_rows[0] = lower_bound_i64(bin_id, d.row_begin, d.row_end, flat_lo);
      s_rows[1] = lower_bound_i64(bin_id, d.row_begin, d.row_end, flat_hi);
    }
    __syncthreads();
    for (int64_t r0 = s_rows[0] + threadIdx.x; r0 < s_rows[1]; r0 += kRowBatch * blockDim.x) {
      int64_t bb[kRowBatch];
      double vv[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int64_t r = r0 + (int64_t)u * blockDim.x;
        bb[u] = r < s_rows[1] ? bin_id[r] : -1;
        vv[u] = r < s_rows[1] ? in[r] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (bb[u] >= 0) tile[bb[u] - flat_lo] = vv[u];
    }
  } else {
    const double* src = (d.src == kSrcInput) ? in : (d.src == kSrcOutput ? out : scratch);
    src += d.point_off;
    double v[kUnroll];
    if (I == 1) {                         // contiguous run of TOe * G elements
      const int cnt = TOe * (int)G;
      const double* base = src + flat_lo;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = threadIdx.x + u * kBlock;
        v[u] = e < cnt ? base[e] : 0.0;
      }
    } else {                              // G rows of TI contiguous elements, stride I
      const double* base = src + o0 * G * I + i0;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = threadIdx.x + u * kBlock;
        v[u] = 0.0;
        if (e < nel) {
          const int g = div_small(e, TI, invTI);
          const int i = e - g * TI;
          if (i < TIe) v[u] = base[(int64_t)g * I + i];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int e = threadIdx.x + u * kBlock;
      if (e < nel) tile[e] = v[u];
    }
  }
  __syncthreads();

  // ---- transform each axis of the group ----
  int stride = TI * (int)G;             // stride of the axis above the current one
  for (int a = 0; a < d.naxes; ++a) {
    const int e = d.ext[a];
    stride /= e;                        // stride of axis a inside the tile
    const double* gm = mats + mat_offset(e - 1);
    // matrices up to 32x32 are staged in LDS; larger ones are read through
    // the cache (every lane of a wave reads the same entry)
    const double* mrow = (EMAX <= 32) ? mat : gm;
    if (EMAX <= 32) {
      for (int k = threadIdx.x; k < e * e; k += blockDim.x) mat[k] = gm[k];
      __syncthreads();
    }
    const int nfib = nel / e;
    for (int f = threadIdx.x; f < nfib; f += blockDim.x) {
      const int low = f % stride;
      const int high = f / stride;
      const int base = high * e * stride + low;
      double x[EMAX];
#pragma unroll
      for (int k = 0; k < EMAX; ++k) x[k] = (k < e) ? tile[base + k * stride] : 0.0;
      for (int m = 0; m < e; ++m) {
        const double* row = mrow + m * e;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < EMAX; ++k)
          if (k < e) acc = fma(row[k], x[k], acc);
        tile[base + m * stride] = acc;
      }
    }
    __syncthreads();
  }

  // ---- store ----
  if (d.dst == kDstGather) {
    if (threadIdx.x == 0) {
      s_rows[0] = lower_bound_i64(bin_id, d.row_begin, d.row_end, flat_lo);
      s_rows[1] = lower_bound_i64(bin_id, d.row_begin, d.row_end, flat_hi);
    }
    __syncthreads();
    for (int64_t r0 = s_rows[0] + threadIdx.x; r0 < s_rows[1]; r0 += kRowBatch * blockDim.x) {
      int64_t bb[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int64_t r = r0 + (int64_t)u * blockDim.x;
        bb[u] = r < s_rows[1] ? bin_id[r] : -1;
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u)
        if (bb[u] >= 0) out[r0 + (int64_t)u * blockDim.x] = tile[bb[u] - flat_lo];
    }
  } else {
    double* dst = ((d.dst == kDstOutput) ? out : scratch) + d.point_off;
    if (I == 1) {
      const int cnt = TOe * (int)G;
      double* base = dst + flat_lo;
      for (int e = threadIdx.x; e < cnt; e += blockDim.x) base[e] = tile[e];
    } else {
      double* base = dst + o0 * G * I + i0;
      for (int e = threadIdx.x; e < nel; e += blockDim.x) {
        const int g = div_small(e, TI, invTI);
        const int i = e - g * TI;
        if (i < TIe) base[(int64_t)g * I + i] = tile[e];
      }
    }
  }
}

}  // namespace

hipError_t launch_dct_level(const DctLevel& lv, const double* in, double* scratch, double* out,
                            const double* mats, const int64_t* bin_id, hipStream_t s) {
  if (lv.tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)lv.tiles), block(kBlock);
  if (lv.emax <= 8) {
    const size_t sh = sizeof(double) * (kTileMax + 8 * 8);
    hipLaunchKernelGGL(dct_pass_kernel<8>, grid, block, sh, s, lv.d_desc, lv.ndesc, in, scratch,
                       out, mats, bin_id);
  } else if (lv.emax <= 16) {
    const size_t sh = sizeof(double) * (kTileMax + 16 * 16);
    hipLaunchKernelGGL(dct_pass_kernel<16>, grid, block, sh, s, lv.d_desc, lv.ndesc, in, scratch,
                       out, mats, bin_id);
  } else if (lv.emax <= 32) {
    const size_t sh = sizeof(double) * (kTileMax + 32 * 32);
    hipLaunchKernelGGL(dct_pass_kernel<32>, grid, block, sh, s, lv.d_desc, lv.ndesc, in, scratch,
                       out, mats, bin_id);
  } else {
    const size_t sh = sizeof(double) * kTileMax;
    hipLaunchKernelGGL(dct_pass_kernel<64>, grid, block, sh, s, lv.d_desc, lv.ndesc, in, scratch,
                       out, mats, bin_id);
  }
  return hipGetLastError();
}

}  // namespace fct
