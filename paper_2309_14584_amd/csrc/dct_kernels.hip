// Separable DCT-I passes over the grids of a plan (Alg. 3, transform step;
// Sec. 3.1, eq. multi_dim_dct), on the matrix cores.
//
// Each grid's tensor is split into groups of consecutive axes.  A pass
// transforms every axis of one group: a workgroup stages a tile
// (TO outer positions x the whole group x TI inner positions) in LDS, applies
// the group's (N+1)x(N+1) matrices one axis at a time, and writes the tile
// back.  Passes of the outer groups run first; the innermost group's pass
// runs last and, for the forward transform, writes only the non-empty bins
// (rows) of its contiguous tile directly into b.  The inverse transform
// (evaluation at the nodes, used to synthesise planted polynomials) runs the
// groups in the opposite order and its first pass scatters the row values
// into a zero tile.  One launch covers the same pass level of every grid of
// every problem: workgroups find their (grid, tile) in a descriptor table.
//
// One axis of the tile is a batch of small matrix products
// Y[m, f] = sum_k C[m, k] X[k, f] over its fibres f, done 16 fibres at a
// time by each wave with 16x16 MFMA tiles: the matrix C is the A operand
// (kept in registers for the whole axis, rows m padded to 16 or 32), 16
// fibres are the B operand (one LDS load per lane and K step) and the
// result is written back in place (a wave reads all of its fibres before it
// writes any of them; waves own disjoint fibres).  Arithmetic modes:
//   F64:    v_mfma_f64_16x16x4 on an FP64 tile;
//   F32:    v_mfma_f32_16x16x4 on an FP32 tile;
//   BF16X3: both operands split into bf16 high and low parts (round to
//           nearest even), Y = C_hi X_hi + C_hi X_lo + C_lo X_hi with
//           v_mfma_f32_16x16x16 and FP32 accumulation, on an FP32 tile.
// Extents above 32 fall back to FP64 FMAs on the vector units.
#include <algorithm>

#include "fct_internal.h"

namespace fct {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

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

// bf16 bits of x, rounded to nearest even (finite inputs).
__device__ __forceinline__ short bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_float(short h) {
  return __uint_as_float(((unsigned)(unsigned short)h) << 16);
}

// ---- one axis on the matrix cores ----------------------------------------
// MB = 16-row blocks of outputs (e <= 16 * MB).
template <int MODE, int MB, typename T>
__device__ __forceinline__ void axis_mfma(T* tile, int nel, int e, int st,
                                          const double* __restrict__ gm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  constexpr int KS = (MODE == FCT_DCT_BF16X3) ? 16 : 4;   // K per MFMA
  constexpr int KBMAX = (16 * MB) / KS;
  const int KB = (e + KS - 1) / KS;
  const int nfib = nel / e;
  const int nbatch = (nfib + 15) >> 4;

  if constexpr (MODE == FCT_DCT_F64 || MODE == FCT_DCT_F32) {
    typedef typename std::conditional<MODE == FCT_DCT_F64, double, float>::type V;
    V a[MB][KBMAX];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int kb = 0; kb < KBMAX; ++kb) {
        const int m = mb * 16 + col, k = kb * 4 + grp;
        a[mb][kb] = (m < e && k < e) ? (V)gm[m * e + k] : (V)0;
      }
    for (int bt = wave; bt < nbatch; bt += nwaves) {
      const int f = bt * 16 + col;
      const bool valid = f < nfib;
      const int base = valid ? (f / st) * e * st + (f % st) : 0;
      typedef typename std::conditional<MODE == FCT_DCT_F64, v4d, v4f>::type Acc;
      Acc acc[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[mb] = (Acc){0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < KBMAX; ++kb) {
        if (kb < KB) {
          const int k = kb * 4 + grp;
          const V bv = (valid && k < e) ? (V)tile[base + k * st] : (V)0;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            if constexpr (MODE == FCT_DCT_F64)
              acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mb][kb], bv, acc[mb], 0, 0, 0);
            else
              acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mb][kb], bv, acc[mb], 0, 0, 0);
          }
        }
      }
      if (valid) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // f64 tiles: lane holds rows grp + 4r; f32 tiles: rows 4 grp + r
            const int m = mb * 16 + (MODE == FCT_DCT_F64 ? grp + 4 * r : 4 * grp + r);
            if (m < e) tile[base + m * st] = (T)acc[mb][r];
          }
      }
    }
  } else {
    v4s ah[MB][KBMAX], al[MB][KBMAX];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int kb = 0; kb < KBMAX; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = mb * 16 + col, k = kb * 16 + 4 * grp + i;
          const float v = (m < e && k < e) ? (float)gm[m * e + k] : 0.0f;
          const short hi = bf16_rne(v);
          ah[mb][kb][i] = hi;
          al[mb][kb][i] = bf16_rne(v - bf16_to_float(hi));
        }
    for (int bt = wave; bt < nbatch; bt += nwaves) {
      const int f = bt * 16 + col;
      const bool valid = f < nfib;
      const int base = valid ? (f / st) * e * st + (f % st) : 0;
      v4f acc[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) acc[mb] = (v4f){0, 0, 0, 0};
#pragma unroll
      for (int kb = 0; kb < KBMAX; ++kb) {
        if (kb < KB) {
          v4s bh, bl;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int k = kb * 16 + 4 * grp + i;
            const float v = (valid && k < e) ? (float)tile[base + k * st] : 0.0f;
            const short hi = bf16_rne(v);
            bh[i] = hi;
            bl[i] = bf16_rne(v - bf16_to_float(hi));
          }
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            // small cross terms first, then the leading product
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[mb][kb], bh, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[mb][kb], bl, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[mb][kb], bh, acc[mb], 0, 0, 0);
          }
        }
      }
      if (valid) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = mb * 16 + 4 * grp + r;
            if (m < e) tile[base + m * st] = (T)acc[mb][r];
          }
      }
    }
  }
}

// ---- one axis on the vector units (FP64, extents up to 64) ---------------
template <typename T>
__device__ __forceinline__ void axis_valu64(T* tile, int nel, int e, int st,
                                            const double* __restrict__ gm) {
  const int nfib = nel / e;
  for (int f = threadIdx.x; f < nfib; f += blockDim.x) {
    const int base = (f / st) * e * st + (f % st);
    double x[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) x[k] = (k < e) ? (double)tile[base + k * st] : 0.0;
    for (int m = 0; m < e; ++m) {
      const double* row = gm + m * e;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 64; ++k)
        if (k < e) acc = fma(row[k], x[k], acc);
      tile[base + m * st] = (T)acc;
    }
  }
}

// MB: 1 (extents <= 16), 2 (<= 32) or 0 (vector units, FP64, <= 64).
template <int MODE, int MB, typename T>
__global__ __launch_bounds__(kBlock) void dct_pass_kernel(
    const PassDesc* __restrict__ descs, int ndesc, const double* __restrict__ in,
    T* scratch, double* out, const double* __restrict__ mats,
    const int64_t* __restrict__ bin_id) {
  // the tile: the level's tile_max elements of dynamic LDS (at most kTileMax)
  extern __shared__ __align__(16) unsigned char dct_smem[];
  T* const tile = reinterpret_cast<T*>(dct_smem);
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
    for (int e = threadIdx.x; e < nel; e += blockDim.x) tile[e] = (T)0;
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
        if (bb[u] >= 0) tile[bb[u] - flat_lo] = (T)vv[u];
    }
  } else {
    T v[kUnroll];
    const int64_t off = d.point_off + (I == 1 ? flat_lo : o0 * G * I + i0);
    // the scratch tensor has the tile type; the caller's buffers are FP64
    if (d.src == kSrcScratch) {
      const T* base = scratch + off;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = threadIdx.x + u * kBlock;
        v[u] = (T)0;
        if (I == 1) {
          if (e < TOe * (int)G) v[u] = base[e];
        } else if (e < nel) {
          const int g = div_small(e, TI, invTI);
          const int i = e - g * TI;
          if (i < TIe) v[u] = base[(int64_t)g * I + i];
        }
      }
    } else {
      const double* base = (d.src == kSrcInput ? in : out) + off;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int e = threadIdx.x + u * kBlock;
        v[u] = (T)0;
        if (I == 1) {
          if (e < TOe * (int)G) v[u] = (T)base[e];
        } else if (e < nel) {
          const int g = div_small(e, TI, invTI);
          const int i = e - g * TI;
          if (i < TIe) v[u] = (T)base[(int64_t)g * I + i];
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
    if constexpr (MB == 0) axis_valu64<T>(tile, nel, e, stride, gm);
    else axis_mfma<MODE, MB, T>(tile, nel, e, stride, gm);
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
        if (bb[u] >= 0) out[r0 + (int64_t)u * blockDim.x] = (double)tile[bb[u] - flat_lo];
    }
  } else {
    const int64_t off = d.point_off + (I == 1 ? flat_lo : o0 * G * I + i0);
    if (d.dst == kDstScratch) {
      T* base = scratch + off;
      if (I == 1) {
        for (int e = threadIdx.x; e < TOe * (int)G; e += blockDim.x) base[e] = tile[e];
      } else {
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
          const int g = div_small(e, TI, invTI);
          const int i = e - g * TI;
          if (i < TIe) base[(int64_t)g * I + i] = tile[e];
        }
      }
    } else {
      double* base = out + off;
      if (I == 1) {
        for (int e = threadIdx.x; e < TOe * (int)G; e += blockDim.x) base[e] = (double)tile[e];
      } else {
        for (int e = threadIdx.x; e < nel; e += blockDim.x) {
          const int g = div_small(e, TI, invTI);
          const int i = e - g * TI;
          if (i < TIe) base[(int64_t)g * I + i] = (double)tile[e];
        }
      }
    }
  }
}

template <int MODE, typename T>
hipError_t launch_mode(const DctLevel& lv, const double* in, void* scratch, double* out,
                       const double* mats, const int64_t* bin_id, hipStream_t s) {
  const dim3 grid((unsigned)lv.tiles), block(kBlock);
  T* sc = static_cast<T*>(scratch);
  const size_t lds = sizeof(T) * (size_t)std::min(lv.tile_max, kTileMax);
  if (lv.emax <= 16) {
    hipLaunchKernelGGL((dct_pass_kernel<MODE, 1, T>), grid, block, lds, s, lv.d_desc, lv.ndesc, in,
                       sc, out, mats, bin_id);
  } else if (lv.emax <= 32) {
    hipLaunchKernelGGL((dct_pass_kernel<MODE, 2, T>), grid, block, lds, s, lv.d_desc, lv.ndesc, in,
                       sc, out, mats, bin_id);
  } else {
    if (MODE != FCT_DCT_F64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((dct_pass_kernel<FCT_DCT_F64, 0, T>), grid, block, lds, s, lv.d_desc,
                       lv.ndesc, in, sc, out, mats, bin_id);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dct_level(const DctLevel& lv, int mode, const double* in, void* scratch,
                            double* out, const double* mats, const int64_t* bin_id,
                            hipStream_t s) {
  if (lv.tiles == 0) return hipSuccess;
  switch (mode) {
    case FCT_DCT_F64: return launch_mode<FCT_DCT_F64, double>(lv, in, scratch, out, mats, bin_id, s);
    case FCT_DCT_F32: return launch_mode<FCT_DCT_F32, float>(lv, in, scratch, out, mats, bin_id, s);
    case FCT_DCT_BF16X3:
      return launch_mode<FCT_DCT_BF16X3, float>(lv, in, scratch, out, mats, bin_id, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fct
