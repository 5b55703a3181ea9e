// Separable DCT-I passes over the grids of a plan (Alg. 3, transform step;
// Sec. 3.1, eq. multi_dim_dct).
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
// every problem: workgroups find their (grid, tile) in a descriptor table,
// and a gathering tile finds its rows in a per-tile table of first rows.
//
// One axis of the tile is a batch of small matrix products
// Y[m, f] = sum_k C[m, k] X[k, f] over its fibres f.  Arithmetic modes:
//   F64:    FP64 products and sums, FP64 tile;
//   F32:    FP32 products and sums (FP32 matrices), FP32 tile;
//   BF16X3: both operands split into bf16 high and low parts (round to
//           nearest even), Y = C_hi X_hi + C_hi X_lo + C_lo X_hi with FP32
//           accumulation, on an FP32 tile (matrix cores only).
// Two engines run the FP64 and FP32 contractions: the vector units (E*E
// multiply-adds per fibre of E points) and the matrix cores (16x16x4 MFMA
// tiles, 16 fibres per wave).  The axes have 2..32 points, mostly 3..8, so
// an MFMA tile is mostly padding while the FP64 and FP32 MFMA peaks equal
// the vector units': the vector engine is the default and the plan's
// tuner times both.  Every value is computed in place: a thread (wave)
// reads all of its fibres before it writes any of them; fibres are
// disjoint.
#include <algorithm>
#include <climits>
#include <cstdint>

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

// Index of the last descriptor in [lo, ndesc) whose tile_begin is <= b
// (tile_begin is non-decreasing and descs[lo].tile_begin <= b), found by one
// wave with a 64-way search: each round tests 64 evenly spaced candidates
// with one load per lane, so n descriptors take ceil(log64 n) dependent
// loads.  Called by all 64 lanes of a wave; the result is the same in every
// lane.
__device__ __forceinline__ int find_desc(const PassDesc* __restrict__ descs, int lo, int ndesc,
                                         int64_t b) {
  const int lane = threadIdx.x & 63;
  int len = ndesc - lo;
  while (len > 1) {
    const int step = (len + 63) >> 6;
    const int off = lane * step;
    const bool ok = off < len && descs[lo + off].tile_begin <= b;
    const unsigned long long m = __ballot(ok);   // lane 0 always holds (descs[lo] <= b)
    const int last = 63 - __clzll((long long)m);
    lo += last * step;
    len = min(step, len - last * step);
  }
  return lo;
}

constexpr int kUnroll = kTileMax / kBlock;   // tile elements per thread
constexpr int kRowBatch = 8;                 // rows gathered / scattered per round
constexpr int kGatherAhead = 4;              // rows per thread whose offsets are loaded early

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

// ---- one axis on the matrix cores -----------------------------------------
// 16 fibres at a time per wave: the matrix is the A operand (registers, rows
// padded to 16 * MB), 16 fibres the B operand (one LDS load per lane and K
// step), the result written back in place.  MB = 16-row blocks of outputs
// (e <= 16 * MB).  FP64: v_mfma_f64_16x16x4; FP32: v_mfma_f32_16x16x4;
// split-BF16x3: v_mfma_f32_16x16x16bf16 on the bf16 high/low parts.
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

// ---- one axis on the vector units ----------------------------------------
// Fibre f of an axis with extent E and stride st inside the tile starts at
// (f / st) * E * st + f % st.  Each thread owns whole fibres: it reads the E
// values, forms the E outputs with E*E fused multiply-adds in the mode's
// precision (A), and writes them back in place.  The matrix is wave-uniform
// (scalar loads, scalar operands of the multiply-adds).
template <int E, typename T, typename A>
__device__ __forceinline__ void axis_small(T* tile, int nel, int st, const A* __restrict__ cm) {
  const int nfib = nel / E;
  const float inv = 1.0f / (float)st;
  for (int f = threadIdx.x; f < nfib; f += kBlock) {
    const int hi = div_small(f, st, inv);
    T* p = tile + (hi * E * st + (f - hi * st));
    A x[E];
#pragma unroll
    for (int k = 0; k < E; ++k) x[k] = (A)p[k * st];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      A y = cm[m * E] * x[0];
#pragma unroll
      for (int k = 1; k < E; ++k) y = fma(cm[m * E + k], x[k], y);
      p[m * st] = (T)y;
    }
  }
}

template <typename T, typename A>
__device__ __forceinline__ void axis_vector(T* tile, int nel, int e, int st,
                                            const A* __restrict__ cm) {
  switch (e) {
    case 2: axis_small<2, T, A>(tile, nel, st, cm); break;
    case 3: axis_small<3, T, A>(tile, nel, st, cm); break;
    case 4: axis_small<4, T, A>(tile, nel, st, cm); break;
    case 5: axis_small<5, T, A>(tile, nel, st, cm); break;
    case 6: axis_small<6, T, A>(tile, nel, st, cm); break;
    case 7: axis_small<7, T, A>(tile, nel, st, cm); break;
    case 8: axis_small<8, T, A>(tile, nel, st, cm); break;
    case 9: axis_small<9, T, A>(tile, nel, st, cm); break;
    case 10: axis_small<10, T, A>(tile, nel, st, cm); break;
    case 11: axis_small<11, T, A>(tile, nel, st, cm); break;
    case 12: axis_small<12, T, A>(tile, nel, st, cm); break;
    case 13: axis_small<13, T, A>(tile, nel, st, cm); break;
    case 14: axis_small<14, T, A>(tile, nel, st, cm); break;
    case 15: axis_small<15, T, A>(tile, nel, st, cm); break;
    case 16: axis_small<16, T, A>(tile, nel, st, cm); break;
    default: break;   // extent 1: identity
  }
}

// Axes longer than 16 (up to EMAX points): the fibre in registers (padded
// to EMAX, predicated), one output row at a time.
template <int EMAX, typename T, typename A>
__device__ __forceinline__ void axis_long(T* tile, int nel, int e, int st,
                                          const A* __restrict__ cm) {
  const int nfib = nel / e;
  const float inv = 1.0f / (float)st;
  for (int f = threadIdx.x; f < nfib; f += kBlock) {
    const int hi = div_small(f, st, inv);
    T* p = tile + (hi * e * st + (f - hi * st));
    A x[EMAX];
#pragma unroll
    for (int k = 0; k < EMAX; ++k) x[k] = (k < e) ? (A)p[k * st] : (A)0;
    for (int m = 0; m < e; ++m) {
      const A* row = cm + m * e;
      A acc = 0;
#pragma unroll
      for (int k = 0; k < EMAX; ++k)
        if (k < e) acc = fma(row[k], x[k], acc);
      p[m * st] = (T)acc;
    }
  }
}

// Geometry of tile t of descriptor k (wave-uniform).
struct TileGeo {
  int64_t off;       // first element of the tile in the grid's tensor buffers
  int64_t flat_lo;   // first flat index of a contiguous (I == 1) tile
  int64_t tl;        // tile index inside the descriptor
  int32_t k;         // descriptor
  int32_t nel;       // TO * G * TI: tile elements (padded)
  int32_t TOe, TIe;  // outer / inner positions actually present
};

__device__ __forceinline__ TileGeo tile_geo(const PassDesc* __restrict__ descs, int k,
                                            int64_t t) {
  const PassDesc& d = descs[k];
  TileGeo g;
  g.k = k;
  g.tl = t - d.tile_begin;
  int64_t o0, i0;
  if (d.I == 1) { o0 = g.tl * d.TO; i0 = 0; }
  else { o0 = g.tl / d.tiles_i; i0 = (g.tl % d.tiles_i) * d.TI; }
  g.TOe = (int)((d.O - o0) < d.TO ? (d.O - o0) : d.TO);
  g.TIe = (int)((d.I - i0) < d.TI ? (d.I - i0) : d.TI);
  g.nel = d.TO * (int)d.G * d.TI;
  g.flat_lo = o0 * d.G;
  g.off = d.point_off + (d.I == 1 ? g.flat_lo : o0 * d.G * d.I + i0);
  return g;
}

// Tile element e = tid + u * kBlock (u < kUnroll) maps to tensor element
// off + gg * I + i (gg = e / TI, i = e % TI); it is present when e < nel and
// i < TIe (contiguous tiles, I == 1: when e < TOe * G).  (gg, i) advance by
// the fixed step kBlock = q TI + r from one u to the next, so no division is
// repeated per element.
struct ElemWalk {
  int gg, i, q, r;
  __device__ __forceinline__ ElemWalk(const PassDesc& d, int tid) {
    const float inv = 1.0f / (float)d.TI;
    gg = div_small(tid, d.TI, inv);
    i = tid - gg * d.TI;
    q = div_small(kBlock, d.TI, inv);
    r = kBlock - q * d.TI;
  }
  __device__ __forceinline__ void next(int TI) {
    gg += q;
    i += r;
    if (i >= TI) { i -= TI; ++gg; }
  }
};

// Issue the global loads of tile `g` (raw bits: FP64 sources as doubles,
// scratch of an FP32 tile as floats in the low word).  Every element's load
// is issued, at a clamped and always valid index, and its raw bits are kept
// in a 64-bit register; fill_tile() masks the absent ones (a load merged
// with a default value would keep a second register alive while in flight).
// Sparse-row sources load nothing here (they are scattered later).
template <typename T>
__device__ __forceinline__ void load_tile(const PassDesc& d, const TileGeo& g,
                                          const double* __restrict__ in, const T* scratch,
                                          const double* out, int tid, uint64_t (&v)[kUnroll]) {
  if (d.src == kSrcRows) return;
  const bool f32 = d.src == kSrcScratch && sizeof(T) == 4;
  const void* src = d.src == kSrcScratch ? static_cast<const void*>(scratch)
                                         : static_cast<const void*>(d.src == kSrcInput ? in : out);
  const uint64_t* b64 = static_cast<const uint64_t*>(src) + g.off;
  const uint32_t* b32 = static_cast<const uint32_t*>(src) + g.off;
  if (d.I == 1) {
    const int last = g.TOe * (int)d.G - 1;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int idx = min(tid + u * kBlock, last);
      v[u] = f32 ? (uint64_t)b32[idx] : b64[idx];
    }
  } else {
    ElemWalk w(d, tid);
    const int gmax = (int)d.G - 1, imax = g.TIe - 1;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t idx = (int64_t)min(w.gg, gmax) * d.I + min(w.i, imax);
      v[u] = f32 ? (uint64_t)b32[idx] : b64[idx];
      w.next(d.TI);
    }
  }
}

// The same loads converted to the tile type at once (one-tile workgroups,
// whose loads are consumed right away: half the registers for FP32 tiles).
template <typename T>
__device__ __forceinline__ void load_tile_typed(const PassDesc& d, const TileGeo& g,
                                                const double* __restrict__ in, const T* scratch,
                                                const double* out, int tid, T (&v)[kUnroll]) {
  if (d.src == kSrcRows) return;
  const double* b64 = (d.src == kSrcInput ? in : out) + g.off;
  const T* bt = scratch + g.off;
  const bool sc = d.src == kSrcScratch;
  if (d.I == 1) {
    const int last = g.TOe * (int)d.G - 1;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int idx = min(tid + u * kBlock, last);
      v[u] = sc ? bt[idx] : (T)b64[idx];
    }
  } else {
    ElemWalk w(d, tid);
    const int gmax = (int)d.G - 1, imax = g.TIe - 1;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t idx = (int64_t)min(w.gg, gmax) * d.I + min(w.i, imax);
      v[u] = sc ? bt[idx] : (T)b64[idx];
      w.next(d.TI);
    }
  }
}

template <typename T>
__device__ __forceinline__ void fill_tile_typed(const PassDesc& d, const TileGeo& g,
                                                const T (&v)[kUnroll], int tid, T* tile) {
  ElemWalk w(d, tid);
  const int lim = d.I == 1 ? g.TOe * (int)d.G : g.nel;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int e = tid + u * kBlock;
    if (e < g.nel) tile[e] = (e < lim && (d.I == 1 || w.i < g.TIe)) ? v[u] : (T)0;
    w.next(d.TI);
  }
}

// Write the loaded raw bits of tile `g` into LDS as T (absent elements 0).
template <typename T>
__device__ __forceinline__ void fill_tile(const PassDesc& d, const TileGeo& g,
                                          const uint64_t (&v)[kUnroll], int tid, T* tile) {
  const bool f32 = d.src == kSrcScratch && sizeof(T) == 4;
  ElemWalk w(d, tid);
  const int lim = d.I == 1 ? g.TOe * (int)d.G : g.nel;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int e = tid + u * kBlock;
    if (e < g.nel) {
      const T x = f32 ? (T)__uint_as_float((uint32_t)v[u])
                      : (T)__longlong_as_double((long long)v[u]);
      const bool here = e < lim && (d.I == 1 || w.i < g.TIe);
      tile[e] = here ? x : (T)0;
    }
    w.next(d.TI);
  }
}

// Rows that tile t gathers: [tile_row[t], tile_row[t + 1]) inside its
// descriptor, up to row_end for the descriptor's last tile.  The first
// kGatherAhead * kBlock of them have their tile offsets loaded into lb.
struct GatherAhead {
  int64_t r_lo, r_hi;
  int32_t lb[kGatherAhead];
};
__device__ __forceinline__ void gather_ahead(const PassDesc& d, const TileGeo& g, int64_t t,
                                             const int32_t* __restrict__ tile_row,
                                             const int64_t* __restrict__ bin_id, int tid,
                                             GatherAhead& ga) {
  ga.r_lo = tile_row[t];
  ga.r_hi = g.tl + 1 < d.ntiles ? (int64_t)tile_row[t + 1] : d.row_end;
#pragma unroll
  for (int u = 0; u < kGatherAhead; ++u) {
    const int64_t r = ga.r_lo + tid + (int64_t)u * kBlock;
    ga.lb[u] = r < ga.r_hi ? (int32_t)(bin_id[r] - g.flat_lo) : -1;
  }
}

// MF (matrix cores; split-BF16x3 always): KIND = 16-row MFMA blocks of the
// outputs (1: extents <= 16, 2: <= 32).  Vector units (FP64, FP32):
// unrolled code for extents <= 16; longer axes (levels of KIND 2: <= 32,
// KIND 0: <= 64) a loop over output rows with the fibre in registers.
//
// PIPE (FP64 tiles): persistent workgroups, as many as are resident, taking
// tiles blockIdx.x, blockIdx.x + gridDim.x, ...; while a tile is
// transformed in LDS and written out, the global loads of the workgroup's
// next tile (and the offsets of the rows it gathers) are already in flight
// in registers.  Without PIPE (FP32 tiles, half the bytes) one workgroup
// per tile, with fewer registers and so more workgroups resident.
template <int MODE, int KIND, typename T, bool PIPE, bool MF>
__global__ __launch_bounds__(kBlock) void dct_pass_kernel(
    const PassDesc* __restrict__ descs, int ndesc, int64_t tiles,
    const double* __restrict__ in, T* scratch, double* out, const double* __restrict__ mats,
    const float* __restrict__ mats32, const int64_t* __restrict__ bin_id,
    const int32_t* __restrict__ tile_row) {
  // the tile: the level's tile_max elements of dynamic LDS (at most kTileMax)
  extern __shared__ __align__(16) unsigned char dct_smem[];
  T* const tile = reinterpret_cast<T*>(dct_smem);

  // this workgroup's tiles: blockIdx.x, blockIdx.x + gridDim.x, ... (the
  // workgroups resident at one time work on neighbouring tiles)
  const int64_t t0 = blockIdx.x;
  const int64_t step = gridDim.x;
  // descriptor of the current tile and the first tile of the next one
  int k = __builtin_amdgcn_readfirstlane(find_desc(descs, 0, ndesc, t0));
  int64_t next_begin = k + 1 < ndesc ? descs[k + 1].tile_begin : INT64_MAX;
  TileGeo nx = tile_geo(descs, k, t0);
  typedef typename std::conditional<PIPE, uint64_t, T>::type R;
  R v[kUnroll];
  GatherAhead ga;
  if constexpr (PIPE) {
    load_tile<T>(descs[k], nx, in, scratch, out, (int)threadIdx.x, v);
    if (descs[k].dst == kDstGather)
      gather_ahead(descs[k], nx, t0, tile_row, bin_id, (int)threadIdx.x, ga);
  }

  for (int64_t tc = t0; tc < tiles; tc += step) {
    const TileGeo g = nx;
    const PassDesc& d = descs[g.k];
    // thread index, opaque to the compiler within this iteration: the
    // per-element indices derived from it are recomputed per tile rather
    // than held in registers across the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    GatherAhead cur;
    if constexpr (PIPE) {
      cur = ga;
    } else {
      load_tile_typed<T>(d, g, in, scratch, out, tid, v);
      if (d.dst == kDstGather) gather_ahead(d, g, tc, tile_row, bin_id, tid, cur);
    }
    __syncthreads();                      // the previous tile's LDS reads are done

    // ---- fill the tile ----
    if (d.src == kSrcRows) {
      for (int e = tid; e < g.nel; e += kBlock) tile[e] = (T)0;
      const int64_t r_lo = tile_row[tc];
      const int64_t r_hi = g.tl + 1 < d.ntiles ? (int64_t)tile_row[tc + 1] : d.row_end;
      __syncthreads();
      for (int64_t r0 = r_lo + tid; r0 < r_hi; r0 += kRowBatch * kBlock) {
        int64_t bb[kRowBatch];
        double vv[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          const int64_t r = r0 + (int64_t)u * kBlock;
          bb[u] = r < r_hi ? bin_id[r] : -1;
          vv[u] = r < r_hi ? in[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          if (bb[u] >= 0) tile[bb[u] - g.flat_lo] = (T)vv[u];
      }
    } else {
      if constexpr (PIPE) fill_tile<T>(d, g, v, tid, tile);
      else fill_tile_typed<T>(d, g, v, tid, tile);
    }
    __syncthreads();

    // ---- the next tile: descriptor, and (PIPE) its loads queued ----
    const int64_t tn = tc + step;
    if (tn < tiles) {
      if (next_begin <= tn) {             // uniform: the next tile is in a later descriptor
        k = __builtin_amdgcn_readfirstlane(find_desc(descs, k + 1, ndesc, tn));
        next_begin = k + 1 < ndesc ? descs[k + 1].tile_begin : INT64_MAX;
      }
      nx = tile_geo(descs, k, tn);
      if constexpr (PIPE) {
        load_tile<T>(descs[k], nx, in, scratch, out, tid, v);
        if (descs[k].dst == kDstGather) gather_ahead(descs[k], nx, tn, tile_row, bin_id, tid, ga);
      }
    }

    // ---- transform each axis of the group ----
    int stride = d.TI * (int)d.G;         // stride of the axis above the current one
    const int naxes = d.naxes;
    for (int a = 0; a < naxes; ++a) {
      const int e = __builtin_amdgcn_readfirstlane(d.ext[a]);
      stride /= e;                        // stride of axis a inside the tile
      const int64_t mo = mat_offset(e - 1);
      if constexpr (MF) {
        axis_mfma<MODE, KIND, T>(tile, g.nel, e, stride, mats + mo);
      } else {
        typedef typename std::conditional<MODE == FCT_DCT_F64, double, float>::type A;
        const A* cm;
        if constexpr (MODE == FCT_DCT_F64) cm = mats + mo; else cm = mats32 + mo;
        if (KIND == 1 || e <= 16) axis_vector<T, A>(tile, g.nel, e, stride, cm);
        else if constexpr (KIND == 2) axis_long<32, T, A>(tile, g.nel, e, stride, cm);
        else if constexpr (KIND == 0) axis_long<64, T, A>(tile, g.nel, e, stride, cm);
      }
      __syncthreads();
    }

    // ---- store ----
    if (d.dst == kDstGather) {
#pragma unroll
      for (int u = 0; u < kGatherAhead; ++u)
        if (cur.lb[u] >= 0)
          out[cur.r_lo + tid + (int64_t)u * kBlock] = (double)tile[cur.lb[u]];
      for (int64_t r0 = cur.r_lo + tid + kGatherAhead * kBlock; r0 < cur.r_hi;
           r0 += kRowBatch * kBlock) {
        int64_t bb[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          const int64_t r = r0 + (int64_t)u * kBlock;
          bb[u] = r < cur.r_hi ? bin_id[r] : -1;
        }
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u)
          if (bb[u] >= 0) out[r0 + (int64_t)u * kBlock] = (double)tile[bb[u] - g.flat_lo];
      }
    } else {
      const int TI = d.TI;
      const int64_t I = d.I;
      const float invTI = 1.0f / (float)TI;
      if (d.dst == kDstScratch) {
        T* base = scratch + g.off;
        if (I == 1) {
          for (int e = tid; e < g.TOe * (int)d.G; e += kBlock) base[e] = tile[e];
        } else {
          for (int e = tid; e < g.nel; e += kBlock) {
            const int gg = div_small(e, TI, invTI);
            const int i = e - gg * TI;
            if (i < g.TIe) base[(int64_t)gg * I + i] = tile[e];
          }
        }
      } else {
        double* base = out + g.off;
        if (I == 1) {
          for (int e = tid; e < g.TOe * (int)d.G; e += kBlock) base[e] = (double)tile[e];
        } else {
          for (int e = tid; e < g.nel; e += kBlock) {
            const int gg = div_small(e, TI, invTI);
            const int i = e - gg * TI;
            if (i < g.TIe) base[(int64_t)gg * I + i] = (double)tile[e];
          }
        }
      }
    }
  }
}

// First row of every tile of the passes that gather (forward, innermost
// group) or scatter (inverse, innermost group) rows: the rows of a grid are
// sorted by flat bin index, so a tile's rows are those from the lower bound
// of its first flat index to the next tile's.  Other passes' entries are
// left unset.  One thread per tile of the level.
__global__ __launch_bounds__(kBlock) void tile_rows_kernel(
    const PassDesc* __restrict__ descs, int ndesc, int64_t tiles,
    const int64_t* __restrict__ bin_id, int32_t* __restrict__ tile_row) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tiles) return;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
  }
  const PassDesc& d = descs[lo];
  if (d.dst != kDstGather && d.src != kSrcRows) return;
  const int64_t flat_lo = (t - d.tile_begin) * d.TO * d.G;   // I == 1 for these passes
  tile_row[t] = (int32_t)lower_bound_i64(bin_id, d.row_begin, d.row_end, flat_lo);
}

// FP64 tiles run persistent and pipelined; FP32 tiles one per workgroup.
template <typename T>
constexpr bool kPipe = sizeof(T) == 8;

// The pass kernel of a level for a mode and engine (null: not available).
template <int MODE, typename T, bool MF>
const void* pass_kernel(int emax) {
  constexpr bool P = kPipe<T>;
  if constexpr (MF) {
    if (emax <= 16) return reinterpret_cast<const void*>(&dct_pass_kernel<MODE, 1, T, P, true>);
    if (emax <= 32) return reinterpret_cast<const void*>(&dct_pass_kernel<MODE, 2, T, P, true>);
    return nullptr;
  } else {
    if (emax <= 16) return reinterpret_cast<const void*>(&dct_pass_kernel<MODE, 1, T, P, false>);
    if (emax <= 32) return reinterpret_cast<const void*>(&dct_pass_kernel<MODE, 2, T, P, false>);
    return reinterpret_cast<const void*>(&dct_pass_kernel<MODE, 0, T, P, false>);
  }
}

template <int MODE, typename T, bool MF>
hipError_t launch_mode(const DctLevel& lv, const double* in, void* scratch, double* out,
                       const double* mats, const float* mats32, const int64_t* bin_id,
                       hipStream_t s) {
  constexpr bool P = kPipe<T>;
  const void* f = pass_kernel<MODE, T, MF>(lv.emax);
  if (!f) return hipErrorInvalidValue;
  const int64_t nwg = P ? std::min<int64_t>(lv.tiles, lv.grid[MODE][MF ? 1 : 0]) : lv.tiles;
  if (nwg <= 0 || nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  if (MODE == FCT_DCT_F32 && !mats32) return hipErrorInvalidValue;
  T* sc = static_cast<T*>(scratch);
  const PassDesc* descs = lv.d_desc;
  int ndesc = lv.ndesc;
  int64_t tiles = lv.tiles;
  const int32_t* tr = lv.d_tile_row;
  void* args[] = {&descs, &ndesc, &tiles, &in, &sc, &out, &mats, &mats32, &bin_id, &tr};
  const size_t lds = sizeof(T) * (size_t)std::min(lv.tile_max, kTileMax);
  return hipLaunchKernel(f, dim3((unsigned)nwg), dim3(kBlock), args, lds, s);
}

// Resident workgroups of one mode's and engine's pass kernel on the device:
// the persistent grid of a level (at least one workgroup per compute unit).
template <int MODE, typename T, bool MF>
hipError_t resident_grid(DctLevel& lv, int cus) {
  const void* f = pass_kernel<MODE, T, MF>(lv.emax);
  int64_t& g = lv.grid[MODE][MF ? 1 : 0];
  if (!f) { g = 0; return hipSuccess; }
  const size_t lds = sizeof(T) * (size_t)std::min(lv.tile_max, kTileMax);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlock, lds);
  if (e != hipSuccess) return e;
  g = (int64_t)std::max(per_cu, 1) * cus;
  return hipSuccess;
}

}  // namespace

hipError_t dct_level_grids(DctLevel& lv, int cus) {
  hipError_t e = resident_grid<FCT_DCT_F64, double, false>(lv, cus);
  if (e == hipSuccess) e = resident_grid<FCT_DCT_F64, double, true>(lv, cus);
  if (e == hipSuccess) e = resident_grid<FCT_DCT_F32, float, false>(lv, cus);
  if (e == hipSuccess) e = resident_grid<FCT_DCT_F32, float, true>(lv, cus);
  if (e == hipSuccess) e = resident_grid<FCT_DCT_BF16X3, float, true>(lv, cus);
  return e;
}

hipError_t launch_tile_rows(const DctLevel& lv, const int64_t* bin_id, hipStream_t s) {
  if (lv.tiles == 0 || !lv.d_tile_row) return hipSuccess;
  const int64_t nb = ceil_div(lv.tiles, (int64_t)kBlock);
  hipLaunchKernelGGL(tile_rows_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, lv.d_desc,
                     lv.ndesc, lv.tiles, bin_id, lv.d_tile_row);
  return hipGetLastError();
}

hipError_t launch_dct_level(const DctLevel& lv, int mode, int engine, const double* in,
                            void* scratch, double* out, const double* mats, const float* mats32,
                            const int64_t* bin_id, hipStream_t s) {
  if (lv.tiles == 0) return hipSuccess;
  if (lv.rows_io && !lv.d_tile_row) return hipErrorInvalidValue;
  const bool mf = engine == FCT_ENGINE_MATRIX;
  switch (mode) {
    case FCT_DCT_F64:
      return mf ? launch_mode<FCT_DCT_F64, double, true>(lv, in, scratch, out, mats, mats32,
                                                           bin_id, s)
                : launch_mode<FCT_DCT_F64, double, false>(lv, in, scratch, out, mats, mats32,
                                                            bin_id, s);
    case FCT_DCT_F32:
      return mf ? launch_mode<FCT_DCT_F32, float, true>(lv, in, scratch, out, mats, mats32,
                                                          bin_id, s)
                : launch_mode<FCT_DCT_F32, float, false>(lv, in, scratch, out, mats, mats32,
                                                           bin_id, s);
    case FCT_DCT_BF16X3:
      if (!mf) return hipErrorInvalidValue;
      return launch_mode<FCT_DCT_BF16X3, float, true>(lv, in, scratch, out, mats, mats32, bin_id,
                                                       s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fct
