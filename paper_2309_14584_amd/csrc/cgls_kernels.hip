// The stacked operator A and the CGLS least-squares iteration (Sec. 3.4,
// Alg. 3: c* = argmin_c || F f - A c ||_2, solved by conjugate gradients on
// the normal equations), for one problem or a batch of independent problems.
//
// A is applied without atomics.  q = A c sums, for each row (non-empty bin),
// the support entries that alias to it; the plan stores those entries
// contiguously (sorted by target bin), so each row is one segmented sum in a
// fixed order.  s = A^T r gathers, for each support entry, the K rows it
// aliases to.  Dot products are reduced per workgroup in a fixed tree and the
// partials are summed in a fixed order by every consumer, so every run gives
// the same bits.
//
// A batch is the block-diagonal system of its problems, but every problem
// keeps its own CG scalars, convergence test and reduction order: a
// workgroup only ever covers rows (or columns) of one problem, and the
// problem's partials are summed over its own workgroups in a fixed order.
// A problem's arithmetic is therefore identical alone and in any batch.
//
// Layout: the row vectors r and q are interleaved as (r, q) pairs and the
// column vectors p and s as (p, s) pairs, so each gather is one 16-byte load.
// The row kernel reads a row's first entries from a 4-wide padded copy of
// perm ("ell"), which saves the dependent load of the row's offset; longer
// rows continue in perm.  Each workgroup finds its problem and range in one
// uniform (scalar) load of its block descriptor.
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
// Per problem, gamma and alpha live in rings of four entries indexed by
// k mod 4, written by the problem's first workgroup and read by the next
// kernel: a launch reads entries k-1 (and k) and writes entry k, so no
// workgroup reads a value that another workgroup of the same launch is
// overwriting.  The iteration number is a device-side base plus a
// launch-time offset, which lets a fixed chunk of iterations be captured
// once in a HIP graph and replayed.
#include <algorithm>

#include "fct_internal.h"

namespace fct {
namespace {

// Sum over the workgroup (up to 16 waves); every thread gets the same value.
// Wave sums use a xor butterfly (each lane adds the same two operands as its
// partner, so all lanes agree bit for bit), then thread 0 adds the wave sums
// in order.  `sh` holds kShSlots doubles.
constexpr int kShSlots = 17;
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
    sh[16] = r;
  }
  __syncthreads();
  const double r = sh[16];
  __syncthreads();
  return r;
}

// This thread's share of a problem's per-workgroup partials.  With at most
// one partial per thread (the usual case) it is a single unconditional load
// from a clamped index, which the compiler can issue next to the kernel's
// other independent loads instead of waiting for it in a loop.
__device__ __forceinline__ double load_partials(const double* __restrict__ part, int32_t off,
                                                int32_t np) {
  if (np <= (int32_t)blockDim.x) {
    const int32_t i = (int32_t)threadIdx.x < np ? (int32_t)threadIdx.x : np - 1;
    const double v = part[off + i];
    return (int32_t)threadIdx.x < np ? v : 0.0;
  }
  double v = 0.0;
  for (int32_t i = threadIdx.x; i < np; i += blockDim.x) v += part[off + i];
  return v;
}

// The partial of ||q||^2 of row block b is the sum of its four per-wave
// partials, in wave order; this thread's share of a problem's row blocks,
// taken as load_partials takes per-block partials.
__device__ __forceinline__ double row_block_partial(const double* __restrict__ part, int32_t b) {
  const double* w = part + 4 * (int64_t)b;
  return ((w[0] + w[1]) + w[2]) + w[3];
}
__device__ __forceinline__ double load_row_partials(const double* __restrict__ part, int32_t off,
                                                    int32_t np) {
  if (np <= (int32_t)blockDim.x) {
    const int32_t i = (int32_t)threadIdx.x < np ? (int32_t)threadIdx.x : np - 1;
    const double v = row_block_partial(part, off + i);
    return (int32_t)threadIdx.x < np ? v : 0.0;
  }
  double v = 0.0;
  for (int32_t i = threadIdx.x; i < np; i += blockDim.x) v += row_block_partial(part, off + i);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double ring_gamma(const double* ring, int p, int k) {
  return ring[p * 8 + (k & 3)];
}
__device__ __forceinline__ double ring_alpha(const double* ring, int p, int k) {
  return ring[p * 8 + 4 + (k & 3)];
}

// (x, y) pairs stored in FP64 (double2) or FP32 (float2); arithmetic in FP64.
__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
// A pair as loaded: double2, or a float2 held as one 64-bit word.  Loads
// that are merged with a default value (masked lanes) keep the raw word in
// registers until it is used; a float2 merged as two floats would make the
// compiler wait for each load before the next one is issued.
template <typename P> struct RawOf { typedef P type; };
template <> struct RawOf<float2> { typedef unsigned long long type; };
__device__ __forceinline__ double2 raw_d2(double2 v) { return v; }
__device__ __forceinline__ double2 raw_d2(unsigned long long v) {
  float2 f;
  __builtin_memcpy(&f, &v, sizeof(f));
  return make_double2(f.x, f.y);
}
template <typename R> __device__ __forceinline__ R raw_zero() { return R{}; }
// What the column kernel gathers per row: the (r, q) pair as loaded, or in
// the FP32 rounds q alone (float); row_d2 widens it to (r, q).
template <bool NR, typename R> struct RowGather { typedef R type; };
template <typename R> struct RowGather<true, R> { typedef float type; };
__device__ __forceinline__ double2 row_d2(double2 v) { return v; }
__device__ __forceinline__ double2 row_d2(unsigned long long v) { return raw_d2(v); }
__device__ __forceinline__ double2 row_d2(float q) { return make_double2(0.0, (double)q); }

// p = s + beta p_prev in FP64, rounded to the pair's storage precision: the
// FP32 rounds use the FP32 value of p everywhere (in q = A p, in the update
// of c and in the next direction), as a unit that stages p in LDS does.
template <typename P> __device__ __forceinline__ double direction(double beta, double2 v);
template <> __device__ __forceinline__ double direction<double2>(double beta, double2 v) {
  return fma(beta, v.x, v.y);
}
template <> __device__ __forceinline__ double direction<float2>(double beta, double2 v) {
  return (double)(float)fma(beta, v.x, v.y);
}

template <typename P> __device__ __forceinline__ P make_pair(double x, double y);
template <> __device__ __forceinline__ double2 make_pair<double2>(double x, double y) {
  return make_double2(x, y);
}
template <> __device__ __forceinline__ float2 make_pair<float2>(double x, double y) {
  return make_float2((float)x, (float)y);
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

__global__ __launch_bounds__(kBlock) void apply_AT_kernel(const ColBlock* __restrict__ cblk,
                                                          const int32_t* __restrict__ rowmap,
                                                          const double* __restrict__ r,
                                                          double* __restrict__ s) {
  const ColBlock bd = cblk[blockIdx.x];
  const int32_t j = bd.col0 + threadIdx.x;          // global column
  if (j >= bd.col_end) return;
  const int32_t jl = j - bd.col_off;                 // column within its problem
  double acc = 0.0;
  for (int l = 0; l < bd.K; ++l) acc += r[rowmap[bd.rmap_off + l * bd.n + jl]];
  s[j] = acc;
}

// r_0 = b - A c_0 (c_0 = 0 unless warm), q = 0; resets the iteration state.
__global__ __launch_bounds__(kBlock) void cgls_init_rows_kernel(CglsArgs a,
                                                                const double* __restrict__ b,
                                                                int warm) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) { a.state[0] = 0; a.state[1] = 0; }
  if (g < a.nprob) { a.done[g] = 0; a.flags[g] = 0; }
  const RowBlock bd = a.rblk[blockIdx.x];
  const int32_t row = bd.row0 + threadIdx.x;
  if (row >= bd.row_end) return;
  double acc = 0.0;
  if (warm) {
    const int32_t t1 = a.seg_off[row + 1];
    for (int32_t t = a.seg_off[row]; t < t1; ++t) acc += a.c[a.perm[t]];
  }
  static_cast<double2*>(a.rq)[row] = make_double2(b[row] - acc, 0.0);
}

// s_0 = A^T r_0, p = 0, c = 0 unless warm, partials of ||s_0||^2.
__global__ __launch_bounds__(kBlock) void cgls_init_cols_kernel(CglsArgs a, int warm) {
  __shared__ double sh[kShSlots];
  const ColBlock bd = a.cblk[blockIdx.x];
  const int32_t j = bd.col0 + threadIdx.x;
  double sv = 0.0;
  if (j < bd.col_end) {
    const int32_t jl = j - bd.col_off;
    const double2* rq = static_cast<const double2*>(a.rq);
    for (int l = 0; l < bd.K; ++l) sv += rq[a.rowmap[bd.rmap_off + l * bd.n + jl]].x;
    static_cast<double2*>(a.ps)[j] = make_double2(0.0, sv);
    if (!warm) a.c[j] = 0.0;
  }
  const double part = block_sum(sv * sv, sh);
  if (threadIdx.x == 0) a.part_s[blockIdx.x] = part;
}

// Registers that prefetch a column's K aliases before the iteration scalars
// are known; further grids continue in a loop.
constexpr int kPrefetch = 4;
// Loads issued together in the loops over long rows and further grids:
// eight for FP32 pairs, six for FP64 pairs (what fits in the 64 registers of
// eight waves per SIMD without spilling).
template <typename P> struct BatchOf { static constexpr int value = 8; };
template <> struct BatchOf<double2> { static constexpr int value = 6; };

// In a batch, whether problem p still iterates, read before any operand is
// loaded so that the workgroups of finished problems cost no memory traffic.
// The value only gates those loads: the decision to return is taken from the
// workgroup's LDS copy of the flag after the first barrier.  A wave that
// sees the flag set during this launch (by the problem's first workgroup)
// belongs to a workgroup that reaches the same stop decision from the same
// scalars before it would use any skipped operand.  A single problem never
// pays for the extra dependent load.
// Block descriptors of the iteration kernels: formed from the arguments for
// a single problem (regular blocks; every load that needs a row or column
// index then waits for no table read), loaded from the tables otherwise.
__device__ __forceinline__ RowBlock row_block(const CglsArgs& a) {
  if (a.reg_M > 0) {
    RowBlock r;
    r.prob = 0;
    r.row0 = (int32_t)blockIdx.x * kBlock;
    r.row_end = min(a.reg_M, r.row0 + kBlock);
    r.cblk_off = 0;
    r.ncblk = (int32_t)a.ncblk;
    r.first = blockIdx.x == 0 ? 1 : 0;
    r.pslot = (int32_t)blockIdx.x;
    r.pad1 = 0;
    return r;
  }
  return a.rblk[blockIdx.x];
}

__device__ __forceinline__ ColBlock col_block(const CglsArgs& a) {
  if (a.reg_n > 0) {
    ColBlock c;
    c.prob = 0;
    c.col0 = (int32_t)blockIdx.x * kBlock;
    c.col_end = min(a.reg_n, c.col0 + kBlock);
    c.col_off = 0;
    c.rblk_off = 0;
    c.nrblk = (int32_t)a.nrblk;
    c.K = a.reg_K;
    c.n = a.reg_n;
    c.rmap_off = 0;
    c.first = blockIdx.x == 0 ? 1 : 0;
    c.pad0 = 0;
    c.pad1 = 0;
    return c;
  }
  return a.cblk[blockIdx.x];
}

__device__ __forceinline__ bool live_problem(const CglsArgs& a, int p) {
  return a.nprob == 1 || __builtin_amdgcn_readfirstlane(a.done[p]) == 0;
}

// NR: the normal-equation form used by the mixed-precision rounds.  The
// residual r is not carried; the column kernel updates s = A^T r by
// s <- s - alpha A^T q, so a round can start from s = A^T (b - A c)
// computed in FP64, which tends to zero at the least-squares solution even
// when the system is inconsistent (r itself does not).
//
// The work of one row block and of one column block is split into a load
// step (every operand that does not depend on the iteration's scalars,
// values kept raw so that the loads are all in flight together) and a
// finish step; the two-kernel iteration and the single-kernel iteration
// (cgls_fused_kernel) run the same steps, so they give the same bits.
template <typename P, bool NR> struct RowOps {
  typedef typename RawOf<P>::type R;
  R rq_raw, r0, r1, r2, r3;
  int4 e;
  int32_t row;
  bool active;
};

template <typename P, bool NR>
__device__ __forceinline__ RowOps<P, NR> rows_load(const CglsArgs& a, const RowBlock& bd,
                                                   bool live) {
  typedef typename RawOf<P>::type R;
  const R* const rqr = static_cast<const R*>(a.rq);
  const R* const psr = static_cast<const R*>(a.ps);
  RowOps<P, NR> o;
  o.row = bd.row0 + threadIdx.x;
  o.active = o.row < bd.row_end && live;
  o.rq_raw = raw_zero<R>();
  o.e = make_int4(-1, -1, -1, -1);
  if (o.active) {
    o.rq_raw = rqr[o.row];
    o.e = a.ell[o.row];
  }
  o.r0 = o.e.x >= 0 ? psr[o.e.x] : raw_zero<R>();
  o.r1 = o.e.y >= 0 ? psr[o.e.y] : raw_zero<R>();
  o.r2 = o.e.z >= 0 ? psr[o.e.z] : raw_zero<R>();
  o.r3 = o.e.w >= 0 ? psr[o.e.w] : raw_zero<R>();
  return o;
}

// q = A p for the block's rows with p_k = s_k + beta p_{k-1} formed on the
// fly, r updated, and the per-wave partials of ||q||^2 (no barrier: the
// consumer adds the four waves of each block in order).
// FP64 rows with more than kLongRow entries (a dimension that most grids do
// not resolve collects many columns in one bin) are summed by the whole
// wave: lane i adds entries i, i + 64, ... of the run in order, then a fixed
// butterfly; shorter rows, and every row of the FP32 rounds, are summed by
// their own lane in perm order.  Either way a row's sum does not depend on
// the launch it is part of.
constexpr int32_t kLongRow = 96;

template <typename P, bool NR>
__device__ __forceinline__ void rows_finish(const CglsArgs& a, const RowBlock& bd,
                                            const RowOps<P, NR>& o, double beta,
                                            double alpha_prev) {
  typedef typename RawOf<P>::type R;
  const R* const psr = static_cast<const R*>(a.ps);
  double qv = 0.0;
  // a row of more than four entries: its run is [t_beg, t_end) in perm (the
  // ELL marker holds the position of its fourth entry)
  int32_t t_beg = 0, t_end = 0;
  if (o.active && o.e.w < -1) {
    t_beg = -(o.e.w + 2) - 3;
    t_end = a.seg_off[o.row + 1];
  }
  const bool is_long = !NR && t_end - t_beg > kLongRow;
  // own rows first (the prefetched pairs are consumed before the wave loop)
  if (o.active && !is_long) {
    const int4 e = o.e;
    const double2 v0 = raw_d2(o.r0), v1 = raw_d2(o.r1), v2 = raw_d2(o.r2), v3 = raw_d2(o.r3);
    // terms in perm order: p_k = s_k + beta p_{k-1} for each aliased column
    if (e.x >= 0) qv += direction<P>(beta, v0);
    if (e.y >= 0) qv += direction<P>(beta, v1);
    if (e.z >= 0) qv += direction<P>(beta, v2);
    if (e.w >= 0) qv += direction<P>(beta, v3);
    if (e.w < -1) {                                  // row of 5..kLongRow: rest of its run
      const int32_t t1 = t_end;
      constexpr int kBatch = BatchOf<P>::value;
      for (int32_t t0 = -(e.w + 2); t0 < t1; t0 += kBatch) {
        // kBatch independent index loads, then kBatch independent gathers,
        // then the sums in perm order
        int32_t jj[kBatch];
        R vv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) jj[u] = t0 + u < t1 ? a.perm[t0 + u] : -1;
#pragma unroll
        for (int u = 0; u < kBatch; ++u) vv[u] = jj[u] >= 0 ? psr[jj[u]] : raw_zero<R>();
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const double2 v = raw_d2(vv[u]);
          if (jj[u] >= 0) qv += direction<P>(beta, v);
        }
      }
    }
  }
  // long rows of the wave, one after another, by all 64 lanes
  if (!NR) {
    uint64_t pending = __ballot(is_long);
    while (pending != 0) {                           // wave-uniform
      const int src = __ffsll((unsigned long long)pending) - 1;
      pending &= pending - 1;
      const int32_t t0 = __shfl(t_beg, src, 64), t1 = __shfl(t_end, src, 64);
      const int lane = (int)(threadIdx.x & 63);
      double part = 0.0;
      for (int32_t t = t0 + lane; t < t1; t += 2 * 64) {
        const int32_t j0 = a.perm[t];
        const int32_t j1 = t + 64 < t1 ? a.perm[t + 64] : -1;
        const R w0 = psr[j0];
        const R w1 = j1 >= 0 ? psr[j1] : raw_zero<R>();
        part += direction<P>(beta, raw_d2(w0));
        if (j1 >= 0) part += direction<P>(beta, raw_d2(w1));
      }
      const double tot = wave_sum(part);
      if (lane == src) qv = tot;
    }
  }
  if (o.active) {
    const double2 rq_old = raw_d2(o.rq_raw);
    if (NR) static_cast<float*>(a.rq)[o.row] = (float)qv;     // q alone, FP32
    else static_cast<P*>(a.rq)[o.row] = make_pair<P>(fma(-alpha_prev, rq_old.y, rq_old.x), qv);
  }
  const double w = wave_sum(qv * qv);
  if ((threadIdx.x & 63) == 0) a.part_q[4 * (int64_t)bd.pslot + (threadIdx.x >> 6)] = w;
}

// gamma_k from the column partials, beta, and the stop test of iteration k.
__device__ __forceinline__ void row_scalars(const CglsArgs& a, int p, int k, double gpart,
                                            double* sh, double* gamma, double* beta,
                                            double* alpha_prev, bool* stop) {
  // k0: first iteration of this run (0, or 1 for a mixed-precision round that
  // continues the previous round's direction; see refine_cols_kernel)
  const int k0 = a.state[1];
  double gprev = 1.0, g0 = 0.0, ap = 0.0;
  if (k > 0) {
    gprev = ring_gamma(a.ring, p, k - 1);
    ap = ring_alpha(a.ring, p, k - 1);
    g0 = a.gamma0[p];
  }
  const double g = block_sum(gpart, sh);
  *gamma = g;
  *beta = k > 0 ? g / gprev : 0.0;
  *alpha_prev = ap;
  // the first iteration only stops on a zero (or non-finite) normal residual
  *stop = k == k0 ? !(g > 0.0) : !(g > a.tol2 * g0);
}

__device__ __forceinline__ void row_scalars_store(const CglsArgs& a, int p, int k, double gamma,
                                                  bool stop) {
  a.ring[p * 8 + (k & 3)] = gamma;
  if (k == a.state[1]) a.gamma0[p] = gamma;
  if (stop) a.done[p] = k + 1;
}

template <typename P, bool NR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
void cgls_rows_kernel(CglsArgs a, int rel) {
  __shared__ double sh[kShSlots];
  __shared__ int s_done;
  const RowBlock bd = row_block(a);                  // uniform
  const int p = bd.prob;
  // the problem's stop flag is read once per workgroup (thread 0, through
  // LDS), so all of its waves take the same branch even if the problem's
  // first workgroup sets the flag during this launch
  if (threadIdx.x == 0) s_done = a.done[p];
  const int base = a.state[0];
  // operands that do not depend on this iteration's scalars; in a batch a
  // problem that has stopped issues none of them
  const RowOps<P, NR> o = rows_load<P, NR>(a, bd, live_problem(a, p));
  const double gpart = load_partials(a.part_s, bd.cblk_off, bd.ncblk);
  __syncthreads();
  if (s_done != 0) return;                           // problem converged or stopped
  const int k = base + rel;
  double gamma, beta, alpha_prev;
  bool stop;
  row_scalars(a, p, k, gpart, sh, &gamma, &beta, &alpha_prev, &stop);
  if (bd.first && threadIdx.x == 0) row_scalars_store(a, p, k, gamma, stop);
  if (stop) return;
  rows_finish<P, NR>(a, bd, o, beta, alpha_prev);
}

template <typename P, bool NR> struct ColOps {
  typedef typename RawOf<P>::type R;
  typedef typename RowGather<NR, R>::type G;
  R ps_raw;
  double c_old;
  G g[kPrefetch];
  int32_t j, jl;
  bool active;
};

template <typename P, bool NR>
__device__ __forceinline__ ColOps<P, NR> cols_load(const CglsArgs& a, const ColBlock& bd,
                                                   bool live) {
  // Unconditional loads from clamped indices (an idle lane reads the
  // block's first column, shared by its whole wave), raw until after the
  // barrier: the index loads and the gathers they feed are each issued
  // together instead of one pair at a time.
  typedef typename RawOf<P>::type R;
  typedef typename RowGather<NR, R>::type G;
  const G* const rqg = static_cast<const G*>(a.rq);
  ColOps<P, NR> o;
  o.j = bd.col0 + threadIdx.x;
  o.active = o.j < bd.col_end && live;
  o.jl = o.j - bd.col_off;
  const int32_t jc = o.active ? o.j : bd.col0;
  const int32_t jlc = jc - bd.col_off;
  o.ps_raw = static_cast<const R*>(a.ps)[jc];
  o.c_old = a.c[jc];
#pragma unroll
  for (int l = 0; l < kPrefetch; ++l)
    o.g[l] = rqg[a.rowmap[bd.rmap_off + (l < bd.K ? l : 0) * bd.n + jlc]];
  return o;
}

// p_k stored, c_{k+1} = c_k + alpha p_k, s_{k+1}, and the block's partial of
// ||s_{k+1}||^2 into part_s[slot].
template <typename P, bool NR, int BATCH = BatchOf<P>::value>
__device__ __forceinline__ void cols_finish(const CglsArgs& a, const ColBlock& bd,
                                            const ColOps<P, NR>& o, double alpha, double beta,
                                            double* sh, int64_t slot) {
  typedef typename RawOf<P>::type R;
  typedef typename RowGather<NR, R>::type G;
  const G* const rqg = static_cast<const G*>(a.rq);
  double sv = 0.0;
  if (o.active) {
    const double2 ps_old = raw_d2(o.ps_raw);
    const double pv = direction<P>(beta, ps_old);
    a.c[o.j] = fma(alpha, pv, o.c_old);
    double qs = 0.0;                                 // NR: (A^T q)_j
#pragma unroll
    for (int l = 0; l < kPrefetch; ++l) {
      const double2 v = row_d2(o.g[l]);
      if (l < bd.K) {
        if (NR) qs += v.y;
        else sv += fma(-alpha, v.y, v.x);
      }
    }
    // further grids kBatch at a time: independent loads, sums in grid order
    constexpr int kBatch = BATCH;
    for (int l0 = kPrefetch; l0 < bd.K; l0 += kBatch) {
      G vv[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u)
        vv[u] = rqg[a.rowmap[bd.rmap_off + min(l0 + u, bd.K - 1) * bd.n + o.jl]];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const double2 v = row_d2(vv[u]);
        if (l0 + u < bd.K) {
          if (NR) qs += v.y;
          else sv += fma(-alpha, v.y, v.x);
        }
      }
    }
    if (NR) sv = fma(-alpha, qs, ps_old.y);
    static_cast<P*>(a.ps)[o.j] = make_pair<P>(pv, sv);
  }
  const double part = block_sum(sv * sv, sh);
  if (threadIdx.x == 0) a.part_s[slot] = part;
}

template <typename P, bool NR, int BATCH = BatchOf<P>::value, int WAVES = 8>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WAVES, 8)))
void cgls_cols_kernel(CglsArgs a, int rel) {
  __shared__ double sh[kShSlots];
  __shared__ int s_done;
  const ColBlock bd = col_block(a);
  const int p = bd.prob;
  if (threadIdx.x == 0) s_done = a.done[p];
  const int base = a.state[0];
  const ColOps<P, NR> o = cols_load<P, NR>(a, bd, live_problem(a, p));
  const double dpart = load_row_partials(a.part_q, bd.rblk_off, bd.nrblk);
  __syncthreads();
  if (s_done != 0) return;
  const int k = base + rel;
  const double gamma = ring_gamma(a.ring, p, k);
  const double gprev = (k > 0) ? ring_gamma(a.ring, p, k - 1) : 1.0;
  const double delta = block_sum(dpart, sh);
  const double beta = (k > 0) ? gamma / gprev : 0.0;
  if (!(delta > 0.0)) {                              // A p = 0: breakdown
    if (bd.first && threadIdx.x == 0) { a.flags[p] = 1; a.done[p] = k + 1; }
    return;
  }
  const double alpha = gamma / delta;
  if (bd.first && threadIdx.x == 0) a.ring[p * 8 + 4 + (k & 3)] = alpha;
  cols_finish<P, NR, BATCH>(a, bd, o, alpha, beta, sh, blockIdx.x);
}

// ---- one problem: the whole iteration in one kernel ----
// For a single problem small enough that every row block and every column
// block has a workgroup of its own, cgls_fused_kernel runs `iters`
// iterations in one launch: row phase, grid barrier, column phase, grid
// barrier.  Every workgroup forms the iteration's scalars itself from the
// same partials in the same order (so all agree on when to stop), and the
// row and column work is exactly that of the two kernels above.
//
// The grid barrier needs every workgroup resident (cooperative launch).
// bar[0] counts arrivals and bar[1] is the generation: a workgroup reads the
// generation, releases its writes, arrives, and waits for the generation to
// change; the last arrival resets the count and advances the generation.
// A wait longer than kSpinLimit polls sets *abort (the host reports a device
// error) and every later wait returns at once, so no wait is unbounded.
constexpr long kSpinLimit = 4000000;

__device__ __forceinline__ void grid_sync(int* bar, int nblocks, int* abort) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const int arrived = __hip_atomic_fetch_add(&bar[0], 1, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (++spins > kSpinLimit) {
          __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();
  }
  __syncthreads();
}

template <typename P, bool NR>
__global__ __launch_bounds__(kBlock) void cgls_fused_kernel(CglsArgs a, int iters, int* bar,
                                                            int* abort) {
  __shared__ double sh[kShSlots];
  __shared__ int s_flag;
  const int nwg = (int)gridDim.x;
  const int w = (int)blockIdx.x;
  const int base = a.state[0];
  for (int rel = 0; rel < iters; ++rel) {
    const int k = base + rel;
    // stopped before (an earlier launch), or a barrier gave up: every
    // workgroup reads the same values here, after the last barrier
    if (threadIdx.x == 0)
      s_flag = __hip_atomic_load(&a.done[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
               __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // row phase
    RowBlock bd;
    RowOps<P, NR> o;
    if (w < a.nrblk) {
      bd = a.rblk[w];
      o = rows_load<P, NR>(a, bd, true);
    }
    const double gpart = load_partials(a.part_s, 0, (int32_t)a.ncblk);
    __syncthreads();
    if (s_flag != 0) break;
    double gamma, beta, alpha_prev;
    bool stop;
    row_scalars(a, 0, k, gpart, sh, &gamma, &beta, &alpha_prev, &stop);
    if (w == 0 && threadIdx.x == 0) row_scalars_store(a, 0, k, gamma, stop);
    if (stop) break;
    for (int64_t b = w; b < a.nrblk; b += nwg) {
      if (b != w) {
        bd = a.rblk[b];
        o = rows_load<P, NR>(a, bd, true);
      }
      rows_finish<P, NR>(a, bd, o, beta, alpha_prev);
    }
    grid_sync(bar, nwg, abort);
    // column phase
    const double dpart = load_row_partials(a.part_q, 0, (int32_t)a.nrblk);
    const double delta = block_sum(dpart, sh);
    if (!(delta > 0.0)) {                            // A p = 0: breakdown
      if (w == 0 && threadIdx.x == 0) { a.flags[0] = 1; a.done[0] = k + 1; }
      break;
    }
    const double alpha = gamma / delta;
    if (w == 0 && threadIdx.x == 0) a.ring[4 + (k & 3)] = alpha;
    for (int64_t c = w; c < a.ncblk; c += nwg) {
      const ColBlock cb = a.cblk[c];
      const ColOps<P, NR> co = cols_load<P, NR>(a, cb, true);
      cols_finish<P, NR>(a, cb, co, alpha, beta, sh, c);
    }
    grid_sync(bar, nwg, abort);
  }
}

// ---- FP32 rounds of a batch: q = A p from LDS ----
// One workgroup of kLdsBlock threads per unit (up to the plan's unit_rows
// consecutive rows of one problem).  The problem's p = fp32(s + beta p_prev)
// is staged in LDS once, then each row sums its entries from LDS.  Every
// value and every reduction is formed exactly as in
// cgls_rows_kernel<float2, true>: gamma from the column partials by the
// first 256 threads in the 256-thread order, the per-row sums in perm order,
// and the per-wave partials of ||q||^2 of each 256-row block with the same
// butterflies, written to that block's slots.  So a problem gives the same
// bits whether its rows run here (in a batch) or in row blocks (alone).
constexpr int kUnitChunks = 6;          // rows per thread in flight (chunks of kLdsBlock rows)

__global__ __launch_bounds__(kLdsBlock) void cgls_rows_unit_kernel(CglsArgs a, int rel) {
  extern __shared__ float lds_p[];                   // [lds_cap]
  __shared__ double sh[kShSlots];
  __shared__ int s_done;
  const RowUnit u = a.units[blockIdx.x];
  const int p = u.prob;
  const int tid = threadIdx.x;
  if (tid == 0) s_done = a.done[p];
  const int base = a.state[0];
  // this thread's share of the column partials, as a 256-thread block takes it
  double gpart = 0.0;
  if (tid < kBlock)
    for (int32_t i = tid; i < u.ncblk; i += kBlock) gpart += a.part_s[u.cblk_off + i];
  __syncthreads();
  if (s_done != 0) return;
  const int k = base + rel;
  const int k0 = a.state[1];
  double gprev = 1.0, g0 = 0.0;
  if (k > 0) {
    gprev = ring_gamma(a.ring, p, k - 1);
    g0 = a.gamma0[p];
  }
  // gamma: butterflies in waves 0..3, then their four sums in order
  {
    const double w = wave_sum(gpart);
    if ((tid & 63) == 0 && tid < kBlock) sh[tid >> 6] = w;
    __syncthreads();
    if (tid == 0) sh[16] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
  }
  const double gamma = sh[16];
  const double beta = k > 0 ? gamma / gprev : 0.0;
  const bool stop = k == k0 ? !(gamma > 0.0) : !(gamma > a.tol2 * g0);
  if (u.first && tid == 0) {
    a.ring[p * 8 + (k & 3)] = gamma;
    if (k == k0) a.gamma0[p] = gamma;
    if (stop) a.done[p] = k + 1;
  }
  if (stop) return;

  // stage p of the problem's columns
  const unsigned long long* psr = static_cast<const unsigned long long*>(a.ps);
  // eight coalesced loads in flight per thread, then their LDS stores
  for (int32_t j0 = 0; j0 < u.n; j0 += 8 * kLdsBlock) {
    unsigned long long raw[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int32_t j = j0 + v * kLdsBlock + tid;
      raw[v] = psr[u.col_off + (j < u.n ? j : 0)];
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int32_t j = j0 + v * kLdsBlock + tid;
      const double2 x = raw_d2(raw[v]);
      if (j < u.n) lds_p[j] = (float)fma(beta, x.x, x.y);
    }
  }
  __syncthreads();

  float* const q = static_cast<float*>(a.rq);
  const int32_t rows_per_round = kUnitChunks * kLdsBlock;
  // the 16-bit ELL entries of kUnitChunks rows per thread, all in flight;
  // the next round's are loaded before this round's sums are formed
  uint4 en[kUnitChunks];
#pragma unroll
  for (int c = 0; c < kUnitChunks; ++c) {
    const int32_t row = u.row0 + c * kLdsBlock + tid;
    en[c] = a.ell16[row < u.row_end ? row : u.row0];
  }
  for (int32_t r0 = u.row0; r0 < u.row_end; r0 += rows_per_round) {
    uint4 e[kUnitChunks];
#pragma unroll
    for (int c = 0; c < kUnitChunks; ++c) {
      e[c] = en[c];
      const int32_t row = r0 + rows_per_round + c * kLdsBlock + tid;
      en[c] = a.ell16[row < u.row_end ? row : u.row0];
    }
    double qv[kUnitChunks];
#pragma unroll
    for (int c = 0; c < kUnitChunks; ++c) {
      const int32_t row = r0 + c * kLdsBlock + tid;
      qv[c] = 0.0;
      if (row < u.row_end) {
        const uint32_t w[4] = {e[c].x, e[c].y, e[c].z, e[c].w};
        // slots in perm order; 0xFFFF empty, slot 7 = 0xFFFE: the run goes on
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t v = (w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
          if (v < 0xFFFEu) qv[c] += (double)lds_p[v];
        }
        if ((w[3] >> 16) == 0xFFFEu) {               // long row: perm from entry 7 on
          const int32_t t1 = a.seg_off[row + 1];
          for (int32_t t0 = a.seg_off[row] + 7; t0 < t1; t0 += 16) {
            int32_t jj[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) jj[v] = a.perm[min(t0 + v, t1 - 1)];
#pragma unroll
            for (int v = 0; v < 16; ++v)
              if (t0 + v < t1) qv[c] += (double)lds_p[jj[v] - u.col_off];
          }
        }
        q[row] = (float)qv[c];
      }
    }
    // per-wave partials of ||q||^2 into the slots of the row blocks, as
    // the row-block kernel writes them (a wave past the unit's end but in
    // its last block writes 0)
#pragma unroll
    for (int c = 0; c < kUnitChunks; ++c) {
      const double w = wave_sum(qv[c] * qv[c]);
      const int32_t wrow = r0 + c * kLdsBlock + (tid & ~63);     // the wave's first row
      const int32_t blk = (wrow - u.row0) / kBlock;
      if ((tid & 63) == 0 && u.row0 + blk * kBlock < u.row_end)
        a.part_q[4 * (int64_t)(u.pslot + blk) + ((wrow - u.row0) % kBlock) / 64] = w;
    }
  }
}

// ---- mixed precision: FP32 CGLS rounds with FP64 residual refinement ----
// r64 = b - A c in FP64 (c is FP64); resets the round's iteration state;
// problems already finished keep their stop flag.
__global__ __launch_bounds__(kBlock) void refine_rows_kernel(CglsArgs a,
                                                             const double* __restrict__ b,
                                                             int start) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) { a.state[0] = start; a.state[1] = start; }
  if (g < a.nprob) { a.done[g] = a.outer_done[g]; a.flags[g] = 0; }
  const RowBlock bd = a.rblk[blockIdx.x];
  const int32_t row = bd.row0 + threadIdx.x;
  if (row >= bd.row_end) return;
  const int4 e = a.ell[row];
  double acc = 0.0;
  if (e.x >= 0) acc += a.c[e.x];
  if (e.y >= 0) acc += a.c[e.y];
  if (e.z >= 0) acc += a.c[e.z];
  if (e.w >= 0) acc += a.c[e.w];
  if (e.w < -1) {
    const int32_t t1 = a.seg_off[row + 1];
    for (int32_t t = -(e.w + 2); t < t1; ++t) acc += a.c[a.perm[t]];
  }
  a.r64[row] = b[row] - acc;
}

// s64 = A^T r64 in FP64 and s = fp32(s64); partials of ||s||^2 (the round's
// CG start) and of ||s64||^2 (the FP64 normal residual).
// A problem with gprev[p] > 0 continues its previous direction (a reliable
// update: only the recurred residual is replaced by the true one): p is
// kept and ring entry 0 receives gamma of the iteration before the previous
// round stopped, so the round's first step (iteration 1) forms
// p = s + (||s||^2 / gprev) p_old.  Otherwise the round restarts with p = 0.
__global__ __launch_bounds__(kBlock) void refine_cols_kernel(CglsArgs a,
                                                             const double* __restrict__ gprev) {
  __shared__ double sh[kShSlots];
  const ColBlock bd = a.cblk[blockIdx.x];
  const int32_t j = bd.col0 + threadIdx.x;
  const bool cont = gprev[bd.prob] > 0.0;
  // a restarting problem gets any finite positive entry (it multiplies p = 0)
  if (bd.first && threadIdx.x == 0) a.ring[bd.prob * 8] = cont ? gprev[bd.prob] : 1.0;
  double s64 = 0.0, s32 = 0.0;
  if (j < bd.col_end) {
    const int32_t jl = j - bd.col_off;
    for (int l = 0; l < bd.K; ++l) s64 += a.r64[a.rowmap[bd.rmap_off + l * bd.n + jl]];
    const float sf = (float)s64;
    s32 = sf;
    float2* ps = static_cast<float2*>(a.ps);
    ps[j] = make_float2(cont ? ps[j].x : 0.0f, sf);
  }
  const double p32 = block_sum(s32 * s32, sh);
  const double p64 = block_sum(s64 * s64, sh);
  if (threadIdx.x == 0) { a.part_s[blockIdx.x] = p32; a.part_true[blockIdx.x] = p64; }
}

// Per problem (one workgroup each): the FP64 normal residual of this round;
// round 0 records it as the reference, later rounds finish the problem when
// it has dropped to tol_outer^2 of the reference (or is zero / not finite).
__global__ __launch_bounds__(kBlock) void refine_check_kernel(CglsArgs a, int round,
                                                              double tol2_outer) {
  __shared__ double sh[kShSlots];
  const int p = blockIdx.x;
  const ProbInfo pi = a.prob[p];
  const double g = block_sum(load_partials(a.part_true, pi.cblk_off, pi.ncblk), sh);
  if (threadIdx.x != 0) return;
  if (a.outer_done[p] != 0) return;
  if (round == 0) a.gtrue0[p] = g;
  a.gtrue[p] = g;
  const double g0 = round == 0 ? g : a.gtrue0[p];
  const bool fin = !(g > 0.0) || !(g > tol2_outer * g0) || !isfinite(g0);
  if (fin) { a.outer_done[p] = round + 1; a.done[p] = 1; }
}

// gamma of the current column partials into ring entry k, for every problem
// that did not stop (one workgroup per problem).
__global__ __launch_bounds__(kBlock) void cgls_gamma_kernel(CglsArgs a, int k) {
  __shared__ double sh[kShSlots];
  const int p = blockIdx.x;
  const ProbInfo pi = a.prob[p];
  const double gamma = block_sum(load_partials(a.part_s, pi.cblk_off, pi.ncblk), sh);
  if (threadIdx.x == 0 && a.done[p] == 0) a.ring[p * 8 + (k & 3)] = gamma;
}

__global__ void cgls_set_base_kernel(int32_t* state, int base) {
  if (threadIdx.x == 0 && blockIdx.x == 0) { state[0] = base; state[1] = 0; }
}

__global__ void cgls_fill_i32_kernel(int32_t* v, int n, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = value;
}

__global__ void cgls_fill_f64_kernel(double* v, int64_t n, double value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = value;
}

__global__ void cgls_advance_kernel(int32_t* state, int chunk) {
  if (threadIdx.x == 0 && blockIdx.x == 0) state[0] += chunk;
}

}  // namespace

hipError_t launch_apply_A(const int32_t* seg_off, const int32_t* perm, int64_t M, const double* c,
                          double* q, hipStream_t s) {
  hipLaunchKernelGGL(apply_A_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0, s,
                     seg_off, perm, M, c, q);
  return hipGetLastError();
}

hipError_t launch_apply_AT(const ColBlock* cblk, int64_t ncblk, const int32_t* rowmap,
                           const double* r, double* out, hipStream_t s) {
  hipLaunchKernelGGL(apply_AT_kernel, dim3((unsigned)ncblk), dim3(kBlock), 0, s, cblk, rowmap, r,
                     out);
  return hipGetLastError();
}

hipError_t launch_cgls_init(const CglsArgs& a, const double* b, bool warm, hipStream_t s) {
  // the row launch also clears the per-problem flags: every problem owns at
  // least one row block, so there are at least nprob >= ceil(nprob/kBlock)
  // workgroups
  hipLaunchKernelGGL(cgls_init_rows_kernel, dim3((unsigned)a.nrblk), dim3(kBlock), 0, s, a, b,
                     warm ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cgls_init_cols_kernel, dim3((unsigned)a.ncblk), dim3(kBlock), 0, s, a,
                     warm ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_cgls_rows(const CglsArgs& a, int rel, hipStream_t s) {
  if (a.fp32) {
    // a batch's LDS units, then the row blocks of the remaining problems
    if (a.nunits > 0) {
      hipLaunchKernelGGL(cgls_rows_unit_kernel, dim3((unsigned)a.nunits), dim3(kLdsBlock),
                         (size_t)a.lds_bytes, s, a, rel);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (a.nrblk32 > 0) {
      CglsArgs b = a;
      b.rblk = a.rblk32;
      hipLaunchKernelGGL((cgls_rows_kernel<float2, true>), dim3((unsigned)a.nrblk32), dim3(kBlock),
                         0, s, b, rel);
    }
  } else {
    hipLaunchKernelGGL((cgls_rows_kernel<double2, false>), dim3((unsigned)a.nrblk), dim3(kBlock), 0, s, a, rel);
  }
  return hipGetLastError();
}

// workgroups of the single-kernel iteration for this plan (0: not possible)
int32_t fused_grid(int device, int64_t nrblk, int64_t ncblk, int fp32) {
  int ncu = 0, nb = 0, coop = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess)
    return 0;
  const hipError_t e = fp32
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&cgls_fused_kernel<float2, true>), kBlock, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&cgls_fused_kernel<double2, false>), kBlock, 0);
  if (e != hipSuccess || !coop) { (void)hipGetLastError(); return 0; }
  const int64_t need = std::max(nrblk, ncblk);
  if (need > (int64_t)nb * ncu) return 0;
  return (int32_t)need;
}

hipError_t launch_cgls_fused(const CglsArgs& a, int iters, int32_t grid, int* bar, int* abort,
                             hipStream_t s) {
  CglsArgs aa = a;
  void* args[] = {&aa, &iters, &bar, &abort};
  if (a.fp32)
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&cgls_fused_kernel<float2, true>),
                                      dim3((unsigned)grid), dim3(kBlock), args, 0, s);
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&cgls_fused_kernel<double2, false>),
                                    dim3((unsigned)grid), dim3(kBlock), args, 0, s);
}

int32_t lds_unit_capacity(int device) {
  int maxsh = 0;
  if (hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
    return 0;
  // static LDS of the unit kernel: sh, s_done
  const int avail = maxsh - (int)(sizeof(double) * kShSlots) - 64;
  int cap = avail / (int)sizeof(float);
  cap = std::min(cap, 40960);
  if (cap < 1024) return 0;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&cgls_rows_unit_kernel),
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          cap * (int)sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return cap;
}

hipError_t launch_cgls_cols(const CglsArgs& a, int rel, hipStream_t s) {
  if (a.fp32)
    hipLaunchKernelGGL((cgls_cols_kernel<float2, true>), dim3((unsigned)a.ncblk), dim3(kBlock), 0, s, a, rel);
  else if (a.max_K > kDeepColsK)
    // many grids per column: deeper batches of independent loads (the sums
    // keep grid order, so the bits are those of the default kernel)
    hipLaunchKernelGGL((cgls_cols_kernel<double2, false, 16, 4>), dim3((unsigned)a.ncblk), dim3(kBlock), 0, s, a, rel);
  else
    hipLaunchKernelGGL((cgls_cols_kernel<double2, false>), dim3((unsigned)a.ncblk), dim3(kBlock), 0, s, a, rel);
  return hipGetLastError();
}

hipError_t launch_refine(const CglsArgs& a, const double* b, const double* gprev, int start,
                         int round, double tol2_outer, hipStream_t s) {
  hipLaunchKernelGGL(refine_rows_kernel, dim3((unsigned)a.nrblk), dim3(kBlock), 0, s, a, b,
                     start);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(refine_cols_kernel, dim3((unsigned)a.ncblk), dim3(kBlock), 0, s, a, gprev);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(refine_check_kernel, dim3((unsigned)a.nprob), dim3(kBlock), 0, s, a, round,
                     tol2_outer);
  return hipGetLastError();
}

hipError_t launch_cgls_iter(const CglsArgs& a, int rel, hipStream_t s) {
  hipError_t e = launch_cgls_rows(a, rel, s);
  if (e != hipSuccess) return e;
  return launch_cgls_cols(a, rel, s);
}

hipError_t launch_cgls_gamma(const CglsArgs& a, int k, hipStream_t s) {
  hipLaunchKernelGGL(cgls_gamma_kernel, dim3((unsigned)a.nprob), dim3(kBlock), 0, s, a, k);
  return hipGetLastError();
}

hipError_t launch_cgls_set_base(int32_t* state, int base, hipStream_t s) {
  hipLaunchKernelGGL(cgls_set_base_kernel, dim3(1), dim3(64), 0, s, state, base);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* v, int n, int value, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cgls_fill_i32_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s,
                     v, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* v, int64_t n, double value, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cgls_fill_f64_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s,
                     v, n, value);
  return hipGetLastError();
}

hipError_t launch_cgls_advance(int32_t* state, int chunk, hipStream_t s) {
  hipLaunchKernelGGL(cgls_advance_kernel, dim3(1), dim3(64), 0, s, state, chunk);
  return hipGetLastError();
}

}  // namespace fct
