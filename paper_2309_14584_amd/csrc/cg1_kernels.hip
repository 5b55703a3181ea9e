// Conjugate gradients on the normal equations A^T A c = A^T b with one
// global reduction per iteration (Chronopoulos and Gear's arrangement of the
// recurrences), for one problem in FP64: the same iterates as CGLS in exact
// arithmetic (Alg. 3's least-squares solve, Sec. 3.4), one kernel per
// iteration instead of two.
//
// Per column j the state is (r, w, s, p) with r = A^T (b - A c) the normal
// residual, w = A^T A r, s = A^T A p, p the direction.  Iteration k, from
// gamma_k = r.r and delta_k = w.r (reduced from the previous launch's
// per-workgroup partials in a fixed order):
//   beta = gamma_k / gamma_{k-1},  alpha = gamma_k / (delta_k - beta gamma_k / alpha_{k-1})
//   p <- r + beta p,  s <- w + beta s,  c <- c + alpha p,  r <- r - alpha s,
//   w <- A^T A r,
// and the partials of the next gamma and delta.  A is 0/1 with every column
// in exactly one row of each of the K grids, so (A^T A r)_j = K r_j plus the
// sum of r over the other members of j's rows (the column's neighbour list,
// a neighbour counted once per shared row).  Each neighbour's new r =
// r - alpha (w + beta s) is linear in its stored values, so the kernel
// gathers the neighbours' (r, w, s) and sums them before the scalars are
// known: one level of dependent loads past the list.  On a Gauss plan A
// has entries in {-1, 0, 1}: a neighbour carries the sign of the product of
// the two entries, and the diagonal is the number of grids where the
// column's entry is nonzero (kept per column).  The state alternates
// between two buffers by iteration parity (workgroups gather the old state
// while others write the new one); so do the partials.
#include "fct_internal.h"

namespace fct {
namespace {

// Sums of two values over the wave (every lane gets both; a fixed butterfly,
// so every workgroup adds in the same order).
__device__ __forceinline__ double2 wave_sum2(double u, double v) {
  for (int off = 32; off > 0; off >>= 1) {
    u += __shfl_xor(u, off, 64);
    v += __shfl_xor(v, off, 64);
  }
  return make_double2(u, v);
}

// This lane's share of np per-workgroup partials (lane t adds t, t + 64,
// ...), eight loads in flight at a time, added in a fixed order.
__device__ __forceinline__ double share(const double* __restrict__ part, int32_t np) {
  constexpr int kU = 8;
  double v[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) v[u] = 0.0;
  for (int32_t b = threadIdx.x; b < np; b += kU * kCg1Block) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int32_t i = b + u * kCg1Block;
      v[u] += i < np ? part[i] : 0.0;
    }
  }
  double r = 0.0;
#pragma unroll
  for (int u = 0; u < kU; ++u) r += v[u];
  return r;
}

// Calls f(m, sign) for every entry of column j's neighbour list: the eight
// slots, then the overflow four at a time (indices loaded before the
// gathers), so that a long list costs few dependent loads.  An entry e >= 0
// is neighbour e with sign +1, e <= -2 neighbour -e - 2 with sign -1 (Gauss
// plans), -1 an empty slot.
template <typename F>
__device__ __forceinline__ void for_neighbours(const CglsArgs& a, int32_t j, F&& f) {
  const int4 e0 = a.nb8[j];
  const int4 e1 = a.nb8[(int64_t)a.cg1_n + j];
  const int32_t t0 = a.nb_off[j], t1 = a.nb_off[j + 1];
  const int32_t m[8] = {e0.x, e0.y, e0.z, e0.w, e1.x, e1.y, e1.z, e1.w};
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (m[u] != -1) f(m[u] >= 0 ? m[u] : -m[u] - 2, m[u] >= 0 ? 1.0 : -1.0);
  for (int32_t t = t0; t < t1; t += 4) {
    int32_t i[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) i[u] = t + u < t1 ? a.nb_ovf[t + u] : -1;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i[u] != -1) f(i[u] >= 0 ? i[u] : -i[u] - 2, i[u] >= 0 ? 1.0 : -1.0);
  }
}

// Weight of entry t of the [K][n] maps (1 without a weight table).
__device__ __forceinline__ int wt(const int8_t* __restrict__ w, int64_t t) {
  return w ? (int)w[t] : 1;
}

// Neighbour counts: the other members of the column's K rows with nonzero
// weight (rows where the column itself has weight 0 add none), and the
// diagonal of A^T A: the number of grids where the column's weight is
// nonzero.  perm entry t belongs to grid t / n.
__global__ __launch_bounds__(kBlock) void cg1_count_kernel(const ColBlock* __restrict__ cblk,
                                                           const int32_t* __restrict__ rowmap,
                                                           const int32_t* __restrict__ seg_off,
                                                           const int32_t* __restrict__ perm,
                                                           const int8_t* __restrict__ w,
                                                           int32_t* __restrict__ cnt,
                                                           int32_t* __restrict__ diag) {
  const ColBlock bd = cblk[blockIdx.x];
  const int32_t j = bd.col0 + threadIdx.x;
  if (j >= bd.col_end) return;
  const int32_t jl = j - bd.col_off;
  int32_t c = 0, dg = 0;
  for (int l = 0; l < bd.K; ++l) {
    const int64_t tj = bd.rmap_off + (int64_t)l * bd.n + jl;
    if (wt(w, tj) == 0) continue;
    ++dg;
    const int32_t row = rowmap[tj];
    if (!w) {
      c += seg_off[row + 1] - seg_off[row] - 1;
      continue;
    }
    for (int32_t t = seg_off[row]; t < seg_off[row + 1]; ++t) {
      const int32_t m = perm[t];
      if (m != j && w[(int64_t)l * bd.n + m] != 0) ++c;
    }
  }
  cnt[j] = c;
  diag[j] = dg;
}

// Neighbour lists in grid order, then run order within a row: slot u of
// column j at int32 element ((u / 4) n + j) 4 + u % 4 of nb8, -1 when unused.
__global__ __launch_bounds__(kBlock) void cg1_fill_kernel(const ColBlock* __restrict__ cblk,
                                                          const int32_t* __restrict__ rowmap,
                                                          const int32_t* __restrict__ seg_off,
                                                          const int32_t* __restrict__ perm,
                                                          const int8_t* __restrict__ w,
                                                          const int32_t* __restrict__ off,
                                                          int32_t n, int32_t* __restrict__ nb8,
                                                          int32_t* __restrict__ ovf) {
  const ColBlock bd = cblk[blockIdx.x];
  const int32_t j = bd.col0 + threadIdx.x;
  if (j >= bd.col_end) return;
  const int32_t jl = j - bd.col_off;
  auto slot = [&](int u) -> int32_t& {
    return nb8[((int64_t)(u >> 2) * n + j) * 4 + (u & 3)];
  };
  for (int u = 0; u < kNbSlots; ++u) slot(u) = -1;
  int32_t idx = 0;
  const int32_t o = off[j], o_end = off[j + 1];
  for (int l = 0; l < bd.K; ++l) {
    const int64_t tj = bd.rmap_off + (int64_t)l * bd.n + jl;
    const int wj = wt(w, tj);
    if (wj == 0) continue;
    const int32_t row = rowmap[tj];
    const int32_t t1 = seg_off[row + 1];
    for (int32_t t = seg_off[row]; t < t1; ++t) {
      const int32_t m = perm[t];
      if (m == j) continue;
      const int wm = wt(w, (int64_t)l * bd.n + m);
      if (wm == 0) continue;
      const int32_t e = wj * wm > 0 ? m : -m - 2;
      if (idx < kNbSlots) slot(idx) = e;
      else if (o + idx - kNbSlots < o_end) ovf[o + idx - kNbSlots] = e;
      ++idx;
    }
  }
}

// q = A c with entry weights (Gauss plans): row r's run in perm, entry t of
// grid t / n, summed in run order.
__global__ __launch_bounds__(kBlock) void apply_A_signed_kernel(
    const int32_t* __restrict__ seg_off, const int32_t* __restrict__ perm,
    const int8_t* __restrict__ w, int64_t M, int64_t n, const double* __restrict__ c,
    double* __restrict__ q) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M) return;
  double acc = 0.0;
  for (int32_t t = seg_off[r]; t < seg_off[r + 1]; ++t) {
    const int32_t j = perm[t];
    acc = fma((double)w[(t / n) * n + j], c[j], acc);
  }
  q[r] = acc;
}

// s = A^T r with entry weights: sum over the grids in order.
__global__ __launch_bounds__(kBlock) void apply_AT_signed_kernel(
    const int32_t* __restrict__ rowmap, const int8_t* __restrict__ w, int32_t K, int64_t n,
    const double* __restrict__ r, double* __restrict__ s) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double acc = 0.0;
  for (int l = 0; l < K; ++l) {
    const int64_t t = (int64_t)l * n + j;
    acc = fma((double)w[t], r[rowmap[t]], acc);
  }
  s[j] = acc;
}

// Gauss plans, start of a solve: r_0 = b - A c_0 into r64 (c_0 = 0 unless
// warm) and the iteration state reset.
__global__ __launch_bounds__(kBlock) void gauss_init_rows_kernel(CglsArgs a,
                                                                 const int8_t* __restrict__ w,
                                                                 const double* __restrict__ b,
                                                                 int64_t M, int warm) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) { a.state[0] = 0; a.state[1] = 0; a.done[0] = 0; a.flags[0] = 0; }
  if (r >= M) return;
  double acc = 0.0;
  if (warm) {
    const int64_t n = a.cg1_n;
    for (int32_t t = a.seg_off[r]; t < a.seg_off[r + 1]; ++t) {
      const int32_t j = a.perm[t];
      acc = fma((double)w[(t / n) * n + j], a.c[j], acc);
    }
  }
  a.r64[r] = b[r] - acc;
}

// s_0 = A^T r_0 into ps.y (ps.x = 0), c = 0 unless warm.
__global__ __launch_bounds__(kBlock) void gauss_init_cols_kernel(CglsArgs a,
                                                                 const int8_t* __restrict__ w,
                                                                 int warm) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = a.cg1_n;
  if (j >= n) return;
  double acc = 0.0;
  for (int l = 0; l < a.cg1_K; ++l) {
    const int64_t t = (int64_t)l * n + j;
    acc = fma((double)w[t], a.r64[a.rowmap[t]], acc);
  }
  static_cast<double2*>(a.ps)[j] = make_double2(0.0, acc);
  if (!warm) a.c[j] = 0.0;
}

// w = A^T A s_0 and gamma_0, delta_0 from the normal residual s_0 that the
// CGLS initialisation left in ps.y: state (r, w, 0, 0) into buffer 0.  One
// wave of kCg1Block columns per workgroup.
__global__ __launch_bounds__(kCg1Block) void cg1_init_kernel(CglsArgs a) {
  const int32_t j = blockIdx.x * kCg1Block + threadIdx.x;
  const double2* ps = static_cast<const double2*>(a.ps);
  double r = 0.0, w = 0.0;
  if (j < a.cg1_n) {
    r = ps[j].y;
    for_neighbours(a, j, [&](int32_t m, double sg) { w = fma(sg, ps[m].y, w); });
    w = fma((double)a.nb_diag[j], r, w);
    a.cg[0][j] = make_double4(r, w, 0.0, 0.0);
  }
  const double2 gd = wave_sum2(r * r, w * r);
  if (threadIdx.x == 0) {
    a.cg_part[blockIdx.x] = gd.x;               // parity 0: gamma, then delta
    a.cg_part[a.cg1_nblk + blockIdx.x] = gd.y;
  }
}

// Launched with an even iteration base (the host queues chunks of even
// length, except a last one that ends at the iteration limit), so the
// buffer parity is that of rel, a launch argument: no operand address waits
// for a load of the base.
__global__ __launch_bounds__(kCg1Block) void cg1_kernel(CglsArgs a, int rel) {
  const int done = a.done[0];
  const int q = rel & 1;
  const double4* cur = a.cg[q];
  double4* nxt = a.cg[q ^ 1];
  const int32_t nb = a.cg1_nblk;
  const double* pin = a.cg_part + (int64_t)q * 2 * nb;
  double* pout = a.cg_part + (int64_t)(q ^ 1) * 2 * nb;

  // operands that do not depend on the scalars of iteration k (issued
  // before the stop flag is tested)
  const int32_t j = blockIdx.x * kCg1Block + threadIdx.x;
  const bool active = j < a.cg1_n;
  const int32_t jc = active ? j : 0;
  const double4 own = cur[jc];
  const double c_old = a.c[jc];
  const double gp = share(pin, nb);
  const double dp = share(pin + nb, nb);
  double R = 0.0, W = 0.0, S = 0.0;
  double dg = 0.0;
  if (active) {
    dg = (double)a.nb_diag[j];
    for_neighbours(a, j, [&](int32_t m, double sg) {
      const double4 v = cur[m];
      R = fma(sg, v.x, R); W = fma(sg, v.y, W); S = fma(sg, v.z, S);
    });
  }
  if (done != 0) return;
  const int k = a.state[0] + rel;

  const double2 gd = wave_sum2(gp, dp);
  const double gamma = gd.x, delta = gd.y;
  const int k0 = a.state[1];
  double beta = 0.0, alpha, g0 = gamma;
  if (k > k0) {
    const double gprev = a.ring[(k - 1) & 3];               // gamma_{k-1}
    const double aprev = a.ring[4 + ((k - 1) & 3)];         // alpha_{k-1}
    beta = gamma / gprev;
    alpha = gamma / (delta - beta * gamma / aprev);
    g0 = a.gamma0[0];
  } else {
    alpha = gamma / delta;
  }
  const bool stop = k == k0 ? !(gamma > 0.0) : !(gamma > a.tol2 * g0);
  const bool broke = !stop && !(alpha > 0.0 && alpha < 1e300);   // A^T A p = 0 direction
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ring[(k & 3)] = gamma;
    a.ring[4 + (k & 3)] = alpha;
    if (k == k0) a.gamma0[0] = gamma;
    if (stop) a.done[0] = k + 1;
    if (broke) { a.flags[0] = 1; a.done[0] = k + 1; }
  }
  if (stop || broke) return;

  double rn = 0.0, wn = 0.0;
  if (active) {
    const double pv = fma(beta, own.w, own.x);       // p = r + beta p
    const double sv = fma(beta, own.z, own.y);       // s = w + beta s
    a.c[j] = fma(alpha, pv, c_old);
    rn = fma(-alpha, sv, own.x);                     // r - alpha s
    // (A^T A)_jj rn plus the neighbours' new r
    wn = fma(dg, rn, R - alpha * fma(beta, S, W));
    nxt[j] = make_double4(rn, wn, sv, pv);
  }
  const double2 o = wave_sum2(rn * rn, wn * rn);
  if (threadIdx.x == 0) {
    pout[blockIdx.x] = o.x;
    pout[nb + blockIdx.x] = o.y;
  }
}

// gamma of iteration k (a run stopped by its iteration limit) into the ring.
__global__ __launch_bounds__(kCg1Block) void cg1_gamma_kernel(CglsArgs a, int k) {
  const double* pin = a.cg_part + (int64_t)(k & 1) * 2 * a.cg1_nblk;
  const double2 g = wave_sum2(share(pin, a.cg1_nblk), 0.0);
  if (threadIdx.x == 0 && a.done[0] == 0) a.ring[k & 3] = g.x;
}

}  // namespace

hipError_t launch_cg1_count(const ColBlock* cblk, int64_t ncblk, const int32_t* rowmap,
                            const int32_t* seg_off, const int32_t* perm, const int8_t* w,
                            int32_t* cnt, int32_t* diag, hipStream_t s) {
  hipLaunchKernelGGL(cg1_count_kernel, dim3((unsigned)ncblk), dim3(kBlock), 0, s, cblk, rowmap,
                     seg_off, perm, w, cnt, diag);
  return hipGetLastError();
}

hipError_t launch_cg1_fill(const ColBlock* cblk, int64_t ncblk, const int32_t* rowmap,
                           const int32_t* seg_off, const int32_t* perm, const int8_t* w,
                           const int32_t* off, int32_t n, int4* nb8, int32_t* ovf,
                           hipStream_t s) {
  hipLaunchKernelGGL(cg1_fill_kernel, dim3((unsigned)ncblk), dim3(kBlock), 0, s, cblk, rowmap,
                     seg_off, perm, w, off, n, reinterpret_cast<int32_t*>(nb8), ovf);
  return hipGetLastError();
}

hipError_t launch_apply_A_signed(const int32_t* seg_off, const int32_t* perm, const int8_t* w,
                                 int64_t M, int64_t n, const double* c, double* q,
                                 hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(apply_A_signed_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0,
                     s, seg_off, perm, w, M, n, c, q);
  return hipGetLastError();
}

hipError_t launch_apply_AT_signed(const int32_t* rowmap, const int8_t* w, int32_t K, int64_t n,
                                  const double* r, double* out, hipStream_t s) {
  hipLaunchKernelGGL(apply_AT_signed_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock),
                     0, s, rowmap, w, K, n, r, out);
  return hipGetLastError();
}

hipError_t launch_gauss_init(const CglsArgs& a, const int8_t* w, const double* b, int64_t M,
                             bool warm, hipStream_t s) {
  hipLaunchKernelGGL(gauss_init_rows_kernel, dim3((unsigned)ceil_div(M > 0 ? M : 1, kBlock)),
                     dim3(kBlock), 0, s, a, w, b, M, warm ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gauss_init_cols_kernel, dim3((unsigned)ceil_div(a.cg1_n, kBlock)),
                     dim3(kBlock), 0, s, a, w, warm ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_cg1_init(const CglsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(cg1_init_kernel, dim3((unsigned)a.cg1_nblk), dim3(kCg1Block), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cg1_iter(const CglsArgs& a, int rel, hipStream_t s) {
  hipLaunchKernelGGL(cg1_kernel, dim3((unsigned)a.cg1_nblk), dim3(kCg1Block), 0, s, a, rel);
  return hipGetLastError();
}

hipError_t launch_cg1_gamma(const CglsArgs& a, int k, hipStream_t s) {
  hipLaunchKernelGGL(cg1_gamma_kernel, dim3(1), dim3(kCg1Block), 0, s, a, k);
  return hipGetLastError();
}

}  // namespace fct
