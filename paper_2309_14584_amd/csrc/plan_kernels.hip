// Plan construction kernels: alias bins, a stable merge sort of
// (grid, bin) keys, segment extraction and the per-degree DCT-I tables.
//
// The alias bin of support row j on grid l is the row-major flat index of
// (fold(n_j1, N_1), ..., fold(n_jD, N_D)); the multi-dimensional entry of
// A^(l) is the product of 1-D entries (Sec. 3.1, eq.
// aliasing_matrix_nd_diff), and each 1-D block has a single 1 in column n at
// row fold(n, N) (Lobatto analogue of Lemma 3.1).  All of it is integer
// work, so the maps are reproducible bit for bit.
#include "fct_internal.h"

namespace fct {
namespace {

__device__ __forceinline__ int64_t fold_dev(int64_t a, int32_t N) {
  if (N == 0) return 0;
  const int64_t p = 2 * (int64_t)N;
  const int64_t r = a % p;
  return r < p - r ? r : p - r;
}

// Gauss grid of N + 1 nodes (Lemma 3.1): T_a equals s T_m on the nodes with
// r = a mod 2(N+1), m = min(r, 2(N+1) - r), s = (-1)^(a div 2(N+1)) for
// r <= N + 1 and its negation beyond; m = N + 1 is the vanishing T_{N+1}
// (weight 0; the entry is kept in bin m = N so that every column still has
// one entry per grid, and adds nothing).
__device__ __forceinline__ int64_t fold_gauss_dev(int64_t a, int32_t N, int& w) {
  const int64_t g = (int64_t)N + 1;
  const int64_t p = 2 * g;
  const int64_t r = a % p;
  const int odd = (int)((a / p) & 1);
  if (r == g) { w = 0; return N; }
  if (r < g) { w *= odd ? -1 : 1; return r; }
  w *= odd ? 1 : -1;
  return p - r;
}

__global__ __launch_bounds__(kBlock) void alias_kernel(
    const int32_t* __restrict__ S, const int32_t* __restrict__ grids,
    const int64_t* __restrict__ strides, int D, int64_t n, int K,
    int64_t* __restrict__ alias, uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
    int8_t* __restrict__ wsign) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)K * n) return;
  const int l = (int)(t / n);
  const int64_t j = t - (int64_t)l * n;
  int64_t bin = 0;
  if (wsign) {
    int w = 1;
    for (int i = 0; i < D; ++i)
      bin += fold_gauss_dev(S[j * D + i], grids[l * D + i], w) * strides[(int64_t)l * D + i];
    wsign[t] = (int8_t)w;
  } else {
    for (int i = 0; i < D; ++i)
      bin += fold_dev(S[j * D + i], grids[l * D + i]) * strides[(int64_t)l * D + i];
  }
  alias[t] = bin;
  keys[t] = ((uint64_t)l << kKeyBinBits) | (uint64_t)bin;
  vals[t] = (int32_t)j;
}

// Number of entries of a[lo, hi) strictly below key (left run rule) or
// not above it (right run rule); equal keys of the left run stay first,
// which makes every merge stable.
template <bool kUpper, typename Ptr>
__device__ __forceinline__ int64_t rank_in(Ptr a, int64_t lo, int64_t hi, uint64_t key) {
  int64_t l = lo, h = hi;
  while (l < h) {
    const int64_t m = (l + h) >> 1;
    const uint64_t v = a[m];
    const bool go_right = kUpper ? (v <= key) : (v < key);
    if (go_right) l = m + 1; else h = m;
  }
  return l - lo;
}

// Sort each tile of kSortTile entries in LDS by repeated pairwise merges;
// padding beyond L holds the largest key and is never written back.
__global__ __launch_bounds__(kBlock) void tile_sort_kernel(uint64_t* __restrict__ keys,
                                                           int32_t* __restrict__ vals,
                                                           int64_t L) {
  __shared__ uint64_t k0[kSortTile], k1[kSortTile];
  __shared__ int32_t v0[kSortTile], v1[kSortTile];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int i = threadIdx.x; i < kSortTile; i += blockDim.x) {
    const int64_t g = base + i;
    k0[i] = g < L ? keys[g] : ~0ull;
    v0[i] = g < L ? vals[g] : -1;
  }
  __syncthreads();
  uint64_t* ka = k0; uint64_t* kb = k1;
  int32_t* va = v0; int32_t* vb = v1;
  for (int w = 1; w < kSortTile; w <<= 1) {
    for (int i = threadIdx.x; i < kSortTile; i += blockDim.x) {
      const int run = i / w;
      const int start = run * w;
      const int pos = i - start;
      int out;
      if ((run & 1) == 0) {
        out = start + pos + (int)rank_in<false>(ka, start + w, start + 2 * w, ka[i]);
      } else {
        out = start - w + pos + (int)rank_in<true>(ka, start - w, start, ka[i]);
      }
      kb[out] = ka[i];
      vb[out] = va[i];
    }
    __syncthreads();
    uint64_t* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  for (int i = threadIdx.x; i < kSortTile; i += blockDim.x) {
    const int64_t g = base + i;
    if (g < L) { keys[g] = ka[i]; vals[g] = va[i]; }
  }
}

// One global merge level: runs of width w are merged pairwise into out.
__global__ __launch_bounds__(kBlock) void merge_level_kernel(
    const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t L, int64_t w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L) return;
  const int64_t run = i / w;
  const int64_t start = run * w;
  const int64_t pos = i - start;
  const uint64_t key = kin[i];
  int64_t out;
  if ((run & 1) == 0) {
    const int64_t lo = start + w;
    const int64_t hi = lo + w < L ? lo + w : L;
    out = start + pos + (lo < L ? rank_in<false>(kin, lo, hi, key) : 0);
  } else {
    out = start - w + pos + rank_in<true>(kin, start - w, start, key);
  }
  kout[out] = key;
  vout[out] = vin[i];
}

constexpr int kSegItems = 4;                      // entries per thread
constexpr int kSegTile = kBlock * kSegItems;      // entries per workgroup

__device__ __forceinline__ int is_head(const uint64_t* keys, int64_t t) {
  return (t == 0 || keys[t] != keys[t - 1]) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void head_count_kernel(const uint64_t* __restrict__ keys,
                                                            int64_t L,
                                                            int32_t* __restrict__ counts) {
  __shared__ int32_t red[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kSegTile + (int64_t)threadIdx.x * kSegItems;
  int c = 0;
  for (int k = 0; k < kSegItems; ++k) {
    const int64_t t = base + k;
    if (t < L) c += is_head(keys, t);
  }
  red[threadIdx.x] = c;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

// Exclusive scan of the per-workgroup head counts, in one workgroup.
__global__ __launch_bounds__(kBlock) void scan_counts_kernel(int32_t* __restrict__ counts,
                                                             int64_t nblocks) {
  __shared__ int32_t buf[kBlock];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblocks; base += kBlock) {
    const int64_t i = base + threadIdx.x;
    const int32_t v = i < nblocks ? counts[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int s = 1; s < kBlock; s <<= 1) {
      const int32_t add = (int)threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    const int32_t incl = buf[threadIdx.x];
    if (i < nblocks) counts[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry += incl;
    __syncthreads();
  }
}

// Row index of every sorted entry = (number of heads up to it) - 1; writes
// perm, seg_off, bin_id, rowmap and the grid row offsets.
__global__ __launch_bounds__(kBlock) void segment_write_kernel(
    const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals, int64_t L,
    int64_t n, const int32_t* __restrict__ block_off, int32_t* __restrict__ perm,
    int32_t* __restrict__ seg_off, int64_t* __restrict__ bin_id,
    int32_t* __restrict__ rowmap, int32_t* __restrict__ row_off, int K) {
  __shared__ int32_t buf[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kSegTile + (int64_t)threadIdx.x * kSegItems;
  int heads[kSegItems];
  int mine = 0;
  for (int k = 0; k < kSegItems; ++k) {
    const int64_t t = base + k;
    heads[k] = t < L ? is_head(keys, t) : 0;
    mine += heads[k];
  }
  buf[threadIdx.x] = mine;
  __syncthreads();
  for (int s = 1; s < kBlock; s <<= 1) {
    const int32_t add = (int)threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
    __syncthreads();
    buf[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t count = block_off[blockIdx.x] + buf[threadIdx.x] - mine;
  const uint64_t mask = (1ull << kKeyBinBits) - 1ull;
  for (int k = 0; k < kSegItems; ++k) {
    const int64_t t = base + k;
    if (t >= L) break;
    count += heads[k];
    const int32_t row = count - 1;
    const uint64_t key = keys[t];
    const int32_t j = vals[t];
    const int l = (int)(key >> kKeyBinBits);
    perm[t] = j;
    rowmap[(int64_t)l * n + j] = row;
    if (heads[k]) {
      seg_off[row] = (int32_t)t;
      bin_id[row] = (int64_t)(key & mask);
    }
    if (t % n == 0) row_off[t / n] = row;
    if (t == L - 1) {
      seg_off[row + 1] = (int32_t)L;
      row_off[K] = row + 1;
    }
  }
}

// Per-degree tables for N = 0..maxdeg:
//   nodes[N*64 + k] = cos(pi k / N), evaluated as sin(pi (N - 2k) / (2N)) so
//                     that x_{N-k} = -x_k exactly;
//   cmat[N][m][k]   = (g_m / N) w_k cos(pi (m k mod 2N) / N), the
//                     interpolation-normalised DCT-I (w_0 = w_N = 1, else 2;
//                     g_0 = g_N = 1/2, else 1);
//   emat[N][k][m]   = cos(pi (m k mod 2N) / N) = T_m(x_k), its inverse.
// Degree 0 is the 1x1 identity and the single node x = 1.
// Gauss grids (Sec. 2, eq. chebyshev_grid; the quadrature of Sec. 3.1 with
// rows n >= 1 doubled):
//   nodes[N*64 + k] = cos(pi (k + 1/2) / (N + 1)) = sin(pi (N - 2k) / (2 (N + 1)));
//   cmat[N][m][k]   = (g_m 2 / (N + 1)) cos(pi (m (2k + 1) mod 4(N+1)) / (2 (N + 1))),
//                     g_0 = 1/2, else 1 (the interpolation-normalised DCT-II);
//   emat[N][k][m]   = cos(pi (m (2k + 1) mod 4(N+1)) / (2 (N + 1))) = T_m(x_k).
// Degree 0 is then the single node x = 0 with the 1x1 identity.
__global__ __launch_bounds__(kBlock) void tables_kernel(int maxdeg, double* __restrict__ nodes,
                                                        double* __restrict__ cmat,
                                                        float* __restrict__ cmat32,
                                                        double* __restrict__ emat, int gauss) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = mat_offset(maxdeg + 1);
  if (t < (int64_t)(maxdeg + 1) * 64) {
    const int N = (int)(t / 64), k = (int)(t % 64);
    double x = 0.0;
    if (k <= N) {
      if (gauss) x = sinpi((double)(N - 2 * k) / (2.0 * (N + 1)));
      else x = (N == 0) ? 1.0 : sinpi((double)(N - 2 * k) / (2.0 * N));
    }
    nodes[t] = x;
  }
  if (t >= total) return;
  int N = 0;
  while (mat_offset(N + 1) <= t) ++N;
  const int64_t local = t - mat_offset(N);
  const int e = N + 1;
  const int row = (int)(local / e), col = (int)(local % e);
  if (gauss) {
    // cmat row = m, col = k; emat row = k, col = m
    const int64_t g = (int64_t)N + 1;
    const int64_t red = ((int64_t)row * (2 * col + 1)) % (4 * g);
    const int64_t red_e = ((int64_t)col * (2 * row + 1)) % (4 * g);
    const double sc = (row == 0 ? 1.0 : 2.0) / (double)g;
    cmat[t] = sc * cospi((double)red / (double)(2 * g));
    cmat32[t] = (float)cmat[t];
    emat[t] = cospi((double)red_e / (double)(2 * g));
    return;
  }
  if (N == 0) {
    cmat[t] = 1.0;
    cmat32[t] = 1.0f;
    emat[t] = 1.0;
    return;
  }
  const int red = (row * col) % (2 * N);
  const double cs = cospi((double)red / (double)N);
  const double w = (col == 0 || col == N) ? 1.0 : 2.0;
  const double g = (row == 0 || row == N) ? 0.5 : 1.0;
  cmat[t] = g / (double)N * w * cs;
  cmat32[t] = (float)cmat[t];
  emat[t] = cs;
}

// Rows by first member: the sort key of entry (l, j) is its grid and the
// first (smallest) column of its row in the (grid, bin) order, so a second
// stable sort keeps every row's run together and in ascending columns while
// ordering each grid's rows by their first column.
__global__ __launch_bounds__(kBlock) void member_keys_kernel(
    const int32_t* __restrict__ rowmap, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ seg_off, int64_t n, int64_t L, uint64_t* __restrict__ keys,
    int32_t* __restrict__ vals) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L) return;
  const int64_t l = t / n;
  const int32_t j = (int32_t)(t - l * n);
  const int32_t first = perm[seg_off[rowmap[t]]];
  keys[t] = ((uint64_t)l << kKeyBinBits) | (uint64_t)first;
  vals[t] = j;
}

// For each row of the new order: its index in the (grid, bin) order (the
// old row of its first member) and its bin.
__global__ __launch_bounds__(kBlock) void row_old_kernel(
    const int32_t* __restrict__ perm_new, const int32_t* __restrict__ seg_new,
    const int32_t* __restrict__ rowmap_old, const int64_t* __restrict__ bin_old, int64_t M,
    int64_t n, int32_t* __restrict__ row_old, int64_t* __restrict__ bin_new) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M) return;
  const int64_t t = seg_new[r];
  const int64_t l = t / n;
  const int32_t ro = rowmap_old[l * n + perm_new[t]];
  row_old[r] = ro;
  bin_new[r] = bin_old[ro];
}

__global__ __launch_bounds__(kBlock) void rows_gather_kernel(const double* __restrict__ src,
                                                             const int32_t* __restrict__ idx,
                                                             int64_t M, double* __restrict__ dst) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M) dst[r] = src[idx[r]];
}

__global__ __launch_bounds__(kBlock) void iota_i32_kernel(int32_t* __restrict__ dst, int64_t count,
                                                          int32_t start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = start + (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void index_inverse_kernel(const int32_t* __restrict__ idx,
                                                               int64_t M,
                                                               int32_t* __restrict__ inv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M) inv[idx[r]] = (int32_t)r;
}

__global__ __launch_bounds__(kBlock) void rows_scatter_kernel(const double* __restrict__ src,
                                                              const int32_t* __restrict__ idx,
                                                              int64_t M, double* __restrict__ dst) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < M) dst[idx[r]] = src[r];
}

__global__ __launch_bounds__(kBlock) void ell_kernel(const int32_t* __restrict__ seg_off,
                                                     const int32_t* __restrict__ perm, int64_t M,
                                                     int4* __restrict__ ell) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M) return;
  const int32_t t0 = seg_off[r], t1 = seg_off[r + 1];
  const int32_t len = t1 - t0;
  int4 e;
  e.x = len > 0 ? perm[t0] : -1;
  e.y = len > 1 ? perm[t0 + 1] : -1;
  e.z = len > 2 ? perm[t0 + 2] : -1;
  e.w = len == 4 ? perm[t0 + 3] : (len > 4 ? -(2 + (t0 + 3)) : -1);
  ell[r] = e;
}

__global__ __launch_bounds__(kBlock) void copy_add_kernel(int32_t* __restrict__ dst,
                                                          const int32_t* __restrict__ src,
                                                          int64_t count, int32_t add) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i] + add;
}

__global__ __launch_bounds__(kBlock) void copy_ell_kernel(int4* __restrict__ dst,
                                                          const int4* __restrict__ src,
                                                          int64_t count, int32_t col_add,
                                                          int32_t perm_add) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int4 e = src[i];
  e.x = e.x >= 0 ? e.x + col_add : e.x;
  e.y = e.y >= 0 ? e.y + col_add : e.y;
  e.z = e.z >= 0 ? e.z + col_add : e.z;
  // -1: empty; <= -2: continuation -(2 + t) at perm position t
  e.w = e.w >= 0 ? e.w + col_add : (e.w <= -2 ? e.w - perm_add : e.w);
  dst[i] = e;
}

// 16-bit ELL of one problem's rows for the LDS units: the first eight
// local columns (column - col_off) of each row, 0xFFFF padded; a row with
// more than eight entries keeps its first seven and marks slot 7 with 0xFFFE
// (the rest is perm[seg_off[row] + 7, seg_off[row + 1])).
__global__ __launch_bounds__(kBlock) void ell16_kernel(const int32_t* __restrict__ seg_off,
                                                       const int32_t* __restrict__ perm,
                                                       int32_t row0, int32_t nrows,
                                                       int32_t col_off, uint4* __restrict__ out) {
  const int32_t i = (int32_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int32_t row = row0 + i;
  const int32_t t0 = seg_off[row], t1 = seg_off[row + 1];
  const int32_t len = t1 - t0;
  uint32_t v[8];
  for (int k = 0; k < 8; ++k) v[k] = 0xFFFFu;
  const int32_t direct = len > 8 ? 7 : len;
  for (int k = 0; k < direct; ++k) v[k] = (uint32_t)(perm[t0 + k] - col_off);
  if (len > 8) v[7] = 0xFFFEu;
  out[row] = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16),
                        v[6] | (v[7] << 16));
}

}  // namespace

hipError_t launch_ell16(const int32_t* seg_off, const int32_t* perm, int32_t row0, int32_t nrows,
                        int32_t col_off, uint4* out, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(ell16_kernel, dim3((unsigned)ceil_div(nrows, kBlock)), dim3(kBlock), 0, s,
                     seg_off, perm, row0, nrows, col_off, out);
  return hipGetLastError();
}

hipError_t launch_copy_add_i32(int32_t* dst, const int32_t* src, int64_t count, int32_t add,
                               hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_add_kernel, dim3((unsigned)ceil_div(count, kBlock)), dim3(kBlock), 0, s,
                     dst, src, count, add);
  return hipGetLastError();
}

hipError_t launch_copy_ell(int4* dst, const int4* src, int64_t count, int32_t col_add,
                           int32_t perm_add, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_ell_kernel, dim3((unsigned)ceil_div(count, kBlock)), dim3(kBlock), 0, s,
                     dst, src, count, col_add, perm_add);
  return hipGetLastError();
}

hipError_t launch_ell(const int32_t* seg_off, const int32_t* perm, int64_t M, int4* ell,
                      hipStream_t s) {
  hipLaunchKernelGGL(ell_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0, s, seg_off,
                     perm, M, ell);
  return hipGetLastError();
}

hipError_t launch_alias(const int32_t* S, const int32_t* grids, const int64_t* strides,
                        int D, int64_t n, int K, int64_t* alias, uint64_t* keys,
                        int32_t* vals, int8_t* wsign, hipStream_t s) {
  const int64_t L = (int64_t)K * n;
  hipLaunchKernelGGL(alias_kernel, dim3((unsigned)ceil_div(L, kBlock)), dim3(kBlock), 0, s,
                     S, grids, strides, D, n, K, alias, keys, vals, wsign);
  return hipGetLastError();
}

hipError_t launch_sort(uint64_t* keys, int32_t* vals, uint64_t* keys_tmp, int32_t* vals_tmp,
                       int64_t L, bool* result_in_tmp, hipStream_t s) {
  const int64_t tiles = ceil_div(L, kSortTile);
  hipLaunchKernelGGL(tile_sort_kernel, dim3((unsigned)tiles), dim3(kBlock), 0, s, keys, vals, L);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint64_t* ka = keys; int32_t* va = vals;
  uint64_t* kb = keys_tmp; int32_t* vb = vals_tmp;
  bool in_tmp = false;
  for (int64_t w = kSortTile; w < L; w <<= 1) {
    hipLaunchKernelGGL(merge_level_kernel, dim3((unsigned)ceil_div(L, kBlock)), dim3(kBlock), 0,
                       s, ka, va, kb, vb, L, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
    in_tmp = !in_tmp;
  }
  *result_in_tmp = in_tmp;
  return hipSuccess;
}

hipError_t launch_segments(const uint64_t* keys, const int32_t* vals, int64_t L, int64_t n,
                           int32_t* block_counts, int64_t nblocks, int32_t* perm,
                           int32_t* seg_off, int64_t* bin_id, int32_t* rowmap,
                           int32_t* row_off, int K, hipStream_t s) {
  hipLaunchKernelGGL(head_count_kernel, dim3((unsigned)nblocks), dim3(kBlock), 0, s, keys, L,
                     block_counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(kBlock), 0, s, block_counts, nblocks);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(segment_write_kernel, dim3((unsigned)nblocks), dim3(kBlock), 0, s, keys,
                     vals, L, n, block_counts, perm, seg_off, bin_id, rowmap, row_off, K);
  return hipGetLastError();
}

hipError_t launch_member_keys(const int32_t* rowmap, const int32_t* perm, const int32_t* seg_off,
                             int64_t n, int K, uint64_t* keys, int32_t* vals, hipStream_t s) {
  const int64_t L = (int64_t)K * n;
  hipLaunchKernelGGL(member_keys_kernel, dim3((unsigned)ceil_div(L, kBlock)), dim3(kBlock), 0, s,
                     rowmap, perm, seg_off, n, L, keys, vals);
  return hipGetLastError();
}

hipError_t launch_row_old(const int32_t* perm_new, const int32_t* seg_new,
                          const int32_t* rowmap_old, const int64_t* bin_old, int64_t M, int64_t n,
                          int32_t* row_old, int64_t* bin_new, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_old_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0, s,
                     perm_new, seg_new, rowmap_old, bin_old, M, n, row_old, bin_new);
  return hipGetLastError();
}

hipError_t launch_rows_gather(const double* src, const int32_t* idx, int64_t M, double* dst,
                              hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(rows_gather_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0, s,
                     src, idx, M, dst);
  return hipGetLastError();
}

hipError_t launch_iota_i32(int32_t* dst, int64_t count, int32_t start, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(iota_i32_kernel, dim3((unsigned)ceil_div(count, kBlock)), dim3(kBlock), 0, s,
                     dst, count, start);
  return hipGetLastError();
}

hipError_t launch_index_inverse(const int32_t* idx, int64_t M, int32_t* inv, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(index_inverse_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0,
                     s, idx, M, inv);
  return hipGetLastError();
}

hipError_t launch_rows_scatter(const double* src, const int32_t* idx, int64_t M, double* dst,
                               hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(rows_scatter_kernel, dim3((unsigned)ceil_div(M, kBlock)), dim3(kBlock), 0,
                     s, src, idx, M, dst);
  return hipGetLastError();
}

hipError_t launch_tables(int maxdeg, double* nodes, double* cmat, float* cmat32, double* emat,
                         int gauss, hipStream_t s) {
  int64_t total = mat_offset(maxdeg + 1);
  const int64_t nn = (int64_t)(maxdeg + 1) * 64;
  if (nn > total) total = nn;
  hipLaunchKernelGGL(tables_kernel, dim3((unsigned)ceil_div(total, kBlock)), dim3(kBlock), 0, s,
                     maxdeg, nodes, cmat, cmat32, emat, gauss);
  return hipGetLastError();
}

int64_t segment_blocks(int64_t L) { return ceil_div(L, kSegTile); }

}  // namespace fct
