// Host side of libfct: the C ABI, argument checks, plan construction,
// DCT pass planning and the CGLS driver.  Every arithmetic step of the
// transform runs in the kernels of the other source files.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <vector>

#include "fct_internal.h"

namespace fct {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

fct_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return e == hipErrorOutOfMemory ? FCT_ENOMEM : FCT_EDEVICE;
}

namespace {

template <typename T>
hipError_t dalloc(T** p, int64_t count, int64_t* bytes) {
  const size_t sz = sizeof(T) * (size_t)(count > 0 ? count : 1);
  hipError_t e = hipMalloc((void**)p, sz);
  if (e == hipSuccess && bytes) *bytes += (int64_t)sz;
  return e;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Gauss grid of N + 1 nodes: the aliased index and the sign (0: T_{N+1}
// vanishes), as in the plan's alias kernel.
int64_t fold_gauss_host(int64_t a, int32_t N, int* w) {
  const int64_t g = (int64_t)N + 1, p = 2 * g, r = a % p;
  const bool odd = ((a / p) & 1) != 0;
  if (r == g) { *w = 0; return N; }
  if (r < g) { *w = odd ? -1 : 1; return r; }
  *w = odd ? 1 : -1;
  return p - r;
}

int64_t fold_host(int64_t a, int32_t N) {
  if (N == 0) return 0;
  const int64_t p = 2 * (int64_t)N;
  const int64_t r = a % p;
  return r < p - r ? r : p - r;
}

// One axis group of one grid: axes [first, last] (extents > 1 listed in ext).
struct Group {
  int first = 0, last = -1;
  std::vector<int32_t> ext;
  int64_t G = 1;
};

// Split grid axes into groups whose LDS tiles fit: the innermost group may
// fill a whole tile (its tiles are contiguous runs of the tensor); the
// other groups leave room for at least kOuterMinInner contiguous inner
// elements per row.  Returned outermost first.
std::vector<Group> make_groups(const int32_t* grid, int D, int64_t tile_max) {
  std::vector<Group> gs;
  Group cur;
  bool inner = true;
  for (int i = D - 1; i >= 0; --i) {
    const int32_t e = grid[i] + 1;
    if (e == 1) continue;
    const int64_t cap = inner ? tile_max : tile_max / kOuterMinInner;
    if (!cur.ext.empty() && (cur.G * e > cap || (int)cur.ext.size() >= kMaxGroupAxes)) {
      gs.push_back(cur);
      cur = Group();
      inner = false;
    }
    if (cur.ext.empty()) cur.last = i;
    cur.first = i;
    cur.ext.insert(cur.ext.begin(), e);
    cur.G *= e;
  }
  if (!cur.ext.empty() || gs.empty()) {
    if (cur.ext.empty()) { cur.first = 0; cur.last = -1; }
    gs.push_back(cur);
  }
  std::reverse(gs.begin(), gs.end());
  return gs;
}

PassDesc make_desc(const int32_t* grid, int D, const Group& g, int64_t point_off,
                   int32_t row_begin, int32_t row_end, int32_t src, int32_t dst,
                   int64_t tile_max) {
  PassDesc d;
  std::memset(&d, 0, sizeof(d));
  int64_t O = 1, I = 1;
  if (g.last >= g.first) {
    for (int i = 0; i < g.first; ++i) O *= grid[i] + 1;
    for (int i = g.last + 1; i < D; ++i) I *= grid[i] + 1;
  } else {
    for (int i = 0; i < D; ++i) O *= grid[i] + 1;   // no axis to transform
  }
  d.O = O; d.G = g.G; d.I = I;
  if (I == 1) {
    d.TI = 1;
    int64_t to = tile_max / g.G;
    if (to > O) to = O;
    if (to < 1) to = 1;
    d.TO = (int32_t)to;
    d.tiles_i = 1;
    d.ntiles = ceil_div(O, to);
  } else {
    d.TO = 1;
    int64_t ti = tile_max / g.G;
    if (ti > I) ti = I;
    if (ti < I && ti > kOuterMinInner) ti -= ti % kOuterMinInner;
    d.TI = (int32_t)ti;
    d.tiles_i = ceil_div(I, ti);
    d.ntiles = O * d.tiles_i;
  }
  d.point_off = point_off;
  d.row_begin = row_begin;
  d.row_end = row_end;
  d.naxes = (int32_t)g.ext.size();
  for (int a = 0; a < d.naxes; ++a) d.ext[a] = g.ext[a];
  d.src = src;
  d.dst = dst;
  return d;
}

// Upload one set of levels; descs[level] lists that level's passes.
fct_status upload_levels(std::vector<std::vector<PassDesc>>& descs,
                         std::vector<DctLevel>& out, int64_t* bytes, int32_t tile_max) {
  out.clear();
  for (auto& lv : descs) {
    DctLevel L;
    int64_t tb = 0;
    int32_t emax = 1;
    for (auto& d : lv) {
      d.tile_begin = tb;
      tb += d.ntiles;
      for (int a = 0; a < d.naxes; ++a) emax = std::max(emax, d.ext[a]);
    }
    if (tb > 0x7fffffffLL) {
      set_error("DCT pass needs %lld workgroups (limit 2^31-1)", (long long)tb);
      return FCT_EINVAL;
    }
    L.ndesc = (int32_t)lv.size();
    L.tiles = tb;
    L.emax = emax;
    L.tile_max = tile_max;
    for (const auto& d : lv) L.rows_io = L.rows_io || d.dst == kDstGather || d.src == kSrcRows;
    out.push_back(L);   // owned by `out` from here (freed with it on error)
    DctLevel& R = out.back();
    FCT_HIP(dalloc(&R.d_desc, (int64_t)lv.size(), bytes));
    FCT_HIP(hipMemcpy(R.d_desc, lv.data(), sizeof(PassDesc) * lv.size(), hipMemcpyHostToDevice));
    if (R.rows_io && R.tiles > 0) FCT_HIP(dalloc(&R.d_tile_row, R.tiles, bytes));
  }
  return FCT_OK;
}

void free_levels(std::vector<DctLevel>& v, int64_t* bytes = nullptr) {
  for (auto& L : v) {
    if (bytes && L.d_desc) *bytes -= (int64_t)sizeof(PassDesc) * std::max<int64_t>(L.ndesc, 1);
    if (bytes && L.d_tile_row) *bytes -= (int64_t)sizeof(int32_t) * L.tiles;
    dfree(L.d_desc);
    dfree(L.d_tile_row);
  }
  v.clear();
}

void destroy_plan(fct_plan* p) {
  if (!p) return;
  dfree(p->d_support); dfree(p->d_grids); dfree(p->d_strides); dfree(p->d_point_off);
  dfree(p->d_alias); dfree(p->d_perm); dfree(p->d_seg_off); dfree(p->d_bin_id);
  dfree(p->d_wsign); dfree(p->d_bin_dct); dfree(p->d_row_old); dfree(p->d_row_new);
  dfree(p->d_rowmap); dfree(p->d_row_off); dfree(p->d_ell); dfree(p->d_nodes); dfree(p->d_cmat);
  dfree(p->d_emat); dfree(p->d_cmat32); dfree(p->d_rblk); dfree(p->d_cblk); dfree(p->d_prob);
  dfree(p->d_units); dfree(p->d_rblk32); dfree(p->d_ell16); dfree(p->d_sdesc);
  free_levels(p->fwd);
  free_levels(p->fwd_full);
  free_levels(p->inv);
  delete p;
}

// Pass levels of every grid for the plan's DCT tile size (p->dct_tile);
// levels built before are replaced.
fct_status build_dct_levels(fct_plan* p) {
  free_levels(p->fwd, &p->device_bytes);
  free_levels(p->fwd_full, &p->device_bytes);
  free_levels(p->inv, &p->device_bytes);
  const int K = p->K;
  const int64_t tm = p->dct_tile;
  std::vector<std::vector<Group>> groups(K);
  int maxlev = 0;
  for (int l = 0; l < K; ++l) {
    groups[l] = make_groups(&p->grids[(size_t)p->grid_goff[l]], p->grid_D[l], tm);
    maxlev = std::max(maxlev, (int)groups[l].size());
  }
  std::vector<std::vector<PassDesc>> fwd(maxlev), full(maxlev), inv(maxlev);
  for (int l = 0; l < K; ++l) {
    const int32_t* g = &p->grids[(size_t)p->grid_goff[l]];
    const int D = p->grid_D[l];
    const auto& gs = groups[l];
    const int np = (int)gs.size();
    const int shift = maxlev - np;   // forward levels aligned at the end
    for (int q = 0; q < np; ++q) {
      const bool first = q == 0, last = q == np - 1;
      fwd[shift + q].push_back(make_desc(g, D, gs[q], p->point_off[l], p->row_off[l],
                                         p->row_off[l + 1], first ? kSrcInput : kSrcScratch,
                                         last ? kDstGather : kDstScratch, tm));
      full[shift + q].push_back(make_desc(g, D, gs[q], p->point_off[l], p->row_off[l],
                                          p->row_off[l + 1], first ? kSrcInput : kSrcOutput,
                                          kDstOutput, tm));
      // inverse: innermost group first (level 0), scattering the row values
      const int lev = np - 1 - q;
      inv[lev].push_back(make_desc(g, D, gs[q], p->point_off[l], p->row_off[l],
                                   p->row_off[l + 1], last ? kSrcRows : kSrcOutput,
                                   kDstOutput, tm));
    }
  }
  fct_status st = upload_levels(fwd, p->fwd, &p->device_bytes, (int32_t)tm);
  if (st != FCT_OK) return st;
  st = upload_levels(full, p->fwd_full, &p->device_bytes, (int32_t)tm);
  if (st != FCT_OK) return st;
  st = upload_levels(inv, p->inv, &p->device_bytes, (int32_t)tm);
  if (st != FCT_OK) return st;
  const int64_t* bins = p->d_bin_dct ? p->d_bin_dct : p->d_bin_id;   // (grid, bin) row order
  for (const auto& L : p->fwd) FCT_HIP(launch_tile_rows(L, bins, nullptr));
  for (const auto& L : p->inv) FCT_HIP(launch_tile_rows(L, bins, nullptr));
  int cus = 0;
  FCT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
  for (auto* set : {&p->fwd, &p->fwd_full, &p->inv})
    for (auto& L : *set) FCT_HIP(dct_level_grids(L, std::max(cus, 1)));
  FCT_HIP(hipDeviceSynchronize());
  return FCT_OK;
}

// Row and column blocks of every problem, and the problem table.  Problem
// p's rows (columns) are cut into blocks of kBlock starting at its own first
// row (column), so the blocking -- and with it every reduction order -- of a
// problem does not depend on the other problems of a batch.  In a batch, the
// FP32 rounds of every problem whose columns fit in a unit's LDS run on LDS
// units of p->unit_rows rows instead (same sums and partials in the same
// order, so a problem gives the same bits alone and in the batch); the
// other problems keep their row blocks (rb32).
fct_status build_blocks(fct_plan* p) {
  dfree(p->d_rblk); dfree(p->d_cblk); dfree(p->d_prob); dfree(p->d_units); dfree(p->d_rblk32);
  dfree(p->d_ell16);
  p->device_bytes -= p->block_bytes;
  const int64_t bytes_before = p->device_bytes;
  std::vector<RowBlock> rb, rb32;
  std::vector<ColBlock> cb;
  std::vector<RowUnit> units;
  p->lds_cap = p->nprob > 1 ? lds_unit_capacity(p->device) : 0;
  for (int32_t q = 0; q < p->nprob; ++q) {
    ProbInfo& pi = p->probs[(size_t)q];
    pi.rblk_off = (int32_t)rb.size();
    pi.nrblk = (int32_t)ceil_div(pi.M, kBlock);
    pi.cblk_off = (int32_t)cb.size();
    pi.ncblk = (int32_t)ceil_div(pi.n, kBlock);
    const bool lds = pi.n <= p->lds_cap;
    const int32_t nunit = lds ? (int32_t)ceil_div(pi.M, p->unit_rows) : 0;
    for (int32_t b = 0; b < pi.nrblk; ++b) {
      RowBlock r;
      std::memset(&r, 0, sizeof(r));
      r.prob = q;
      r.row0 = pi.row_off + b * kBlock;
      r.row_end = std::min(pi.row_off + pi.M, r.row0 + kBlock);
      r.cblk_off = pi.cblk_off;
      r.ncblk = pi.ncblk;
      r.first = b == 0;
      r.pslot = (int32_t)rb.size();
      rb.push_back(r);
      if (!lds) rb32.push_back(r);
    }
    for (int32_t u = 0; u < nunit; ++u) {
      RowUnit t;
      std::memset(&t, 0, sizeof(t));
      t.prob = q;
      t.row0 = pi.row_off + u * p->unit_rows;
      t.row_end = std::min(pi.row_off + pi.M, t.row0 + p->unit_rows);
      t.first = u == 0;
      t.pslot = pi.rblk_off + u * (p->unit_rows / kBlock);
      t.cblk_off = pi.cblk_off;
      t.ncblk = pi.ncblk;
      t.col_off = pi.col_off;
      t.n = pi.n;
      units.push_back(t);
    }
    for (int32_t b = 0; b < pi.ncblk; ++b) {
      ColBlock c;
      std::memset(&c, 0, sizeof(c));
      c.prob = q;
      c.col0 = pi.col_off + b * kBlock;
      c.col_end = std::min(pi.col_off + pi.n, c.col0 + kBlock);
      c.col_off = pi.col_off;
      c.rblk_off = pi.rblk_off;
      c.nrblk = pi.nrblk;
      c.K = pi.K;
      c.n = pi.n;
      c.rmap_off = pi.rmap_off;
      c.first = b == 0;
      cb.push_back(c);
    }
  }
  p->nrblk = (int64_t)rb.size();
  p->ncblk = (int64_t)cb.size();
  if (p->nrblk > 0x7fffffffLL || p->ncblk > 0x7fffffffLL) {
    set_error("too many CGLS blocks");
    return FCT_EINVAL;
  }
  int64_t* bytes = &p->device_bytes;
  FCT_HIP(dalloc(&p->d_rblk, p->nrblk, bytes));
  FCT_HIP(dalloc(&p->d_cblk, p->ncblk, bytes));
  FCT_HIP(dalloc(&p->d_prob, (int64_t)p->nprob, bytes));
  FCT_HIP(hipMemcpy(p->d_rblk, rb.data(), sizeof(RowBlock) * rb.size(), hipMemcpyHostToDevice));
  FCT_HIP(hipMemcpy(p->d_cblk, cb.data(), sizeof(ColBlock) * cb.size(), hipMemcpyHostToDevice));
  FCT_HIP(hipMemcpy(p->d_prob, p->probs.data(), sizeof(ProbInfo) * p->probs.size(),
                    hipMemcpyHostToDevice));
  p->nunits = (int64_t)units.size();
  p->nrblk32 = (int64_t)rb32.size();
  if (p->nunits > 0) {
    FCT_HIP(dalloc(&p->d_units, p->nunits, bytes));
    FCT_HIP(hipMemcpy(p->d_units, units.data(), sizeof(RowUnit) * units.size(),
                      hipMemcpyHostToDevice));
    FCT_HIP(dalloc(&p->d_ell16, p->M, bytes));
    for (const ProbInfo& pi : p->probs)
      if (pi.n <= p->lds_cap)
        FCT_HIP(launch_ell16(p->d_seg_off, p->d_perm, pi.row_off, pi.M, pi.col_off, p->d_ell16,
                             nullptr));
    FCT_HIP(hipDeviceSynchronize());
  }
  if (p->nrblk32 > 0) {
    FCT_HIP(dalloc(&p->d_rblk32, p->nrblk32, bytes));
    FCT_HIP(hipMemcpy(p->d_rblk32, rb32.data(), sizeof(RowBlock) * rb32.size(),
                      hipMemcpyHostToDevice));
  }
  p->block_bytes = p->device_bytes - bytes_before;
  return FCT_OK;
}

fct_status build_tables(fct_plan* p, hipStream_t stream) {
  int64_t* bytes = &p->device_bytes;
  FCT_HIP(dalloc(&p->d_nodes, (int64_t)(p->maxdeg + 1) * 64, bytes));
  FCT_HIP(dalloc(&p->d_cmat, mat_offset(p->maxdeg + 1), bytes));
  FCT_HIP(dalloc(&p->d_cmat32, mat_offset(p->maxdeg + 1), bytes));
  FCT_HIP(dalloc(&p->d_emat, mat_offset(p->maxdeg + 1), bytes));
  FCT_HIP(launch_tables(p->maxdeg, p->d_nodes, p->d_cmat, p->d_cmat32, p->d_emat, p->gauss,
                        stream));
  return FCT_OK;
}

fct_status validate_inputs(int32_t D, int64_t n, const int32_t* S, int32_t K, const int32_t* G,
                           uint32_t flags) {
  if (D < 1 || D > FCT_MAX_DIM) { set_error("D=%d outside [1, %d]", D, FCT_MAX_DIM); return FCT_EINVAL; }
  if (n < 1) { set_error("n_support must be >= 1"); return FCT_EINVAL; }
  if (K < 1 || K >= (1 << 19)) { set_error("K=%d outside [1, 2^19)", K); return FCT_EINVAL; }
  if (!S || !G) { set_error("support and grids must be non-NULL host arrays"); return FCT_EINVAL; }
  if ((int64_t)K * n >= 0x7fffffffLL) { set_error("K * n_support must be < 2^31"); return FCT_EINVAL; }
  for (int64_t t = 0; t < n * D; ++t)
    if (S[t] < 0) { set_error("support entry %lld is negative", (long long)t); return FCT_EINVAL; }
  for (int64_t l = 0; l < K; ++l) {
    double pts = 1.0;
    for (int i = 0; i < D; ++i) {
      const int32_t N = G[l * D + i];
      if (N < 0 || N > FCT_MAX_DEGREE) {
        set_error("grid %lld dim %d: degree %d outside [0, %d]", (long long)l, i, N, FCT_MAX_DEGREE);
        return FCT_EINVAL;
      }
      pts *= (double)(N + 1);
    }
    if (pts >= 17592186044416.0) {  // 2^44
      set_error("grid %lld has %.3g points (limit 2^44)", (long long)l, pts);
      return FCT_EINVAL;
    }
  }
  // duplicate support rows
  {
    std::vector<int64_t> idx((size_t)n);
    for (int64_t j = 0; j < n; ++j) idx[(size_t)j] = j;
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      return std::lexicographical_compare(S + a * D, S + a * D + D, S + b * D, S + b * D + D);
    });
    for (int64_t j = 1; j < n; ++j)
      if (std::equal(S + idx[j] * D, S + idx[j] * D + D, S + idx[j - 1] * D)) {
        set_error("support rows %lld and %lld are equal", (long long)idx[j - 1], (long long)idx[j]);
        return FCT_EINVAL;
      }
  }
  if (flags & ~(FCT_PLAN_ALLOW_RANK_DEFICIENT | FCT_PLAN_GAUSS | FCT_PLAN_ROWS_BY_MEMBER)) {
    set_error("unknown plan flags 0x%x", flags);
    return FCT_EINVAL;
  }
  if ((flags & FCT_PLAN_GAUSS) && (flags & FCT_PLAN_ROWS_BY_MEMBER)) {
    set_error("FCT_PLAN_GAUSS and FCT_PLAN_ROWS_BY_MEMBER do not combine");
    return FCT_EINVAL;
  }
  if ((flags & FCT_PLAN_GAUSS) && !(flags & FCT_PLAN_ALLOW_RANK_DEFICIENT)) {
    // per dimension, the signed 1-D rows of every degree over the K grids
    // must be nonzero and pairwise independent (not equal up to sign)
    for (int i = 0; i < D; ++i) {
      int32_t mx = 0;
      for (int64_t j = 0; j < n; ++j) mx = std::max(mx, S[j * D + i]);
      std::set<std::vector<int64_t>> seen;
      for (int32_t a = 0; a <= mx; ++a) {
        std::vector<int64_t> key((size_t)K);
        int64_t first = 0;
        for (int64_t l = 0; l < K; ++l) {
          int w = 1;
          const int64_t m = fold_gauss_host(a, G[l * D + i], &w);
          key[(size_t)l] = w == 0 ? 0 : w * (m + 1);
          if (first == 0) first = key[(size_t)l];
        }
        if (first == 0) {
          set_error("rank pre-check: dimension %d, degree %d vanishes on every grid", i, a);
          return FCT_ERANK;
        }
        if (first < 0) for (auto& v : key) v = -v;
        if (!seen.insert(key).second) {
          set_error("rank pre-check: dimension %d, degree %d aliases an earlier degree (up to "
                    "sign) on every grid", i, a);
          return FCT_ERANK;
        }
      }
    }
  } else if (!(flags & FCT_PLAN_ALLOW_RANK_DEFICIENT)) {
    // per dimension, the K folds must tell apart every degree that occurs
    for (int i = 0; i < D; ++i) {
      int32_t mx = 0;
      for (int64_t j = 0; j < n; ++j) mx = std::max(mx, S[j * D + i]);
      std::set<std::vector<int64_t>> seen;
      for (int32_t a = 0; a <= mx; ++a) {
        std::vector<int64_t> key((size_t)K);
        for (int64_t l = 0; l < K; ++l) key[(size_t)l] = fold_host(a, G[l * D + i]);
        if (!seen.insert(key).second) {
          set_error("rank pre-check: dimension %d, degree %d aliases an earlier degree on "
                    "every grid", i, a);
          return FCT_ERANK;
        }
      }
    }
  }
  return FCT_OK;
}

bool dev_ok(const fct_plan* p) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != p->device) {
    set_error("the current HIP device (%d) is not the plan's device (%d)", cur, p->device);
    return false;
  }
  return true;
}

struct DevGuard {
  std::vector<void*> ptrs;
  ~DevGuard() { for (void* q : ptrs) if (q) (void)hipFree(q); }
};

}  // namespace

// A c and A^T r of a plan, with the entry weights of a Gauss plan.
hipError_t plan_apply_A(const fct_plan* p, const double* c, double* q, hipStream_t s) {
  if (p->gauss) return launch_apply_A_signed(p->d_seg_off, p->d_perm, p->d_wsign, p->M, p->n, c, q, s);
  return launch_apply_A(p->d_seg_off, p->d_perm, p->M, c, q, s);
}

hipError_t plan_apply_AT(const fct_plan* p, const double* r, double* out, hipStream_t s) {
  if (p->gauss) return launch_apply_AT_signed(p->d_rowmap, p->d_wsign, p->K, p->n, r, out, s);
  return launch_apply_AT(p->d_cblk, p->ncblk, p->d_rowmap, r, out, s);
}

}  // namespace fct

using namespace fct;

extern "C" {

const char* fct_last_error(void) { return g_last_error.c_str(); }

const char* fct_status_string(fct_status s) {
  switch (s) {
    case FCT_OK: return "FCT_OK";
    case FCT_EINVAL: return "FCT_EINVAL";
    case FCT_ENOMEM: return "FCT_ENOMEM";
    case FCT_EDEVICE: return "FCT_EDEVICE";
    case FCT_ERANK: return "FCT_ERANK";
    case FCT_ENOCONV: return "FCT_ENOCONV";
    case FCT_ENONFINITE: return "FCT_ENONFINITE";
  }
  return "FCT_UNKNOWN";
}

int32_t fct_abi_version(void) { return FCT_ABI_VERSION; }

fct_status fct_plan_create(int32_t D, int64_t n, const int32_t* support, int32_t K,
                           const int32_t* grids, uint32_t flags, hipStream_t stream,
                           fct_plan** out) {
  g_last_error.clear();
  if (!out) { set_error("out is NULL"); return FCT_EINVAL; }
  *out = nullptr;
  fct_status st = validate_inputs(D, n, support, K, grids, flags);
  if (st != FCT_OK) return st;

  fct_plan* p = new (std::nothrow) fct_plan();
  if (!p) { set_error("host allocation failed"); return FCT_ENOMEM; }
  struct Guard {
    fct_plan* p;
    uint64_t *k0 = nullptr, *k1 = nullptr;
    int32_t *v0 = nullptr, *v1 = nullptr, *bc = nullptr;
    ~Guard() {
      dfree(k0); dfree(k1); dfree(v0); dfree(v1); dfree(bc);
      if (p) destroy_plan(p);
    }
  } guard{p};

  FCT_HIP(hipGetDevice(&p->device));
  p->gauss = (flags & FCT_PLAN_GAUSS) ? 1 : 0;
  p->rows_by_member = (flags & FCT_PLAN_ROWS_BY_MEMBER) ? 1 : 0;
  p->nprob = 1;
  p->D = D; p->K = K; p->n = n;
  p->grids.assign(grids, grids + (size_t)K * D);
  for (int64_t t = 0; t < n * D; ++t) p->smax = std::max(p->smax, support[t]);
  p->grid_D.assign((size_t)K, D);
  p->grid_goff.resize((size_t)K + 1);
  for (int l = 0; l <= K; ++l) p->grid_goff[(size_t)l] = (int64_t)l * D;
  p->points.resize(K);
  p->point_off.assign((size_t)K + 1, 0);
  std::vector<int64_t> strides((size_t)K * D);
  p->maxdeg = 0;
  for (int l = 0; l < K; ++l) {
    int64_t st_ = 1;
    for (int i = D - 1; i >= 0; --i) {
      strides[(size_t)l * D + i] = st_;
      st_ *= grids[(size_t)l * D + i] + 1;
      p->maxdeg = std::max(p->maxdeg, grids[(size_t)l * D + i]);
    }
    p->points[l] = st_;
    p->point_off[l + 1] = p->point_off[l] + st_;
    p->max_points = std::max(p->max_points, st_);
  }
  p->total_points = p->point_off[K];
  const int64_t L = (int64_t)K * n;
  int64_t* bytes = &p->device_bytes;

  FCT_HIP(dalloc(&p->d_support, n * D, bytes));
  FCT_HIP(dalloc(&p->d_grids, (int64_t)K * D, bytes));
  FCT_HIP(dalloc(&p->d_strides, (int64_t)K * D, bytes));
  FCT_HIP(dalloc(&p->d_point_off, (int64_t)K + 1, bytes));
  FCT_HIP(dalloc(&p->d_alias, L, bytes));
  if (p->gauss) FCT_HIP(dalloc(&p->d_wsign, L, bytes));
  FCT_HIP(dalloc(&p->d_perm, L, bytes));
  FCT_HIP(dalloc(&p->d_seg_off, L + 1, bytes));
  FCT_HIP(dalloc(&p->d_bin_id, L, bytes));
  FCT_HIP(dalloc(&p->d_rowmap, L, bytes));
  FCT_HIP(dalloc(&p->d_row_off, (int64_t)K + 1, bytes));
  FCT_HIP(dalloc(&guard.k0, L, nullptr));
  FCT_HIP(dalloc(&guard.k1, L, nullptr));
  FCT_HIP(dalloc(&guard.v0, L, nullptr));
  FCT_HIP(dalloc(&guard.v1, L, nullptr));
  const int64_t nb = segment_blocks(L);
  FCT_HIP(dalloc(&guard.bc, nb, nullptr));

  FCT_HIP(hipMemcpyAsync(p->d_support, support, sizeof(int32_t) * n * D, hipMemcpyHostToDevice, stream));
  FCT_HIP(hipMemcpyAsync(p->d_grids, grids, sizeof(int32_t) * K * D, hipMemcpyHostToDevice, stream));
  FCT_HIP(hipMemcpyAsync(p->d_strides, strides.data(), sizeof(int64_t) * K * D, hipMemcpyHostToDevice, stream));
  FCT_HIP(hipMemcpyAsync(p->d_point_off, p->point_off.data(), sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice, stream));

  st = build_tables(p, stream);
  if (st != FCT_OK) return st;
  FCT_HIP(launch_alias(p->d_support, p->d_grids, p->d_strides, D, n, K, p->d_alias, guard.k0,
                       guard.v0, p->d_wsign, stream));
  bool in_tmp = false;
  FCT_HIP(launch_sort(guard.k0, guard.v0, guard.k1, guard.v1, L, &in_tmp, stream));
  const uint64_t* ks = in_tmp ? guard.k1 : guard.k0;
  const int32_t* vs = in_tmp ? guard.v1 : guard.v0;
  FCT_HIP(launch_segments(ks, vs, L, n, guard.bc, nb, p->d_perm, p->d_seg_off, p->d_bin_id,
                          p->d_rowmap, p->d_row_off, K, stream));
  p->row_off.assign((size_t)K + 1, 0);
  FCT_HIP(hipMemcpyAsync(p->row_off.data(), p->d_row_off, sizeof(int32_t) * (K + 1),
                         hipMemcpyDeviceToHost, stream));
  FCT_HIP(hipStreamSynchronize(stream));
  p->M = p->row_off[K];
  if (p->rows_by_member) {
    // second stable sort by (grid, first member of the row): same rows, each
    // grid's rows ordered by their smallest column; the (grid, bin) order
    // stays behind for the DCT (d_bin_dct) with the map between the two
    int32_t *perm2 = nullptr, *seg2 = nullptr, *rowmap2 = nullptr;
    int64_t* bin2 = nullptr;
    struct G2 {
      int32_t **a, **b, **c; int64_t** d;
      ~G2() { dfree(*a); dfree(*b); dfree(*c); dfree(*d); }
    } g2{&perm2, &seg2, &rowmap2, &bin2};
    FCT_HIP(dalloc(&perm2, L, nullptr));
    FCT_HIP(dalloc(&seg2, L + 1, nullptr));
    FCT_HIP(dalloc(&rowmap2, L, nullptr));
    FCT_HIP(dalloc(&bin2, L, nullptr));
    FCT_HIP(dalloc(&p->d_row_old, p->M, bytes));
    FCT_HIP(launch_member_keys(p->d_rowmap, p->d_perm, p->d_seg_off, n, K, guard.k0, guard.v0,
                               stream));
    bool in_tmp2 = false;
    FCT_HIP(launch_sort(guard.k0, guard.v0, guard.k1, guard.v1, L, &in_tmp2, stream));
    FCT_HIP(launch_segments(in_tmp2 ? guard.k1 : guard.k0, in_tmp2 ? guard.v1 : guard.v0, L, n,
                            guard.bc, nb, perm2, seg2, bin2, rowmap2, p->d_row_off, K, stream));
    FCT_HIP(launch_row_old(perm2, seg2, p->d_rowmap, p->d_bin_id, p->M, n, p->d_row_old, bin2,
                           stream));
    FCT_HIP(dalloc(&p->d_row_new, p->M, bytes));
    FCT_HIP(launch_index_inverse(p->d_row_old, p->M, p->d_row_new, stream));
    FCT_HIP(hipStreamSynchronize(stream));
    p->d_bin_dct = p->d_bin_id;
    p->d_bin_id = bin2;
    bin2 = nullptr;
    std::swap(p->d_perm, perm2);
    std::swap(p->d_seg_off, seg2);
    std::swap(p->d_rowmap, rowmap2);
  }
  FCT_HIP(dalloc(&p->d_ell, p->M, bytes));
  FCT_HIP(launch_ell(p->d_seg_off, p->d_perm, p->M, p->d_ell, stream));
  FCT_HIP(hipStreamSynchronize(stream));

  ProbInfo pi;
  std::memset(&pi, 0, sizeof(pi));
  pi.row_off = 0; pi.M = (int32_t)p->M; pi.col_off = 0; pi.n = (int32_t)n;
  pi.K = K; pi.rmap_off = 0; pi.grid_off = 0;
  p->probs.assign(1, pi);
  p->prob_point_off = {0, p->total_points};
  st = build_blocks(p);
  if (st != FCT_OK) return st;
  st = build_dct_levels(p);
  if (st != FCT_OK) return st;
  {
    std::vector<SampleDesc> sd;
    make_sample_descs(p->grids, D, K, p->point_off, &sd, &p->sample_tiles);
    if (p->sample_tiles > 0x7fffffffLL) {
      set_error("sampling needs %lld workgroups (limit 2^31-1)", (long long)p->sample_tiles);
      return FCT_EINVAL;
    }
    FCT_HIP(dalloc(&p->d_sdesc, (int64_t)sd.size(), bytes));
    FCT_HIP(hipMemcpy(p->d_sdesc, sd.data(), sizeof(SampleDesc) * sd.size(),
                      hipMemcpyHostToDevice));
  }
  guard.p = nullptr;
  *out = p;
  return FCT_OK;
}

fct_status fct_batch_create(int32_t count, const fct_plan* const* plans, hipStream_t stream,
                            fct_plan** out) {
  g_last_error.clear();
  if (!out || !plans || count < 1) { set_error("need count >= 1 plans and an output"); return FCT_EINVAL; }
  *out = nullptr;
  int dev = -1;
  FCT_HIP(hipGetDevice(&dev));
  int64_t Lsum = 0, Msum = 0, nsum = 0, Ksum = 0;
  for (int32_t q = 0; q < count; ++q) {
    const fct_plan* s = plans[q];
    if (!s || s->nprob != 1) { set_error("plan %d is NULL or already a batch", q); return FCT_EINVAL; }
    if (s->gauss) { set_error("plan %d is a Gauss-grid plan (not batched)", q); return FCT_EINVAL; }
    if (s->device != dev) { set_error("plan %d lives on another device", q); return FCT_EINVAL; }
    Lsum += (int64_t)s->K * s->n;
    Msum += s->M;
    nsum += s->n;
    Ksum += s->K;
  }
  if (Lsum >= 0x7fffffffLL || Msum >= 0x7fffffffLL || Ksum >= (1 << 24)) {
    set_error("batch too large (sum K*n = %lld, rows = %lld)", (long long)Lsum, (long long)Msum);
    return FCT_EINVAL;
  }
  fct_plan* p = new (std::nothrow) fct_plan();
  if (!p) { set_error("host allocation failed"); return FCT_ENOMEM; }
  struct Guard { fct_plan* p; ~Guard() { if (p) destroy_plan(p); } } guard{p};
  p->device = dev;
  p->nprob = count;
  p->K = (int32_t)Ksum;
  p->n = nsum;
  p->M = Msum;
  int64_t* bytes = &p->device_bytes;
  FCT_HIP(dalloc(&p->d_perm, Lsum, bytes));
  FCT_HIP(dalloc(&p->d_seg_off, Msum + 1, bytes));
  FCT_HIP(dalloc(&p->d_bin_id, Msum, bytes));
  FCT_HIP(dalloc(&p->d_rowmap, Lsum, bytes));
  FCT_HIP(dalloc(&p->d_ell, Msum, bytes));
  // a batch with a plan whose rows are ordered by first member keeps the
  // (grid, bin) order of every problem for its transforms, with the maps
  // between the two (identity for the other problems)
  for (int32_t q = 0; q < count; ++q) p->rows_by_member |= plans[q]->rows_by_member;
  if (p->rows_by_member) {
    FCT_HIP(dalloc(&p->d_bin_dct, Msum, bytes));
    FCT_HIP(dalloc(&p->d_row_old, Msum, bytes));
    FCT_HIP(dalloc(&p->d_row_new, Msum, bytes));
  }

  p->grid_goff.push_back(0);
  p->point_off.push_back(0);
  p->row_off.push_back(0);
  p->prob_point_off.push_back(0);
  int64_t loff = 0, moff = 0, noff = 0;
  for (int32_t q = 0; q < count; ++q) {
    const fct_plan* s = plans[q];
    const int64_t Lq = (int64_t)s->K * s->n;
    ProbInfo pi;
    std::memset(&pi, 0, sizeof(pi));
    pi.row_off = (int32_t)moff; pi.M = (int32_t)s->M;
    pi.col_off = (int32_t)noff; pi.n = (int32_t)s->n;
    pi.K = s->K; pi.rmap_off = (int32_t)loff;
    pi.grid_off = (int32_t)p->points.size();
    p->probs.push_back(pi);
    FCT_HIP(launch_copy_add_i32(p->d_perm + loff, s->d_perm, Lq, (int32_t)noff, stream));
    FCT_HIP(launch_copy_add_i32(p->d_seg_off + moff, s->d_seg_off, s->M, (int32_t)loff, stream));
    FCT_HIP(launch_copy_add_i32(p->d_rowmap + loff, s->d_rowmap, Lq, (int32_t)moff, stream));
    FCT_HIP(launch_copy_ell(p->d_ell + moff, s->d_ell, s->M, (int32_t)noff, (int32_t)loff, stream));
    FCT_HIP(hipMemcpyAsync(p->d_bin_id + moff, s->d_bin_id, sizeof(int64_t) * s->M,
                           hipMemcpyDeviceToDevice, stream));
    if (p->rows_by_member) {
      FCT_HIP(hipMemcpyAsync(p->d_bin_dct + moff, s->d_bin_dct ? s->d_bin_dct : s->d_bin_id,
                             sizeof(int64_t) * s->M, hipMemcpyDeviceToDevice, stream));
      if (s->rows_by_member) {
        FCT_HIP(launch_copy_add_i32(p->d_row_old + moff, s->d_row_old, s->M, (int32_t)moff, stream));
        FCT_HIP(launch_copy_add_i32(p->d_row_new + moff, s->d_row_new, s->M, (int32_t)moff, stream));
      } else {
        FCT_HIP(launch_iota_i32(p->d_row_old + moff, s->M, (int32_t)moff, stream));
        FCT_HIP(launch_iota_i32(p->d_row_new + moff, s->M, (int32_t)moff, stream));
      }
    }
    for (int32_t l = 0; l < s->K; ++l) {
      const int32_t D = s->grid_D[(size_t)l];
      const int32_t* g = &s->grids[(size_t)s->grid_goff[(size_t)l]];
      p->grids.insert(p->grids.end(), g, g + D);
      p->grid_D.push_back(D);
      p->grid_goff.push_back((int64_t)p->grids.size());
      p->points.push_back(s->points[(size_t)l]);
      p->point_off.push_back(p->point_off.back() + s->points[(size_t)l]);
      p->row_off.push_back((int32_t)(moff + s->row_off[(size_t)l + 1]));
      p->max_points = std::max(p->max_points, s->points[(size_t)l]);
    }
    p->prob_point_off.push_back(p->point_off.back());
    p->D = std::max(p->D, s->D);
    p->maxdeg = std::max(p->maxdeg, s->maxdeg);
    loff += Lq; moff += s->M; noff += s->n;
  }
  p->total_points = p->point_off.back();
  const int32_t end = (int32_t)Lsum;
  FCT_HIP(hipMemcpyAsync(p->d_seg_off + Msum, &end, sizeof(int32_t), hipMemcpyHostToDevice, stream));
  FCT_HIP(dalloc(&p->d_grids, (int64_t)p->grids.size(), bytes));
  FCT_HIP(dalloc(&p->d_point_off, (int64_t)p->K + 1, bytes));
  FCT_HIP(dalloc(&p->d_row_off, (int64_t)p->K + 1, bytes));
  FCT_HIP(hipMemcpyAsync(p->d_grids, p->grids.data(), sizeof(int32_t) * p->grids.size(),
                         hipMemcpyHostToDevice, stream));
  FCT_HIP(hipMemcpyAsync(p->d_point_off, p->point_off.data(), sizeof(int64_t) * (p->K + 1),
                         hipMemcpyHostToDevice, stream));
  FCT_HIP(hipMemcpyAsync(p->d_row_off, p->row_off.data(), sizeof(int32_t) * (p->K + 1),
                         hipMemcpyHostToDevice, stream));
  fct_status st = build_tables(p, stream);
  if (st != FCT_OK) return st;
  FCT_HIP(hipStreamSynchronize(stream));
  st = build_blocks(p);
  if (st != FCT_OK) return st;
  st = build_dct_levels(p);
  if (st != FCT_OK) return st;
  guard.p = nullptr;
  *out = p;
  return FCT_OK;
}

void fct_plan_destroy(fct_plan* plan) { destroy_plan(plan); }

fct_status fct_plan_get_info(const fct_plan* p, fct_plan_info* o) {
  if (!p || !o) { set_error("NULL argument"); return FCT_EINVAL; }
  std::memset(o, 0, sizeof(*o));
  o->D = p->D; o->K = p->K; o->n_support = p->n; o->total_points = p->total_points;
  o->total_rows = p->M; o->max_points = p->max_points; o->max_degree = p->maxdeg;
  o->dct_levels = (int32_t)p->fwd.size(); o->device_bytes = p->device_bytes;
  o->problems = p->nprob;
  for (const auto& pi : p->probs) o->entries += (int64_t)pi.K * pi.n;
  return FCT_OK;
}

fct_status fct_plan_grid(const fct_plan* p, int32_t l, int64_t* points, int64_t* rows,
                         int64_t* point_offset, int64_t* row_offset) {
  if (!p || l < 0 || l >= p->K) { set_error("bad plan or grid index"); return FCT_EINVAL; }
  if (points) *points = p->points[l];
  if (rows) *rows = p->row_off[l + 1] - p->row_off[l];
  if (point_offset) *point_offset = p->point_off[l];
  if (row_offset) *row_offset = p->row_off[l];
  return FCT_OK;
}

fct_status fct_plan_problem(const fct_plan* p, int32_t q, int64_t* n, int64_t* rows,
                            int64_t* col_offset, int64_t* row_offset, int64_t* point_offset,
                            int64_t* points) {
  if (!p || q < 0 || q >= p->nprob) { set_error("bad plan or problem index"); return FCT_EINVAL; }
  const ProbInfo& pi = p->probs[(size_t)q];
  if (n) *n = pi.n;
  if (rows) *rows = pi.M;
  if (col_offset) *col_offset = pi.col_off;
  if (row_offset) *row_offset = pi.row_off;
  if (point_offset) *point_offset = p->prob_point_off[(size_t)q];
  if (points) *points = p->prob_point_off[(size_t)q + 1] - p->prob_point_off[(size_t)q];
  return FCT_OK;
}

fct_status fct_plan_export(const fct_plan* p, int64_t* d_alias, int32_t* d_perm,
                           int32_t* d_seg_off, int64_t* d_bin_id, int32_t* d_rowmap,
                           hipStream_t s) {
  if (!p) { set_error("NULL plan"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  int64_t L = 0;
  for (const auto& pi : p->probs) L += (int64_t)pi.K * pi.n;
  if (d_alias && !p->d_alias) { set_error("alias bins are kept for single-problem plans only"); return FCT_EINVAL; }
  if (d_alias) FCT_HIP(hipMemcpyAsync(d_alias, p->d_alias, sizeof(int64_t) * L, hipMemcpyDeviceToDevice, s));
  if (d_perm) FCT_HIP(hipMemcpyAsync(d_perm, p->d_perm, sizeof(int32_t) * L, hipMemcpyDeviceToDevice, s));
  if (d_seg_off) FCT_HIP(hipMemcpyAsync(d_seg_off, p->d_seg_off, sizeof(int32_t) * (p->M + 1), hipMemcpyDeviceToDevice, s));
  if (d_bin_id) FCT_HIP(hipMemcpyAsync(d_bin_id, p->d_bin_id, sizeof(int64_t) * p->M, hipMemcpyDeviceToDevice, s));
  if (d_rowmap) FCT_HIP(hipMemcpyAsync(d_rowmap, p->d_rowmap, sizeof(int32_t) * L, hipMemcpyDeviceToDevice, s));
  return FCT_OK;
}

fct_status fct_plan_weights(const fct_plan* p, int8_t* d_w, hipStream_t s) {
  if (!p || !d_w) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  if (p->nprob != 1) { set_error("entry weights are kept for single-problem plans only"); return FCT_EINVAL; }
  const int64_t L = (int64_t)p->K * p->n;
  if (p->gauss) FCT_HIP(hipMemcpyAsync(d_w, p->d_wsign, (size_t)L, hipMemcpyDeviceToDevice, s));
  else FCT_HIP(hipMemsetAsync(d_w, 1, (size_t)L, s));
  return FCT_OK;
}

fct_status fct_grid_nodes(const fct_plan* p, int32_t grid, int32_t dim, double* host_out) {
  if (!p || !host_out || grid < 0 || grid >= p->K || dim < 0 || dim >= p->grid_D[(size_t)grid]) {
    set_error("bad arguments");
    return FCT_EINVAL;
  }
  if (!dev_ok(p)) return FCT_EINVAL;
  const int N = p->grids[(size_t)p->grid_goff[(size_t)grid] + dim];
  FCT_HIP(hipMemcpy(host_out, p->d_nodes + (int64_t)N * 64, sizeof(double) * (N + 1),
                    hipMemcpyDeviceToHost));
  return FCT_OK;
}

fct_status fct_ws_create(const fct_plan* p, fct_ws** out) {
  if (!p || !out) { set_error("NULL argument"); return FCT_EINVAL; }
  *out = nullptr;
  if (!dev_ok(p)) return FCT_EINVAL;
  fct_ws* w = new (std::nothrow) fct_ws();
  if (!w) { set_error("host allocation failed"); return FCT_ENOMEM; }
  struct G { fct_ws* w; ~G() { if (w) fct_ws_destroy(w); } } guard{w};
  w->device = p->device;
  w->plan = p;
  const int64_t P = p->nprob;
  FCT_HIP(dalloc(&w->d_scratch, p->total_points, nullptr));
  FCT_HIP(dalloc(&w->d_rq, p->M, nullptr));
  FCT_HIP(dalloc(&w->d_ps, p->n, nullptr));
  FCT_HIP(dalloc(&w->d_ctmp, p->n, nullptr));
  FCT_HIP(dalloc(&w->d_r64, p->M, nullptr));
  FCT_HIP(dalloc(&w->d_part_true, p->ncblk, nullptr));
  FCT_HIP(dalloc(&w->d_gtrue, 2 * P, nullptr));
  FCT_HIP(dalloc(&w->d_outer, P, nullptr));
  FCT_HIP(hipHostMalloc((void**)&w->h_outer, sizeof(int32_t) * P, hipHostMallocDefault));
  FCT_HIP(dalloc(&w->d_gprev, P, nullptr));
  FCT_HIP(hipHostMalloc((void**)&w->h_gprev, sizeof(double) * P, hipHostMallocDefault));
  FCT_HIP(hipHostMalloc((void**)&w->h_gtrue, sizeof(double) * 2 * P, hipHostMallocDefault));
  FCT_HIP(dalloc(&w->d_part_q, 4 * p->nrblk, nullptr));   // one per wave of a row block
  FCT_HIP(dalloc(&w->d_part_s, p->ncblk, nullptr));
  if (p->rows_by_member) FCT_HIP(dalloc(&w->d_bperm, p->M, nullptr));
  if (P == 1) {
    FCT_HIP(dalloc(&w->d_cg, 2 * p->n, nullptr));
    FCT_HIP(dalloc(&w->d_cg_part, 4 * ceil_div(p->n, kCg1Block), nullptr));
  }
  FCT_HIP(dalloc(&w->d_status, (int64_t)status_bytes(P), nullptr));
  {
    const StatusView v = status_view(w->d_status, P);
    w->d_ring = v.ring; w->d_gamma0 = v.gamma0; w->d_done = v.done; w->d_flags = v.flags;
  }
  FCT_HIP(dalloc(&w->d_done_tmp, P, nullptr));
  FCT_HIP(dalloc(&w->d_state, 4, nullptr));
  FCT_HIP(dalloc(&w->d_state_tmp, 4, nullptr));
  FCT_HIP(dalloc(&w->d_bar, 4, nullptr));
  FCT_HIP(hipMemset(w->d_bar, 0, sizeof(int32_t) * 4));
  FCT_HIP(hipHostMalloc((void**)&w->h_status, 3 * status_bytes(P), hipHostMallocDefault));
  w->h_flags = status_view(w->h_status + 2 * status_bytes(P), P).flags;
  for (auto& e : w->ev) FCT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  FCT_HIP(hipStreamCreateWithFlags(&w->graph_stream, hipStreamNonBlocking));
  guard.w = nullptr;
  *out = w;
  return FCT_OK;
}

void fct_ws_destroy(fct_ws* w) {
  if (!w) return;
  for (auto& g : w->graph_exec) if (g) (void)hipGraphExecDestroy(g);
  if (w->graph_stream) (void)hipStreamDestroy(w->graph_stream);
  for (auto& e : w->ev) if (e) (void)hipEventDestroy(e);
  dfree(w->d_scratch); dfree(w->d_rq); dfree(w->d_ps); dfree(w->d_ctmp);
  dfree(w->d_part_q); dfree(w->d_part_s); dfree(w->d_status);
  dfree(w->d_cg); dfree(w->d_cg_part); dfree(w->d_bperm); dfree(w->d_nb8); dfree(w->d_nb_off); dfree(w->d_nb_ovf); dfree(w->d_nb_diag);
  dfree(w->d_done_tmp); dfree(w->d_state);
  dfree(w->d_state_tmp); dfree(w->d_bar); dfree(w->d_r64); dfree(w->d_part_true); dfree(w->d_gtrue);
  dfree(w->d_outer);
  if (w->h_outer) (void)hipHostFree(w->h_outer);
  dfree(w->d_gprev);
  if (w->h_gprev) (void)hipHostFree(w->h_gprev);
  if (w->h_gtrue) (void)hipHostFree(w->h_gtrue);
  if (w->h_status) (void)hipHostFree(w->h_status);
  delete w;
}

static fct_status check_ws(const fct_plan* p, const fct_ws* w) {
  if (!w) { set_error("this call needs a workspace"); return FCT_EINVAL; }
  if (w->plan != p) { set_error("workspace was created for another plan"); return FCT_EINVAL; }
  return FCT_OK;
}

fct_status fct_sample(const fct_plan* p, int32_t family, const double* params, int32_t n_params,
                      const double* d_coeffs, double* d_samples, fct_ws* ws, hipStream_t s) {
  if (!p || !d_samples) { set_error("NULL plan or output"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  if (family == FCT_F_PLANTED) {
    if (!d_coeffs) { set_error("planted family needs d_coeffs"); return FCT_EINVAL; }
    fct_status st = check_ws(p, ws);
    if (st != FCT_OK) return st;
    // q = A c at the non-empty bins, then evaluation at the nodes
    double* q = reinterpret_cast<double*>(ws->d_rq);   // M doubles of scratch
    if (p->rows_by_member) {
      // q in the plan's row order, then scattered to the (grid, bin) order
      FCT_HIP(plan_apply_A(p, d_coeffs, ws->d_bperm, s));
      FCT_HIP(launch_rows_gather(ws->d_bperm, p->d_row_new, p->M, q, s));
    } else {
      FCT_HIP(plan_apply_A(p, d_coeffs, q, s));
    }
    const int64_t* bins = p->d_bin_dct ? p->d_bin_dct : p->d_bin_id;
    for (const auto& lv : p->inv)
      FCT_HIP(launch_dct_level(lv, FCT_DCT_F64, FCT_ENGINE_VECTOR, q, nullptr, d_samples,
                                       p->d_emat, nullptr, bins, s));
    return FCT_OK;
  }
  if (p->nprob != 1) {
    set_error("analytic families are sampled per problem (use each problem's own plan)");
    return FCT_EINVAL;
  }
  const int D = p->D;
  int need = 0;
  switch (family) {
    case FCT_F_EXPCOS: need = 2 * D; break;
    case FCT_F_GAUSS: need = 1 + D; break;
    case FCT_F_RUNGE: need = 1; break;
    case FCT_F_OSC: need = 0; break;
    default: set_error("unknown family %d", family); return FCT_EINVAL;
  }
  if (n_params < need || (need > 0 && !params)) {
    set_error("family %d needs %d parameters, got %d", family, need, n_params);
    return FCT_EINVAL;
  }
  SampleParams prm;
  std::memset(&prm, 0, sizeof(prm));
  for (int i = 0; i < need; ++i) prm.v[i] = params[i];
  FCT_HIP(launch_sample(family, prm, D, p->d_sdesc, p->K, p->sample_tiles, p->d_grids,
                        p->d_nodes, d_samples, s));
  return FCT_OK;
}

static fct_status check_mode(const fct_plan* p, int32_t mode) {
  if (mode != FCT_DCT_F64 && mode != FCT_DCT_F32 && mode != FCT_DCT_BF16X3) {
    set_error("unknown DCT mode %d", mode);
    return FCT_EINVAL;
  }
  if (mode != FCT_DCT_F64 && p->maxdeg > 31) {
    set_error("DCT mode %d needs every degree <= 31 (plan has %d)", mode, p->maxdeg);
    return FCT_EINVAL;
  }
  return FCT_OK;
}

fct_status fct_dct(const fct_plan* p, const double* d_samples, double* d_b, int32_t mode,
                   fct_ws* ws, hipStream_t s) {
  if (!p || !d_samples || !d_b) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  fct_status st = check_mode(p, mode);
  if (st != FCT_OK) return st;
  void* scratch = nullptr;
  if (p->fwd.size() > 1 || p->rows_by_member) {
    st = check_ws(p, ws);
    if (st != FCT_OK) return st;
    scratch = ws->d_scratch;
  }
  // rows by first member: the passes write b in (grid, bin) order, then the
  // rows are gathered into the plan's order
  double* out = p->rows_by_member ? ws->d_bperm : d_b;
  const int64_t* bins = p->d_bin_dct ? p->d_bin_dct : p->d_bin_id;
  for (const auto& lv : p->fwd)
    FCT_HIP(launch_dct_level(lv, mode, p->dct_engine[mode], d_samples, scratch, out,
                                     p->d_cmat, p->d_cmat32, bins, s));
  if (p->rows_by_member) FCT_HIP(launch_rows_gather(ws->d_bperm, p->d_row_old, p->M, d_b, s));
  return FCT_OK;
}

fct_status fct_dct_full(const fct_plan* p, const double* d_samples, double* d_out, int32_t mode,
                        fct_ws* ws, hipStream_t s) {
  (void)ws;
  if (!p || !d_samples || !d_out) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  fct_status st = check_mode(p, mode);
  if (st != FCT_OK) return st;
  for (const auto& lv : p->fwd_full)
    FCT_HIP(launch_dct_level(lv, mode, p->dct_engine[mode], d_samples, nullptr, d_out,
                                     p->d_cmat, p->d_cmat32,
                                     p->d_bin_dct ? p->d_bin_dct : p->d_bin_id, s));
  return FCT_OK;
}

fct_status fct_eval(const fct_plan* p, const double* d_c, int64_t m, const double* d_x,
                    double* d_f, fct_ws* ws, hipStream_t s) {
  if (!p) { set_error("NULL plan"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  if (p->nprob != 1 || !p->d_support) {
    set_error("evaluation needs a single-problem plan (use each problem's own plan)");
    return FCT_EINVAL;
  }
  if (m < 0) { set_error("m = %lld < 0", (long long)m); return FCT_EINVAL; }
  if (m == 0) return FCT_OK;
  if (!d_c || !d_x || !d_f) { set_error("NULL argument"); return FCT_EINVAL; }
  const int nk = p->smax + 1;
  if (eval_chunk(p->D, nk) == 0 || p->D * nk > 65535) {
    set_error("evaluation table of D * (max degree + 1) = %d values per point exceeds the LDS",
              p->D * nk);
    return FCT_EINVAL;
  }
  if (ws) {
    fct_status st = check_ws(p, ws);
    if (st != FCT_OK) return st;
  }
  const int slices = eval_slices(p->n, p->D, nk, m, ws ? p->total_points : 0);
  FCT_HIP(launch_eval(p->d_support, d_c, p->n, p->D, nk, m, d_x, d_f, slices,
                      ws ? ws->d_scratch : nullptr, s));
  return FCT_OK;
}

// ---- condition estimate and grid-count selection (Alg. 2) ---------------

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..k) and off-diagonal b[0..k-1) (Sturm sequence of the LDL^T
// pivots).
static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, int k,
                       double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i > 0 ? off / d : 0.0);
    if (d == 0.0) d = -1e-300;            // a zero pivot counts as negative
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// The idx-th smallest eigenvalue (0-based) of the tridiagonal, by bisection
// inside its Gershgorin interval.
static double tridiag_eig(const std::vector<double>& a, const std::vector<double>& b, int k,
                          int idx) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 400 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, k, mid) > idx) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Lanczos on A^T A from d_v0 with full reorthogonalisation (two classical
// Gram-Schmidt passes against every earlier vector), on `s`, synchronous.
static fct_status lanczos_condition(const fct_plan* p, const double* d_v0, int32_t max_steps,
                                    double tol, double rank_tol, hipStream_t s,
                                    fct_cond_info* out) {
  const int64_t n = p->n;
  const int kmax = (int)std::max<int64_t>(1, std::min<int64_t>(max_steps, n));
  if ((double)(kmax + 1) * (double)n * 8.0 > 32.0 * (1ull << 30)) {
    set_error("condition estimate: %d steps of %lld-vectors exceed 32 GiB", kmax,
              (long long)n);
    return FCT_EINVAL;
  }
  double *V = nullptr, *w = nullptr, *q = nullptr, *part = nullptr, *h = nullptr, *ab = nullptr;
  struct G {
    double** v[6];
    ~G() { for (auto x : v) dfree(*x); }
  } guard{{&V, &w, &q, &part, &h, &ab}};
  const int64_t ldp = kmax + 1;
  FCT_HIP(dalloc(&V, (int64_t)(kmax + 1) * n, nullptr));
  FCT_HIP(dalloc(&w, n, nullptr));
  FCT_HIP(dalloc(&q, std::max<int64_t>(p->M, 1), nullptr));
  FCT_HIP(dalloc(&part, (int64_t)cond_dot_blocks(n) * ldp, nullptr));
  FCT_HIP(dalloc(&h, ldp, nullptr));
  FCT_HIP(dalloc(&ab, 3, nullptr));      // per step: the two passes' h[j], ||w||^2
  std::vector<double> hh((size_t)ldp), alpha, beta;
  // v_1 = v0 / ||v0||
  FCT_HIP(launch_multi_dot(d_v0, n, 1, d_v0, n, part, ldp, h, s));
  FCT_HIP(hipMemcpyAsync(hh.data(), h, sizeof(double), hipMemcpyDeviceToHost, s));
  FCT_HIP(hipStreamSynchronize(s));
  if (!(hh[0] > 0.0) || !std::isfinite(hh[0])) {
    set_error("condition estimate: the start vector is zero or not finite");
    return FCT_EINVAL;
  }
  FCT_HIP(launch_scale(d_v0, 1.0 / std::sqrt(hh[0]), V, n, s));
  double lmin = 0.0, lmax = 0.0, lmin_prev = 0.0, lmax_prev = 0.0;
  int steps = 0;
  for (int j = 0; j < kmax; ++j) {
    const double* vj = V + (int64_t)j * n;
    FCT_HIP(plan_apply_A(p, vj, q, s));
    FCT_HIP(plan_apply_AT(p, q, w, s));
    for (int pass = 0; pass < 2; ++pass) {
      FCT_HIP(launch_multi_dot(V, n, j + 1, w, n, part, ldp, h, s));
      FCT_HIP(launch_orth_update(V, n, j + 1, h, w, n, s));
      FCT_HIP(hipMemcpyAsync(ab + pass, h + j, sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    FCT_HIP(launch_multi_dot(w, n, 1, w, n, part, ldp, ab + 2, s));
    FCT_HIP(hipMemcpyAsync(hh.data(), ab, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    FCT_HIP(hipStreamSynchronize(s));
    const double a = hh[0] + hh[1];
    const double bn = std::sqrt(std::max(hh[2], 0.0));
    alpha.push_back(a);
    steps = j + 1;
    const bool check = steps % 8 == 0 || steps == kmax;
    const double scale = std::max(lmax, std::fabs(a));
    const bool breakdown = !(bn > 1e-13 * std::max(scale, 1e-300)) || steps == n;
    if (check || breakdown) {
      lmin = tridiag_eig(alpha, beta, steps, 0);
      lmax = tridiag_eig(alpha, beta, steps, steps - 1);
      if (breakdown) break;               // T is A^T A on an invariant subspace
      if (tol > 0.0 && steps >= 16 && std::fabs(lmin - lmin_prev) <= tol * lmax &&
          std::fabs(lmax - lmax_prev) <= tol * lmax)
        break;
      lmin_prev = lmin;
      lmax_prev = lmax;
    }
    if (steps == kmax) break;
    beta.push_back(bn);
    FCT_HIP(launch_scale(w, 1.0 / bn, V + (int64_t)(j + 1) * n, n, s));
  }
  fct_cond_info info;
  std::memset(&info, 0, sizeof(info));
  info.lambda_min = lmin;
  info.lambda_max = lmax;
  info.steps = steps;
  info.full_rank = lmin > rank_tol * lmax ? 1 : 0;
  info.kappa = (info.full_rank && lmin > 0.0) ? std::sqrt(lmax / lmin) : HUGE_VAL;
  if (out) *out = info;
  return FCT_OK;
}

fct_status fct_plan_condition(const fct_plan* p, const double* d_v0, int32_t max_steps,
                              double tol, double rank_tol, hipStream_t s, fct_cond_info* out) {
  if (!p || !d_v0) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  if (p->nprob != 1) { set_error("condition estimate needs a single-problem plan"); return FCT_EINVAL; }
  if (max_steps < 1 || !(tol >= 0.0) || !(rank_tol >= 0.0)) {
    set_error("bad max_steps %d, tol or rank_tol", max_steps);
    return FCT_EINVAL;
  }
  return lanczos_condition(p, d_v0, max_steps, tol, rank_tol, s, out);
}

fct_status fct_select_grids(int32_t D, int64_t n, const int32_t* support, int32_t n_cand,
                            const int32_t* candidates, double kappa0, const double* d_v0,
                            int32_t max_steps, double tol, double rank_tol, hipStream_t s,
                            int32_t* out_L, fct_cond_info* out) {
  if (!out_L || !candidates || !support || !d_v0 || n_cand < 1 || !(kappa0 >= 1.0)) {
    set_error("bad argument to fct_select_grids");
    return FCT_EINVAL;
  }
  *out_L = 0;
  fct_cond_info info;
  std::memset(&info, 0, sizeof(info));
  for (int32_t L = 1; L <= n_cand; ++L) {
    fct_plan* p = nullptr;
    fct_status st = fct_plan_create(D, n, support, L, candidates, FCT_PLAN_ALLOW_RANK_DEFICIENT,
                                    s, &p);
    if (st != FCT_OK) return st;
    st = fct_plan_condition(p, d_v0, max_steps, tol, rank_tol, s, &info);
    fct_plan_destroy(p);
    if (st != FCT_OK) return st;
    if (info.full_rank && info.kappa <= kappa0) {
      *out_L = L;
      if (out) *out = info;
      return FCT_OK;
    }
  }
  if (out) *out = info;
  set_error("no prefix of the %d candidate grids reaches kappa <= %g", n_cand, kappa0);
  return FCT_ENOCONV;
}

fct_status fct_apply_A(const fct_plan* p, const double* d_c, double* d_q, hipStream_t s) {
  if (!p || !d_c || !d_q) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  FCT_HIP(plan_apply_A(p, d_c, d_q, s));
  return FCT_OK;
}

fct_status fct_apply_AT(const fct_plan* p, const double* d_r, double* d_s, hipStream_t s) {
  if (!p || !d_r || !d_s) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  FCT_HIP(plan_apply_AT(p, d_r, d_s, s));
  return FCT_OK;
}

// Neighbour lists of the one-reduction solve (built on its first use with
// this workspace): counts on the device, overflow offsets on the host.
static fct_status ensure_neighbours(const fct_plan* p, fct_ws* ws, hipStream_t s) {
  if (ws->d_nb8) return FCT_OK;
  dfree(ws->d_nb_off);
  dfree(ws->d_nb_ovf);
  dfree(ws->d_nb_diag);
  const int64_t n = p->n;
  FCT_HIP(dalloc(&ws->d_nb_off, n + 1, nullptr));
  FCT_HIP(dalloc(&ws->d_nb_diag, n, nullptr));
  FCT_HIP(launch_cg1_count(p->d_cblk, p->ncblk, p->d_rowmap, p->d_seg_off, p->d_perm, p->d_wsign,
                           ws->d_nb_off, ws->d_nb_diag, s));
  std::vector<int32_t> h((size_t)n + 1, 0);
  FCT_HIP(hipMemcpyAsync(h.data(), ws->d_nb_off, sizeof(int32_t) * (size_t)n,
                         hipMemcpyDeviceToHost, s));
  FCT_HIP(hipStreamSynchronize(s));
  int64_t tot = 0;
  for (int64_t j = 0; j < n; ++j) {
    const int32_t c = h[(size_t)j];
    h[(size_t)j] = (int32_t)tot;
    tot += c > kNbSlots ? c - kNbSlots : 0;
    if (tot > INT32_MAX) {
      set_error("one_reduction: neighbour lists exceed 2^31 entries");
      return FCT_EINVAL;
    }
  }
  h[(size_t)n] = (int32_t)tot;
  FCT_HIP(hipMemcpyAsync(ws->d_nb_off, h.data(), sizeof(int32_t) * (size_t)(n + 1),
                         hipMemcpyHostToDevice, s));
  FCT_HIP(dalloc(&ws->d_nb_ovf, tot, nullptr));
  int4* nb8 = nullptr;
  FCT_HIP(dalloc(&nb8, 2 * n, nullptr));
  hipError_t e = launch_cg1_fill(p->d_cblk, p->ncblk, p->d_rowmap, p->d_seg_off, p->d_perm,
                                 p->d_wsign, ws->d_nb_off, (int32_t)n, nb8, ws->d_nb_ovf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dfree(nb8);
    FCT_HIP(e);
  }
  ws->d_nb8 = nb8;
  return FCT_OK;
}

// One iteration: two kernels (CGLS), or one (the one-reduction variant).
static hipError_t launch_iteration(const CglsArgs& a, int rel, hipStream_t s) {
  return a.cg1 ? launch_cg1_iter(a, rel, s) : launch_cgls_iter(a, rel, s);
}

// Graph of `chunk` CGLS iterations for the given arguments (cached per
// precision in the workspace; rebuilt when the chunk or any argument
// changes -- the output, the tolerance, or the plan's block tables, which
// retuning reallocates).  Callers zero CglsArgs before filling it, so the
// byte comparison sees no stale padding.
static fct_status ensure_graph(fct_ws* ws, const CglsArgs& a, int chunk) {
  const int g = a.fp32 ? 1 : 0;
  if (ws->graph_exec[g] && ws->graph_chunk[g] == chunk &&
      std::memcmp(&ws->graph_args[g], &a, sizeof(CglsArgs)) == 0)
    return FCT_OK;
  if (ws->graph_exec[g]) { (void)hipGraphExecDestroy(ws->graph_exec[g]); ws->graph_exec[g] = nullptr; }
  hipGraph_t gr = nullptr;
  FCT_HIP(hipStreamBeginCapture(ws->graph_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int rel = 0; rel < chunk && e == hipSuccess; ++rel) e = launch_iteration(a, rel, ws->graph_stream);
  if (e == hipSuccess) e = launch_cgls_advance(a.state, chunk, ws->graph_stream);
  hipError_t e2 = hipStreamEndCapture(ws->graph_stream, &gr);
  if (e != hipSuccess) { if (gr) (void)hipGraphDestroy(gr); return hip_fail(e, "graph capture", __FILE__, __LINE__); }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture", __FILE__, __LINE__);
  e = hipGraphInstantiate(&ws->graph_exec[g], gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) { ws->graph_exec[g] = nullptr; return hip_fail(e, "hipGraphInstantiate", __FILE__, __LINE__); }
  ws->graph_chunk[g] = chunk;
  ws->graph_args[g] = a;
  return FCT_OK;
}

// CGLS iterations until every problem has stopped or `maxit` iterations ran.
// Chunks of iterations are kept two deep in the stream: while chunk i runs,
// the host reads the per-problem convergence state copied after chunk i-1.
// From each running problem's observed decrease of ||A^T r||^2 the host
// predicts how many iterations remain and shortens the next chunk
// accordingly, so few (early-exiting) launches run after the last problem
// has converged.  Returns the number of iterations enqueued.
constexpr int kWarmChunks = 3;   // short chunks at the start of a CGLS run

static fct_status cgls_loop(const fct_plan* p, fct_ws* ws, const CglsArgs& a, int k0, int maxit,
                            int chunk, bool use_graph, int32_t fused, hipStream_t s,
                            int* queued_out) {
  const int P = p->nprob;
  const int g = a.fp32 ? 1 : 0;
  if (fused > 0) use_graph = false;
  if (use_graph) {
    fct_status st = ensure_graph(ws, a, chunk);
    if (st != FCT_OK) return st;
  }
  int upto[2] = {0, 0};
  int head = 0, inflight = 0, queued = 0;
  std::vector<int> kprev((size_t)P, -1), klast((size_t)P, -1);
  std::vector<double> gprev((size_t)P, 0.0), glast((size_t)P, 0.0);
  int target = maxit;
  // The first chunks are short: iterations queued past a problem's stop are
  // wasted for a single problem (its kernels issue their loads before they
  // read the stop flag), and the remaining-iteration estimate needs two
  // finished chunks, so a run of a few tens of iterations would otherwise
  // queue two full chunks before the first feedback.
  const int warm = std::max(4, chunk / 4);
  int nchunks = 0;
  while (true) {
    while (inflight < 2 && queued < maxit && queued < target) {
      // near the predicted end, queue half of what remains: the estimate
      // tends to run long (CG converges faster near the end), so the last
      // chunks shrink and a stop is seen before many iterations are wasted
      const int remaining = std::min(maxit, target) - queued;
      int want = nchunks < kWarmChunks ? std::min(warm, chunk) : chunk;
      if (target < maxit && remaining <= 2 * chunk)
        want = std::min(want, std::max(warm / 2, (remaining + 1) / 2));
      int c = std::min(want, remaining);
      if (c < 1) c = 1;
      // the one-reduction kernel takes its buffer parity from rel: keep every
      // chunk's base even (only a chunk that ends at maxit may be odd)
      if (a.cg1 && (c & 1) && queued + c < maxit) ++c;
      ++nchunks;
      if (fused > 0) {
        FCT_HIP(launch_cgls_fused(a, c, fused, ws->d_bar, ws->d_bar + 2, s));
        FCT_HIP(launch_cgls_advance(a.state, c, s));
      } else if (use_graph && c == chunk) {
        FCT_HIP(hipGraphLaunch(ws->graph_exec[g], s));
      } else {
        for (int rel = 0; rel < c; ++rel) FCT_HIP(launch_iteration(a, rel, s));
        FCT_HIP(launch_cgls_advance(a.state, c, s));
      }
      queued += c;
      const int sl = (head + inflight) & 1;
      upto[sl] = queued;
      // ring, gamma0 and done of every problem in one copy
      FCT_HIP(hipMemcpyAsync(ws->h_status + (size_t)sl * status_bytes(P), ws->d_status,
                             (size_t)76 * P, hipMemcpyDeviceToHost, s));
      FCT_HIP(hipEventRecord(ws->ev[sl], s));
      ++inflight;
    }
    if (inflight == 0) break;
    const int sl = head;
    FCT_HIP(hipEventSynchronize(ws->ev[sl]));
    head ^= 1;
    --inflight;
    const StatusView hv = status_view(ws->h_status + (size_t)sl * status_bytes(P), P);
    const int32_t* hd = hv.done;
    const double* hr = hv.ring;
    const double* hg0 = hv.gamma0;
    const int k = k0 + upto[sl] - 1;             // last iteration of that chunk
    bool all_done = true;
    int need_max = -1;
    for (int q = 0; q < P; ++q) {
      if (hd[q] != 0) continue;
      all_done = false;
      kprev[q] = klast[q]; gprev[q] = glast[q];
      klast[q] = k; glast[q] = hr[q * 8 + (k & 3)];
      const double g0 = hg0[q];
      if (kprev[q] >= 0 && glast[q] > 0.0 && gprev[q] > glast[q] && g0 > 0.0) {
        const double lrate = (std::log(glast[q]) - std::log(gprev[q])) / (double)(k - kprev[q]);
        const double need = (std::log(a.tol2 * g0) - std::log(glast[q])) / lrate;
        if (std::isfinite(need) && need >= 0.0) {
          const double t = (double)(k - k0) + need + 2.0;    // iterations of this run
          need_max = std::max(need_max, t < (double)maxit ? (int)t + 1 : maxit);
        } else {
          need_max = maxit;
        }
      } else {
        need_max = maxit;
      }
    }
    if (all_done) break;
    target = std::max(need_max, queued + 1);
  }
  FCT_HIP(hipStreamSynchronize(s));
  *queued_out = queued;
  return FCT_OK;
}

// Mean kernel times from back-to-back launches bracketed by HIP events on
// this stream, after the results were read: every problem re-runs
// iteration k (stop test off, its own stop flags untouched), first the row
// kernel, then the column kernel with its coefficient update directed into
// scratch, so d_c keeps the solution.
static fct_status time_kernels(fct_ws* ws, const CglsArgs& a, int k, int P, hipStream_t s,
                               double* rows_us, double* cols_us) {
  constexpr int kReps = 200;
  CglsArgs t = a;
  t.tol2 = 0.0;
  t.c = ws->d_ctmp;
  t.done = ws->d_done_tmp;
  t.state = ws->d_state_tmp;
  FCT_HIP(launch_fill_i32(ws->d_done_tmp, P, 0, s));
  FCT_HIP(launch_cgls_set_base(ws->d_state_tmp, k, s));
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  struct EG { hipEvent_t* e; ~EG() { for (int i = 0; i < 3; ++i) if (e[i]) (void)hipEventDestroy(e[i]); } } eg{ev};
  for (auto& e : ev) FCT_HIP(hipEventCreate(&e));
  FCT_HIP(hipEventRecord(ev[0], s));
  for (int i = 0; i < kReps; ++i)
    FCT_HIP(t.cg1 ? launch_cg1_iter(t, 0, s) : launch_cgls_rows(t, 0, s));
  FCT_HIP(hipEventRecord(ev[1], s));
  if (!t.cg1)
    for (int i = 0; i < kReps; ++i) FCT_HIP(launch_cgls_cols(t, 0, s));
  FCT_HIP(hipEventRecord(ev[2], s));
  FCT_HIP(hipEventSynchronize(ev[2]));
  float m1 = 0.f, m2 = 0.f;
  FCT_HIP(hipEventElapsedTime(&m1, ev[0], ev[1]));
  FCT_HIP(hipEventElapsedTime(&m2, ev[1], ev[2]));
  *rows_us = 1e3 * m1 / kReps;
  *cols_us = t.cg1 ? 0.0 : 1e3 * m2 / kReps;
  return FCT_OK;
}

fct_status fct_solve(const fct_plan* p, const double* d_b, double* d_c,
                     const fct_solve_opts* opts_in, fct_solve_info* info, fct_ws* ws,
                     hipStream_t s) {
  if (!p || !d_b || !d_c) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  fct_status st = check_ws(p, ws);
  if (st != FCT_OK) return st;
  fct_solve_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opts_in) o = *opts_in;
  if (o.mode != FCT_SOLVE_F64 && o.mode != FCT_SOLVE_F32_REFINE && o.mode != FCT_SOLVE_F32) {
    set_error("unknown solve mode %d", o.mode);
    return FCT_EINVAL;
  }
  const bool mixed = o.mode != FCT_SOLVE_F64;
  if (o.maxit <= 0) o.maxit = 4000;
  if (o.check_every <= 0) o.check_every = 32;
  if (o.tol <= 0.0) o.tol = o.mode == FCT_SOLVE_F32 ? 2e-7 : 1e-14;
  if (o.check_every > 4096) o.check_every = 4096;
  if (o.maxit > (1 << 30)) { set_error("maxit too large"); return FCT_EINVAL; }
  if (p->gauss) {
    if (mixed || o.single_kernel > 0) {
      set_error("a Gauss-grid plan is solved in FP64 by the one-reduction CG "
                "(no FP32 modes, no single kernel)");
      return FCT_EINVAL;
    }
    o.one_reduction = 1;
  }
  if (o.one_reduction != 0 &&
      (mixed || p->nprob != 1 || o.single_kernel > 0 || !ws->d_cg)) {
    set_error("one_reduction needs an FP64 solve of a single-problem plan (two-kernel form)");
    return FCT_EINVAL;
  }
  if (o.max_refine <= 0) o.max_refine = 12;
  if (o.inner_tol <= 0.0) o.inner_tol = 1e-5;
  const int P = p->nprob;
  CglsArgs a;
  std::memset(&a, 0, sizeof(a));
  a.rblk = p->d_rblk; a.cblk = p->d_cblk; a.prob = p->d_prob;
  a.units = p->d_units; a.nunits = p->nunits; a.ell16 = p->d_ell16;
  a.rblk32 = p->d_rblk32; a.nrblk32 = p->nrblk32;
  a.lds_bytes = p->lds_cap * (int32_t)sizeof(float);
  a.nrblk = p->nrblk; a.ncblk = p->ncblk; a.nprob = P;
  a.ell = p->d_ell; a.seg_off = p->d_seg_off; a.perm = p->d_perm; a.rowmap = p->d_rowmap;
  a.rq = ws->d_rq; a.ps = ws->d_ps; a.c = d_c; a.fp32 = mixed ? 1 : 0;
  a.part_q = ws->d_part_q; a.part_s = ws->d_part_s;
  a.ring = ws->d_ring; a.gamma0 = ws->d_gamma0; a.done = ws->d_done; a.flags = ws->d_flags;
  a.state = ws->d_state;
  a.r64 = ws->d_r64; a.part_true = ws->d_part_true; a.gtrue0 = ws->d_gtrue;
  a.gtrue = ws->d_gtrue + P; a.outer_done = ws->d_outer;
  for (const auto& pi : p->probs) a.max_K = std::max(a.max_K, pi.K);
  if (P == 1) {
    a.reg_M = (int32_t)p->M;
    a.reg_n = (int32_t)p->n;
    a.reg_K = p->K;
  }
  if (o.one_reduction != 0) {
    st = ensure_neighbours(p, ws, s);
    if (st != FCT_OK) return st;
    a.cg1 = 1;
    a.nb8 = ws->d_nb8;
    a.nb_off = ws->d_nb_off;
    a.nb_ovf = ws->d_nb_ovf;
    a.nb_diag = ws->d_nb_diag;
    a.cg1_n = (int32_t)p->n;
    a.cg1_K = p->K;
    a.cg1_nblk = (int32_t)ceil_div(p->n, kCg1Block);
    a.cg[0] = ws->d_cg;
    a.cg[1] = ws->d_cg + p->n;
    a.cg_part = ws->d_cg_part;
  }
  const int chunk = o.check_every;
  // on request, one problem whose blocks each fit a resident workgroup: one
  // kernel per chunk of iterations (grid barriers between the phases)
  int32_t fused = 0;
  if (P == 1 && o.single_kernel > 0) {
    const int g = mixed ? 1 : 0;
    if (ws->fused[g] < 0) ws->fused[g] = fused_grid(p->device, p->nrblk, p->ncblk, mixed ? 1 : 0);
    fused = ws->fused[g];
  }
  if (fused > 0) FCT_HIP(launch_fill_i32(ws->d_bar, 4, 0, s));

  std::vector<int> iters((size_t)P, 0), rounds((size_t)P, 0);
  const StatusView fin = status_view(ws->h_status + 2 * status_bytes(P), P);
  int32_t* fd = fin.done;
  double* fr = fin.ring;
  double* fg0 = fin.gamma0;
  int total_queued = 0, last_queued = 0;
  if (!mixed) {
    a.tol2 = o.tol * o.tol;
    if (p->gauss) FCT_HIP(launch_gauss_init(a, p->d_wsign, d_b, p->M, o.warm_start != 0, s));
    else FCT_HIP(launch_cgls_init(a, d_b, o.warm_start != 0, s));
    if (a.cg1) FCT_HIP(launch_cg1_init(a, s));
    st = cgls_loop(p, ws, a, 0, o.maxit, chunk, o.use_graph != 0, fused, s, &last_queued);
    if (st != FCT_OK) return st;
    total_queued = last_queued;
    // gamma of the last queued iteration into the ring of every problem that
    // has not stopped (the kernel checks done itself), then the final status
    FCT_HIP(a.cg1 ? launch_cg1_gamma(a, last_queued, s) : launch_cgls_gamma(a, last_queued, s));
    FCT_HIP(hipMemcpyAsync(ws->h_status + 2 * status_bytes(P), ws->d_status, status_bytes(P),
                           hipMemcpyDeviceToHost, s));
    FCT_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < P; ++q) iters[(size_t)q] = fd[q] != 0 ? fd[q] - 1 : last_queued;
  } else {
    // FP32 CGLS rounds, each started from the FP64 residual of the FP64
    // iterate; the outer test is the FP64 normal residual.  A round after
    // the first continues each problem's last direction (reliable update)
    // unless o.restart_rounds is set or the problem broke down.
    a.tol2 = o.inner_tol * o.inner_tol;
    const double tol2_outer = o.tol * o.tol;
    const bool restart = o.restart_rounds != 0;
    if (!o.warm_start) FCT_HIP(launch_fill_f64(d_c, p->n, 0.0, s));
    FCT_HIP(launch_fill_i32(ws->d_outer, P, 0, s));
    FCT_HIP(launch_fill_f64(ws->d_gprev, P, 0.0, s));
    const int nround = o.mode == FCT_SOLVE_F32 ? 1 : o.max_refine;
    int budget = o.maxit;
    int start = 0;
    for (int round = 0; round <= nround; ++round) {
      FCT_HIP(launch_refine(a, d_b, ws->d_gprev, start, round, tol2_outer, s));
      FCT_HIP(hipMemcpyAsync(ws->h_outer, ws->d_outer, sizeof(int32_t) * P, hipMemcpyDeviceToHost, s));
      FCT_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (int q = 0; q < P; ++q) all &= ws->h_outer[q] != 0;
      if (all || round == nround || budget <= 0) break;
      if (o.mode == FCT_SOLVE_F32) a.tol2 = o.tol * o.tol;   // one round to the requested tol
      st = cgls_loop(p, ws, a, start, budget, chunk, o.use_graph != 0, fused, s, &last_queued);
      if (st != FCT_OK) return st;
      total_queued += last_queued;
      budget -= last_queued;
      FCT_HIP(hipMemcpyAsync(ws->h_status + 2 * status_bytes(P), ws->d_status,
                             status_bytes(P), hipMemcpyDeviceToHost, s));
      FCT_HIP(hipStreamSynchronize(s));
      bool any_cont = false;
      for (int q = 0; q < P; ++q) {
        ws->h_gprev[q] = 0.0;
        if (ws->h_outer[q] != 0) continue;
        iters[(size_t)q] += fd[q] != 0 ? fd[q] - 1 - start : last_queued;
        rounds[(size_t)q] = round + 1;
        // stopped at iteration ks after at least one step of this round: the
        // next round continues p_{ks-1} with gamma_{ks-1} from the ring
        const int ks = fd[q] - 1;
        if (!restart && fd[q] != 0 && ws->h_flags[q] == 0 && ks - 1 >= start) {
          const double gp = fr[q * 8 + ((ks - 1) & 3)];
          if (gp > 0.0 && std::isfinite(gp)) { ws->h_gprev[q] = gp; any_cont = true; }
        }
      }
      start = any_cont ? 1 : 0;
      FCT_HIP(hipMemcpyAsync(ws->d_gprev, ws->h_gprev, sizeof(double) * P, hipMemcpyHostToDevice, s));
    }
    FCT_HIP(hipMemcpyAsync(ws->h_outer, ws->d_outer, sizeof(int32_t) * P, hipMemcpyDeviceToHost, s));
    FCT_HIP(hipMemcpyAsync(ws->h_gtrue, ws->d_gtrue, sizeof(double) * 2 * P, hipMemcpyDeviceToHost, s));
    FCT_HIP(hipStreamSynchronize(s));
  }

  if (fused > 0) {
    int32_t abort_flag = 0;
    FCT_HIP(hipMemcpyAsync(&abort_flag, ws->d_bar + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FCT_HIP(hipStreamSynchronize(s));
    if (abort_flag != 0) {
      set_error("single-kernel CGLS: a grid barrier waited too long (workgroups not resident?)");
      return FCT_EDEVICE;
    }
  }
  ws->last.assign((size_t)P, fct_solve_info());
  fct_solve_info agg;
  std::memset(&agg, 0, sizeof(agg));
  agg.problems = P;
  bool nonfinite = false;
  int max_iter = 0;
  for (int q = 0; q < P; ++q) {
    fct_solve_info& r = ws->last[(size_t)q];
    std::memset(&r, 0, sizeof(r));
    const int it = iters[(size_t)q];
    double g0, gk;
    if (!mixed) {
      g0 = fg0[q];
      gk = fr[q * 8 + (it & 3)];
      r.converged = (fd[q] != 0 && ws->h_flags[q] == 0) ? 1 : 0;
      if (fd[q] == 1 && g0 == 0.0) r.converged = 1;   // A^T b = 0: c_0 is exact
    } else {
      g0 = ws->h_gtrue[q];
      gk = ws->h_gtrue[P + q];
      r.converged = (ws->h_outer[q] != 0 && std::isfinite(gk)) ? 1 : 0;
      // pure FP32: its one round met the tolerance on its own (FP32)
      // normal residual, or the FP64 normal residual is below it
      if (o.mode == FCT_SOLVE_F32)
        r.converged = (gk <= o.tol * o.tol * g0 ||
                       (rounds[(size_t)q] > 0 && fd[q] != 0 && ws->h_flags[q] == 0)) ? 1 : 0;
      r.refinements = rounds[(size_t)q];
    }
    r.iterations = it;
    r.normal_residual0 = std::sqrt(g0);
    r.rel_normal_residual = g0 > 0 ? std::sqrt(gk / g0) : 0.0;
    r.problems = 1;
    r.problems_converged = r.converged;
    if (!std::isfinite(g0)) { nonfinite = true; r.converged = 0; r.problems_converged = 0; }
    max_iter = std::max(max_iter, it);
    agg.problems_converged += r.converged;
    agg.refinements = std::max(agg.refinements, r.refinements);
    agg.rel_normal_residual = std::max(agg.rel_normal_residual, r.rel_normal_residual);
    agg.normal_residual0 = std::max(agg.normal_residual0, r.normal_residual0);
  }
  agg.iterations = max_iter;
  agg.converged = agg.problems_converged == P ? 1 : 0;
  if (o.timing && last_queued > 0) {
    // the one-reduction kernel is timed as its first iteration (no ring
    // entries of earlier ones needed)
    st = time_kernels(ws, a, a.cg1 ? 0 : std::max(0, last_queued - 1), P, s, &agg.rows_kernel_us,
                      &agg.cols_kernel_us);
    if (st != FCT_OK) return st;
  }
  if (info) *info = agg;
  if (nonfinite) { set_error("||A^T b|| is not finite"); return FCT_ENONFINITE; }
  if (!agg.converged) {
    set_error("CGLS: %d of %d problems did not converge within %d iterations "
              "(largest relative normal residual %.3e)", P - agg.problems_converged, P,
              total_queued, agg.rel_normal_residual);
    return FCT_ENOCONV;
  }
  return FCT_OK;
}

// Autotuner: times the forward DCT for each LDS tile size and, for a batch,
// the FP32 row kernels for each unit size, on this plan's own shapes, and
// keeps the fastest of each.  Both choices only change the work
// decomposition, never a result.
fct_status fct_plan_tune(fct_plan* p, fct_ws* ws, int32_t dct_mode, hipStream_t s,
                         fct_tune_info* out) {
  if (!p || !ws) { set_error("NULL argument"); return FCT_EINVAL; }
  if (!dev_ok(p)) return FCT_EINVAL;
  fct_status st = check_ws(p, ws);
  if (st != FCT_OK) return st;
  st = check_mode(p, dct_mode);
  if (st != FCT_OK) return st;
  fct_tune_info info;
  std::memset(&info, 0, sizeof(info));
  double* d_x = nullptr;
  double* d_b = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  struct G {
    double** x; double** b; hipEvent_t* e;
    ~G() { dfree(*x); dfree(*b); for (int i = 0; i < 2; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
  } guard{&d_x, &d_b, ev};
  FCT_HIP(dalloc(&d_x, p->total_points, nullptr));
  FCT_HIP(dalloc(&d_b, std::max<int64_t>(p->M, 1), nullptr));
  FCT_HIP(hipMemsetAsync(d_x, 0, sizeof(double) * (size_t)p->total_points, s));
  for (auto& e : ev) FCT_HIP(hipEventCreate(&e));
  auto timed = [&](auto&& body, int reps, double* us) -> fct_status {
    fct_status r = body();                                   // warm-up
    if (r != FCT_OK) return r;
    FCT_HIP(hipEventRecord(ev[0], s));
    for (int i = 0; i < reps; ++i) {
      r = body();
      if (r != FCT_OK) return r;
    }
    FCT_HIP(hipEventRecord(ev[1], s));
    FCT_HIP(hipEventSynchronize(ev[1]));
    float ms = 0.f;
    FCT_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    *us = 1e3 * ms / reps;
    return FCT_OK;
  };

  // DCT tile size and engine
  const int32_t tiles[3] = {1024, 2048, 4096};
  const bool vec_ok = dct_mode != FCT_DCT_BF16X3;
  const bool mat_ok = p->maxdeg <= 31;
  int best_tile = -1, best_engine = -1;
  double best_us = 0.0;
  for (int c = 0; c < 3; ++c) {
    p->dct_tile = tiles[c];
    st = build_dct_levels(p);
    if (st != FCT_OK) return st;
    for (int eng = FCT_ENGINE_VECTOR; eng <= FCT_ENGINE_MATRIX; ++eng) {
      if ((eng == FCT_ENGINE_VECTOR && !vec_ok) || (eng == FCT_ENGINE_MATRIX && !mat_ok)) continue;
      p->dct_engine[dct_mode] = eng;
      double* slot = eng == FCT_ENGINE_VECTOR ? &info.dct_us[c] : &info.dct_matrix_us[c];
      st = timed([&]() { return fct_dct(p, d_x, d_b, dct_mode, ws, s); }, 3, slot);
      if (st != FCT_OK) return st;
      if (best_tile < 0 || *slot < best_us) { best_tile = c; best_engine = eng; best_us = *slot; }
    }
  }
  p->dct_tile = tiles[best_tile];
  p->dct_engine[dct_mode] = best_engine;
  st = build_dct_levels(p);
  if (st != FCT_OK) return st;
  info.dct_tile = p->dct_tile;
  info.dct_engine = best_engine;

  // rows per LDS unit (FP32 rounds of a batch)
  if (p->nunits > 0) {
    const int32_t rows[4] = {4096, 8192, 16384, 32768};
    const int P = p->nprob;
    // every problem running, positive gamma, zero vectors: the timed launches
    // do the work of a full-batch iteration
    FCT_HIP(launch_fill_f64(ws->d_part_s, p->ncblk, 1.0, s));
    FCT_HIP(launch_fill_f64(ws->d_ring, 8 * (int64_t)P, 1.0, s));
    FCT_HIP(launch_fill_f64(ws->d_gamma0, P, 1.0, s));
    FCT_HIP(launch_fill_f64(reinterpret_cast<double*>(ws->d_ps), 2 * p->n, 0.0, s));
    FCT_HIP(launch_fill_i32(ws->d_done_tmp, P, 0, s));
    FCT_HIP(launch_cgls_set_base(ws->d_state_tmp, 1, s));
    int bu = -1;
    for (int c = 0; c < 4; ++c) {
      p->unit_rows = rows[c];
      st = build_blocks(p);
      if (st != FCT_OK) return st;
      CglsArgs a;
      std::memset(&a, 0, sizeof(a));
      a.rblk = p->d_rblk; a.cblk = p->d_cblk; a.prob = p->d_prob;
      a.nrblk = p->nrblk; a.ncblk = p->ncblk; a.nprob = P;
      a.units = p->d_units; a.nunits = p->nunits; a.ell16 = p->d_ell16;
      a.rblk32 = p->d_rblk32; a.nrblk32 = p->nrblk32;
      a.lds_bytes = p->lds_cap * (int32_t)sizeof(float);
      a.ell = p->d_ell; a.seg_off = p->d_seg_off; a.perm = p->d_perm; a.rowmap = p->d_rowmap;
      a.rq = ws->d_rq; a.ps = ws->d_ps; a.fp32 = 1; a.c = ws->d_ctmp;
      a.part_q = ws->d_part_q; a.part_s = ws->d_part_s; a.ring = ws->d_ring;
      a.gamma0 = ws->d_gamma0; a.done = ws->d_done_tmp; a.flags = ws->d_flags;
      a.state = ws->d_state_tmp; a.tol2 = 0.0;
      st = timed([&]() -> fct_status { FCT_HIP(launch_cgls_rows(a, 0, s)); return FCT_OK; }, 10,
                 &info.rows_us[c]);
      if (st != FCT_OK) return st;
      if (bu < 0 || info.rows_us[c] < info.rows_us[bu]) bu = c;
    }
    p->unit_rows = rows[bu];
    st = build_blocks(p);
    if (st != FCT_OK) return st;
    info.unit_rows = p->unit_rows;
  }
  FCT_HIP(hipStreamSynchronize(s));
  if (out) *out = info;
  return FCT_OK;
}

fct_status fct_plan_set_dct_engine(fct_plan* p, int32_t dct_mode, int32_t engine) {
  if (!p) { set_error("NULL plan"); return FCT_EINVAL; }
  if (dct_mode < FCT_DCT_F64 || dct_mode > FCT_DCT_BF16X3) {
    set_error("unknown DCT mode %d", dct_mode);
    return FCT_EINVAL;
  }
  if (engine != FCT_ENGINE_VECTOR && engine != FCT_ENGINE_MATRIX) {
    set_error("unknown DCT engine %d", engine);
    return FCT_EINVAL;
  }
  if (engine == FCT_ENGINE_VECTOR && dct_mode == FCT_DCT_BF16X3) {
    set_error("the split-BF16x3 DCT runs on the matrix cores only");
    return FCT_EINVAL;
  }
  if (engine == FCT_ENGINE_MATRIX && p->maxdeg > 31) {
    set_error("the matrix engine needs every degree <= 31 (plan has %d)", p->maxdeg);
    return FCT_EINVAL;
  }
  p->dct_engine[dct_mode] = engine;
  return FCT_OK;
}

fct_status fct_ws_problem_info(const fct_ws* w, int32_t q, fct_solve_info* out) {
  if (!w || !out || q < 0 || q >= (int32_t)w->last.size()) {
    set_error("bad workspace, problem index or no solve yet");
    return FCT_EINVAL;
  }
  *out = w->last[(size_t)q];
  return FCT_OK;
}

}  // extern "C"
