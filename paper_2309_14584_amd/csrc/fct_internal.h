// Internal declarations of libfct (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fct.h"

namespace fct {

constexpr int kBlock = 256;          // threads per workgroup for every kernel
constexpr int kMaxGroupAxes = 12;    // axes transformed together in one DCT pass
constexpr int kTileMax = 4096;       // doubles in one DCT LDS tile (32 KiB)
constexpr int kOuterMinInner = 16;   // contiguous elements per row of an outer-pass tile
constexpr int kKeyBinBits = 44;      // sort key = (grid << 44) | flat bin
constexpr int kSortTile = 1024;      // elements sorted per workgroup before global merges
constexpr int kMaxHistory = 65536;   // CGLS scalar history length (iteration cap)

// Where a DCT pass reads its tile from and writes it to.
enum PassSrc : int32_t { kSrcInput = 0, kSrcScratch = 1, kSrcRows = 2, kSrcOutput = 3 };
enum PassDst : int32_t { kDstScratch = 1, kDstOutput = 2, kDstGather = 3 };

// One axis-group pass over one grid.  The grid tensor is viewed as
// (O, G, I): O outer positions, the G = prod(ext) positions of the group's
// axes, and I inner positions.  A workgroup owns a tile of TO outer
// positions x G x TI inner positions, staged whole in LDS.
struct PassDesc {
  int64_t O, G, I;
  int64_t tiles_i;       // ceil(I / TI)
  int64_t tile_begin;    // first tile index of this descriptor in its launch
  int64_t ntiles;        // tiles of this descriptor
  int64_t point_off;     // offset of the grid's tensor in the point buffers
  int32_t row_begin;     // global rows of the grid (gather / sparse load)
  int32_t row_end;
  int32_t TO, TI;
  int32_t naxes;         // axes in the group (all with extent > 1)
  int32_t src, dst;
  int32_t pad;
  int32_t ext[kMaxGroupAxes];   // extents of the group axes, outer to inner
};

struct DctLevel {
  PassDesc* d_desc = nullptr;
  int32_t ndesc = 0;
  int64_t tiles = 0;
  int32_t emax = 0;      // largest extent among the level's axes
  int32_t tile_max = kTileMax;  // LDS tile elements of this level's passes
  bool rows_io = false;  // some pass gathers (forward) or scatters (inverse) rows
  int32_t* d_tile_row = nullptr;  // tiles entries: first row of each such tile
  int64_t grid[3][2] = {};        // persistent workgroups per DCT mode and engine
};

// Thread-local error message.
void set_error(const char* fmt, ...);
fct_status hip_fail(hipError_t e, const char* what, const char* file, int line);

#define FCT_HIP(call)                                                   \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) return ::fct::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
// Offset of the (N+1) x (N+1) matrix of degree N in the packed tables:
// sum_{j=1}^{N} j^2.
inline __host__ __device__ int64_t mat_offset(int N) {
  return (int64_t)N * (N + 1) * (2 * N + 1) / 6;
}

// ---- kernel launchers (each enqueues on `stream`, returns hipError_t) ----

// plan construction
// wsign (Gauss plans, else nullptr): weight in {-1, 0, 1} of every entry
hipError_t launch_alias(const int32_t* S, const int32_t* grids, const int64_t* strides,
                        int D, int64_t n, int K, int64_t* alias, uint64_t* keys,
                        int32_t* vals, int8_t* wsign, hipStream_t s);
hipError_t launch_sort(uint64_t* keys, int32_t* vals, uint64_t* keys_tmp,
                       int32_t* vals_tmp, int64_t L, bool* result_in_tmp, hipStream_t s);
hipError_t launch_segments(const uint64_t* keys, const int32_t* vals, int64_t L,
                           int64_t n, int32_t* block_counts, int64_t nblocks,
                           int32_t* perm, int32_t* seg_off, int64_t* bin_id,
                           int32_t* rowmap, int32_t* row_off, int K, hipStream_t s);
// cmat32: the forward matrices rounded to FP32 (the FP32 DCT mode's operands)
// Rows by first member (plan flag): keys of the second sort, then each new
// row's (grid, bin)-order index and bin; row permutations of M doubles
// (dst[r] = src[idx[r]], and dst[idx[r]] = src[r])
hipError_t launch_member_keys(const int32_t* rowmap, const int32_t* perm, const int32_t* seg_off,
                             int64_t n, int K, uint64_t* keys, int32_t* vals, hipStream_t s);
hipError_t launch_row_old(const int32_t* perm_new, const int32_t* seg_new,
                          const int32_t* rowmap_old, const int64_t* bin_old, int64_t M, int64_t n,
                          int32_t* row_old, int64_t* bin_new, hipStream_t s);
hipError_t launch_rows_gather(const double* src, const int32_t* idx, int64_t M, double* dst,
                              hipStream_t s);
hipError_t launch_rows_scatter(const double* src, const int32_t* idx, int64_t M, double* dst,
                               hipStream_t s);
// dst[i] = start + i
hipError_t launch_iota_i32(int32_t* dst, int64_t count, int32_t start, hipStream_t s);
// inv[idx[r]] = r for a permutation idx of 0..M-1
hipError_t launch_index_inverse(const int32_t* idx, int64_t M, int32_t* inv, hipStream_t s);
// gauss: Chebyshev-Gauss nodes and the DCT-II instead of Lobatto and DCT-I
hipError_t launch_tables(int maxdeg, double* nodes, double* cmat, float* cmat32, double* emat,
                         int gauss, hipStream_t s);
// ell[r] = first four entries of row r's run in perm, -1 padded; a row with
// more than four entries stores -(2 + t) in the last slot, t = perm index
// where its remaining entries continue
hipError_t launch_ell(const int32_t* seg_off, const int32_t* perm, int64_t M, int4* ell,
                      hipStream_t s);

// DCT passes
// mode: fct_dct_mode; scratch holds doubles (FP64) or floats (other modes)
// engine: fct_dct_engine; mats32: FP32 copy of mats (FP32 mode only; may be
// null otherwise)
hipError_t launch_dct_level(const DctLevel& lv, int mode, int engine, const double* in,
                            void* scratch, double* out, const double* mats, const float* mats32,
                            const int64_t* bin_id, hipStream_t s);
// fills lv.grid: resident workgroups of each mode's pass kernel (cus: compute units)
hipError_t dct_level_grids(DctLevel& lv, int cus);
// fills lv.d_tile_row (allocated by the caller when lv.rows_io)
hipError_t launch_tile_rows(const DctLevel& lv, const int64_t* bin_id, hipStream_t s);

// sampler: family parameters travel by value in the kernel arguments
struct SampleParams {
  double v[2 * FCT_MAX_DIM + 2];
};
// One sampler workgroup covers R rows of one grid's tensor viewed as
// O rows x I inner positions (the trailing axes split .. D-1).
constexpr int kSampleInnerMax = 512;   // inner positions tabulated in LDS
constexpr int kSampleRowsMax = 256;    // rows per workgroup
constexpr int kSamplePoints = 8192;    // target points per workgroup
struct SampleDesc {
  int64_t point_off;     // offset of the grid's tensor
  int64_t O;             // rows
  int64_t tile_begin;    // first workgroup of this grid
  int32_t grid;          // grid index (degrees at grids + grid * D)
  int32_t split;         // first inner axis
  int32_t I;             // inner positions per row (<= kSampleInnerMax, or one axis)
  int32_t R;             // rows per workgroup (R * I <= max(kSamplePoints, I))
};
void make_sample_descs(const std::vector<int32_t>& grids, int D, int K,
                       const std::vector<int64_t>& point_off, std::vector<SampleDesc>* out,
                       int64_t* tiles);
hipError_t launch_sample(int family, const SampleParams& prm, int D, const SampleDesc* descs,
                         int ndesc, int64_t tiles, const int32_t* grids, const double* nodes,
                         double* out, hipStream_t s);

// evaluation of the expansion at arbitrary points (nk = max support entry + 1)
constexpr int kEvalLdsMax = 160 * 1024;   // LDS of one workgroup
int eval_chunk(int D, int nk);            // 0: the per-point table does not fit
size_t eval_lds_bytes(int D, int nk, int chunk);
// support slices for m points given scratch_elems doubles of scratch (>= 1)
int eval_slices(int64_t n, int D, int nk, int64_t m, int64_t scratch_elems);
hipError_t launch_eval(const int32_t* support, const double* c, int64_t n, int D, int nk,
                       int64_t m, const double* X, double* f, int slices, double* scratch,
                       hipStream_t s);

// condition estimate (Lanczos on A^T A): part holds cond_dot_blocks(n) x ldp
// doubles; out[i] = sum_e X[i][e] w[e] for i < cnt (cnt <= ldp)
int cond_dot_blocks(int64_t n);
hipError_t launch_multi_dot(const double* X, int64_t ld, int cnt, const double* w, int64_t n,
                            double* part, int64_t ldp, double* out, hipStream_t s);
// w -= sum_{i < cnt} X[i] h[i]
hipError_t launch_orth_update(const double* X, int64_t ld, int cnt, const double* h, double* w,
                              int64_t n, hipStream_t s);
hipError_t launch_scale(const double* x, double a, double* y, int64_t n, hipStream_t s);

// Work decomposition of the CGLS kernels.  A plan holds one or more
// independent problems (a batch); every workgroup of the row (column)
// kernel covers up to kBlock rows (columns) of a single problem.
struct RowBlock {
  int32_t prob;       // problem index
  int32_t row0;       // first global row of the block
  int32_t row_end;    // one past the last row of the block
  int32_t cblk_off;   // the problem's column blocks [cblk_off, cblk_off + ncblk)
  int32_t ncblk;
  int32_t first;      // 1 for the problem's first row block (writes its scalars)
  int32_t pslot;      // slot of this block's partials of ||q||^2 (4 per block)
  int32_t pad1;
};
struct ColBlock {
  int32_t prob;
  int32_t col0;       // first global column of the block
  int32_t col_end;
  int32_t col_off;    // first global column of the problem
  int32_t rblk_off;   // first slot of the problem's row partials
  int32_t nrblk;      // row partials of the FP64 row kernel
  int32_t K;          // grids of the problem
  int32_t n;          // columns of the problem
  int32_t rmap_off;   // offset of the problem's rowmap block [K][n]
  int32_t first;
  int32_t pad0, pad1;
};
// In a batch, FP32 rounds compute q = A p for every problem whose p vector
// fits in LDS with one workgroup of kLdsBlock threads per unit of up to
// kUnitRows rows: the unit stages p once and gathers from LDS.
constexpr int kLdsBlock = 1024;
constexpr int kUnitRows = 16384;   // default rows per unit (a multiple of kLdsBlock)
struct RowUnit {
  int32_t prob;
  int32_t row0, row_end;   // global rows of the unit
  int32_t first;           // 1 for the problem's first unit
  int32_t pslot;           // first row-partial slot of the unit (its first row block)
  int32_t cblk_off, ncblk; // the problem's column partials
  int32_t col_off, n;      // the problem's columns
  int32_t pad0, pad1, pad2;
};
struct ProbInfo {
  int32_t row_off, M;     // global rows of the problem
  int32_t col_off, n;     // global columns
  int32_t K, rmap_off;    // grids, rowmap (and perm) offset
  int32_t rblk_off, nrblk;
  int32_t cblk_off, ncblk;
  int32_t grid_off;       // first grid of the problem
  int32_t pad0;
};

// operator
hipError_t launch_apply_A(const int32_t* seg_off, const int32_t* perm, int64_t M,
                          const double* c, double* q, hipStream_t s);
hipError_t launch_apply_AT(const ColBlock* cblk, int64_t ncblk, const int32_t* rowmap,
                           const double* r, double* out, hipStream_t s);

// CGLS
struct CglsArgs {
  const RowBlock* rblk;
  const ColBlock* cblk;
  const ProbInfo* prob;
  int64_t nrblk, ncblk;
  int32_t nprob;
  const int4* ell;    // [M] first four columns of each row (see plan)
  const int32_t* seg_off;
  const int32_t* perm;
  const int32_t* rowmap;
  void* rq;           // [M] (r, q) per row as double2; FP32 rounds: q as float
  void* ps;           // [n] (p, s) per column: double2, or float2 when fp32
  int32_t fp32;       // nonzero: FP32 storage of (r, q) and (p, s)
  double* c;          // [n]
  double* part_q;     // [4 nrblk] ||q||^2 per wave of each row block
  double* part_s;     // [ncblk]
  double* ring;       // [nprob][8]: gamma ring (k mod 4), alpha ring (k mod 4)
  double* gamma0;     // [nprob] ||A^T r_0||^2
  int32_t* done;      // [nprob] iteration+1 at which the problem stopped, 0 while running
  int32_t* flags;     // [nprob] 1 = breakdown (A p = 0)
  int32_t* state;     // [0] iteration base
  double tol2;
  // mixed precision (FP32 rounds refined in FP64)
  double* r64;        // [M] FP64 residual b - A c of the round
  double* part_true;  // [ncblk] partials of the FP64 normal residual
  double* gtrue0;     // [nprob] FP64 ||A^T r||^2 of round 0
  double* gtrue;      // [nprob] FP64 ||A^T r||^2 of the latest round
  int32_t* outer_done;// [nprob] round+1 at which the problem finished, 0 while refining
  // FP32 rounds of a batch: LDS units, and the row blocks of the other problems
  const uint4* ell16;   // [M] 16-bit local-column ELL of the units' rows
  const RowUnit* units;
  int64_t nunits;
  const RowBlock* rblk32;
  int64_t nrblk32;
  int32_t lds_bytes;  // dynamic LDS of the unit kernel
  // one-reduction CG (one problem, FP64): (r, w, s, p) per column in two
  // buffers by iteration parity, [2 parities][gamma, delta][cg1_nblk] partials,
  // and each column's neighbour list (the other members of its K rows, in
  // grid order, repeated when two columns share several rows): the first
  // eight in nb8 ([2][n] int4, -1 padded), the rest in
  // nb_ovf[nb_off[j] .. nb_off[j+1])
  int32_t cg1;
  double4* cg[2];
  double* cg_part;
  const int4* nb8;
  const int32_t* nb_off;
  const int32_t* nb_ovf;
  const int32_t* nb_diag;   // [n] diagonal of A^T A
  // a single problem's row and column blocks are regular (block b covers
  // [b kBlock, min(end, (b + 1) kBlock))): its rows, columns and grids, so
  // the iteration kernels form their descriptors instead of loading them
  // (0: read the block tables)
  int32_t reg_M, reg_n, reg_K;
  int32_t max_K;      // most grids of a problem (column-kernel batch depth)
  int32_t cg1_n;      // columns
  int32_t cg1_K;      // grids
  int32_t cg1_nblk;   // one-wave workgroups (kCg1Block columns each)
};
constexpr int kCg1Block = 64;
constexpr int kDeepColsK = 64;    // above: the FP64 column kernel loads 16 grids at a time
constexpr int kNbSlots = 8;
hipError_t launch_cgls_init(const CglsArgs& a, const double* b, bool warm, hipStream_t s);
// one-reduction CG: init after launch_cgls_init, one kernel per iteration
hipError_t launch_cg1_init(const CglsArgs& a, hipStream_t s);
// neighbour lists of a single-problem plan: counts (other members over the
// K rows of each column) into cnt[n], then the lists from the overflow
// offsets off[n+1] (entries beyond the eighth)
// (w: entry weights of a Gauss plan, else nullptr; diag[n] gets the
// diagonal of A^T A)
hipError_t launch_cg1_count(const ColBlock* cblk, int64_t ncblk, const int32_t* rowmap,
                            const int32_t* seg_off, const int32_t* perm, const int8_t* w,
                            int32_t* cnt, int32_t* diag, hipStream_t s);
hipError_t launch_cg1_fill(const ColBlock* cblk, int64_t ncblk, const int32_t* rowmap,
                           const int32_t* seg_off, const int32_t* perm, const int8_t* w,
                           const int32_t* off, int32_t n, int4* nb8, int32_t* ovf,
                           hipStream_t s);
// A c and A^T r of a Gauss plan (entry weights w [K][n]), and the start of
// its solve: r_0 = b - A c_0 into a.r64, s_0 = A^T r_0 into a.ps.y, state reset
hipError_t launch_apply_A_signed(const int32_t* seg_off, const int32_t* perm, const int8_t* w,
                                 int64_t M, int64_t n, const double* c, double* q,
                                 hipStream_t s);
hipError_t launch_apply_AT_signed(const int32_t* rowmap, const int8_t* w, int32_t K, int64_t n,
                                  const double* r, double* out, hipStream_t s);
hipError_t launch_gauss_init(const CglsArgs& a, const int8_t* w, const double* b, int64_t M,
                             bool warm, hipStream_t s);
hipError_t launch_cg1_iter(const CglsArgs& a, int rel, hipStream_t s);
hipError_t launch_cg1_gamma(const CglsArgs& a, int k, hipStream_t s);
hipError_t launch_cgls_iter(const CglsArgs& a, int rel, hipStream_t s);
hipError_t launch_cgls_rows(const CglsArgs& a, int rel, hipStream_t s);
hipError_t launch_cgls_cols(const CglsArgs& a, int rel, hipStream_t s);
hipError_t launch_cgls_advance(int32_t* state, int chunk, hipStream_t s);
// ring entry k = ||s||^2 of the current column partials, for running problems
hipError_t launch_cgls_gamma(const CglsArgs& a, int k, hipStream_t s);
hipError_t launch_cgls_set_base(int32_t* state, int base, hipStream_t s);
// columns of p a unit can stage (0: no LDS units on this device)
int32_t lds_unit_capacity(int device);
// single-kernel iterations of one problem: workgroups (0: not possible) and launch
int32_t fused_grid(int device, int64_t nrblk, int64_t ncblk, int fp32);
hipError_t launch_cgls_fused(const CglsArgs& a, int iters, int32_t grid, int* bar, int* abort,
                             hipStream_t s);
hipError_t launch_fill_i32(int32_t* v, int n, int value, hipStream_t s);
hipError_t launch_fill_f64(double* v, int64_t n, double value, hipStream_t s);
// one refinement round's start: r64 = b - A c, (p, s) = (0, A^T r), FP64 test
hipError_t launch_refine(const CglsArgs& a, const double* b, const double* gprev, int start,
                         int round, double tol2_outer, hipStream_t s);
int64_t segment_blocks(int64_t L);

// batch construction: dst[i] = src[i] + add (i < count)
hipError_t launch_copy_add_i32(int32_t* dst, const int32_t* src, int64_t count, int32_t add,
                               hipStream_t s);
// 16-bit local-column ELL (8 slots) of rows [row0, row0 + nrows) of one problem
hipError_t launch_ell16(const int32_t* seg_off, const int32_t* perm, int32_t row0, int32_t nrows,
                        int32_t col_off, uint4* out, hipStream_t s);
// ELL entries shifted to global columns (col_add) and perm positions (perm_add)
hipError_t launch_copy_ell(int4* dst, const int4* src, int64_t count, int32_t col_add,
                           int32_t perm_add, hipStream_t s);

}  // namespace fct

// ---- opaque handles ----------------------------------------------------

struct fct_plan {
  int device = 0;
  int32_t nprob = 1;               // problems (1, or the size of a batch)
  int32_t D = 0;                   // dimension (largest over a batch)
  int32_t K = 0;                   // grids over all problems
  int64_t n = 0;                   // columns over all problems
  int64_t M = 0;                   // rows over all problems
  int64_t total_points = 0;
  int64_t max_points = 0;
  int32_t maxdeg = 0;
  int32_t smax = 0;                // largest support entry (single problem)
  int32_t gauss = 0;               // Gauss grids / DCT-II operator (single problem)
  int32_t rows_by_member = 0;      // rows ordered by first member (in a batch: some problem's)
  std::vector<int32_t> grid_D;     // [K] dimension of each grid's problem
  std::vector<int64_t> grid_goff;  // [K+1] offsets of each grid's degrees in `grids`
  std::vector<int32_t> grids;      // degrees, grid after grid
  std::vector<int64_t> points;     // [K]
  std::vector<int64_t> point_off;  // [K+1]
  std::vector<int32_t> row_off;    // [K+1]
  std::vector<fct::ProbInfo> probs;      // [nprob]
  std::vector<int64_t> prob_point_off;   // [nprob+1]
  int64_t nrblk = 0, ncblk = 0;

  int32_t* d_support = nullptr;    // [n][D]      (single problem only)
  int64_t* d_strides = nullptr;    // [K][D]      (single problem only)
  int64_t* d_alias = nullptr;      // [K*n]       (single problem only)
  int8_t* d_wsign = nullptr;       // [K*n]       entry weights of a Gauss plan
  int64_t* d_bin_dct = nullptr;    // [M] bins in (grid, bin) row order (rows_by_member plans)
  int32_t* d_row_old = nullptr;    // [M] (grid, bin)-order index of each row (rows_by_member)
  int32_t* d_row_new = nullptr;    // [M] its inverse: the row of each (grid, bin)-order index
  int32_t* d_grids = nullptr;      // degrees, as `grids`
  int64_t* d_point_off = nullptr;  // [K+1]
  fct::SampleDesc* d_sdesc = nullptr;  // [K] sampler split of each grid (single problem)
  int64_t sample_tiles = 0;        // sampler workgroups
  int32_t* d_perm = nullptr;       // [sum K n]   global columns
  int32_t* d_seg_off = nullptr;    // [M+1]       offsets into perm
  int64_t* d_bin_id = nullptr;     // [M]
  int32_t* d_rowmap = nullptr;     // [sum K n]   global rows, block [K_p][n_p] per problem
  int32_t* d_row_off = nullptr;    // [K+1]
  int4* d_ell = nullptr;           // [M]
  fct::RowBlock* d_rblk = nullptr; // [nrblk]
  fct::RowUnit* d_units = nullptr; // [nunits]  FP32 rounds of a batch: LDS units
  uint4* d_ell16 = nullptr;        // [M]       16-bit ELL of the units' rows
  fct::RowBlock* d_rblk32 = nullptr; // [nrblk32] FP32 rounds: row blocks outside the units
  int64_t nunits = 0, nrblk32 = 0;
  int32_t lds_cap = 0;             // columns a unit stages (floats in LDS)
  int32_t dct_tile = fct::kTileMax;     // tuned: LDS tile elements of the DCT passes
  int32_t dct_engine[3] = {FCT_ENGINE_VECTOR, FCT_ENGINE_VECTOR, FCT_ENGINE_MATRIX};  // per mode
  int32_t unit_rows = fct::kUnitRows;   // tuned: rows per LDS unit
  int64_t block_bytes = 0;         // device bytes of the block descriptors, units and ell16
  fct::ColBlock* d_cblk = nullptr; // [ncblk]
  fct::ProbInfo* d_prob = nullptr; // [nprob]
  double* d_nodes = nullptr;       // [(maxdeg+1) * 64]
  double* d_cmat = nullptr;        // packed forward DCT-I matrices, degrees 0..maxdeg
  float* d_cmat32 = nullptr;       // the same rounded to FP32
  double* d_emat = nullptr;        // packed evaluation matrices
  std::vector<fct::DctLevel> fwd; // forward passes, outer groups first, gather into b
  std::vector<fct::DctLevel> fwd_full; // forward passes writing whole tensors
  std::vector<fct::DctLevel> inv; // inverse passes, inner group first
  int64_t device_bytes = 0;
};

// Layout of the solve status block of nprob problems (bytes).
inline size_t status_bytes(int64_t P) { return (size_t)80 * (size_t)P; }
struct StatusView {
  double* ring;      // [P][8]
  double* gamma0;    // [P]
  int32_t* done;     // [P]
  int32_t* flags;    // [P]
};
inline StatusView status_view(unsigned char* base, int64_t P) {
  return {reinterpret_cast<double*>(base), reinterpret_cast<double*>(base + 64 * P),
          reinterpret_cast<int32_t*>(base + 72 * P), reinterpret_cast<int32_t*>(base + 76 * P)};
}

struct fct_ws {
  int device = 0;
  const fct_plan* plan = nullptr;
  double* d_scratch = nullptr;     // [total_points]
  double2* d_rq = nullptr;         // [M]
  double2* d_ps = nullptr;         // [n]
  double* d_ctmp = nullptr;        // [n] coefficient sink of timing launches
  double* d_r64 = nullptr;         // [M]
  double* d_part_true = nullptr;   // [ncblk]
  double* d_gtrue = nullptr;       // [2][nprob] reference and latest FP64 normal residual
  int32_t* d_outer = nullptr;      // [nprob]
  int32_t* h_outer = nullptr;      // pinned [nprob]
  double* h_gtrue = nullptr;       // pinned [2][nprob]
  double* d_gprev = nullptr;       // [nprob] gamma before the previous round stopped (0: restart)
  double* h_gprev = nullptr;       // pinned [nprob]
  double* d_part_q = nullptr;      // [4 nrblk] per-wave partials of ||q||^2
  double* d_part_s = nullptr;      // [ncblk]
  double4* d_cg = nullptr;         // [2][n] one-reduction CG state (single problem)
  double* d_cg_part = nullptr;     // [2][2][ceil(n/kCg1Block)] its partials
  int4* d_nb8 = nullptr;           // [2][n] neighbour lists (built on first use)
  int32_t* d_nb_off = nullptr;     // [n+1]
  int32_t* d_nb_ovf = nullptr;     // [max(1, overflow entries)]
  int32_t* d_nb_diag = nullptr;    // [n]
  double* d_bperm = nullptr;       // [M] rows in (grid, bin) order (rows_by_member plans)
  // per-problem solve status, one allocation so that a chunk check copies it
  // to the host at once: ring [nprob][8], gamma0 [nprob] (doubles), then
  // done [nprob], flags [nprob] (int32); the four pointers are views of it
  unsigned char* d_status = nullptr;
  double* d_ring = nullptr;
  double* d_gamma0 = nullptr;
  int32_t* d_done = nullptr;
  int32_t* d_flags = nullptr;
  int32_t* d_done_tmp = nullptr;   // [nprob] (timing launches)
  int32_t* d_state = nullptr;      // [4]
  int32_t* d_state_tmp = nullptr;  // [4]   (timing launches)
  int32_t* d_bar = nullptr;        // [4]   grid barrier (count, generation), abort flag
  int32_t fused[2] = {-1, -1};     // single-kernel workgroups per precision (-1: not yet known)
  // pinned host copies of the status block: two in-flight chunk checks,
  // then the final state (slot 2); h_flags is slot 2's flags
  unsigned char* h_status = nullptr;   // [3][status_bytes(nprob)]
  int32_t* h_flags = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};   // FP64, FP32 iteration chunks
  hipStream_t graph_stream = nullptr;
  int graph_chunk[2] = {0, 0};
  fct::CglsArgs graph_args[2];     // arguments the cached graphs were captured with
  // per-problem results of the last solve
  std::vector<fct_solve_info> last;
};
