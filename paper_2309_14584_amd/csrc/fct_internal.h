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
hipError_t launch_alias(const int32_t* S, const int32_t* grids, const int64_t* strides,
                        int D, int64_t n, int K, int64_t* alias, uint64_t* keys,
                        int32_t* vals, hipStream_t s);
hipError_t launch_sort(uint64_t* keys, int32_t* vals, uint64_t* keys_tmp,
                       int32_t* vals_tmp, int64_t L, bool* result_in_tmp, hipStream_t s);
hipError_t launch_segments(const uint64_t* keys, const int32_t* vals, int64_t L,
                           int64_t n, int32_t* block_counts, int64_t nblocks,
                           int32_t* perm, int32_t* seg_off, int64_t* bin_id,
                           int32_t* rowmap, int32_t* row_off, int K, hipStream_t s);
hipError_t launch_tables(int maxdeg, double* nodes, double* cmat, double* emat,
                         hipStream_t s);
// ell[r] = first four entries of row r's run in perm, -1 padded; a row with
// more than four entries stores -(2 + t) in the last slot, t = perm index
// where its remaining entries continue
hipError_t launch_ell(const int32_t* seg_off, const int32_t* perm, int64_t M, int4* ell,
                      hipStream_t s);

// DCT passes
hipError_t launch_dct_level(const DctLevel& lv, const double* in, double* scratch,
                            double* out, const double* mats, const int64_t* bin_id,
                            hipStream_t s);

// sampler: family parameters travel by value in the kernel arguments
struct SampleParams {
  double v[2 * FCT_MAX_DIM + 2];
};
hipError_t launch_sample(int family, const SampleParams& prm, int D, int K,
                         const int32_t* grids, const int64_t* point_off,
                         int64_t total_points, const double* nodes, double* out,
                         hipStream_t s);

// operator
hipError_t launch_apply_A(const int32_t* seg_off, const int32_t* perm, int64_t M,
                          const double* c, double* q, hipStream_t s);
hipError_t launch_apply_AT(const int32_t* rowmap, int K, int64_t n, const double* r,
                           double* out, hipStream_t s);

// CGLS
struct CglsArgs {
  const int32_t* seg_off;
  const int32_t* perm;
  const int4* ell;    // [M] first four columns of each row (see plan)
  const int32_t* rowmap;
  int64_t M, n;
  int32_t K;
  double2* rq;        // [M] (r, q) per row
  double2* ps;        // [n] (p, s) per column
  double* c;          // [n]
  double* part_q;     // [nblocks rows]
  double* part_s;     // [nblocks cols]
  double* hist_gamma; // [kMaxHistory]
  double* hist_alpha; // [kMaxHistory]
  int32_t* state;     // [0] done flag (iteration+1), [1] iteration base
  double tol2;
};
hipError_t launch_cgls_init(const CglsArgs& a, const double* b, bool warm, hipStream_t s);
hipError_t launch_cgls_iter(const CglsArgs& a, int rel, hipStream_t s);
hipError_t launch_cgls_rows(const CglsArgs& a, int rel, hipStream_t s);
hipError_t launch_cgls_cols(const CglsArgs& a, int rel, hipStream_t s);
hipError_t launch_cgls_advance(int32_t* state, int chunk, hipStream_t s);
// hist_gamma[k] = ||s||^2 from the current column partials
hipError_t launch_cgls_gamma(const CglsArgs& a, int k, hipStream_t s);
// timing support: state = (running, base k); then back to the recorded stop
hipError_t launch_cgls_timing_state(int32_t* state, int k, hipStream_t s);
hipError_t launch_cgls_timing_state_restore(int32_t* state, int stop, int breakdown,
                                            hipStream_t s);
int64_t segment_blocks(int64_t L);
int64_t cgls_row_blocks(int64_t M);
int64_t cgls_col_blocks(int64_t n);

}  // namespace fct

// ---- opaque handles ----------------------------------------------------

struct fct_plan {
  int device = 0;
  int32_t D = 0, K = 0;
  int64_t n = 0;
  int64_t M = 0;
  int64_t total_points = 0;
  int64_t max_points = 0;
  int32_t maxdeg = 0;
  std::vector<int32_t> grids;      // [K][D]
  std::vector<int64_t> points;     // [K]
  std::vector<int64_t> point_off;  // [K+1]
  std::vector<int32_t> row_off;    // [K+1]

  int32_t* d_support = nullptr;    // [n][D]
  int32_t* d_grids = nullptr;      // [K][D]
  int64_t* d_strides = nullptr;    // [K][D]
  int64_t* d_point_off = nullptr;  // [K+1]
  int64_t* d_alias = nullptr;      // [K*n]
  int32_t* d_perm = nullptr;       // [K*n]
  int32_t* d_seg_off = nullptr;    // [M+1]
  int64_t* d_bin_id = nullptr;     // [M]
  int32_t* d_rowmap = nullptr;     // [K*n]
  int32_t* d_row_off = nullptr;    // [K+1]
  int4* d_ell = nullptr;           // [M]
  double* d_nodes = nullptr;       // [(maxdeg+1) * 64]
  double* d_cmat = nullptr;        // packed forward DCT-I matrices, degrees 0..maxdeg
  double* d_emat = nullptr;        // packed evaluation matrices
  std::vector<fct::DctLevel> fwd; // forward passes, outer groups first, gather into b
  std::vector<fct::DctLevel> fwd_full; // forward passes writing whole tensors
  std::vector<fct::DctLevel> inv; // inverse passes, inner group first
  int64_t device_bytes = 0;
};

struct fct_ws {
  int device = 0;
  const fct_plan* plan = nullptr;
  double* d_scratch = nullptr;     // [total_points]
  double2* d_rq = nullptr;         // [M]
  double2* d_ps = nullptr;         // [n]
  double* d_ctmp = nullptr;        // [n] coefficient sink of timing launches
  double* d_part_q = nullptr;
  double* d_part_s = nullptr;
  double* d_hist_gamma = nullptr;
  double* d_hist_alpha = nullptr;
  double* d_params = nullptr;      // [2 * FCT_MAX_DIM + 8] sampler parameters
  int32_t* d_state = nullptr;      // [4]
  int32_t* h_state = nullptr;      // pinned [2][4]: state copies of two in-flight chunks
  double* h_gamma = nullptr;       // pinned [6]: per chunk (gamma_last, gamma_0), then final pair
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t graph_stream = nullptr;
  int graph_chunk = 0;
  const double* graph_b = nullptr;
  double* graph_c = nullptr;
  double graph_tol2 = -1.0;
};
