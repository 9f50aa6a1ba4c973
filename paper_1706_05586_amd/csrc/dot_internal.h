// Internal declarations shared by the dotpath HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/dotpath.h"

namespace dot {

// pairs per chunk of the contraction (a chunk never spans two RBFs)
constexpr int64_t DOT_PAIR_CHUNK = 512;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define DOT_FAIL(code, ...)          \
  do {                               \
    ::dot::set_error(__VA_ARGS__);   \
    return (code);                   \
  } while (0)

#define DOT_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::dot::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                      \
      return DOT_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

#define DOT_LAUNCH_CHECK() DOT_HIP(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Block-wide exclusive prefix sum of a 0/1 flag over 256 threads; returns the
// position and sets *total.  Order follows threadIdx.x, so compaction is
// deterministic.
__device__ __forceinline__ int block_scan_flag256(int flag, int* s_wave, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(flag);
  const int before = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) s_wave[wave] = __popcll(bal);
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) off += s_wave[w];
    tot += s_wave[w];
  }
  *total = tot;
  return off + before;
}

// ---------------------------------------------------------------- handle
struct GridDims {
  int dim;
  int nx, ny, nz;
  int64_t nxy, N;
  double h;
  double hd;   // h^d (cell volume)
};

struct dot_state_arrays;

// ---------------------------------------------------------------- multigrid
// Geometric hierarchy for the V-cycle preconditioner (2D and 3D grids):
// level l + 1 aggregates 2 x 2 x 2 cells of level l (2 x 2 in 2D; the last
// aggregate of an odd side is one cell thick along it) and is the same
// finite-volume discretization on the coarse cells, with D and mu averaged
// over the children.  Every level is kept in the symmetrically scaled form
// (unit diagonal): couplings to +x, +y, +z in binary64 and binary32.
constexpr int DOT_MG_MAXLEV = 12;

struct MgLevel {
  GridDims g;
  // level 0 points at the operator's arrays; coarse levels own theirs
  double* D = nullptr;     // diffusion
  double* mu = nullptr;    // absorption (mass h^d mu)
  double* cx = nullptr;
  double* cy = nullptr;
  double* cz = nullptr;
  double* b0 = nullptr;
  double* diag = nullptr;
  double* sd = nullptr;    // sqrt(diag)
  float* sd32 = nullptr;   // sd rounded to binary32 (owned on every level)
  double* sx = nullptr;
  double* sy = nullptr;
  double* sz = nullptr;
  float* sx32 = nullptr;
  float* sy32 = nullptr;
  float* sz32 = nullptr;
  // all but the coarsest: sd(cell) / sd_{l+1}(parent), the prolongation weight
  double* q = nullptr;
  float* q32 = nullptr;
};

}  // namespace dot

struct dot_op {
  dot::GridDims g;
  int bc[6];
  int device;
  // binary64 operator (unscaled): face coefficients to the +axis neighbour
  // (zero on the last layer), boundary diagonal b0, full diagonal.
  double* cx = nullptr;
  double* cy = nullptr;
  double* cz = nullptr;
  double* b0 = nullptr;
  double* diag = nullptr;
  // symmetric Jacobi scaling: sd = sqrt(diag); scaled coefficients
  // T / (sd_c sd_c'), unit diagonal (binary64 and binary32 copies).
  double* sd = nullptr;
  double* sx = nullptr;
  double* sy = nullptr;
  double* sz = nullptr;
  float* sx32 = nullptr;
  float* sy32 = nullptr;
  float* sz32 = nullptr;
  // diffusion from the level set (dot_pals_mua_diffusion): D0 then holds
  // D(theta), Dbuild the coefficient given to dot_build_operator, restored by
  // dot_pals_mua and dot_set_mua
  bool diff_mode = false;
  double mus_in = 0.0, mus_out = 0.0;
  double* Dbuild = nullptr;
  // contraction rows and pairs with the face terms of dA/dp (diffusion mode):
  // 1 + 2 dim rows per band cell (the cell, then its faces -x, +x, -y, +y,
  // -z, +z): row cell, neighbour across the face (-1: none) and the weight of
  // the adjoint-field difference; every (RBF, cell) pair repeated per row
  int32_t* vrow_cell = nullptr;
  int32_t* vrow_nbr = nullptr;
  double* vrow_w = nullptr;
  int64_t vrow_cap = 0, n_vrows = 0;
  int32_t* vpair_band = nullptr;
  double* vpair_g = nullptr;
  float* vpair_g32 = nullptr;
  int64_t vpair_cap = 0, n_vpairs = 0;
  int64_t* vchunk_begin = nullptr;
  int32_t* vrbf_chunk0 = nullptr;
  int64_t vchunk_cap = 0, n_vchunks = 0;
  int vrbf_cap = 0;
  // level-set state from the last dot_pals_mua call
  double* phi = nullptr;
  double* theta = nullptr;      // copy of theta (m0 x (2 + dim))
  int64_t theta_cap = 0;
  dot_pals pals{};
  bool have_pals = false;
  // per-RBF cell lists where d mu / d p is nonzero: cells sorted by RBF then
  // cell index; rbf_start[m]..rbf_start[m+1]; chunk table for the contraction
  int32_t* pair_cell = nullptr;
  int64_t pair_cap = 0;
  int64_t n_pairs = 0;
  int64_t* rbf_start = nullptr;  // device, m0 + 1
  int32_t* chunk_rbf = nullptr;  // device, per chunk: RBF index
  int64_t* chunk_begin = nullptr;  // device, per chunk: first pair
  int32_t* rbf_chunk0 = nullptr;   // device, m0 + 1: first chunk of each RBF
  int64_t chunk_cap = 0;
  int64_t n_chunks = 0;            // chunks hold at most DOT_PAIR_CHUNK pairs
  int64_t rbf_cap = 0;
  int64_t* rbf_sub = nullptr;    // device: per (RBF, scan range) counts, then starts
  int64_t rbf_sub_cap = 0;
  // per pair: h^d d mu / d p of its RBF's active parameters (pair-major), and
  // its row in the band-cell list (every cell of any list, in cell order),
  // through which the contraction reads U and Z rows packed cell-major
  double* pair_g = nullptr;
  int64_t pair_g_cap = 0;        // doubles
  float* pair_g32 = nullptr;     // the same values rounded to binary32
  int64_t pair_g32_cap = 0;
  int32_t* pair_band = nullptr;
  int64_t pair_band_cap = 0;
  int32_t* band_idx = nullptr;   // N: band row of a cell, -1 elsewhere
  int32_t* band_cells = nullptr; // cell of each band row
  int64_t band_cap = 0;
  int64_t n_band = 0;            // valid once band_pending is false (band_count)
  bool band_pending = false;     // n_band is still on its way to pinned_band
  hipEvent_t band_ev = nullptr;  // recorded after that copy
  int64_t* pinned_band = nullptr;
  // pinned staging of the per-RBF list tables, reused once lists_ev (the
  // previous upload) has completed
  char* stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t lists_ev = nullptr;
  bool lists_pending = false;
  int64_t* band_part = nullptr;  // per 2048-cell block: band cells before it
  int64_t band_part_cap = 0;
  // optode cell lists on the device, keyed by the host list's content (the
  // same sources and detectors come back every step, so a repeated list
  // costs no copy): the cells in the caller's order, the points sorted
  // stably by cell, the distinct cells and each one's run of points
  struct CellList {
    std::vector<int32_t> key;     // the host list
    int32_t* dev = nullptr;       // [n] cells, [n] sorted points, [n_u] cells, [n_u + 1] runs
    int64_t cap = 0;              // int32 slots of dev
    int n = 0, n_u = 0;
    uint64_t used = 0;            // last use, for replacement
  };
  CellList cell_lists[4];
  uint64_t cell_clock = 0;
  // small device/pinned staging
  double* small_dev = nullptr;    // small device scratch (scalars)
  void* prof = nullptr;           // kernel timing state (solve.hip)
  int32_t* pinned = nullptr;      // pinned host mailbox (counters/flags)
  double* pinned_d = nullptr;     // pinned host doubles (misfit, small results)
  hipEvent_t poll_ev[2] = {};     // the solver's pending flag snapshots
  // multigrid hierarchy (levels 0 .. mg_nlev - 1; mg_nlev < 2: not available)
  double* D0 = nullptr;           // copy of the frozen diffusion field
  double* mu0 = nullptr;          // absorption of the current diagonal
  int mg_nlev = 0;
  bool mg_ok = false;             // every level's diagonal positive and finite
  int* mg_flag = nullptr;         // device flag of that check
  dot::MgLevel mg[dot::DOT_MG_MAXLEV];
};

namespace dot {

int validate_grid(const dot_grid* g, GridDims* out, const char** why);
void destroy_profile(dot_op* op);
int profile_begin(dot_op* op, int kind, hipStream_t s, hipEvent_t* e0, hipEvent_t* e1,
                  unsigned long long** cols);
int profile_end(dot_op* op, int kind, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
constexpr int kPinnedInts = 4 * DOT_MAX_COLUMNS + 64;
// the device copy of an optode cell list (host, n entries, each in [0, N));
// *out is valid until the next call with a different list
int cells_on_device(dot_op* op, int n, const int32_t* cells_host, hipStream_t s,
                    const dot_op::CellList** out);
// after the pair lists of dot_pals_mua: per-pair d mu / d p and band rows
int jac_prepare(dot_op* op, hipStream_t s);
// rows of the band lists (waits for the count of the last jac_prepare)
int64_t band_count(dot_op* op);
// the face rows and pairs of diffusion mode (after jac_prepare)
int jac_prepare_faces(dot_op* op, hipStream_t s);
// multigrid: levels of the grid (0 or 1: none), hierarchy (re)build after
// the diagonal changed, and one V-cycle z = M^-1 r on the scaled system
int mg_levels_for(const GridDims& g, GridDims* levels);
int mg_refresh(dot_op* op, hipStream_t s);
void mg_free(dot_op* op);

// bfloat16 storage of V-cycle vectors whose arithmetic is binary32: the
// upper half of the binary32 pattern, rounded to nearest even when stored
struct bf16s {
  unsigned short u;
};

// Work vectors of one V-cycle: per level l >= 1 a right-hand side, an
// iterate and a result (N_l columns apart); on level 0 one iterate, or two
// when the vectors are stored in a narrower type than the arithmetic (the
// right-hand side and the result are the caller's).
template <typename T>
struct MgWork {
  int nlev = 0;
  T* b[DOT_MG_MAXLEV] = {};
  T* x[DOT_MG_MAXLEV] = {};
  T* z[DOT_MG_MAXLEV] = {};
  int64_t ld[DOT_MG_MAXLEV] = {};
};
// bytes of MgWork<T> for k columns on op's hierarchy (0 without one);
// carve the vectors from base (256-aligned); ld0: the level-0 stride
// (level0_iterates: 1, or 2 for narrower storage)
size_t mg_work_bytes(const dot_op* op, int k, int64_t ld0, size_t elem, int level0_iterates = 1);
template <typename T>
void mg_work_layout(const dot_op* op, int k, int64_t ld0, char* base, MgWork<T>* w,
                    int level0_iterates = 1);
// algorithmic bytes per column of one V-cycle: the level-0 right-hand side
// and result in elements of elem0 bytes, every other vector of elem bytes
double mg_cycle_stream_bytes(const dot_op* op, size_t elem0, size_t elem);
// partial slots per column of the level-0 smoothing kernel (the dot (r, z))
int mg_partial_slots(const dot_op* op, int k);
// z0 = V-cycle applied to r0 (both k columns ld0 apart; columns outside
// `active` are skipped); partial[0][j][slot] receives r0_j . z0_j
// (prof_cols: optional, receives the number of active columns)
// (T: the arithmetic and r0, z0; S: the stored work vectors, T or bf16s)
template <typename T, typename S>
int mg_vcycle(dot_op* op, const MgWork<S>& w, int k, const T* r0, int64_t ld0, T* z0,
              const int* active, double* partial, hipStream_t s,
              unsigned long long* prof_cols = nullptr);

constexpr int kWave = 64;

// The hardware deals a grid's blocks to the 8 XCDs in turn (block b runs on
// XCD b mod 8).  Maps block b to a logical block so that each XCD runs one
// contiguous range of the logical order and neighbours in that order share
// the XCD's L2.
__device__ __forceinline__ int xcd_remap_block(int b, int total) {
  const int per = total >> 3, rem = total & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * per + min(xcd, rem) + idx;
}

}  // namespace dot
