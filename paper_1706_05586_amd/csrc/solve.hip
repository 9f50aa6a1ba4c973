// Multi-right-hand-side solves with the matrix-free 7-point (5-point in 2D)
// operator: the forward solves A z_i = B w_i and the adjoint solves
// A^T y_j = C v_j of Section 3.3 (A is symmetric here).
//
// Method: Jacobi-preconditioned CG from x0 = 0.  With S = diag(A)^{1/2} the
// iteration is carried out on the symmetrically scaled system
// (S^-1 A S^-1) x^ = S^-1 b (unit diagonal), whose CG iterates are those of
// Jacobi-PCG on A with x = S^-1 x^.  Each iteration is two stencil sweeps:
//   pass 1: p = r + beta p_old (formed on the fly at the halo too), q = A^ p,
//           partial sums of p.q; p written to the other buffer
//   pass 2: q = A^ p recomputed, x += alpha p, r -= alpha q, partial sums of
//           r.r and |S r|^2 (the unscaled residual norm)
// so the vector traffic is 8 streams per column per iteration.  Per-column
// alpha, beta, norms and the convergence mask live on the device; the host
// polls the number of active columns every few iterations.
//
// Preconditioner: wherever the grid coarsens (every side >= 5), a geometric multigrid
// V-cycle on the scaled system (mg.hip) by default: pass 1 then forms
// p = z + beta p_old from z = M^-1 r, the V-cycle runs after pass 2 and its
// last kernel forms r.z, so an iteration is the two sweeps plus one V-cycle.
// Elsewhere (and on request) the Jacobi preconditioning of the scaling alone.
//
// Mixed precision: binary32 CG on the scaled system with binary64 reliable
// updates (solve_mixed below): the binary32 correction is folded into the
// binary64 x^ and the binary32 residual is replaced by the binary64 b^ - A^ x^
// whenever it has dropped by inner_rtol; the search direction is kept, and
// every stopping decision is taken on the binary64 residual.
//
// Kernel layout for gfx950: a block is a 64 x TY tile in (x, y) (one wave per
// x row) marching through a chunk of z planes; z neighbours stay in
// registers, x/y neighbours come from a double-buffered LDS plane with a
// one-cell halo that is prefetched one plane ahead.  A block processes a
// group of RG columns so each coefficient is loaded once per cell per group;
// the column group varies fastest in the block order, so the groups of one
// tile run together and share its coefficients in L2, and the tiles are
// spread over the 8 XCDs in contiguous runs.  Reductions are deterministic:
// wave shuffles, then LDS in fixed order, then per-block partials summed in
// fixed order by a finalize kernel (one block per column).
#include <algorithm>
#include <vector>

#include "dot_internal.h"

namespace dot {

// Launch geometry
constexpr int kTileRows = 4;        // rows per tile
constexpr int kColsPerBlock = 4;    // columns per block (both precisions)
constexpr int64_t kZWant = 2048;    // blocks aimed at per column group when choosing z chunks
constexpr int kZMin = 8;            // fewest planes per z chunk
constexpr int64_t kColumnPad = 1088;  // work-vector column stride is N + kColumnPad
constexpr int TX = 64;              // one wave per x row
constexpr int TY = kTileRows;
constexpr int NT = TX * TY;
constexpr int NHALO = 2 * TX + 2 * TY;
static_assert(NT >= NHALO, "every halo cell of a tile needs a thread of its block");
constexpr int RG = kColsPerBlock;  // columns per block, binary64 sweeps and elementwise passes
template <typename T>
struct ColsPerBlock {
  static constexpr int value = kColsPerBlock;
};
template <>
struct ColsPerBlock<float> {
  static constexpr int value = kColsPerBlock;
};

enum SweepMode { M_APPLY = 0, M_TRUE = 1, M_PCG1 = 2, M_PCG2 = 3, M_RESID = 4 };
enum EltMode { E_INIT = 0, E_REPLACE = 1, E_FOLD = 2, E_UNSCALE = 3, E_FINISH = 4 };
enum FinMode {
  F_INIT = 0,      // bnorm, rho, scale = |b^|, activity
  F_ALPHA = 1,     // alpha = rho / p.q
  F_BETA = 2,      // binary64 PCG: relres, convergence, beta
  F_BETA_RU = 3,   // binary32 CG: beta, reliable-update schedule
  F_RESID = 4,     // true binary64 residual: convergence
  F_REPLACE = 5,   // residual replaced: rho, beta
  F_TRUE = 6,      // final true relres
  F_RHO_MG = 7,    // multigrid: rho = r.z, beta = rho / rho_old (0 on the first)
  F_BETA_MG = 8,   // multigrid, binary64: relres and convergence only
  F_RU_MG = 9,     // multigrid, binary32: reliable-update schedule only
  F_REPLACE_MG = 10  // multigrid: residual replaced (rho and beta follow from r.z)
};

enum { FLAG_BREAKDOWN = 1, FLAG_NONFINITE = 2 };

#define DOT_TRY(...)               \
  do {                             \
    int rc_ = (__VA_ARGS__);       \
    if (rc_ != DOT_OK) return rc_; \
  } while (0)

struct Geom {
  int nx, ny, nz;
  int64_t nxy, N;
  int64_t ldw;   // column stride of the library's own work vectors (>= N)
  int tiles_x, ntiles, zc, nzc, k;
  int nblk_col;  // ntiles * nzc: partial slots per column
};

__host__ __device__ inline int n_groups(const Geom& G, int rg) { return (G.k + rg - 1) / rg; }

struct ColState {
  double* rho;       // r.z of the current iteration
  double* rho_prev;  // r.z of the previous iteration (reliable updates)
  double* alpha;
  double* beta;
  double* bnorm;     // ||b||_2
  double* relres;    // last relative residual (estimate or true)
  double* scale;     // binary32 scaling of the residual (||b^||)
  double* rmax;      // largest binary32 residual norm since the last update
  int* active;       // column still iterating
  int* upd;          // reliable update due
  int* iters;        // iterations per column
  int* flags;        // FLAG_* per column
  // binary32 CG: x^ (xnew) or the correction d (dnew) holds no value of
  // this solve yet and reads as zero, so the set-up writes no zeros
  int* xnew;
  int* dnew;
};

template <typename T>
struct SweepArgs {
  Geom G;
  const T* cx;
  const T* cy;
  const T* cz;
  const double* diag;  // unscaled diagonal (APPLY/TRUE); unit diagonal otherwise
  const double* sd;    // sqrt(diag)
  const int* active;   // per column, NULL = all
  const double* coef;  // beta (PCG1), alpha (PCG2)
  // column strides of in0, in1, out0, out1 (0 = N, the caller's layout)
  int64_t ld_in0, ld_in1, ld_out0, ld_out1;
  bool norm_s;         // PCG2: also accumulate |S r|^2 (reads sqrt(diag))
  const T* in0;        // APPLY/TRUE: x; PCG1: r; PCG2: p; RESID: x^
  const T* in1;        // PCG1: p_old (not read for a column whose beta is 0)
  const double* b;     // TRUE/RESID: right-hand side
  T* out0;             // APPLY: y; PCG1: p_new; PCG2: x (in place); RESID: r64
  T* out1;             // PCG2: r (in place)
  const int* dnew;     // PCG2: columns whose out0 holds no value yet (read as 0)
  double* partial;     // [2][k][nblk_col]
  unsigned long long* prof_cols;  // optional: sum of active columns over launches
  // RESID with out2: instead of r64, the binary32 residual r / scale[j] (column
  // stride ld_out2) and its norms (as the replacement pass forms them) into
  // partial2
  float* out2;
  const double* scale;
  int64_t ld_out2;
  double* partial2;
};

// Logical block -> (tile, z chunk, column group).  The column group varies
// fastest: the blocks of all groups of one tile and z chunk are neighbours in
// the logical order, so they run together on one XCD and share that tile's
// coefficient and halo cache lines in its L2.
__device__ __forceinline__ void block_coords(int logical, const Geom& G, int ngroups, int* tile,
                                             int* zci, int* grp) {
  *grp = logical % ngroups;
  const int rest = logical / ngroups;
  *tile = rest % G.ntiles;
  *zci = rest / G.ntiles;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block reduction of acc[RG][2] over NT threads into the per-block partial
// slots.  Deterministic: fixed shuffle tree, then waves summed in order.
template <int RG>
__device__ __forceinline__ void block_partials(double (&acc)[RG][2], const Geom& G, int grp,
                                               int slot, double* partial) {
  __shared__ double red[TY][RG][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < RG; ++r) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const double v = wave_sum(acc[r][a]);
      if (lane == 0) red[wave][r][a] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < RG * 2) {
    const int r = threadIdx.x >> 1, a = threadIdx.x & 1;
    const int j = grp * RG + r;
    if (j < G.k) {
      double s = 0.0;
      for (int w = 0; w < TY; ++w) s += red[w][r][a];
      partial[((int64_t)a * G.k + j) * G.nblk_col + slot] = s;
    }
  }
}

// Load of element c (32-bit byte offset) from a block-uniform column base.
template <typename T>
__device__ __forceinline__ T ld(const T* base, uint32_t c) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + c * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st(T* base, uint32_t c, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + c * (uint32_t)sizeof(T)) = v;
}

// v, or +0 when keep is false, without a branch: the load stays
// unconditional and a stale NaN or Inf pattern is cleared exactly
template <typename T>
__device__ __forceinline__ T zero_unless(T v, bool keep) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float(__float_as_uint(v) & (keep ? 0xffffffffu : 0u));
  } else {
    return __longlong_as_double(__double_as_longlong(v) & (keep ? ~0ll : 0ll));
  }
}

template <int MODE, typename T>
__global__ __launch_bounds__(NT) void sweep_kernel(SweepArgs<T> a) {
  constexpr int RG = ColsPerBlock<T>::value;
  // pass 1 stages p = r + beta p_old: two raw loads per staged value, combined
  // only where the value is consumed so that no load is waited for early
  constexpr bool TWO = MODE == M_PCG1;
  const int ngroups = (a.G.k + RG - 1) / RG;
  // two LDS planes: plane z is written to sm[(z - z0) & 1] while the other
  // buffer may still be read by slower waves of plane z - 1, so one barrier
  // per plane suffices
  __shared__ T sm[2][RG][TY + 2][TX + 2];
  const Geom& G = a.G;
  const int logical = xcd_remap_block((int)blockIdx.x, (int)gridDim.x);
  int tile, zci, grp;
  block_coords(logical, G, ngroups, &tile, &zci, &grp);
  const int slot = tile + G.ntiles * zci;
  const int x0 = (tile % G.tiles_x) * TX, y0 = (tile / G.tiles_x) * TY;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int x = x0 + tx, y = y0 + ty;
  const bool in = x < G.nx && y < G.ny;
  const int z0 = zci * G.zc, z1 = min(G.nz, z0 + G.zc);
  const uint32_t nxy = (uint32_t)G.nxy;

  // per-column state; the column base pointers are block-uniform, so cell
  // offsets stay 32-bit
  bool act[RG];
  T cf[RG];
  const T* in0[RG];
  const T* in1[RG];
  T* out0[RG];
  T* out1[RG];
  const double* bcol[RG];
  float* out2c[RG];
  double scl[RG];
  bool keep0[RG];
  bool any = false;
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    const int j = grp * RG + r;
    act[r] = j < G.k && (a.active == nullptr || a.active[j] != 0);
    cf[r] = (act[r] && a.coef) ? (T)a.coef[j] : T(0);
    const int64_t jj = j < G.k ? j : 0;
    in0[r] = a.in0 + (a.ld_in0 ? a.ld_in0 : G.N) * jj;
    // beta = 0 (the first direction): p_old may hold anything, so the term
    // cf * p_old reads the first operand instead (0 * finite = 0)
    in1[r] = TWO ? (cf[r] == T(0) ? in0[r] : a.in1 + (a.ld_in1 ? a.ld_in1 : G.N) * jj) : nullptr;
    keep0[r] = !(MODE == M_PCG2 && a.dnew && j < G.k && a.dnew[j] != 0);
    out0[r] = a.out0 ? a.out0 + (a.ld_out0 ? a.ld_out0 : G.N) * jj : nullptr;
    out1[r] = a.out1 ? a.out1 + (a.ld_out1 ? a.ld_out1 : G.N) * jj : nullptr;
    bcol[r] = a.b ? a.b + G.N * jj : nullptr;
    out2c[r] = a.out2 ? a.out2 + a.ld_out2 * jj : nullptr;
    scl[r] = (act[r] && a.scale) ? a.scale[j] : 1.0;
    any |= act[r];
  }
  if (!any) return;  // uniform over the block
  if (a.prof_cols && tile == 0 && zci == 0 && threadIdx.x == 0) {
    int n = 0;
#pragma unroll
    for (int r = 0; r < RG; ++r) n += act[r] ? 1 : 0;
    atomicAdd(a.prof_cols, (unsigned long long)n);
  }

  // halo slot owned by this thread (if any)
  int hx = -1, hy = -1, hsy = 0, hsx = 0;
  const bool hthread = threadIdx.x < NHALO;
  if (hthread) {
    const int s = threadIdx.x;
    if (s < TX) {
      hx = x0 + s; hy = y0 - 1; hsy = 0; hsx = s + 1;
    } else if (s < 2 * TX) {
      hx = x0 + s - TX; hy = y0 + TY; hsy = TY + 1; hsx = s - TX + 1;
    } else if (s < 2 * TX + TY) {
      hx = x0 - 1; hy = y0 + s - 2 * TX; hsy = s - 2 * TX + 1; hsx = 0;
    } else {
      hx = x0 + TX; hy = y0 + s - 2 * TX - TY; hsy = s - 2 * TX - TY + 1; hsx = TX + 1;
    }
  }
  const bool hin = hx >= 0 && hx < G.nx && hy >= 0 && hy < G.ny;
  // clamped cell indices: loads are unconditional and always in bounds,
  // results of out-of-domain cells are discarded
  const uint32_t hbase = hin ? (uint32_t)(hx + G.nx * hy) : 0u;
  const uint32_t base = in ? (uint32_t)(x + G.nx * y) : 0u;
  const uint32_t nx = (uint32_t)G.nx;

  T vm[RG], vc[RG];        // staged values of planes z-1 and z
  T pr0[RG], pr1[RG];      // raw loads of the own cell, plane z+1
  T hr0[RG], hr1[RG];      // raw loads of the halo cell, next plane
  double acc[RG][2], acc2[RG][2];
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    acc[r][0] = acc[r][1] = 0.0;
    acc2[r][0] = acc2[r][1] = 0.0;
    const uint32_t cm = base + (uint32_t)(z0 > 0 ? z0 - 1 : z0) * nxy;
    const uint32_t c0 = base + (uint32_t)z0 * nxy;
    const uint32_t h0 = hbase + (uint32_t)z0 * nxy;
    T m0 = ld(in0[r], cm), q0 = ld(in0[r], c0), g0 = ld(in0[r], h0);
    if constexpr (TWO) {
      m0 += cf[r] * ld(in1[r], cm);
      q0 += cf[r] * ld(in1[r], c0);
      hr1[r] = ld(in1[r], h0);
    } else {
      hr1[r] = T(0);
    }
    hr0[r] = g0;
    vm[r] = (z0 > 0 && in) ? m0 : T(0);
    vc[r] = in ? q0 : T(0);
  }
  T cD = (z0 > 0) ? ld(a.cz, base + (uint32_t)(z0 - 1) * nxy) : T(0);

  for (int z = z0; z < z1; ++z) {
    const int buf = (z - z0) & 1;
    const uint32_t c = base + (uint32_t)z * nxy;
    const bool has_up = z + 1 < G.nz;
    const uint32_t cu = has_up ? c + nxy : c;
    // plane z into LDS: own values and the halo loaded one plane ago
#pragma unroll
    for (int r = 0; r < RG; ++r) sm[buf][r][ty + 1][tx + 1] = vc[r];
    if (hthread) {
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        T h = hr0[r];
        if constexpr (TWO) h += cf[r] * hr1[r];
        sm[buf][r][hsy][hsx] = hin ? h : T(0);
      }
    }
    // loads issued before the barrier, in the order they are needed: own
    // plane z+1, coefficients and per-cell operands of plane z (used after
    // the barrier), then the halo of plane z+1 last, which stays in flight
    // until the next plane's LDS write (vmcnt retires in order)
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      pr0[r] = ld(in0[r], cu);
      if constexpr (TWO) pr1[r] = ld(in1[r], cu);
    }
    // every load is unconditional (clamped index, result selected) so the
    // compiler's in-order vmcnt bookkeeping stays exact across the loop body
    const bool has_w = in && x > 0, has_s = in && y > 0;
    const T cE = ld(a.cx, c);
    const T cWl = ld(a.cx, has_w ? c - 1 : c);
    const T cN = ld(a.cy, c);
    const T cSl = ld(a.cy, has_s ? c - nx : c);
    const T cU = ld(a.cz, c);
    const T cW = has_w ? cWl : T(0);
    const T cS = has_s ? cSl : T(0);
    T dd = T(1);
    double sdc = 1.0;
    if constexpr (MODE == M_APPLY || MODE == M_TRUE) dd = (T)ld(a.diag, c);
    if constexpr (MODE == M_RESID) sdc = ld(a.sd, c);
    // block-uniform: the sqrt(diag) stream is read only when the caller
    // wants the unscaled norm of this iteration
    if constexpr (MODE == M_PCG2) sdc = a.norm_s ? ld(a.sd, c) : 1.0;
    T o0[RG], o1[RG];
    double bo[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      if constexpr (MODE == M_PCG2) {
        o0[r] = zero_unless(ld((const T*)out0[r], c), keep0[r]);
        o1[r] = ld((const T*)out1[r], c);
      }
      if constexpr (MODE == M_RESID || MODE == M_TRUE) bo[r] = ld(bcol[r], c);
    }
    {
      const uint32_t hc = hbase + (uint32_t)min(z + 1, G.nz - 1) * nxy;
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        hr0[r] = ld(in0[r], hc);
        if constexpr (TWO) hr1[r] = ld(in1[r], hc);
      }
    }
    __syncthreads();
    T vp[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      T v = pr0[r];
      if constexpr (TWO) v += cf[r] * pr1[r];
      vp[r] = (has_up && in) ? v : T(0);
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      if (!act[r]) continue;  // block-uniform
      const T vW = sm[buf][r][ty + 1][tx], vE = sm[buf][r][ty + 1][tx + 2];
      const T vS = sm[buf][r][ty][tx + 1], vN = sm[buf][r][ty + 2][tx + 1];
      const T Av = dd * vc[r] - cW * vW - cE * vE - cS * vS - cN * vN - cD * vm[r] - cU * vp[r];
      if constexpr (MODE == M_APPLY) {
        if (in) st(out0[r], c, Av);
      } else if constexpr (MODE == M_TRUE) {
        const double rr = bo[r] - (double)Av;
        if (in) acc[r][0] += rr * rr;
      } else if constexpr (MODE == M_PCG1) {
        if (in) {
          st(out0[r], c, vc[r]);
          acc[r][0] += (double)vc[r] * (double)Av;
        }
      } else if constexpr (MODE == M_PCG2) {
        const T al = cf[r];
        const T xn = o0[r] + al * vc[r];
        const T rn = o1[r] - al * Av;
        if (in) {
          st(out0[r], c, xn);
          st(out1[r], c, rn);
          const double rd = (double)rn;
          acc[r][0] += rd * rd;
          if (a.norm_s) {
            const double t = sdc * rd;
            acc[r][1] += t * t;
          }
        }
      } else if constexpr (MODE == M_RESID) {
        const double rr = bo[r] / sdc - (double)Av;
        if (in) {
          acc[r][0] += rr * rr;
          const double t = sdc * rr;
          acc[r][1] += t * t;
          if (out2c[r]) {
            const float rv = (float)(rr / scl[r]);
            out2c[r][c] = rv;
            const double rd = (double)rv;
            acc2[r][0] += rd * rd;
            const double t2 = sdc * rd;
            acc2[r][1] += t2 * t2;
          } else {
            st(out0[r], c, (T)rr);
          }
        }
      }
    }
    cD = cU;
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      vm[r] = vc[r];
      vc[r] = vp[r];
    }
  }
  if constexpr (MODE != M_APPLY) block_partials<RG>(acc, G, grp, slot, a.partial);
  if constexpr (MODE == M_RESID) {
    if (a.out2) {  // uniform
      __syncthreads();  // block_partials' LDS is read above
      block_partials<RG>(acc2, G, grp, slot, a.partial2);
    }
  }
}

// Elementwise passes on the same block decomposition (same partial slots).
struct EltArgs {
  Geom G;
  const double* sd;
  const int* mask;      // columns to process (NULL = all)
  const double* scale;  // per column scale
  const double* b;      // INIT: rhs
  double* xh;           // x^ (binary64; INIT: cleared unless NULL)
  double* r64;          // INIT: binary64 residual b^ (or NULL: not kept)
  float* r32;           // inner residual
  float* d32;           // inner correction
  double* p64z;         // INIT: binary64 direction buffer to clear (or NULL)
  float* p32z;          // INIT: binary32 direction buffer to clear (or NULL)
  const int* xnew;      // FOLD / FINISH: columns whose x^ reads as 0 (or NULL)
  const int* dnew;      // FOLD / FINISH: columns whose d reads as 0 (or NULL)
  const int* fold;      // FINISH: columns whose d is folded (the others only unscaled)
  double* partial;
};

constexpr int EU = 4;  // planes per step of the elementwise passes

template <int MODE>
__global__ __launch_bounds__(NT) void elt_kernel(EltArgs a) {
  const Geom& G = a.G;
  const int ngroups = (G.k + RG - 1) / RG;
  const int logical = xcd_remap_block((int)blockIdx.x, (int)gridDim.x);
  int tile, zci, grp;
  block_coords(logical, G, ngroups, &tile, &zci, &grp);
  const int slot = tile + G.ntiles * zci;
  const int x = (tile % G.tiles_x) * TX + (threadIdx.x & 63);
  const int y = (tile / G.tiles_x) * TY + (threadIdx.x >> 6);
  const bool in = x < G.nx && y < G.ny;
  const int z0 = zci * G.zc, z1 = min(G.nz, z0 + G.zc);
  bool act[RG], hx[RG], hd[RG];
  int col[RG];
  double sc[RG];
  bool any = false;
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    const int j = grp * RG + r;
    col[r] = j;
    act[r] = j < G.k && (a.mask == nullptr || a.mask[j] != 0);
    sc[r] = (act[r] && a.scale) ? a.scale[j] : 0.0;
    // x^ and d hold values (block-uniform); FINISH folds d only where asked
    hx[r] = act[r] && !(a.xnew && a.xnew[j] != 0);
    hd[r] = act[r] && !(a.dnew && a.dnew[j] != 0) && (MODE != E_FINISH || (a.fold && a.fold[j] != 0));
    // FOLD: nothing to add to a valid x^
    if (MODE == E_FOLD && hx[r] && !hd[r]) act[r] = false;
    any |= act[r];
  }
  if (!any) return;
  double acc[RG][2];
#pragma unroll
  for (int r = 0; r < RG; ++r) acc[r][0] = acc[r][1] = 0.0;
  if (in) {
    const int64_t base = x + (int64_t)G.nx * y;
    // EU planes per step: every load of the step's planes and columns is
    // issued before any of them is used (the last step's surplus planes
    // load the chunk's last plane again and are dropped); sqrt(diag) is
    // loaded once per plane for the block's columns
    constexpr bool LB = MODE == E_INIT || MODE == E_REPLACE;
    constexpr bool LS = MODE != E_FOLD;
    bool lx[RG], lddd[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      lx[r] = act[r] && (MODE == E_UNSCALE || ((MODE == E_FOLD || MODE == E_FINISH) && hx[r]));
      lddd[r] = act[r] && (MODE == E_FOLD || MODE == E_FINISH) && hd[r];
    }
    for (int z = z0; z < z1; z += EU) {
      double vb[RG][EU], vs[EU], vx[RG][EU];
      float vd[RG][EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const int64_t c = base + (int64_t)min(z + u, z1 - 1) * G.nxy;
        vs[u] = LS ? a.sd[c] : 1.0;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
          const int64_t o = c + G.N * (int64_t)col[r], w = c + G.ldw * (int64_t)col[r];
          vb[r][u] = (LB && act[r]) ? a.b[o] : 0.0;
          vx[r][u] = lx[r] ? a.xh[o] : 0.0;
          vd[r][u] = lddd[r] ? a.d32[w] : 0.0f;
        }
      }
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        if (z + u >= z1) break;
        const int64_t c = base + (int64_t)(z + u) * G.nxy;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
          if (!act[r]) continue;  // block-uniform
          const int64_t o = c + G.N * (int64_t)col[r];     // caller's arrays
          const int64_t w = c + G.ldw * (int64_t)col[r];   // work vectors
          if constexpr (MODE == E_INIT) {
            const double bv = vb[r][u];
            const double rv = bv / vs[u];
            if (a.xh) a.xh[o] = 0.0;
            if (a.r64) a.r64[w] = rv;
            if (a.d32) a.d32[w] = 0.0f;
            if (a.p64z) a.p64z[w] = 0.0;
            if (a.p32z) a.p32z[w] = 0.0f;
            acc[r][0] += rv * rv;
            acc[r][1] += bv * bv;
          } else if constexpr (MODE == E_REPLACE) {
            // the first binary32 residual (b^ / scale, x = 0), formed from b
            // as E_INIT forms b^
            const float rv = (float)((vb[r][u] / vs[u]) / sc[r]);
            a.r32[w] = rv;
            const double rd = (double)rv;
            acc[r][0] += rd * rd;
            const double t = vs[u] * rd;
            acc[r][1] += t * t;
          } else if constexpr (MODE == E_FOLD) {
            // d is not cleared: the columns folded here are marked as
            // holding no correction, which the next CG pass 2 reads as zero
            a.xh[o] = hd[r] ? vx[r][u] + sc[r] * (double)vd[r][u] : vx[r][u];
          } else if constexpr (MODE == E_UNSCALE) {
            a.xh[o] = vx[r][u] / vs[u];
          } else if constexpr (MODE == E_FINISH) {
            // pending correction folded (columns stopped by the iteration
            // cap) and x = x^ / sqrt(diag) in one pass
            double xv = vx[r][u];
            if (hd[r]) xv += sc[r] * (double)vd[r][u];
            a.xh[o] = xv / vs[u];
          }
        }
      }
    }
  }
  if constexpr (MODE == E_INIT || MODE == E_REPLACE) block_partials<RG>(acc, G, grp, slot, a.partial);
}

// One block per column: sum that column's per-block partials in fixed order
// and update its state.  Columns outside `live` are left untouched.
struct FinArgs {
  int mode;
  int k, nblk;
  const double* partial;
  const int* live;
  ColState st;
  double rtol, delta;
  int have_s;   // F_BETA_RU / F_RU_MG: the sweep accumulated |S r|^2; F_RHO_MG: first
};

__global__ __launch_bounds__(256) void finalize_kernel(FinArgs a) {
  __shared__ double red[2][256];
  const int j = blockIdx.x;
  if (j >= a.k) return;
  if (a.live && a.live[j] == 0) return;  // uniform over the block
  const ColState& st = a.st;
  for (int q = 0; q < 2; ++q) {
    const double* p = a.partial + ((int64_t)q * a.k + j) * a.nblk;
    double s = 0.0;
    for (int i = threadIdx.x; i < a.nblk; i += 256) s += p[i];
    red[q][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s0 = red[0][0], s1 = red[1][0];
  const bool fin = isfinite(s0) && isfinite(s1);
  switch (a.mode) {
    case F_INIT: {
      const double bn = sqrt(s1);
      st.bnorm[j] = bn;
      st.rho[j] = s0;
      st.rho_prev[j] = 0.0;
      st.scale[j] = sqrt(s0);
      st.rmax[j] = 0.0;
      st.beta[j] = 0.0;
      st.iters[j] = 0;
      st.flags[j] = 0;
      st.upd[j] = 0;
      st.xnew[j] = 1;
      st.dnew[j] = 1;
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
        st.relres[j] = NAN;
      } else {
        st.active[j] = bn > 0.0 ? 1 : 0;
        st.relres[j] = bn > 0.0 ? 1.0 : 0.0;
      }
      break;
    }
    case F_ALPHA: {
      if (!fin || !(s0 > 0.0)) {
        st.flags[j] |= fin ? FLAG_BREAKDOWN : FLAG_NONFINITE;
        st.alpha[j] = 0.0;
        st.active[j] = 0;
      } else {
        st.alpha[j] = st.rho[j] / s0;
      }
      break;
    }
    case F_BETA: {  // binary64 PCG: stopping test on the recursive residual
      st.iters[j] += 1;
      const double rel = sqrt(s1) / st.bnorm[j];
      st.relres[j] = rel;
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
      } else if (rel <= a.rtol) {
        st.active[j] = 0;
      } else {
        st.beta[j] = s0 / st.rho[j];
        st.rho[j] = s0;
      }
      break;
    }
    case F_BETA_RU: {  // binary32 CG: schedule a reliable update when due
      st.iters[j] += 1;
      st.dnew[j] = 0;  // CG pass 2 has written d
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
        break;
      }
      const double rn = sqrt(s0);
      // the unscaled estimate exists on the iterations the host polls,
      // which are the only ones whose update flags it acts on
      bool claims = false;
      if (a.have_s) {
        const double est = st.scale[j] * sqrt(s1) / st.bnorm[j];
        st.relres[j] = est;
        claims = est <= a.rtol;
      }
      st.rho_prev[j] = st.rho[j];
      st.beta[j] = s0 / st.rho[j];
      st.rho[j] = s0;
      st.rmax[j] = fmax(st.rmax[j], rn);
      if (rn < a.delta * st.rmax[j] || claims) st.upd[j] = 1;
      break;
    }
    case F_RESID: {  // true binary64 residual after folding the correction
      st.xnew[j] = 0;
      st.dnew[j] = 1;
      const double rel = sqrt(s1) / st.bnorm[j];
      st.relres[j] = rel;
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
        st.upd[j] = 0;
      } else if (rel <= a.rtol) {
        st.active[j] = 0;
        st.upd[j] = 0;
      }
      break;
    }
    case F_REPLACE: {  // residual replaced by the true one; keep the direction
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
      } else {
        st.beta[j] = st.rho_prev[j] > 0.0 ? s0 / st.rho_prev[j] : 0.0;
        st.rho[j] = s0;
        st.rmax[j] = sqrt(s0);
      }
      st.upd[j] = 0;
      break;
    }
    case F_TRUE: {
      const double bn = st.bnorm[j];
      st.relres[j] = bn > 0.0 ? sqrt(s0) / bn : sqrt(s0);
      break;
    }
    case F_RHO_MG: {  // r.z of the preconditioned residual
      if (!fin || !(s0 > 0.0)) {
        st.flags[j] |= fin ? FLAG_BREAKDOWN : FLAG_NONFINITE;
        st.active[j] = 0;
        st.upd[j] = 0;
      } else {
        st.beta[j] = a.have_s ? 0.0 : s0 / st.rho[j];
        st.rho[j] = s0;
      }
      break;
    }
    case F_BETA_MG: {
      st.iters[j] += 1;
      const double rel = sqrt(s1) / st.bnorm[j];
      st.relres[j] = rel;
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
      } else if (rel <= a.rtol) {
        st.active[j] = 0;
      }
      break;
    }
    case F_RU_MG: {
      st.iters[j] += 1;
      st.dnew[j] = 0;  // CG pass 2 has written d
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
        break;
      }
      const double rn = sqrt(s0);
      bool claims = false;
      if (a.have_s) {
        const double est = st.scale[j] * sqrt(s1) / st.bnorm[j];
        st.relres[j] = est;
        claims = est <= a.rtol;
      }
      st.rmax[j] = fmax(st.rmax[j], rn);
      if (rn < a.delta * st.rmax[j] || claims) st.upd[j] = 1;
      break;
    }
    case F_REPLACE_MG: {
      if (!fin) {
        st.flags[j] |= FLAG_NONFINITE;
        st.active[j] = 0;
      } else {
        st.rmax[j] = sqrt(s0);
      }
      st.upd[j] = 0;
      break;
    }
  }
}

// ---------------------------------------------------------------- host side
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static Geom make_geom(const GridDims& g, int k) {
  Geom G;
  G.nx = g.nx;
  G.ny = g.ny;
  G.nz = g.nz;
  G.nxy = g.nxy;
  G.N = g.N;
  // work-vector columns kColumnPad elements apart beyond N, so that the columns
  // of a group and the vectors of one sweep do not sit a power of two apart
  G.ldw = g.N + kColumnPad;
  G.k = k;
  G.tiles_x = (g.nx + TX - 1) / TX;
  const int tiles_y = (g.ny + TY - 1) / TY;
  G.ntiles = G.tiles_x * tiles_y;
  // z chunk: aim for kZWant blocks of kColsPerBlock columns, chunks of at least
  // kZMin planes.  The chunking does not depend on the column group size,
  // so every kernel of a solve shares the partial slots.
  const int64_t want = kZWant;
  const int64_t per_z = (int64_t)G.ntiles * n_groups(G, kColsPerBlock);
  int nzc = (int)std::min<int64_t>(g.nz, std::max<int64_t>(1, (want + per_z - 1) / per_z));
  int zc = (g.nz + nzc - 1) / nzc;
  zc = std::max(zc, std::min(kZMin, g.nz));
  G.zc = zc;
  G.nzc = (g.nz + zc - 1) / zc;
  G.nblk_col = G.ntiles * G.nzc;
  return G;
}

struct Workspace {
  double* r64;
  double* p64[2];
  float* r32;
  float* p32[2];
  float* d32;
  // multigrid (when the operator has a hierarchy): z = M^-1 r and the V-cycle
  double* z64;
  float* z32;
  MgWork<double> mg64;
  MgWork<float> mg32;   // DOT_MIXED with binary32 V-cycle vectors
  MgWork<bf16s> mgh;    // DOT_MIXED with bfloat16 V-cycle vectors (the default)
  bool mg_half;
  int mg_slots;      // partial slots per column of the V-cycle's r.z
  double* partial;
  size_t partial_stride;  // elements; the second set starts there
  ColState st;
  size_t bytes;
};

static size_t layout_workspace(const dot_op* op, const Geom& G, int precision, char* base,
                               Workspace* w, bool mg_half = true) {
  const size_t Nk = (size_t)G.ldw * G.k;
  const bool mg = op->mg_nlev >= 2;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  Workspace ws{};
  if (precision == DOT_FP64) {
    ws.r64 = (double*)take(Nk * 8);
    ws.p64[0] = (double*)take(Nk * 8);
    ws.p64[1] = (double*)take(Nk * 8);
    if (mg) {
      ws.z64 = (double*)take(Nk * 8);
      char* m = take(mg_work_bytes(op, G.k, G.ldw, 8));
      if (base) mg_work_layout<double>(op, G.k, G.ldw, m, &ws.mg64);
    }
  } else {
    ws.r32 = (float*)take(Nk * 4);
    ws.p32[0] = (float*)take(Nk * 4);
    ws.p32[1] = (float*)take(Nk * 4);
    ws.d32 = (float*)take(Nk * 4);
    if (mg) {
      ws.z32 = (float*)take(Nk * 4);
      // room for either storage of the V-cycle's vectors
      char* m = take(std::max(mg_work_bytes(op, G.k, G.ldw, 4),
                              mg_work_bytes(op, G.k, G.ldw, sizeof(bf16s), 2)));
      ws.mg_half = mg_half;
      if (base && mg_half) mg_work_layout<bf16s>(op, G.k, G.ldw, m, &ws.mgh, 2);
      else if (base) mg_work_layout<float>(op, G.k, G.ldw, m, &ws.mg32);
    }
  }
  ws.mg_slots = mg ? mg_partial_slots(op, G.k) : 0;
  // two sets of [2][k][slots] partials: the residual sweep of a reliable
  // update fills both (its own norms and those of the replaced residual)
  ws.partial_stride = (size_t)2 * G.k * std::max(G.nblk_col, ws.mg_slots);
  ws.partial = (double*)take(2 * ws.partial_stride * 8);
  const size_t k = (size_t)G.k;
  ws.st.rho = (double*)take(k * 8);
  ws.st.rho_prev = (double*)take(k * 8);
  ws.st.alpha = (double*)take(k * 8);
  ws.st.beta = (double*)take(k * 8);
  ws.st.bnorm = (double*)take(k * 8);
  ws.st.relres = (double*)take(k * 8);
  ws.st.scale = (double*)take(k * 8);
  ws.st.rmax = (double*)take(k * 8);
  ws.st.active = (int*)take(k * 4);
  ws.st.upd = (int*)take(k * 4);
  ws.st.iters = (int*)take(k * 4);
  ws.st.flags = (int*)take(k * 4);
  ws.st.xnew = (int*)take(k * 4);
  ws.st.dnew = (int*)take(k * 4);
  ws.bytes = off;
  if (w) *w = ws;
  return off;
}

// ------------------------------------------------------------ profiling
// Timed launches: an event pair each and, for launches whose kernels count
// their active columns, a device slot of that count.  A counted launch that
// found no active column (a launch queued after every column had stopped,
// see LagPoll) is left out of the totals.
constexpr int kProfSlots = 2048;
struct ProfState {
  bool on = false;
  unsigned mask = ~0u;  // kinds timed (bit 1 << kind)
  std::vector<hipEvent_t> pool;
  struct Pending {
    int kind;
    hipEvent_t e0, e1;
    bool counted;
  };
  std::vector<Pending> pending;
  double ms[DOT_PROF_KINDS] = {};
  int64_t launches[DOT_PROF_KINDS] = {};
  unsigned long long cols[DOT_PROF_KINDS] = {};
  unsigned long long* cols_dev = nullptr;  // kProfSlots, slot i for pending[i]
};

static ProfState* prof_of(dot_op* op) { return reinterpret_cast<ProfState*>(op->prof); }

static int prof_drain(dot_op* op) {
  ProfState* p = prof_of(op);
  if (!p) return DOT_OK;
  const size_t n = p->pending.size();
  if (n == 0) return DOT_OK;
  for (auto& q : p->pending) DOT_HIP(hipEventSynchronize(q.e1));
  std::vector<unsigned long long> slot(n);
  DOT_HIP(hipMemcpy(slot.data(), p->cols_dev, n * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  DOT_HIP(hipMemset(p->cols_dev, 0, n * sizeof(unsigned long long)));
  for (size_t i = 0; i < n; ++i) {
    const auto& q = p->pending[i];
    if (!q.counted || slot[i] > 0) {
      float ms = 0.0f;
      DOT_HIP(hipEventElapsedTime(&ms, q.e0, q.e1));
      p->ms[q.kind] += ms;
      p->launches[q.kind] += 1;
      p->cols[q.kind] += slot[i];
    }
    p->pool.push_back(q.e0);
    p->pool.push_back(q.e1);
  }
  p->pending.clear();
  return DOT_OK;
}

static int prof_begin(dot_op* op, int kind, hipStream_t s, hipEvent_t* e0, hipEvent_t* e1,
                      unsigned long long** cols) {
  *e0 = *e1 = nullptr;
  *cols = nullptr;
  ProfState* p = prof_of(op);
  if (!p || !p->on || kind < 0 || !((p->mask >> kind) & 1u)) return DOT_OK;
  if (p->pending.size() >= (size_t)kProfSlots) DOT_TRY(prof_drain(op));
  for (hipEvent_t* e : {e0, e1}) {
    if (p->pool.empty()) {
      hipEvent_t ev;
      DOT_HIP(hipEventCreate(&ev));
      p->pool.push_back(ev);
    }
    *e = p->pool.back();
    p->pool.pop_back();
  }
  *cols = p->cols_dev + p->pending.size();
  DOT_HIP(hipEventRecord(*e0, s));
  return DOT_OK;
}

static int prof_end(dot_op* op, int kind, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                    bool counted = false) {
  if (!e0) return DOT_OK;
  DOT_HIP(hipEventRecord(e1, s));
  prof_of(op)->pending.push_back({kind, e0, e1, counted});
  return DOT_OK;
}

template <int MODE, typename T>
static int launch_sweep(dot_op* op, SweepArgs<T> a, hipStream_t s, int kind = -1) {
  hipEvent_t e0, e1;
  DOT_TRY(prof_begin(op, kind, s, &e0, &e1, &a.prof_cols));
  const int blocks = a.G.nblk_col * n_groups(a.G, ColsPerBlock<T>::value);
  hipLaunchKernelGGL((sweep_kernel<MODE, T>), dim3(blocks), dim3(NT), 0, s, a);
  DOT_LAUNCH_CHECK();
  return prof_end(op, kind, s, e0, e1, true);
}

template <int MODE>
static int launch_elt(const EltArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((elt_kernel<MODE>), dim3(a.G.nblk_col * n_groups(a.G, RG)), dim3(NT), 0, s, a);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

static int launch_fin(int mode, const Geom& G, const Workspace& ws, const int* live, double rtol,
                      double delta, hipStream_t s, int have_s = 1, int set = 0) {
  FinArgs f;
  f.have_s = have_s;
  f.mode = mode;
  f.k = G.k;
  f.nblk = mode == F_RHO_MG ? ws.mg_slots : G.nblk_col;
  f.partial = ws.partial + (set ? ws.partial_stride : 0);
  f.live = live;
  f.st = ws.st;
  f.rtol = rtol;
  f.delta = delta;
  hipLaunchKernelGGL(finalize_kernel, dim3(G.k), dim3(256), 0, s, f);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

// Copy the activity (and update) flags to pinned host memory and count them.
static int poll(dot_op* op, const Workspace& ws, int k, hipStream_t s, int* n_active,
                int* n_upd) {
  DOT_HIP(hipMemcpyAsync(op->pinned, ws.st.active, k * sizeof(int), hipMemcpyDeviceToHost, s));
  if (n_upd)
    DOT_HIP(hipMemcpyAsync(op->pinned + k, ws.st.upd, k * sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  DOT_TRY(prof_drain(op));
  int na = 0, nu = 0;
  for (int j = 0; j < k; ++j) {
    na += op->pinned[j] != 0;
    if (n_upd) nu += op->pinned[k + j] != 0;
  }
  *n_active = na;
  if (n_upd) *n_upd = nu;
  return DOT_OK;
}

// Flag snapshots read one poll late: at a poll the activity and update
// flags are copied to one of two pinned slots behind an event, and the
// previous poll's slot is then read, so the host waits for the stream only
// when it is a poll interval behind and the GPU keeps the next iterations
// queued.  Iterations enqueued after the last column has stopped run with
// every column masked off and cost a few microseconds per launch.
struct LagPoll {
  int pending = -1;  // slot of the snapshot not read yet (-1: none)
  int next = 0;
};

static int poll_snapshot(dot_op* op, const Workspace& ws, int k, hipStream_t s, LagPoll& lp) {
  int32_t* slot = op->pinned + 2 * k * lp.next;
  DOT_HIP(hipMemcpyAsync(slot, ws.st.active, k * sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipMemcpyAsync(slot + k, ws.st.upd, k * sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipEventRecord(op->poll_ev[lp.next], s));
  return DOT_OK;
}

// reads the pending snapshot (waiting for it) and makes the one just taken pending
static int poll_read(dot_op* op, int k, LagPoll& lp, bool advance, int* n_active, int* n_upd) {
  if (lp.pending >= 0) {
    DOT_HIP(hipEventSynchronize(op->poll_ev[lp.pending]));
    const int32_t* slot = op->pinned + 2 * k * lp.pending;
    int na = 0, nu = 0;
    for (int j = 0; j < k; ++j) {
      na += slot[j] != 0;
      nu += slot[k + j] != 0;
    }
    *n_active = na;
    *n_upd = nu;
  }
  lp.pending = advance ? lp.next : -1;
  if (advance) lp.next ^= 1;
  return DOT_OK;
}

static SweepArgs<double> base_args64(dot_op* op, const Geom& G) {
  SweepArgs<double> a{};
  a.G = G;
  a.cx = op->sx;
  a.cy = op->sy;
  a.cz = op->sz;
  a.sd = op->sd;
  return a;
}

static SweepArgs<float> base_args32(dot_op* op, const Geom& G) {
  SweepArgs<float> a{};
  a.G = G;
  a.cx = op->sx32;
  a.cy = op->sy32;
  a.cz = op->sz32;
  a.sd = op->sd;
  return a;
}

// x = x^ / sqrt(diag) (or the binary32 CG's finishing pass `fin`), then the
// true residual of x in binary64
static int finish_true(dot_op* op, const Geom& G, const Workspace& ws, const double* rhs,
                       double* x, hipStream_t s, const EltArgs* fin = nullptr) {
  EltArgs e{};
  e.G = G;
  e.sd = op->sd;
  e.xh = x;
  if (fin) DOT_TRY(launch_elt<E_FINISH>(*fin, s));
  else DOT_TRY(launch_elt<E_UNSCALE>(e, s));
  SweepArgs<double> t{};
  t.G = G;
  t.cx = op->cx;
  t.cy = op->cy;
  t.cz = op->cz;
  t.diag = op->diag;
  t.in0 = x;
  t.b = rhs;
  t.partial = ws.partial;
  DOT_TRY(launch_sweep<M_TRUE, double>(op, t, s));
  DOT_TRY(launch_fin(F_TRUE, G, ws, nullptr, 0.0, 0.0, s));
  return DOT_OK;
}

static int solve_fp64(dot_op* op, const Geom& G, const Workspace& ws, const double* rhs, double* x,
                      const dot_solve_opts& o, bool mg, hipStream_t s, int* iters_done) {
  EltArgs e{};
  e.G = G;
  e.sd = op->sd;
  e.b = rhs;
  e.xh = x;
  e.r64 = ws.r64;
  e.p64z = ws.p64[0];
  e.partial = ws.partial;
  DOT_TRY(launch_elt<E_INIT>(e, s));
  DOT_TRY(launch_fin(F_INIT, G, ws, nullptr, o.rtol, 0.0, s));
  // z = M^-1 r and rho = r.z (the first beta is zero)
  auto precondition = [&](int first) -> int {
    hipEvent_t e0, e1;
    unsigned long long* cols;
    DOT_TRY(prof_begin(op, DOT_PROF_VCYCLE_FP64, s, &e0, &e1, &cols));
    DOT_TRY(mg_vcycle<double>(op, ws.mg64, G.k, ws.r64, G.ldw, ws.z64, ws.st.active, ws.partial, s,
                              cols));
    DOT_TRY(prof_end(op, DOT_PROF_VCYCLE_FP64, s, e0, e1, true));
    return launch_fin(F_RHO_MG, G, ws, ws.st.active, o.rtol, 0.0, s, first);
  };
  if (mg) DOT_TRY(precondition(1));
  int n_active = 0;
  DOT_TRY(poll(op, ws, G.k, s, &n_active, nullptr));
  LagPoll lp;
  int it = 0;
  int cur = 0;
  while (n_active > 0 && it < o.max_iter) {
    SweepArgs<double> p1 = base_args64(op, G);
    p1.active = ws.st.active;
    p1.coef = ws.st.beta;
    p1.in0 = mg ? ws.z64 : ws.r64;
    p1.in1 = ws.p64[cur];
    p1.out0 = ws.p64[cur ^ 1];
    p1.ld_in0 = p1.ld_in1 = p1.ld_out0 = G.ldw;
    p1.partial = ws.partial;
    DOT_TRY(launch_sweep<M_PCG1, double>(op, p1, s, DOT_PROF_PCG1_FP64));
    DOT_TRY(launch_fin(F_ALPHA, G, ws, ws.st.active, o.rtol, 0.0, s));
    cur ^= 1;
    SweepArgs<double> p2 = base_args64(op, G);
    p2.active = ws.st.active;
    p2.coef = ws.st.alpha;
    p2.in0 = ws.p64[cur];
    p2.out0 = x;
    p2.out1 = ws.r64;
    p2.ld_in0 = p2.ld_out1 = G.ldw;
    p2.norm_s = true;
    p2.partial = ws.partial;
    DOT_TRY(launch_sweep<M_PCG2, double>(op, p2, s, DOT_PROF_PCG2_FP64));
    DOT_TRY(launch_fin(mg ? F_BETA_MG : F_BETA, G, ws, ws.st.active, o.rtol, 0.0, s));
    if (mg) DOT_TRY(precondition(0));
    ++it;
    if (it % o.check_every == 0 || it == o.max_iter) {
      int nu = 0;
      DOT_TRY(poll_snapshot(op, ws, G.k, s, lp));
      DOT_TRY(poll_read(op, G.k, lp, true, &n_active, &nu));
    }
  }
  *iters_done = it;
  return finish_true(op, G, ws, rhs, x, s);
}

// Binary32 CG with binary64 reliable updates: the correction d is accumulated
// in binary32; when the binary32 residual of a column has dropped by `delta`
// since its last update, or claims convergence, the correction is folded
// into x^ in binary64 (x^ += s d), the true residual b^ - A^ x^ is recomputed
// in binary64 and replaces the binary32 residual.  The search direction is
// kept, so the Krylov information is not discarded as in a restart.  Every
// convergence decision is made on the binary64 residual.  With multigrid the
// binary32 V-cycle preconditions the binary32 residual (after a replacement,
// the replaced one).
static int solve_mixed(dot_op* op, const Geom& G, const Workspace& ws, const double* rhs,
                       double* x, const dot_solve_opts& o, bool mg, hipStream_t s, int* iters_done,
                       int* outer_done) {
  const double delta = o.inner_rtol;
  EltArgs e{};
  e.G = G;
  e.sd = op->sd;
  e.b = rhs;
  e.xh = x;
  e.r32 = ws.r32;
  e.d32 = ws.d32;
  e.scale = ws.st.scale;
  e.partial = ws.partial;
  e.xnew = ws.st.xnew;
  e.dnew = ws.st.dnew;
  // norms of b^ and b only: x^, d and the first direction are not cleared
  // (F_INIT marks x^ and d as holding no value; the first CG pass 1 does not
  // read p_old, its beta being 0)
  EltArgs e0 = e;
  e0.xh = nullptr;
  e0.d32 = nullptr;
  DOT_TRY(launch_elt<E_INIT>(e0, s));
  DOT_TRY(launch_fin(F_INIT, G, ws, nullptr, o.rtol, delta, s));
  EltArgs er = e;
  er.mask = ws.st.active;
  DOT_TRY(launch_elt<E_REPLACE>(er, s));
  DOT_TRY(launch_fin(mg ? F_REPLACE_MG : F_REPLACE, G, ws, ws.st.active, o.rtol, delta, s));
  auto precondition = [&](int first) -> int {
    hipEvent_t e0, e1;
    unsigned long long* cols;
    DOT_TRY(prof_begin(op, DOT_PROF_VCYCLE_FP32, s, &e0, &e1, &cols));
    if (ws.mg_half)
      DOT_TRY(mg_vcycle<float>(op, ws.mgh, G.k, ws.r32, G.ldw, ws.z32, ws.st.active, ws.partial, s,
                               cols));
    else
      DOT_TRY(mg_vcycle<float>(op, ws.mg32, G.k, ws.r32, G.ldw, ws.z32, ws.st.active, ws.partial, s,
                               cols));
    DOT_TRY(prof_end(op, DOT_PROF_VCYCLE_FP32, s, e0, e1, true));
    return launch_fin(F_RHO_MG, G, ws, ws.st.active, o.rtol, delta, s, first);
  };
  if (mg) DOT_TRY(precondition(1));
  int n_active = 0, n_upd = 0;
  DOT_TRY(poll(op, ws, G.k, s, &n_active, nullptr));
  LagPoll lp;
  int it = 0, updates = 0, cur = 0;
  auto count = [&](bool advance) -> int {
    n_upd = 0;
    DOT_TRY(poll_read(op, G.k, lp, advance, &n_active, &n_upd));
    if (n_upd > 0) ++updates;
    return DOT_OK;
  };
  while (n_active > 0 && it < o.max_iter) {
    SweepArgs<float> p1 = base_args32(op, G);
    p1.active = ws.st.active;
    p1.coef = ws.st.beta;
    p1.in0 = mg ? ws.z32 : ws.r32;
    p1.in1 = ws.p32[cur];
    p1.out0 = ws.p32[cur ^ 1];
    p1.ld_in0 = p1.ld_in1 = p1.ld_out0 = G.ldw;
    p1.partial = ws.partial;
    DOT_TRY(launch_sweep<M_PCG1, float>(op, p1, s, DOT_PROF_PCG1_FP32));
    DOT_TRY(launch_fin(F_ALPHA, G, ws, ws.st.active, o.rtol, delta, s));
    cur ^= 1;
    SweepArgs<float> p2 = base_args32(op, G);
    p2.active = ws.st.active;
    p2.coef = ws.st.alpha;
    p2.in0 = ws.p32[cur];
    p2.out0 = ws.d32;
    p2.out1 = ws.r32;
    p2.ld_in0 = p2.ld_out0 = p2.ld_out1 = G.ldw;
    p2.dnew = ws.st.dnew;
    p2.partial = ws.partial;
    const bool polled = (it + 1) % o.check_every == 0 || it + 1 == o.max_iter;
    p2.norm_s = polled;
    DOT_TRY(launch_sweep<M_PCG2, float>(op, p2, s, DOT_PROF_PCG2_FP32));
    DOT_TRY(launch_fin(mg ? F_RU_MG : F_BETA_RU, G, ws, ws.st.active, o.rtol, delta, s,
                       polled ? 1 : 0));
    ++it;
    if (polled) {
      DOT_TRY(poll_snapshot(op, ws, G.k, s, lp));
      // reliable update of the flagged columns (every kernel masked by the
      // update flags: a no-op where none is set)
      EltArgs ef = e;
      ef.mask = ws.st.upd;
      DOT_TRY(launch_elt<E_FOLD>(ef, s));
      // binary64 residual and, in the same sweep, the binary32 residual
      // that replaces the recurrence's (r / scale) with the norms of both
      SweepArgs<double> rs = base_args64(op, G);
      rs.active = ws.st.upd;
      rs.in0 = x;
      rs.b = rhs;
      rs.out2 = ws.r32;
      rs.ld_out2 = G.ldw;
      rs.scale = ws.st.scale;
      rs.partial = ws.partial;
      rs.partial2 = ws.partial + ws.partial_stride;
      DOT_TRY(launch_sweep<M_RESID, double>(op, rs, s, DOT_PROF_RESID));
      DOT_TRY(launch_fin(F_RESID, G, ws, ws.st.upd, o.rtol, delta, s));
      DOT_TRY(launch_fin(mg ? F_REPLACE_MG : F_REPLACE, G, ws, ws.st.upd, o.rtol, delta, s, 1, 1));
    }
    if (mg) DOT_TRY(precondition(0));
    if (polled) DOT_TRY(count(true));
  }
  DOT_TRY(count(false));
  // columns stopped by the iteration cap fold their pending correction in
  // the pass that unscales x
  EltArgs ef = e;
  ef.fold = ws.st.active;
  *iters_done = it;
  *outer_done = updates;
  return finish_true(op, G, ws, rhs, x, s, &ef);
}

}  // namespace dot

using namespace dot;

extern "C" {

size_t dot_solve_workspace_bytes(const dot_op* op, int k, int precision) {
  if (!op || k < 1 || k > DOT_MAX_COLUMNS || (precision != DOT_FP64 && precision != DOT_MIXED))
    return 0;
  Geom G = make_geom(op->g, k);
  return layout_workspace(op, G, precision, nullptr, nullptr);
}

int dot_apply(dot_op* op, int k, const double* X_dev, double* Y_dev, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (k < 1) DOT_FAIL(DOT_EINVAL, "k must be >= 1");
  if (!X_dev || !Y_dev) DOT_FAIL(DOT_EINVAL, "X_dev/Y_dev is NULL");
  const size_t bytes = (size_t)op->g.N * k * sizeof(double);
  const char* xa = (const char*)X_dev;
  const char* ya = (const char*)Y_dev;
  if (xa < ya + bytes && ya < xa + bytes) DOT_FAIL(DOT_EINVAL, "X_dev and Y_dev overlap");
  Geom G = make_geom(op->g, k);
  SweepArgs<double> a{};
  a.G = G;
  a.cx = op->cx;
  a.cy = op->cy;
  a.cz = op->cz;
  a.diag = op->diag;
  a.in0 = X_dev;
  a.out0 = Y_dev;
  return launch_sweep<M_APPLY, double>(op, a, as_stream(stream));
}

int dot_multigrid_levels(const dot_op* op) {
  return (op && op->mg_nlev >= 2 && op->mg_ok) ? op->mg_nlev : 0;
}

double dot_multigrid_cycle_bytes(const dot_op* op, int precision) {
  if (dot_multigrid_levels(op) == 0 || (precision != DOT_FP64 && precision != DOT_MIXED))
    return 0.0;
  return precision == DOT_FP64 ? mg_cycle_stream_bytes(op, sizeof(double), sizeof(double))
                                : mg_cycle_stream_bytes(op, sizeof(float), sizeof(bf16s));
}

// scaled vectors, r^ and z^, then the V-cycle's work vectors and dot slots
static size_t mg_apply_layout(const dot_op* op, int k, char* base, double** rh, double** zh,
                              MgWork<double>* w, double** partial) {
  const size_t nk = (size_t)op->g.N * k * sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  char* a = take(nk);
  char* b = take(nk);
  char* m = take(mg_work_bytes(op, k, op->g.N, sizeof(double)));
  char* p = take((size_t)2 * k * std::max(1, mg_partial_slots(op, k)) * sizeof(double));
  if (base) {
    *rh = (double*)a;
    *zh = (double*)b;
    mg_work_layout<double>(op, k, op->g.N, m, w);
    *partial = (double*)p;
  }
  return off;
}

size_t dot_multigrid_workspace_bytes(const dot_op* op, int k) {
  if (dot_multigrid_levels(op) == 0 || k < 1 || k > DOT_MAX_COLUMNS) return 0;
  return mg_apply_layout(op, k, nullptr, nullptr, nullptr, nullptr, nullptr);
}

// out[c + N j] = in[c + N j] / sd[c]
__global__ void div_sd_kernel(int64_t N, int k, const double* __restrict__ in,
                              const double* __restrict__ sd, double* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N * k) return;
  out[t] = in[t] / sd[t % N];
}

int dot_multigrid_apply(dot_op* op, int k, const double* R_dev, double* Z_dev, void* work_dev,
                        size_t work_bytes, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (dot_multigrid_levels(op) == 0) DOT_FAIL(DOT_EINVAL, "no multigrid hierarchy for this operator");
  if (k < 1 || k > DOT_MAX_COLUMNS) DOT_FAIL(DOT_EINVAL, "k must be in [1, %d]", DOT_MAX_COLUMNS);
  if (!R_dev || !Z_dev) DOT_FAIL(DOT_EINVAL, "R_dev/Z_dev is NULL");
  const size_t need = mg_apply_layout(op, k, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (!work_dev || work_bytes < need)
    DOT_FAIL(DOT_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
  if (((uintptr_t)work_dev & 255) != 0) DOT_FAIL(DOT_EINVAL, "work_dev must be 256-byte aligned");
  double *rh = nullptr, *zh = nullptr, *partial = nullptr;
  MgWork<double> w;
  mg_apply_layout(op, k, (char*)work_dev, &rh, &zh, &w, &partial);
  hipStream_t s = as_stream(stream);
  const unsigned blocks = (unsigned)((op->g.N * k + 255) / 256);
  hipLaunchKernelGGL(div_sd_kernel, dim3(blocks), dim3(256), 0, s, op->g.N, k, R_dev, op->sd, rh);
  DOT_LAUNCH_CHECK();
  DOT_TRY(mg_vcycle<double>(op, w, k, rh, op->g.N, zh, nullptr, partial, s));
  hipLaunchKernelGGL(div_sd_kernel, dim3(blocks), dim3(256), 0, s, op->g.N, k, zh, op->sd, Z_dev);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

int dot_solve_multi_rhs(dot_op* op, int trans, int k, const double* rhs_dev, double* x_dev,
                        const dot_solve_opts* opts, void* work_dev, size_t work_bytes,
                        dot_solve_info* info, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (trans != 0 && trans != 1) DOT_FAIL(DOT_EINVAL, "trans must be 0 or 1");
  if (k < 1 || k > DOT_MAX_COLUMNS) DOT_FAIL(DOT_EINVAL, "k must be in [1, %d]", DOT_MAX_COLUMNS);
  if (!rhs_dev || !x_dev) DOT_FAIL(DOT_EINVAL, "rhs_dev/x_dev is NULL");
  if (!opts) DOT_FAIL(DOT_EINVAL, "opts is NULL");
  if (opts->precision != DOT_FP64 && opts->precision != DOT_MIXED)
    DOT_FAIL(DOT_EINVAL, "opts.precision must be DOT_FP64 or DOT_MIXED");
  if (!(opts->rtol > 0.0) || !(opts->rtol < 1.0)) DOT_FAIL(DOT_EINVAL, "opts.rtol must be in (0, 1)");
  if (opts->max_iter < 1) DOT_FAIL(DOT_EINVAL, "opts.max_iter must be >= 1");
  if (opts->check_every < 1) DOT_FAIL(DOT_EINVAL, "opts.check_every must be >= 1");
  if (opts->precision == DOT_MIXED && (!(opts->inner_rtol > 0.0) || !(opts->inner_rtol < 1.0)))
    DOT_FAIL(DOT_EINVAL, "opts.inner_rtol must be in (0, 1)");
  const size_t bytes = (size_t)op->g.N * k * sizeof(double);
  const char* ra = (const char*)rhs_dev;
  const char* xa = (const char*)x_dev;
  if (ra < xa + bytes && xa < ra + bytes) DOT_FAIL(DOT_EINVAL, "rhs_dev and x_dev overlap");
  if (opts->precond != DOT_PRECOND_AUTO && opts->precond != DOT_PRECOND_JACOBI &&
      opts->precond != DOT_PRECOND_MG && opts->precond != DOT_PRECOND_MG_F32)
    DOT_FAIL(DOT_EINVAL, "opts.precond must be DOT_PRECOND_AUTO, _JACOBI, _MG or _MG_F32");
  const bool mg_req = opts->precond == DOT_PRECOND_MG || opts->precond == DOT_PRECOND_MG_F32;
  if (mg_req && op->mg_nlev < 2)
    DOT_FAIL(DOT_EINVAL, "no multigrid hierarchy for this grid (every side must be >= 5)");
  if (mg_req && !op->mg_ok)
    DOT_FAIL(DOT_EINVAL, "multigrid hierarchy has a non-positive diagonal on some level");
  const bool mg = op->mg_nlev >= 2 && op->mg_ok && opts->precond != DOT_PRECOND_JACOBI;
  Geom G = make_geom(op->g, k);
  const size_t need = layout_workspace(op, G, opts->precision, nullptr, nullptr);
  if (!work_dev || work_bytes < need)
    DOT_FAIL(DOT_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
  if (((uintptr_t)work_dev & 255) != 0) DOT_FAIL(DOT_EINVAL, "work_dev must be 256-byte aligned");
  const char* wa = (const char*)work_dev;
  if ((wa < xa + bytes && xa < wa + need) || (wa < ra + bytes && ra < wa + need))
    DOT_FAIL(DOT_EINVAL, "workspace overlaps rhs_dev or x_dev");
  Workspace ws;
  layout_workspace(op, G, opts->precision, (char*)work_dev, &ws,
                   opts->precond != DOT_PRECOND_MG_F32);
  hipStream_t s = as_stream(stream);
  int iters = 0, outer = 0;
  int rc = opts->precision == DOT_FP64
               ? solve_fp64(op, G, ws, rhs_dev, x_dev, *opts, mg, s, &iters)
               : solve_mixed(op, G, ws, rhs_dev, x_dev, *opts, mg, s, &iters, &outer);
  if (rc != DOT_OK) return rc;
  // per-column results
  std::vector<int> it_col(k), flags(k);
  std::vector<double> rel(k);
  DOT_HIP(hipMemcpyAsync(it_col.data(), ws.st.iters, k * sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipMemcpyAsync(flags.data(), ws.st.flags, k * sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipMemcpyAsync(rel.data(), ws.st.relres, k * sizeof(double), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  DOT_TRY(prof_drain(op));
  int imax = 0, fl = 0;
  bool conv = true;
  for (int j = 0; j < k; ++j) {
    imax = std::max(imax, it_col[j]);
    fl |= flags[j];
    if (!(rel[j] <= opts->rtol)) conv = false;
  }
  if (info) {
    info->iters_max = imax;
    info->outer = outer;
    if (info->iters_host)
      for (int j = 0; j < k; ++j) info->iters_host[j] = it_col[j];
    if (info->relres_host)
      for (int j = 0; j < k; ++j) info->relres_host[j] = rel[j];
  }
  if (fl & FLAG_NONFINITE) DOT_FAIL(DOT_ENONFINITE, "non-finite values in the solve");
  if (fl & FLAG_BREAKDOWN) DOT_FAIL(DOT_EBREAKDOWN, "CG breakdown: p^T A p <= 0 or r^T M^-1 r <= 0");
  if (!conv) {
    set_error("not converged: max relres above rtol after %d iterations", iters);
    return DOT_NOT_CONVERGED;
  }
  return DOT_OK;
}

int dot_profile_enable(dot_op* op, int enable) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  ProfState* p = prof_of(op);
  if (!p) {
    p = new ProfState();
    op->prof = p;
    hipError_t e = hipMalloc(&p->cols_dev, kProfSlots * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(p->cols_dev, 0, kProfSlots * sizeof(unsigned long long));
    if (e != hipSuccess) DOT_FAIL(DOT_EHIP, "hipMalloc: %s", hipGetErrorString(e));
  }
  DOT_TRY(prof_drain(op));
  p->on = enable != 0;
  p->mask = ~0u;
  for (int i = 0; i < DOT_PROF_KINDS; ++i) {
    p->ms[i] = 0.0;
    p->launches[i] = 0;
    p->cols[i] = 0;
  }
  return DOT_OK;
}

int dot_profile_kinds(dot_op* op, unsigned mask) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  ProfState* p = prof_of(op);
  if (!p) DOT_FAIL(DOT_EINVAL, "profiling was never enabled on this handle");
  p->mask = mask;
  return DOT_OK;
}

int dot_profile_read(dot_op* op, int kind, double* ms_total, int64_t* launches,
                     int64_t* column_sweeps) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (kind < 0 || kind >= DOT_PROF_KINDS) DOT_FAIL(DOT_EINVAL, "unknown profile kind %d", kind);
  ProfState* p = prof_of(op);
  if (!p) DOT_FAIL(DOT_EINVAL, "profiling was never enabled on this handle");
  DOT_HIP(hipDeviceSynchronize());
  DOT_TRY(prof_drain(op));
  if (ms_total) *ms_total = p->ms[kind];
  if (launches) *launches = p->launches[kind];
  if (column_sweeps) *column_sweeps = (int64_t)p->cols[kind];
  return DOT_OK;
}

}  // extern "C"

namespace dot {
void destroy_profile(dot_op* op) {
  ProfState* p = prof_of(op);
  if (!p) return;
  for (auto& q : p->pending) {
    (void)hipEventDestroy(q.e0);
    (void)hipEventDestroy(q.e1);
  }
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  if (p->cols_dev) (void)hipFree(p->cols_dev);
  delete p;
  op->prof = nullptr;
}

// Used by the contraction to time itself when profiling is on.
int profile_begin(dot_op* op, int kind, hipStream_t s, hipEvent_t* e0, hipEvent_t* e1,
                  unsigned long long** cols) {
  return prof_begin(op, kind, s, e0, e1, cols);
}
int profile_end(dot_op* op, int kind, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return prof_end(op, kind, s, e0, e1);
}
}  // namespace dot
