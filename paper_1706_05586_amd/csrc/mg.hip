// Geometric multigrid V-cycle: the preconditioner of the multi-right-hand-side
// CG (the forward and adjoint solves of Section 3.3), on 3D and 2D grids.
//
// The CG runs on the symmetrically scaled system A^ = S^-1 A S^-1 (S =
// sqrt(diag A)); its preconditioner is z = S V(S r), V one V-cycle for A.
// Every level is kept in scaled form (unit diagonal), so with P the
// piecewise-constant prolongation (a coarse value copied to the 2 x 2 x 2
// children of its aggregate; 2 x 2 in 2D, fewer in the last aggregate of an
// odd side) the transfers between level l (scaling S_l)
// and level l + 1 (S_{l+1}) are
//     prolongation  x^_l += S_l P S_{l+1}^-1 x^_{l+1}   (weight q = sd / sd_parent)
//     restriction   b^_{l+1} = S_{l+1}^-1 P^T S_l r^_l   (its transpose)
// and the coarse operator is the same finite-volume discretization on the
// coarse cells (D and mu averaged over the children).  One V-cycle, with
// nu_l damped Jacobi steps J(v) = v + w (b - A^ v) each way on level l:
//     down, level l:  x = J^(nu_l - 1)(w b);  b_{l+1} = R (b - A^ x)
//     coarsest:       NU_C Jacobi steps from zero
//     up, level l:    z = J^nu_l(x + P z_{l+1})
// with w = MG_OMEGA.  Every kernel does one step or the restriction, forming
// w b from b rather than storing it.  Pre- and post-smoothing are the same
// symmetric Jacobi step, equally many, and R = P^T, so the preconditioner is
// symmetric; it is positive definite because w < 2 / lambda_max(A^) for
// these diagonally dominant operators (lambda_max <= 2) and every coarse
// correction is positive semidefinite.  The coarse levels, where steps cost
// little, take more of them.  The last step on level 0 also forms r . z per
// column.
//
// Kernel layout: a block is a 64 x 4 (x, y) tile, one wave per row of 64
// cells (a bfloat16 row is one full 128-byte line), marching through an even
// chunk of z planes with the z neighbours in registers and the x/y
// neighbours from a double-buffered LDS plane; a block handles MRG columns
// so coefficients are read once per group.  A 2 x 2 aggregate of a plane is
// lanes l, l ^ 1 of two waves: the x pair is a wave shuffle, the z pair is
// summed in registers, and the odd row hands its sum to the even row through
// LDS at the next barrier.  Results are deterministic: the coarse sums are
// formed in a fixed order and the dot products reduce through wave shuffles
// and per-block partial slots.
#include <algorithm>
#include <type_traits>

#include "dot_internal.h"

namespace dot {

constexpr int MTX = 64;                 // tile width: one wave
constexpr int MTY = 4;                  // tile rows: one per wave
constexpr int MNT = MTX * MTY;          // 256 threads
constexpr int MNH = 2 * MTX + 2 * MTY;  // halo cells of a tile
static_assert(MNT >= MNH, "every halo cell needs a thread");
constexpr int MRG = 4;                  // columns per block
constexpr int MG_NU_C = 8;              // Jacobi steps on the coarsest level

constexpr int MG_NU0 = 2;               // smoothing steps each way on the finest level
constexpr int MG_NU1 = 3;               // ... on level 1
constexpr int MG_NU2 = 5;               // ... and on the coarser levels above the coarsest
#define MG_OMEGA 0.85

__host__ __device__ inline int mg_nu(int level) {
  return level == 0 ? MG_NU0 : (level == 1 ? MG_NU1 : MG_NU2);
}

// MG_DOWN: restriction of the residual of the staged iterate;
// MG_SMOOTH: one damped Jacobi step from the staged iterate
enum MgMode { MG_DOWN = 0, MG_SMOOTH = 1 };

struct MgGeom {
  int nx, ny, nz;
  int64_t nxy;
  int tiles_x, ntiles, zc, nzc;  // zc even
  int cnx, cny;                  // coarse level (down: written, up: read)
  int64_t cnxy;
};

// T: arithmetic and coefficients; TB: the right-hand side b; TS: the
// stored iterates and coarse vectors; TO: the smoothing result
template <typename T, typename TB, typename TS, typename TO>
struct MgArgs {
  MgGeom G;
  int k;
  const T* sx;
  const T* sy;
  const T* sz;
  const T* sd;         // down: sqrt(diag) of this level
  const T* sdc;        // down: sqrt(diag) of the coarse level
  const T* q;          // prolongation: sd / sd_coarse(parent)
  const int* active;   // columns to process (NULL = all)
  const TB* b;         // right-hand side of this level (ld)
  const TS* x;         // staged iterate (ld; the kernels without it form w b)
  const TS* xc;        // coarse correction added to it (cld)
  TO* out;             // smoothing: result (ld)
  TS* bc;              // down: coarse right-hand side (cld)
  int64_t ld, cld;
  double* partial;     // smoothing: [2][k][nblk] slots of b . out (or NULL)
  unsigned long long* prof_cols;  // optional: += active columns of the launch
  int nblk;
};

static MgGeom mg_geom(const GridDims& g, const GridDims* gc, int k) {
  MgGeom G{};
  G.nx = g.nx;
  G.ny = g.ny;
  G.nz = g.nz;
  G.nxy = g.nxy;
  G.tiles_x = (g.nx + MTX - 1) / MTX;
  G.ntiles = G.tiles_x * ((g.ny + MTY - 1) / MTY);
  // z chunks: aim for about 1280 blocks (at 128^3 x 40 columns two chunks of
  // 64 planes per tile and column group; 640 blocks or 960 gave fewer chunks
  // on the coarse levels and were slower, 2048 took 1.5% longer per
  // V-cycle), chunks of an even number of planes
  const int groups = (k + MRG - 1) / MRG;
  const int64_t per_z = (int64_t)G.ntiles * groups;
  int nzc = (int)std::min<int64_t>(std::max(1, g.nz / 2), std::max<int64_t>(1, (1280 + per_z - 1) / per_z));
  int zc = (g.nz + nzc - 1) / nzc;
  zc += zc & 1;
  G.zc = zc;
  G.nzc = (g.nz + zc - 1) / zc;
  if (gc) {
    G.cnx = gc->nx;
    G.cny = gc->ny;
    G.cnxy = gc->nxy;
  }
  return G;
}

template <typename T>
__device__ __forceinline__ T mg_ld(const T* p, int64_t i) {
  return p[i];
}
// loads and stores of the work vectors in their storage type
template <typename T>
__device__ __forceinline__ T mg_ldv(const float* p, int64_t i) {
  return (T)p[i];
}
template <typename T>
__device__ __forceinline__ T mg_ldv(const double* p, int64_t i) {
  return (T)p[i];
}
template <typename T>
__device__ __forceinline__ T mg_ldv(const bf16s* p, int64_t i) {
  return (T)__uint_as_float((unsigned)p[i].u << 16);
}
__device__ __forceinline__ void mg_stv(float* p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void mg_stv(double* p, int64_t i, double v) { p[i] = v; }
__device__ __forceinline__ void mg_stv(bf16s* p, int64_t i, float v) {
  unsigned u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  p[i].u = (unsigned short)(u >> 16);
}

// The staged iterate v of a level kernel is x (HX) or w b, plus q xc(parent)
// with the prolongation (HC).  MG_DOWN writes the restriction of b - A^ v,
// MG_SMOOTH writes v + w (b - A^ v).
template <int MODE, bool HX, bool HC, typename T, typename TB, typename TS, typename TO>
__global__ __launch_bounds__(MNT) void mg_level_kernel(MgArgs<T, TB, TS, TO> a) {
  const MgGeom& G = a.G;
  const int groups = (a.k + MRG - 1) / MRG;
  // column groups fastest, then tiles: the blocks of one tile and its x
  // neighbours run on one XCD and share coefficient and halo lines in its L2
  const int logical = xcd_remap_block((int)blockIdx.x, (int)gridDim.x);
  const int grp = logical % groups;
  const int rest = logical / groups;
  const int tile = rest % G.ntiles, zci = rest / G.ntiles;
  const int slot = tile + G.ntiles * zci;
  const int x0 = (tile % G.tiles_x) * MTX, y0 = (tile / G.tiles_x) * MTY;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tx = lane, ty = wave;
  const int x = x0 + tx, y = y0 + ty;
  const bool in = x < G.nx && y < G.ny;
  const int z0 = zci * G.zc, z1 = min(G.nz, z0 + G.zc);
  const T w = (T)MG_OMEGA;
  __shared__ T sm[2][MRG][MTY + 2][MTX + 2];
  // restriction: the odd rows' sums over a completed aggregate (even lanes)
  __shared__ T xr[MODE == MG_DOWN ? MRG : 1][MTY / 2][MTX / 2];

  bool act[MRG];
  int64_t col[MRG];
  bool any = false;
#pragma unroll
  for (int r = 0; r < MRG; ++r) {
    const int j = grp * MRG + r;
    act[r] = j < a.k && (a.active == nullptr || a.active[j] != 0);
    col[r] = j < a.k ? j : 0;
    any |= act[r];
  }
  if (!any) return;  // uniform over the block
  if (a.prof_cols && tile == 0 && zci == 0 && threadIdx.x == 0) {
    int n = 0;
#pragma unroll
    for (int r = 0; r < MRG; ++r) n += act[r] ? 1 : 0;
    atomicAdd(a.prof_cols, (unsigned long long)n);
  }

  // halo cell owned by this thread (if any)
  int hx = -1, hy = -1, hsy = 0, hsx = 0;
  const bool hthread = threadIdx.x < MNH;
  if (hthread) {
    const int s = threadIdx.x;
    if (s < MTX) {
      hx = x0 + s; hy = y0 - 1; hsy = 0; hsx = s + 1;
    } else if (s < 2 * MTX) {
      hx = x0 + s - MTX; hy = y0 + MTY; hsy = MTY + 1; hsx = s - MTX + 1;
    } else if (s < 2 * MTX + MTY) {
      hx = x0 - 1; hy = y0 + s - 2 * MTX; hsy = s - 2 * MTX + 1; hsx = 0;
    } else {
      hx = x0 + MTX; hy = y0 + s - 2 * MTX - MTY; hsy = s - 2 * MTX - MTY + 1; hsx = MTX + 1;
    }
  }
  const bool hin = hx >= 0 && hx < G.nx && hy >= 0 && hy < G.ny;
  // clamped cells: every load is in bounds, values of cells outside the
  // domain are replaced by zero where they are used
  const int64_t hbase = hin ? hx + (int64_t)G.nx * hy : 0;
  const int64_t base = in ? x + (int64_t)G.nx * y : 0;
  // parents (up): coarse (x/2, y/2) of the own and the halo cell
  const int64_t pbase = in ? (x >> 1) + (int64_t)G.cnx * (y >> 1) : 0;
  const int64_t phbase = hin ? (hx >> 1) + (int64_t)G.cnx * (hy >> 1) : 0;

  // Raw loads of a cell's staged value (b, and x, q and xc(parent) where the
  // kernel has them) are combined only where the value is used: the own
  // cell's next plane after the barrier, the halo cell's next plane at the
  // following plane's LDS store, so no load is waited for before the barrier
  // that follows it.  The own cell's raw b of plane z is carried to the
  // residual b - A^ v of that plane.
  struct Raw {
    T v[MRG];
    T x[MRG];
    T xc[MRG];
    T q;
  };
  // Every load is unconditional: the odd plane reloads its aggregate's
  // parent (a cache hit) rather than keep the even plane's, because a load
  // issued on one path only makes the compiler wait for every load in
  // flight (the counter retires in order) where the paths join.
  auto load_raw = [&](int64_t c, int64_t p, Raw& o) {
#pragma unroll
    for (int r = 0; r < MRG; ++r) {
      o.v[r] = mg_ldv<T>(a.b, c + a.ld * col[r]);
      if constexpr (HX) o.x[r] = mg_ldv<T>(a.x, c + a.ld * col[r]);
      if constexpr (HC) o.xc[r] = mg_ldv<T>(a.xc, p + a.cld * col[r]);
    }
    if constexpr (HC) o.q = mg_ld(a.q, c);
  };
  auto staged = [&](const Raw& o, int r) -> T {
    T v;
    if constexpr (HX) {
      v = o.x[r];
    } else {
      v = w * o.v[r];
    }
    if constexpr (HC) v += o.q * o.xc[r];
    return v;
  };

  T vm[MRG], vc[MRG], bcur[MRG];
  Raw pr;  // own cell, plane z + 1 (its coarse values carried between planes)
  {
    Raw om;
    const int zm = z0 > 0 ? z0 - 1 : z0;
    load_raw(base + zm * G.nxy, pbase + (zm >> 1) * G.cnxy, om);
    load_raw(base + z0 * G.nxy, pbase + (z0 >> 1) * G.cnxy, pr);
#pragma unroll
    for (int r = 0; r < MRG; ++r) {
      vm[r] = (z0 > 0 && in) ? staged(om, r) : T(0);
      vc[r] = in ? staged(pr, r) : T(0);
      bcur[r] = pr.v[r];
    }
  }
  Raw hr;  // halo cell, plane z
  load_raw(hbase + z0 * G.nxy, phbase + (z0 >> 1) * G.cnxy, hr);
  T cD = z0 > 0 ? mg_ld(a.sz, base + (z0 - 1) * G.nxy) : T(0);
  T sdc_next = T(1);
  T zacc[MRG];
  double acc[MRG];
#pragma unroll
  for (int r = 0; r < MRG; ++r) {
    zacc[r] = T(0);
    acc[r] = 0.0;
  }
  // restriction: an aggregate completed on the previous plane (its coarse
  // plane and sqrt(diag)) is written by the even row once the barrier has
  // made the odd row's sum visible
  bool pend = false;
  int pzc = 0;
  T psdc = T(1);
  auto write_coarse = [&]() {
    if constexpr (MODE == MG_DOWN) {
      if ((ty & 1) == 0 && in && (lane & 1) == 0) {
        const int64_t C = (x >> 1) + (int64_t)G.cnx * (y >> 1) + G.cnxy * pzc;
#pragma unroll
        for (int r = 0; r < MRG; ++r) {
          if (!act[r]) continue;
          mg_stv(a.bc, C + a.cld * col[r], (zacc[r] + xr[r][ty >> 1][lane >> 1]) / psdc);
        }
      }
    }
  };

  for (int z = z0; z < z1; ++z) {
    const int buf = (z - z0) & 1;
    const int64_t c = base + z * G.nxy;
    const bool has_up = z + 1 < G.nz;
    const int zu = has_up ? z + 1 : z;
#pragma unroll
    for (int r = 0; r < MRG; ++r) sm[buf][r][ty + 1][tx + 1] = vc[r];
    if (hthread) {
#pragma unroll
      for (int r = 0; r < MRG; ++r) sm[buf][r][hsy][hsx] = hin ? staged(hr, r) : T(0);
    }
    // loads for after the barrier: own cell of plane z + 1, this plane's
    // right-hand side and coefficients; then the halo of plane z + 1
    load_raw(base + zu * G.nxy, pbase + (zu >> 1) * G.cnxy, pr);
    const bool has_w = in && x > 0, has_s = in && y > 0;
    const T cE = mg_ld(a.sx, c);
    const T cWl = mg_ld(a.sx, has_w ? c - 1 : c);
    const T cN = mg_ld(a.sy, c);
    const T cSl = mg_ld(a.sy, has_s ? c - G.nx : c);
    const T cU = mg_ld(a.sz, c);
    const T sdv = MODE == MG_DOWN ? mg_ld(a.sd, c) : T(0);
    // the aggregate's coarse sqrt(diag), loaded on the even plane for the
    // odd plane's write
    if (MODE == MG_DOWN && (z & 1) == 0)
      sdc_next = mg_ld(a.sdc, in ? (x >> 1) + (int64_t)G.cnx * (y >> 1) + G.cnxy * (z >> 1) : 0);
    load_raw(hbase + zu * G.nxy, phbase + (zu >> 1) * G.cnxy, hr);
    __syncthreads();
    if constexpr (MODE == MG_DOWN) {
      if (pend) write_coarse();  // block-uniform
      pend = false;
    }
    const T cW = has_w ? cWl : T(0);
    const T cS = has_s ? cSl : T(0);
    T vp[MRG];
#pragma unroll
    for (int r = 0; r < MRG; ++r) vp[r] = (has_up && in) ? staged(pr, r) : T(0);
#pragma unroll
    for (int r = 0; r < MRG; ++r) {
      if (!act[r]) continue;  // block-uniform
      const T vW = sm[buf][r][ty + 1][tx], vE = sm[buf][r][ty + 1][tx + 2];
      const T vS = sm[buf][r][ty][tx + 1], vN = sm[buf][r][ty + 2][tx + 1];
      const T Av = vc[r] - cW * vW - cE * vE - cS * vS - cN * vN - cD * vm[r] - cU * vp[r];
      const T bv = bcur[r];
      if constexpr (MODE == MG_DOWN) {
        // restriction: S_l (b - A^ x) summed over the aggregate (cells
        // outside the grid contribute zero): the x pair here, the z pair
        // in registers, the y pair at the coarse write
        const T e = in ? sdv * (bv - Av) : T(0);
        const T s2 = e + __shfl_xor(e, 1, 64);
        if ((z & 1) == 0) zacc[r] = s2;
        else zacc[r] += s2;
        // the aggregate is complete after its odd plane, or after an even
        // plane that is the last of an odd n_z (also the one plane in 2D)
        if (((z & 1) == 1 || z + 1 == G.nz) && (ty & 1) == 1 && (lane & 1) == 0)
          xr[r][ty >> 1][lane >> 1] = zacc[r];
      } else {
        const T zv = vc[r] + w * (bv - Av);
        if (in) {
          mg_stv(a.out, c + a.ld * col[r], zv);
          acc[r] += (double)bv * (double)zv;
        }
      }
    }
    if constexpr (MODE == MG_DOWN) {
      if ((z & 1) == 1 || z + 1 == G.nz) {
        pend = true;
        pzc = z >> 1;
        psdc = sdc_next;
      }
    }
    cD = cU;
#pragma unroll
    for (int r = 0; r < MRG; ++r) {
      vm[r] = vc[r];
      vc[r] = vp[r];
      bcur[r] = pr.v[r];
    }
  }
  if constexpr (MODE == MG_DOWN) {
    if (pend) {  // the chunk's last aggregate
      __syncthreads();
      write_coarse();
    }
  }
  if constexpr (MODE == MG_SMOOTH) {
    if (a.partial) {
      __shared__ double red[MNT / 64][MRG];
#pragma unroll
      for (int r = 0; r < MRG; ++r) {
        double v = acc[r];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][r] = v;
      }
      __syncthreads();
      if (threadIdx.x < MRG) {
        const int r = threadIdx.x;
        const int j = grp * MRG + r;
        if (j < a.k) {
          double s = 0.0;
          for (int q = 0; q < MNT / 64; ++q) s += red[q][r];
          a.partial[(int64_t)j * a.nblk + slot] = s;
          a.partial[((int64_t)a.k + j) * a.nblk + slot] = 0.0;
        }
      }
    }
  }
}

// One damped Jacobi step on the coarsest level, one thread per cell and
// column: out = in + w (b - A^ in), or out = w b when in is NULL.
template <typename T, typename TS>
__global__ __launch_bounds__(256) void mg_jacobi_kernel(GridDims g, int k, const T* __restrict__ sx,
                                                        const T* __restrict__ sy,
                                                        const T* __restrict__ sz,
                                                        const int* __restrict__ active,
                                                        const TS* __restrict__ b,
                                                        const TS* __restrict__ xin,
                                                        TS* __restrict__ out, int64_t ld) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= g.N * k) return;
  const int j = (int)(t / g.N);
  const int64_t c = t - (int64_t)j * g.N;
  if (active && active[j] == 0) return;
  const T w = (T)MG_OMEGA;
  const TS* bj = b + ld * j;
  TS* oj = out + ld * j;
  if (!xin) {
    mg_stv(oj, c, w * mg_ldv<T>(bj, c));
    return;
  }
  const TS* xj = xin + ld * j;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / g.nxy);
  auto X = [&](int64_t i) { return mg_ldv<T>(xj, i); };
  T Av = X(c) - sx[c] * (x + 1 < g.nx ? X(c + 1) : T(0)) - sy[c] * (y + 1 < g.ny ? X(c + g.nx) : T(0)) -
         sz[c] * (z + 1 < g.nz ? X(c + g.nxy) : T(0));
  if (x > 0) Av -= sx[c - 1] * X(c - 1);
  if (y > 0) Av -= sy[c - g.nx] * X(c - g.nx);
  if (z > 0) Av -= sz[c - g.nxy] * X(c - g.nxy);
  mg_stv(oj, c, X(c) + w * (mg_ldv<T>(bj, c) - Av));
}

// The coarse tail of the V-cycle in one launch: the levels from the first
// one of at most MG_TAIL_MAXN cells down to the coarsest, one block per
// column with every vector of those levels in LDS (b, and two iterates per
// level).  Each thread owns the cells tid + MG_TAIL_THREADS i of a level
// and keeps their coefficients in registers while it works on that level.
// The arithmetic is that of the level kernels (the same steps, the
// restriction summed over the eight children in a fixed order).
constexpr int MG_TAIL_THREADS = 512;
constexpr int MG_TAIL_CPT = 8;
constexpr int MG_TAIL_MAXN = MG_TAIL_THREADS * MG_TAIL_CPT;
constexpr size_t MG_TAIL_MAXBYTES = 144 * 1024;

template <typename T>
struct MgTailLevel {
  int nx, ny, nz, N;
  const T* sx;
  const T* sy;
  const T* sz;
  const double* sd;  // sqrt(diag)
  const T* q;        // prolongation weights (all but the coarsest)
  int off;           // LDS element offset of b; the iterates follow at off + N, off + 2 N
  int nu;            // smoothing steps each way
};

template <typename T, typename TS>
struct MgTailArgs {
  int nl;  // tail levels; L[nl - 1] is the coarsest
  MgTailLevel<T> L[DOT_MG_MAXLEV];
  int k;
  const int* active;
  const TS* b;  // right-hand side of L[0] (global, ldb)
  TS* z;        // result of L[0] (global, ldz)
  int64_t ldb, ldz;
};

template <typename T, typename TS>
__global__ __launch_bounds__(MG_TAIL_THREADS) void mg_tail_kernel(MgTailArgs<T, TS> a) {
  extern __shared__ __align__(16) unsigned char mg_tail_smem[];
  T* S = reinterpret_cast<T*>(mg_tail_smem);
  const int j = blockIdx.x;
  if (j >= a.k || (a.active && a.active[j] == 0)) return;  // uniform
  const int t = threadIdx.x;
  const T w = (T)MG_OMEGA;

  // per-thread cells of the current level: coefficients and neighbour flags
  T cE[MG_TAIL_CPT], cW[MG_TAIL_CPT], cN[MG_TAIL_CPT], cS[MG_TAIL_CPT], cU[MG_TAIL_CPT],
      cD[MG_TAIL_CPT];
  int fl[MG_TAIL_CPT];  // bit 0..5: has -x, +x, -y, +y, -z, +z neighbour
  auto prepare = [&](const MgTailLevel<T>& L) {
#pragma unroll
    for (int i = 0; i < MG_TAIL_CPT; ++i) {
      const int c = t + MG_TAIL_THREADS * i;
      fl[i] = 0;
      cE[i] = cW[i] = cN[i] = cS[i] = cU[i] = cD[i] = T(0);
      if (c < L.N) {
        const int x = c % L.nx, y = (c / L.nx) % L.ny, z = c / (L.nx * L.ny);
        const int nxy = L.nx * L.ny;
        fl[i] = (x > 0) | ((x + 1 < L.nx) << 1) | ((y > 0) << 2) | ((y + 1 < L.ny) << 3) |
                ((z > 0) << 4) | ((z + 1 < L.nz) << 5);
        cE[i] = L.sx[c];
        cN[i] = L.sy[c];
        cU[i] = L.sz[c];
        if (x > 0) cW[i] = L.sx[c - 1];
        if (y > 0) cS[i] = L.sy[c - L.nx];
        if (z > 0) cD[i] = L.sz[c - nxy];
      }
    }
  };
  // A^ v at owned cell i (c) of a level from the LDS vector v
  auto apply = [&](const MgTailLevel<T>& L, const T* v, int i, int c) -> T {
    const int nxy = L.nx * L.ny;
    const int f = fl[i];
    const T vW = v[(f & 1) ? c - 1 : c], vE = v[(f & 2) ? c + 1 : c];
    const T vS = v[(f & 4) ? c - L.nx : c], vN = v[(f & 8) ? c + L.nx : c];
    const T vD = v[(f & 16) ? c - nxy : c], vU = v[(f & 32) ? c + nxy : c];
    return v[c] - cW[i] * vW - cE[i] * vE - cS[i] * vS - cN[i] * vN - cD[i] * vD - cU[i] * vU;
  };
  // out = J(in) = in + w (b - A^ in); in == NULL: in = w b
  auto jstep = [&](const MgTailLevel<T>& L, const T* b, const T* in, T* out) {
    if (in == nullptr) {
      for (int c = t; c < L.N; c += MG_TAIL_THREADS) out[c] = w * b[c];
      __syncthreads();
      return;
    }
#pragma unroll
    for (int i = 0; i < MG_TAIL_CPT; ++i) {
      const int c = t + MG_TAIL_THREADS * i;
      if (c < L.N) out[c] = in[c] + w * (b[c] - apply(L, in, i, c));
    }
    __syncthreads();
  };

  const MgTailLevel<T>& L0 = a.L[0];
  for (int c = t; c < L0.N; c += MG_TAIL_THREADS) S[L0.off + c] = mg_ldv<T>(a.b, c + a.ldb * j);
  __syncthreads();
  const T* pre[DOT_MG_MAXLEV];
  // down: x = J^(nu - 1)(w b), restriction of b - A^ x
  for (int l = 0; l + 1 < a.nl; ++l) {
    const MgTailLevel<T>& L = a.L[l];
    const MgTailLevel<T>& C = a.L[l + 1];
    T* b = S + L.off;
    T* buf[2] = {S + L.off + L.N, S + L.off + 2 * L.N};
    prepare(L);
    jstep(L, b, nullptr, buf[0]);
    int cur = 0;
    for (int s = 1; s < L.nu; ++s) {
      jstep(L, b, buf[cur], buf[cur ^ 1]);
      cur ^= 1;
    }
    const T* x = buf[cur];
    T* r = buf[cur ^ 1];
#pragma unroll
    for (int i = 0; i < MG_TAIL_CPT; ++i) {
      const int c = t + MG_TAIL_THREADS * i;
      if (c < L.N) r[c] = (T)L.sd[c] * (b[c] - apply(L, x, i, c));
    }
    __syncthreads();
    T* bc = S + C.off;
    const int nxy = L.nx * L.ny;
    for (int cc = t; cc < C.N; cc += MG_TAIL_THREADS) {
      const int X = cc % C.nx, Y = (cc / C.nx) % C.ny, Z = cc / (C.nx * C.ny);
      const int f0 = 2 * X + L.nx * (2 * Y) + nxy * (2 * Z);
      const int ex = min(2, L.nx - 2 * X), ey = min(2, L.ny - 2 * Y), ez = min(2, L.nz - 2 * Z);
      T s = T(0);
      for (int dz = 0; dz < ez; ++dz)
        for (int dy = 0; dy < ey; ++dy)
          for (int dx = 0; dx < ex; ++dx) s += r[f0 + dx + L.nx * dy + nxy * dz];
      bc[cc] = s / (T)C.sd[cc];
    }
    __syncthreads();
    pre[l] = x;
  }
  // coarsest: MG_NU_C steps from zero
  const T* zc;
  {
    const MgTailLevel<T>& L = a.L[a.nl - 1];
    T* b = S + L.off;
    T* buf[2] = {S + L.off + L.N, S + L.off + 2 * L.N};
    prepare(L);
    jstep(L, b, nullptr, buf[0]);
    int cur = 0;
    for (int s = 1; s < MG_NU_C; ++s) {
      jstep(L, b, buf[cur], buf[cur ^ 1]);
      cur ^= 1;
    }
    zc = buf[cur];
  }
  // up: y = x + P z_{l+1}, then nu steps
  for (int l = a.nl - 2; l >= 0; --l) {
    const MgTailLevel<T>& L = a.L[l];
    const MgTailLevel<T>& C = a.L[l + 1];
    T* b = S + L.off;
    T* buf[2] = {S + L.off + L.N, S + L.off + 2 * L.N};
    const int xi = pre[l] == buf[0] ? 0 : 1;
    T* y = buf[xi ^ 1];
    const int nxy = L.nx * L.ny;
    for (int c = t; c < L.N; c += MG_TAIL_THREADS) {
      const int x = c % L.nx, yy = (c / L.nx) % L.ny, z = c / nxy;
      const int p = (x >> 1) + C.nx * ((yy >> 1) + C.ny * (z >> 1));
      y[c] = pre[l][c] + L.q[c] * zc[p];
    }
    __syncthreads();
    prepare(L);
    int cur = xi ^ 1;
    for (int s = 0; s < L.nu; ++s) {
      jstep(L, b, buf[cur], buf[cur ^ 1]);
      cur ^= 1;
    }
    zc = buf[cur];
  }
  for (int c = t; c < L0.N; c += MG_TAIL_THREADS) mg_stv(a.z, c + a.ldz * j, zc[c]);
}

static size_t mg_al(size_t v) { return (v + 255) & ~(size_t)255; }

// Column stride of a coarse level's vectors: a larger level's columns are
// padded so that the columns of a block's group do not sit a power of two
// apart.
static int64_t mg_ld_of(int64_t N) { return N >= 8192 ? N + 1088 : N; }

size_t mg_work_bytes(const dot_op* op, int k, int64_t ld0, size_t elem, int level0_iterates) {
  if (op->mg_nlev < 2) return 0;
  size_t off = MG_NU0 >= 2 ? (size_t)level0_iterates * mg_al((size_t)ld0 * k * elem) : 0;
  for (int l = 1; l < op->mg_nlev; ++l) off += 3 * mg_al((size_t)mg_ld_of(op->mg[l].g.N) * k * elem);
  return off;
}

template <typename T>
void mg_work_layout(const dot_op* op, int k, int64_t ld0, char* base, MgWork<T>* w,
                    int level0_iterates) {
  *w = MgWork<T>{};
  if (op->mg_nlev < 2) return;
  w->nlev = op->mg_nlev;
  w->ld[0] = ld0;
  size_t off = 0;
  if (MG_NU0 >= 2) {
    const size_t bytes = mg_al((size_t)ld0 * k * sizeof(T));
    w->x[0] = reinterpret_cast<T*>(base);
    off += bytes;
    if (level0_iterates > 1) {
      w->z[0] = reinterpret_cast<T*>(base + off);
      off += bytes;
    }
  }
  for (int l = 1; l < op->mg_nlev; ++l) {
    w->ld[l] = mg_ld_of(op->mg[l].g.N);
    const size_t bytes = mg_al((size_t)w->ld[l] * k * sizeof(T));
    w->b[l] = reinterpret_cast<T*>(base + off);
    off += bytes;
    w->x[l] = reinterpret_cast<T*>(base + off);
    off += bytes;
    w->z[l] = reinterpret_cast<T*>(base + off);
    off += bytes;
  }
}
template void mg_work_layout<float>(const dot_op*, int, int64_t, char*, MgWork<float>*, int);
template void mg_work_layout<double>(const dot_op*, int, int64_t, char*, MgWork<double>*, int);
template void mg_work_layout<bf16s>(const dot_op*, int, int64_t, char*, MgWork<bf16s>*, int);

int mg_partial_slots(const dot_op* op, int k) {
  if (op->mg_nlev < 2) return 0;
  const MgGeom G = mg_geom(op->mg[0].g, &op->mg[1].g, k);
  return G.ntiles * G.nzc;
}

template <typename T>
struct MgCoef;
template <>
struct MgCoef<double> {
  static const double* sx(const MgLevel& L) { return L.sx; }
  static const double* sy(const MgLevel& L) { return L.sy; }
  static const double* sz(const MgLevel& L) { return L.sz; }
  static const double* q(const MgLevel& L) { return L.q; }
  static const double* sd(const MgLevel& L) { return L.sd; }
};
template <>
struct MgCoef<float> {
  static const float* sx(const MgLevel& L) { return L.sx32; }
  static const float* sy(const MgLevel& L) { return L.sy32; }
  static const float* sz(const MgLevel& L) { return L.sz32; }
  static const float* q(const MgLevel& L) { return L.q32; }
  static const float* sd(const MgLevel& L) { return L.sd32; }
};

template <int MODE, bool HX, bool HC, typename T, typename TB, typename TS, typename TO>
static void mg_launch(const MgArgs<T, TB, TS, TO>& a, int groups, hipStream_t s) {
  const int blocks = a.G.ntiles * a.G.nzc * groups;
  hipLaunchKernelGGL((mg_level_kernel<MODE, HX, HC, T, TB, TS, TO>), dim3(blocks), dim3(MNT), 0, s, a);
}

// The coarse tail run by mg_tail_kernel: levels t0 .. nl - 1 (t0 >= 1), the
// levels of at most MG_TAIL_MAXN cells whose three vectors fit in LDS
// together; t0 = nl: none, the coarsest level then takes MG_NU_C Jacobi
// launches.  *tail_bytes receives the LDS bytes of the tail.
static int mg_tail_start(const dot_op* op, size_t elem, size_t* tail_bytes) {
  const int nl = op->mg_nlev;
  int t0 = nl;
  size_t tb = 0;
  for (int l = nl - 1; l >= 1; --l) {
    const size_t bytes = tb + 3 * (size_t)op->mg[l].g.N * elem;
    if (op->mg[l].g.N > MG_TAIL_MAXN || bytes > MG_TAIL_MAXBYTES) break;
    tb = bytes;
    t0 = l;
  }
  *tail_bytes = tb;
  return t0;
}

// Level 0's smoothing outputs: with S = T they alternate between z0 and
// w.x[0], the first and the last in z0 (2 nu - 1 of them); with a narrower
// S they alternate between w.z[0] and w.x[0] and the last one is z0.  Every
// coarser level alternates between w.z[l] and w.x[l], the last in w.z[l],
// where the level above reads the correction.
template <typename T, typename S>
int mg_vcycle(dot_op* op, const MgWork<S>& w, int k, const T* r0, int64_t ld0, T* z0,
              const int* active, double* partial, hipStream_t s, unsigned long long* prof_cols) {
  constexpr bool same = std::is_same<T, S>::value;
  const int nl = op->mg_nlev;
  if (nl < 2 || w.nlev != nl) DOT_FAIL(DOT_EINVAL, "multigrid hierarchy not available");
  if (MG_NU0 >= 2 && (!w.x[0] || (!same && !w.z[0])))
    DOT_FAIL(DOT_EINVAL, "multigrid work vectors missing");
  const int groups = (k + MRG - 1) / MRG;
  auto geom = [&](int l) { return mg_geom(op->mg[l].g, l + 1 < nl ? &op->mg[l + 1].g : nullptr, k); };
  // common fields of a level's launch
  auto fill = [&](auto& a, int l) {
    const MgLevel& L = op->mg[l];
    a.G = geom(l);
    a.k = k;
    a.sx = MgCoef<T>::sx(L);
    a.sy = MgCoef<T>::sy(L);
    a.sz = MgCoef<T>::sz(L);
    a.q = MgCoef<T>::q(L);
    a.active = active;
    a.ld = l == 0 ? ld0 : w.ld[l];
    if (l + 1 < nl) a.cld = w.ld[l + 1];
    a.nblk = a.G.ntiles * a.G.nzc;
  };
  // one smoothing step of level l with right-hand side b, staged iterate x
  // (NULL: w b) and coarse correction xc (NULL: none), result to out
  auto launch_smooth = [&](auto* b, const S* x, const S* xc, auto* out, int l, double* part) {
    using TB = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
    using TO = std::remove_pointer_t<decltype(out)>;
    MgArgs<T, TB, S, TO> a{};
    fill(a, l);
    a.b = b;
    a.x = x;
    a.xc = xc;
    a.out = out;
    a.partial = part;
    a.prof_cols = part ? prof_cols : nullptr;
    if (x && xc) mg_launch<MG_SMOOTH, true, true>(a, groups, s);
    else if (x) mg_launch<MG_SMOOTH, true, false>(a, groups, s);
    else if (xc) mg_launch<MG_SMOOTH, false, true>(a, groups, s);
    else mg_launch<MG_SMOOTH, false, false>(a, groups, s);
  };
  auto launch_down = [&](auto* b, const S* x, int l) {
    using TB = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
    MgArgs<T, TB, S, S> a{};
    fill(a, l);
    a.sd = MgCoef<T>::sd(op->mg[l]);
    a.sdc = MgCoef<T>::sd(op->mg[l + 1]);
    a.b = b;
    a.x = x;
    a.bc = w.b[l + 1];
    if (x) mg_launch<MG_DOWN, true, false>(a, groups, s);
    else mg_launch<MG_DOWN, false, false>(a, groups, s);
  };
  size_t tail_bytes = 0;
  const int t0 = mg_tail_start(op, sizeof(T), &tail_bytes);
  const int ndown = t0 < nl ? t0 : nl - 1;  // levels with a down and an up pass
  int outputs[DOT_MG_MAXLEV] = {};
  // the S buffer of level l's next non-final output
  auto next_buf = [&](int l) -> S* {
    const bool first_kind = (outputs[l]++ & 1) == 0;
    if (l == 0 && same) return first_kind ? reinterpret_cast<S*>(z0) : w.x[0];
    return first_kind ? w.z[l] : w.x[l];
  };
  // down the hierarchy: nu - 1 steps after x = w b, then the restriction
  const S* pre[DOT_MG_MAXLEV] = {};
  for (int l = 0; l < ndown; ++l) {
    const S* x = nullptr;
    for (int i = 1; i < mg_nu(l); ++i) {
      S* o = next_buf(l);
      if (l == 0) launch_smooth(r0, x, nullptr, o, 0, nullptr);
      else launch_smooth(static_cast<const S*>(w.b[l]), x, nullptr, o, l, nullptr);
      DOT_LAUNCH_CHECK();
      x = o;
    }
    pre[l] = x;
    if (l == 0) launch_down(r0, x, 0);
    else launch_down(static_cast<const S*>(w.b[l]), x, l);
    DOT_LAUNCH_CHECK();
  }
  if (t0 < nl) {
    MgTailArgs<T, S> ta{};
    ta.nl = nl - t0;
    int off = 0;
    for (int i = 0; i < ta.nl; ++i) {
      const MgLevel& L = op->mg[t0 + i];
      MgTailLevel<T>& d = ta.L[i];
      d.nx = L.g.nx;
      d.ny = L.g.ny;
      d.nz = L.g.nz;
      d.N = (int)L.g.N;
      d.sx = MgCoef<T>::sx(L);
      d.sy = MgCoef<T>::sy(L);
      d.sz = MgCoef<T>::sz(L);
      d.sd = L.sd;
      d.q = MgCoef<T>::q(L);
      d.off = off;
      d.nu = mg_nu(t0 + i);
      off += 3 * d.N;
    }
    ta.k = k;
    ta.active = active;
    ta.b = w.b[t0];
    ta.ldb = w.ld[t0];
    ta.z = w.z[t0];
    ta.ldz = w.ld[t0];
    if (tail_bytes > 65536)
      DOT_HIP(hipFuncSetAttribute((const void*)mg_tail_kernel<T, S>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)tail_bytes));
    hipLaunchKernelGGL((mg_tail_kernel<T, S>), dim3(k), dim3(MG_TAIL_THREADS), tail_bytes, s, ta);
    DOT_LAUNCH_CHECK();
  } else {
    // coarsest level: MG_NU_C Jacobi steps from zero, ending in z
    const int l = nl - 1;
    const MgLevel& L = op->mg[l];
    const unsigned blocks = (unsigned)((L.g.N * k + 255) / 256);
    S* bufs[2] = {w.x[l], w.z[l]};
    // step i writes bufs[(MG_NU_C - 1 - i) & 1], so the last one lands in z
    const S* prev = nullptr;
    for (int i = 0; i < MG_NU_C; ++i) {
      S* o = bufs[(MG_NU_C - 1 - i) & 1 ? 0 : 1];
      hipLaunchKernelGGL((mg_jacobi_kernel<T, S>), dim3(blocks), dim3(256), 0, s, L.g, k,
                         MgCoef<T>::sx(L), MgCoef<T>::sy(L), MgCoef<T>::sz(L), active, w.b[l], prev,
                         o, w.ld[l]);
      DOT_LAUNCH_CHECK();
      prev = o;
    }
  }
  // up the hierarchy: the prolongation with the first of nu steps; on level
  // 0 the last step writes z0 and forms r0 . z0
  for (int l = ndown - 1; l >= 0; --l) {
    const S* x = pre[l];
    const int nu = mg_nu(l);
    for (int i = 0; i < nu; ++i) {
      const S* xc = i == 0 ? w.z[l + 1] : nullptr;
      if (l == 0 && i == nu - 1) {
        launch_smooth(r0, x, xc, z0, 0, partial);
        DOT_LAUNCH_CHECK();
        break;
      }
      S* o = next_buf(l);
      if (l == 0) launch_smooth(r0, x, xc, o, 0, nullptr);
      else launch_smooth(static_cast<const S*>(w.b[l]), x, xc, o, l, nullptr);
      DOT_LAUNCH_CHECK();
      x = o;
    }
  }
  return DOT_OK;
}
// Algorithmic HBM bytes per column of one V-cycle (mg_vcycle's launches):
// every vector a level kernel must read or write once, the operator's
// coefficients (shared by the columns of a block) not counted.  A smoothing
// step reads b and, except the first, the staged iterate, reads the parent
// values with the prolongation, and writes its result; the restriction reads
// b and the iterate and writes the coarse right-hand side; the tail kernel
// reads its top level's right-hand side and writes its result (the deeper
// levels live in LDS); the Jacobi steps of a coarsest level without a tail
// read b and the previous iterate and write.  Level 0's right-hand side and
// its last result take elem0 bytes, every other vector elem.
double mg_cycle_stream_bytes(const dot_op* op, size_t elem0, size_t elem) {
  const int nl = op->mg_nlev;
  if (nl < 2) return 0.0;
  size_t tail_bytes = 0;
  const int t0 = mg_tail_start(op, elem0, &tail_bytes);
  const int ndown = t0 < nl ? t0 : nl - 1;
  const double e0 = (double)elem0, e = (double)elem;
  double v = 0.0;   // bytes
  for (int l = 0; l < ndown; ++l) {
    const double n = (double)op->mg[l].g.N, nc = (double)op->mg[l + 1].g.N;
    const double eb = l == 0 ? e0 : e;   // this level's right-hand side
    const int nu = mg_nu(l);
    bool have_x = false;
    for (int i = 1; i < nu; ++i) {
      v += n * (eb + (have_x ? e : 0.0) + e);
      have_x = true;
    }
    v += n * (eb + (have_x ? e : 0.0)) + nc * e;            // restriction
    for (int i = 0; i < nu; ++i) {
      const double eo = (l == 0 && i == nu - 1) ? e0 : e;
      v += n * (eb + (have_x ? e : 0.0) + eo) + (i == 0 ? nc * e : 0.0);
      have_x = true;
    }
  }
  if (t0 < nl) {
    v += 2.0 * (double)op->mg[t0].g.N * e;
  } else {
    const double n = (double)op->mg[nl - 1].g.N;
    v += (2.0 * n + (MG_NU_C - 1) * 3.0 * n) * e;
  }
  return v;
}

template int mg_vcycle<float, float>(dot_op*, const MgWork<float>&, int, const float*, int64_t,
                                     float*, const int*, double*, hipStream_t, unsigned long long*);
template int mg_vcycle<float, bf16s>(dot_op*, const MgWork<bf16s>&, int, const float*, int64_t,
                                     float*, const int*, double*, hipStream_t, unsigned long long*);
template int mg_vcycle<double, double>(dot_op*, const MgWork<double>&, int, const double*, int64_t,
                                       double*, const int*, double*, hipStream_t,
                                       unsigned long long*);

}  // namespace dot
