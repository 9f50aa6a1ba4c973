// Frequency-domain solves (Section 2, eq. PDE with omega > 0 and eq.
// compmeas): (A + i kappa E) x = b with kappa = omega / nu.  In the
// cell-centred finite-volume scheme every unknown is a cell average, so the
// frequency term integrates to E = h^d I on every row (the zero rows of the
// paper's E belong to boundary nodes of its vertex-centred scheme, which this
// one does not have).  A_w = A + i kappa h^d I is complex symmetric
// (A_w^T = A_w, not Hermitian), so the adjoint solves of Section 3.3 use the
// same matrix, and the solver is conjugate orthogonal CG (COCG: CG with the
// unconjugated bilinear form x^T y), preconditioned by a real symmetric
// positive definite M applied to the real and imaginary parts alike.
//
// As in the real solver the iteration runs on the symmetrically scaled
// system S^-1 A_w S^-1 x^ = S^-1 b (S = diag(A)^1/2): unit real diagonal
// plus i kappa h^d / diag(A)_c, with M the multigrid V-cycle of the real part
// (mg.hip, on 2k real columns) or the identity (Jacobi).  Per iteration:
//   apply  : q = A_w^ p, partial sums of sigma = p^T q
//   update : x^ += alpha p, r^ -= alpha q (alpha = rho / sigma), partial
//            sums of ||S r^||^2 (the unscaled residual, conjugated norm) and,
//            without a V-cycle, rho = r^T r
//   V-cycle: z = M r^, then partial sums of rho = r^T z
//   dir    : p = z + beta p, beta = rho / rho_old
// Per-column scalars (complex alpha, beta, rho) live on the device and are
// formed by one block per column from the per-block partials in fixed order
// (deterministic).  With DOT_MIXED the V-cycle runs in binary32 (binary32
// work vectors: with bfloat16 ones, as in the real mixed solve, COCG lost
// its short-recurrence orthogonality and stalled) on a binary32 copy of
// r^ / ||b|| (per column) that the update pass writes beside r^; z comes
// back in binary32 and is scaled by ||b|| where the r^T z and direction
// passes read it.  Every recurrence and the convergence test stay binary64:
// the preconditioner only steers the iteration.
// An N x k complex block is stored as an N x 2k real block:
// the real parts in columns 0 .. k-1, the imaginary parts in columns
// k .. 2k-1 (so either half is an ordinary real field block).
#include <algorithm>
#include <vector>

#include "dot_internal.h"

namespace dot {

#define DOT_TRY_C(...)             \
  do {                             \
    int rc_ = (__VA_ARGS__);       \
    if (rc_ != DOT_OK) return rc_; \
  } while (0)

constexpr int CZ_T = 256;   // threads per block, one cell each
constexpr int CZ_RG = 4;    // complex columns per block (coefficients read once per cell)
constexpr int64_t CZ_PAD = 1088;

struct CzArgs {
  GridDims g;
  int64_t ld;            // work-vector plane stride
  int k, nblk;           // complex columns, blocks per column group
  const double* sx;      // scaled couplings to +x, +y, +z
  const double* sy;
  const double* sz;
  const double* diag;    // unscaled diagonal
  const double* sd;      // sqrt(diag)
  double wk;             // kappa h^d
  const int* active;     // per complex column
  const double* coef;    // complex per column: alpha (update), beta (dir)
  const double* in0;
  const double* in1;
  double* out0;
  double* out1;
  double* partial;       // [4][k][nblk]
  int jacobi;            // update also forms rho = r^T r
  int first;             // dir: the first direction p = z
  float* r32;            // update: also r^ / ||b|| in binary32 (or NULL)
  const float* z32;      // rz, dir: z in binary32, times ||b|| (or NULL: in1 / in0)
  const double* bnorm;   // ||b|| per complex column (with r32 / z32)
};

__device__ __forceinline__ double cz_bscale(const CzArgs& a, int j) {
  const double b = a.bnorm[j];
  return b > 0.0 ? b : 1.0;
}

__device__ __forceinline__ double cz_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block reduction of acc[CZ_RG][NA] into partial[a][j][blk].
template <int NA>
__device__ __forceinline__ void cz_partials(double (&acc)[CZ_RG][NA], const CzArgs& a, int grp,
                                            int a0) {
  __shared__ double red[CZ_T / 64][CZ_RG][NA];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r)
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const double v = cz_wave_sum(acc[r][q]);
      if (lane == 0) red[wave][r][q] = v;
    }
  __syncthreads();
  if (threadIdx.x < CZ_RG * NA) {
    const int r = threadIdx.x / NA, q = threadIdx.x % NA;
    const int j = grp * CZ_RG + r;
    if (j < a.k) {
      double s = 0.0;
      for (int w = 0; w < CZ_T / 64; ++w) s += red[w][r][q];
      a.partial[((int64_t)(a0 + q) * a.k + j) * a.nblk + blockIdx.x] = s;
    }
  }
}

// q = A_w^ p for the active columns; partial sums of sigma = p^T q.
__global__ __launch_bounds__(CZ_T) void cz_apply_kernel(CzArgs a) {
  const int grp = blockIdx.y;
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  const bool in = c < a.g.N;
  const int64_t cc = in ? c : 0;
  const int x = (int)(cc % a.g.nx), y = (int)((cc / a.g.nx) % a.g.ny),
            z = (int)(cc / a.g.nxy);
  const bool hw = x > 0, he = x + 1 < a.g.nx, hs = y > 0, hn = y + 1 < a.g.ny;
  const bool hd = z > 0, hu = z + 1 < a.g.nz;
  const int64_t iw = hw ? cc - 1 : cc, ie = he ? cc + 1 : cc;
  const int64_t is = hs ? cc - a.g.nx : cc, in_ = hn ? cc + a.g.nx : cc;
  const int64_t id = hd ? cc - a.g.nxy : cc, iu = hu ? cc + a.g.nxy : cc;
  const double cE = he ? a.sx[cc] : 0.0, cW = hw ? a.sx[iw] : 0.0;
  const double cN = hn ? a.sy[cc] : 0.0, cS = hs ? a.sy[is] : 0.0;
  const double cU = hu ? a.sz[cc] : 0.0, cD = hd ? a.sz[id] : 0.0;
  const double wi = a.wk / a.diag[cc];
  double acc[CZ_RG][2];
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    acc[r][0] = acc[r][1] = 0.0;
    const int j = grp * CZ_RG + r;
    if (j >= a.k || !a.active[j]) continue;   // block-uniform
    const double* pr = a.in0 + (int64_t)j * a.ld;
    const double* pi = pr + (int64_t)a.k * a.ld;
    const double vr = pr[cc], vi = pi[cc];
    const double Ar = vr - cW * pr[iw] - cE * pr[ie] - cS * pr[is] - cN * pr[in_] -
                      cD * pr[id] - cU * pr[iu];
    const double Ai = vi - cW * pi[iw] - cE * pi[ie] - cS * pi[is] - cN * pi[in_] -
                      cD * pi[id] - cU * pi[iu];
    const double qr = Ar - wi * vi, qi = Ai + wi * vr;
    if (in) {
      double* qo = a.out0 + (int64_t)j * a.ld;
      qo[c] = qr;
      qo[c + (int64_t)a.k * a.ld] = qi;
      acc[r][0] = vr * qr - vi * qi;
      acc[r][1] = vr * qi + vi * qr;
    }
  }
  cz_partials<2>(acc, a, grp, 0);
}

// x^ += alpha p, r^ -= alpha q; partials: ||S r^||^2 and (Jacobi) r^T r.
// in0 = p, in1 = q, out0 = x^, out1 = r^.
__global__ __launch_bounds__(CZ_T) void cz_update_kernel(CzArgs a) {
  const int grp = blockIdx.y;
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  const bool in = c < a.g.N;
  const double s = in ? a.sd[c] : 0.0;
  double acc[CZ_RG][3];
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
    const int j = grp * CZ_RG + r;
    if (j >= a.k || !a.active[j]) continue;
    if (!in) continue;
    const double ar = a.coef[2 * j], ai = a.coef[2 * j + 1];
    const int64_t o = (int64_t)j * a.ld + c;
    const int64_t oi = o + (int64_t)a.k * a.ld;
    const double pr = a.in0[o], pi = a.in0[oi];
    const double qr = a.in1[o], qi = a.in1[oi];
    const double xr = a.out0[o] + (ar * pr - ai * pi);
    const double xi = a.out0[oi] + (ar * pi + ai * pr);
    const double rr = a.out1[o] - (ar * qr - ai * qi);
    const double ri = a.out1[oi] - (ar * qi + ai * qr);
    a.out0[o] = xr;
    a.out0[oi] = xi;
    a.out1[o] = rr;
    a.out1[oi] = ri;
    if (a.r32) {  // block-uniform
      const double inv = 1.0 / cz_bscale(a, j);
      a.r32[o] = (float)(rr * inv);
      a.r32[oi] = (float)(ri * inv);
    }
    acc[r][0] = s * s * (rr * rr + ri * ri);
    if (a.jacobi) {
      acc[r][1] = rr * rr - ri * ri;
      acc[r][2] = 2.0 * rr * ri;
    }
  }
  cz_partials<3>(acc, a, grp, 0);
}

// partial sums of rho = r^T z (in0 = r, in1 = z) into slots 1, 2.
__global__ __launch_bounds__(CZ_T) void cz_rz_kernel(CzArgs a) {
  const int grp = blockIdx.y;
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  const bool in = c < a.g.N;
  double acc[CZ_RG][2];
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    acc[r][0] = acc[r][1] = 0.0;
    const int j = grp * CZ_RG + r;
    if (j >= a.k || !a.active[j] || !in) continue;
    const int64_t o = (int64_t)j * a.ld + c;
    const int64_t oi = o + (int64_t)a.k * a.ld;
    const double rr = a.in0[o], ri = a.in0[oi];
    double zr, zi;
    if (a.z32) {  // block-uniform
      const double bs = cz_bscale(a, j);
      zr = bs * (double)a.z32[o];
      zi = bs * (double)a.z32[oi];
    } else {
      zr = a.in1[o];
      zi = a.in1[oi];
    }
    acc[r][0] = rr * zr - ri * zi;
    acc[r][1] = rr * zi + ri * zr;
  }
  cz_partials<2>(acc, a, grp, 1);
}

// p = z + beta p (in0 = z, out0 = p); the first direction is p = z.
__global__ __launch_bounds__(CZ_T) void cz_dir_kernel(CzArgs a) {
  const int grp = blockIdx.y;
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  if (c >= a.g.N) return;
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    const int j = grp * CZ_RG + r;
    if (j >= a.k || !a.active[j]) continue;
    const int64_t o = (int64_t)j * a.ld + c;
    const int64_t oi = o + (int64_t)a.k * a.ld;
    double zr, zi;
    if (a.z32) {  // block-uniform
      const double bs = cz_bscale(a, j);
      zr = bs * (double)a.z32[o];
      zi = bs * (double)a.z32[oi];
    } else {
      zr = a.in0[o];
      zi = a.in0[oi];
    }
    if (a.first) {
      a.out0[o] = zr;
      a.out0[oi] = zi;
      continue;
    }
    const double br = a.coef[2 * j], bi = a.coef[2 * j + 1];
    const double pr = a.out0[o], pi = a.out0[oi];
    a.out0[o] = zr + (br * pr - bi * pi);
    a.out0[oi] = zi + (br * pi + bi * pr);
  }
}

// r32 = r^ / ||b|| for the first V-cycle (the update pass writes it after
// that); in0 = r^.
__global__ __launch_bounds__(CZ_T) void cz_r32_kernel(CzArgs a) {
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  if (c >= a.g.N) return;
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    const int j = blockIdx.y * CZ_RG + r;
    if (j >= a.k || !a.active[j]) continue;
    const double inv = 1.0 / cz_bscale(a, j);
    const int64_t o = (int64_t)j * a.ld + c;
    const int64_t oi = o + (int64_t)a.k * a.ld;
    a.r32[o] = (float)(a.in0[o] * inv);
    a.r32[oi] = (float)(a.in0[oi] * inv);
  }
}

__global__ void cz_zero_int_kernel(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// r^ = S^-1 b (in0 = b, caller layout), x^ = 0; partials ||b||^2 (slot 0)
// and, for Jacobi, rho = r^T r (slots 1, 2).
__global__ __launch_bounds__(CZ_T) void cz_init_kernel(CzArgs a) {
  const int grp = blockIdx.y;
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  const bool in = c < a.g.N;
  const double s = in ? a.sd[c] : 1.0;
  double acc[CZ_RG][3];
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
    const int j = grp * CZ_RG + r;
    if (j >= a.k || !in) continue;
    const double br = a.in0[(int64_t)j * a.g.N + c];
    const double bi = a.in0[(int64_t)(a.k + j) * a.g.N + c];
    const double rr = br / s, ri = bi / s;
    const int64_t o = (int64_t)j * a.ld + c;
    const int64_t oi = o + (int64_t)a.k * a.ld;
    a.out0[o] = 0.0;
    a.out0[oi] = 0.0;
    a.out1[o] = rr;
    a.out1[oi] = ri;
    acc[r][0] = br * br + bi * bi;
    acc[r][1] = rr * rr - ri * ri;
    acc[r][2] = 2.0 * rr * ri;
  }
  cz_partials<3>(acc, a, grp, 0);
}

// x = S^-1 x^ into the caller's layout (in0 = x^, out0 = x).
__global__ __launch_bounds__(CZ_T) void cz_unscale_kernel(CzArgs a) {
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  if (c >= a.g.N) return;
  const double s = a.sd[c];
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    const int j = blockIdx.y * CZ_RG + r;
    if (j >= a.k) continue;
    for (int h = 0; h < 2; ++h)
      a.out0[(int64_t)(h * a.k + j) * a.g.N + c] = a.in0[(int64_t)(h * a.k + j) * a.ld + c] / s;
  }
}

// ||b - A_w x||^2 with the unscaled operator (in0 = x, in1 = b, caller
// layout; sx/sy/sz here are the unscaled couplings, diag the full diagonal).
__global__ __launch_bounds__(CZ_T) void cz_true_kernel(CzArgs a) {
  const int grp = blockIdx.y;
  const int64_t c = blockIdx.x * (int64_t)CZ_T + threadIdx.x;
  const bool in = c < a.g.N;
  const int64_t cc = in ? c : 0;
  const int x = (int)(cc % a.g.nx), y = (int)((cc / a.g.nx) % a.g.ny),
            z = (int)(cc / a.g.nxy);
  const bool hw = x > 0, he = x + 1 < a.g.nx, hs = y > 0, hn = y + 1 < a.g.ny;
  const bool hd = z > 0, hu = z + 1 < a.g.nz;
  const int64_t iw = hw ? cc - 1 : cc, ie = he ? cc + 1 : cc;
  const int64_t is = hs ? cc - a.g.nx : cc, in_ = hn ? cc + a.g.nx : cc;
  const int64_t id = hd ? cc - a.g.nxy : cc, iu = hu ? cc + a.g.nxy : cc;
  const double cE = he ? a.sx[cc] : 0.0, cW = hw ? a.sx[iw] : 0.0;
  const double cN = hn ? a.sy[cc] : 0.0, cS = hs ? a.sy[is] : 0.0;
  const double cU = hu ? a.sz[cc] : 0.0, cD = hd ? a.sz[id] : 0.0;
  const double dd = a.diag[cc];
  double acc[CZ_RG][1];
#pragma unroll
  for (int r = 0; r < CZ_RG; ++r) {
    acc[r][0] = 0.0;
    const int j = grp * CZ_RG + r;
    if (j >= a.k || !in) continue;
    const double* xr = a.in0 + (int64_t)j * a.g.N;
    const double* xi = xr + (int64_t)a.k * a.g.N;
    const double Ar = dd * xr[cc] - cW * xr[iw] - cE * xr[ie] - cS * xr[is] - cN * xr[in_] -
                      cD * xr[id] - cU * xr[iu] - a.wk * xi[cc];
    const double Ai = dd * xi[cc] - cW * xi[iw] - cE * xi[ie] - cS * xi[is] - cN * xi[in_] -
                      cD * xi[id] - cU * xi[iu] + a.wk * xr[cc];
    const double rr = a.in1[(int64_t)j * a.g.N + c] - Ar;
    const double ri = a.in1[(int64_t)(a.k + j) * a.g.N + c] - Ai;
    acc[r][0] = rr * rr + ri * ri;
  }
  cz_partials<1>(acc, a, grp, 0);
}

// Per-column scalars from the partials (one block per column, fixed order).
enum CzFin { CZ_F_INIT = 0, CZ_F_ALPHA = 1, CZ_F_RES = 2, CZ_F_BETA = 3, CZ_F_RHO0 = 4 };

struct CzState {
  double* rho;      // complex
  double* alpha;    // complex
  double* beta;     // complex
  double* bnorm;
  double* relres;
  int* active;      // per complex column
  int* active2;     // per real plane (V-cycle mask)
  int* iters;
  int* flags;
  int* n_active;    // device count of active columns
};

__global__ __launch_bounds__(256) void cz_fin_kernel(int mode, int k, int nblk,
                                                     const double* __restrict__ partial,
                                                     CzState st, double rtol) {
  const int j = blockIdx.x;
  __shared__ double red[4][256];
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256)
#pragma unroll
    for (int q = 0; q < 3; ++q) s[q] += partial[((int64_t)q * k + j) * nblk + b];
#pragma unroll
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s0 = red[0][0], s1 = red[1][0], s2 = red[2][0];
  if (mode == CZ_F_INIT) {
    st.bnorm[j] = sqrt(s0);
    st.iters[j] = 0;
    st.flags[j] = 0;
    st.relres[j] = s0 > 0.0 ? 1.0 : 0.0;
    const int act = s0 > 0.0 ? 1 : 0;
    st.active[j] = act;
    st.active2[j] = st.active2[k + j] = act;
    st.rho[2 * j] = s1;
    st.rho[2 * j + 1] = s2;
    st.beta[2 * j] = st.beta[2 * j + 1] = 0.0;
    if (act) atomicAdd(st.n_active, 1);
    return;
  }
  if (!st.active[j]) return;
  if (mode == CZ_F_ALPHA) {
    // alpha = rho / sigma (complex division); sigma = 0 is a breakdown
    const double sr = s0, si = s1;
    const double den = sr * sr + si * si;
    const double rr = st.rho[2 * j], ri = st.rho[2 * j + 1];
    if (!(den > 0.0) || !isfinite(den)) {
      st.flags[j] |= 1;
      st.active[j] = 0;
      st.active2[j] = st.active2[k + j] = 0;
      atomicSub(st.n_active, 1);
      st.alpha[2 * j] = st.alpha[2 * j + 1] = 0.0;
      return;
    }
    st.alpha[2 * j] = (rr * sr + ri * si) / den;
    st.alpha[2 * j + 1] = (ri * sr - rr * si) / den;
  } else if (mode == CZ_F_RES) {
    // unscaled residual norm after the update; Jacobi: rho_new in s1, s2
    st.iters[j] += 1;
    const double rel = sqrt(s0) / st.bnorm[j];
    st.relres[j] = rel;
    if (!isfinite(rel)) st.flags[j] |= 2;
    if (rel <= rtol || !isfinite(rel)) {
      st.active[j] = 0;
      st.active2[j] = st.active2[k + j] = 0;
      atomicSub(st.n_active, 1);
      return;
    }
  } else if (mode == CZ_F_BETA) {
    // beta = rho_new / rho_old
    const double nr = s1, ni = s2;
    const double orr = st.rho[2 * j], oi = st.rho[2 * j + 1];
    const double den = orr * orr + oi * oi;
    if (!(den > 0.0)) {
      st.flags[j] |= 1;
      st.active[j] = 0;
      st.active2[j] = st.active2[k + j] = 0;
      atomicSub(st.n_active, 1);
      return;
    }
    st.beta[2 * j] = (nr * orr + ni * oi) / den;
    st.beta[2 * j + 1] = (ni * orr - nr * oi) / den;
    st.rho[2 * j] = nr;
    st.rho[2 * j + 1] = ni;
  } else if (mode == CZ_F_RHO0) {
    st.rho[2 * j] = s1;
    st.rho[2 * j + 1] = s2;
  }
}

// true relative residual of every column (also the inactive ones)
__global__ __launch_bounds__(256) void cz_true_fin_kernel(int k, int nblk,
                                                          const double* __restrict__ partial,
                                                          CzState st) {
  const int j = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(int64_t)j * nblk + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) st.relres[j] = st.bnorm[j] > 0.0 ? sqrt(red[0]) / st.bnorm[j] : 0.0;
}

// --------------------------------------------------------------- workspace
struct CzWork {
  int64_t ld;
  double *x, *r, *p, *q, *z;
  double* partial;
  double *rho, *alpha, *beta, *bnorm, *relres;
  int *active, *active2, *iters, *flags, *n_active;
  double* mgpart;
  MgWork<double> mg;
  bool use_mg;
  bool mixed;        // binary32 V-cycle: r32 / z32 and mg32 instead of z and mg
  float *r32, *z32;
  MgWork<float> mg32;
};

static size_t al256z(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t cz_layout(const dot_op* op, int k, bool use_mg, bool mixed, char* base, CzWork* w) {
  mixed = mixed && use_mg;
  const int64_t N = op->g.N;
  const int64_t ld = N + CZ_PAD;
  const int nblk = (int)((N + CZ_T - 1) / CZ_T);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += al256z(bytes);
    return p;
  };
  const size_t vec = (size_t)2 * k * ld * sizeof(double);
  double* x = (double*)take(vec);
  double* r = (double*)take(vec);
  double* p = (double*)take(vec);
  double* q = (double*)take(vec);
  double* z = (use_mg && !mixed) ? (double*)take(vec) : nullptr;
  float* r32 = mixed ? (float*)take(vec / 2) : nullptr;
  float* z32 = mixed ? (float*)take(vec / 2) : nullptr;
  double* partial = (double*)take((size_t)4 * k * nblk * sizeof(double));
  double* sc = (double*)take((size_t)8 * k * sizeof(double));
  int* iv = (int*)take((size_t)(6 * k + 8) * sizeof(int));
  double* mgpart = nullptr;
  char* mgbase = nullptr;
  if (use_mg) {
    mgpart = (double*)take((size_t)2 * (2 * k) * mg_partial_slots(op, 2 * k) * sizeof(double));
    mgbase = take(mixed ? mg_work_bytes(op, 2 * k, ld, sizeof(float))
                        : mg_work_bytes(op, 2 * k, ld, sizeof(double)));
  }
  if (w) {
    w->ld = ld;
    w->x = x; w->r = r; w->p = p; w->q = q; w->z = z;
    w->partial = partial;
    w->rho = sc; w->alpha = sc + 2 * k; w->beta = sc + 4 * k; w->bnorm = sc + 6 * k;
    w->relres = sc + 7 * k;
    w->active = iv; w->active2 = iv + k; w->iters = iv + 3 * k; w->flags = iv + 4 * k;
    w->n_active = iv + 5 * k;
    w->mgpart = mgpart;
    w->use_mg = use_mg;
    w->mixed = mixed;
    w->r32 = r32;
    w->z32 = z32;
    if (mixed) mg_work_layout<float>(op, 2 * k, ld, mgbase, &w->mg32, 1);
    else if (use_mg) mg_work_layout<double>(op, 2 * k, ld, mgbase, &w->mg);
  }
  return off + 256;
}

static CzArgs cz_args(const dot_op* op, int k, double wk, const CzWork& w) {
  CzArgs a{};
  a.g = op->g;
  a.ld = w.ld;
  a.k = k;
  a.nblk = (int)((op->g.N + CZ_T - 1) / CZ_T);
  a.sx = op->sx;
  a.sy = op->sy;
  a.sz = op->sz;
  a.diag = op->diag;
  a.sd = op->sd;
  a.wk = wk;
  a.active = w.active;
  a.partial = w.partial;
  a.bnorm = w.bnorm;
  return a;
}

}  // namespace dot

using namespace dot;

extern "C" {

size_t dot_solve_complex_workspace_bytes(const dot_op* op, int k, int precond) {
  if (!op || k < 1 || k > DOT_MAX_COLUMNS / 2) return 0;
  const bool mg = precond != DOT_PRECOND_JACOBI && dot_multigrid_levels(op) > 0;
  return std::max(cz_layout(op, k, mg, false, nullptr, nullptr),
                  cz_layout(op, k, mg, true, nullptr, nullptr));
}

int dot_solve_complex(dot_op* op, double kappa, int k, const double* rhs_dev, double* x_dev,
                      const dot_solve_opts* opts, void* work_dev, size_t work_bytes,
                      dot_solve_info* info, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (k < 1 || k > DOT_MAX_COLUMNS / 2)
    DOT_FAIL(DOT_EINVAL, "k must be in [1, %d]", DOT_MAX_COLUMNS / 2);
  if (!rhs_dev || !x_dev) DOT_FAIL(DOT_EINVAL, "rhs_dev/x_dev is NULL");
  if (!opts) DOT_FAIL(DOT_EINVAL, "opts is NULL");
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) DOT_FAIL(DOT_EINVAL, "kappa must be finite, >= 0");
  if (!(opts->rtol > 0.0) || opts->max_iter < 1 || opts->check_every < 1)
    DOT_FAIL(DOT_EINVAL, "rtol > 0, max_iter >= 1 and check_every >= 1 are required");
  if (opts->precision != DOT_FP64 && opts->precision != DOT_MIXED)
    DOT_FAIL(DOT_EINVAL, "precision must be DOT_FP64 or DOT_MIXED");
  if (opts->precond != DOT_PRECOND_AUTO && opts->precond != DOT_PRECOND_JACOBI &&
      opts->precond != DOT_PRECOND_MG)
    DOT_FAIL(DOT_EINVAL, "unknown preconditioner");
  const int levels = dot_multigrid_levels(op);
  if (opts->precond == DOT_PRECOND_MG && levels == 0)
    DOT_FAIL(DOT_EINVAL, "no multigrid hierarchy for this operator");
  const bool use_mg = opts->precond != DOT_PRECOND_JACOBI && levels > 0;
  const bool mixed = opts->precision == DOT_MIXED;
  const size_t need = cz_layout(op, k, use_mg, mixed, nullptr, nullptr);
  if (!work_dev || work_bytes < need)
    DOT_FAIL(DOT_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
  if (((uintptr_t)work_dev & 255) != 0) DOT_FAIL(DOT_EINVAL, "work_dev must be 256-byte aligned");
  const char* lo = (const char*)rhs_dev;
  const char* xo = (const char*)x_dev;
  const size_t span = (size_t)op->g.N * 2 * k * sizeof(double);
  if (lo < xo + span && xo < lo + span) DOT_FAIL(DOT_EINVAL, "rhs_dev and x_dev overlap");

  hipStream_t s = as_stream(stream);
  CzWork w;
  cz_layout(op, k, use_mg, mixed, (char*)work_dev, &w);
  const double wk = kappa * op->g.hd;
  const CzArgs a = cz_args(op, k, wk, w);
  const CzState st{w.rho, w.alpha, w.beta, w.bnorm, w.relres, w.active, w.active2, w.iters,
                   w.flags, w.n_active};
  const dim3 grid((unsigned)a.nblk, (unsigned)((k + CZ_RG - 1) / CZ_RG));
  const int nblk = a.nblk;
  auto fin = [&](int mode) -> int {
    hipLaunchKernelGGL(cz_fin_kernel, dim3(k), dim3(256), 0, s, mode, k, nblk, w.partial, st,
                       opts->rtol);
    DOT_LAUNCH_CHECK();
    return DOT_OK;
  };
  // z = M r^ and rho = r^T z into partial slots 1, 2 (multigrid only; with
  // Jacobi the update pass forms rho = r^T r in the same slots)
  auto precondition = [&]() -> int {
    if (!use_mg) return DOT_OK;
    if (w.mixed)
      DOT_TRY_C(mg_vcycle<float, float>(op, w.mg32, 2 * k, w.r32, w.ld, w.z32, w.active2,
                                        w.mgpart, s));
    else
      DOT_TRY_C(mg_vcycle<double>(op, w.mg, 2 * k, w.r, w.ld, w.z, w.active2, w.mgpart, s));
    CzArgs b = a;
    b.in0 = w.r;
    b.in1 = w.z;
    b.z32 = w.z32;
    hipLaunchKernelGGL(cz_rz_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
    return DOT_OK;
  };
  auto direction = [&](bool first) -> int {
    CzArgs b = a;
    b.in0 = use_mg ? w.z : w.r;
    b.z32 = use_mg ? w.z32 : nullptr;
    b.out0 = w.p;
    b.coef = w.beta;
    b.first = first ? 1 : 0;
    hipLaunchKernelGGL(cz_dir_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
    return DOT_OK;
  };

  // r^ = S^-1 b, x^ = 0, ||b||, the columns to solve, rho, p = z
  hipLaunchKernelGGL(cz_zero_int_kernel, dim3(1), dim3(64), 0, s, w.n_active);
  DOT_LAUNCH_CHECK();
  {
    CzArgs b = a;
    b.in0 = rhs_dev;
    b.out0 = w.x;
    b.out1 = w.r;
    hipLaunchKernelGGL(cz_init_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
  }
  DOT_TRY_C(fin(CZ_F_INIT));
  if (w.mixed) {  // the first binary32 residual, now that ||b|| is known
    CzArgs b = a;
    b.in0 = w.r;
    b.r32 = w.r32;
    hipLaunchKernelGGL(cz_r32_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
  }
  DOT_TRY_C(precondition());
  if (use_mg) DOT_TRY_C(fin(CZ_F_RHO0));
  DOT_TRY_C(direction(true));

  int it = 0, n_active = 1;
  while (it < opts->max_iter && n_active > 0) {
    CzArgs b = a;
    b.in0 = w.p;
    b.out0 = w.q;
    hipLaunchKernelGGL(cz_apply_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
    DOT_TRY_C(fin(CZ_F_ALPHA));
    b = a;
    b.in0 = w.p;
    b.in1 = w.q;
    b.out0 = w.x;
    b.out1 = w.r;
    b.coef = w.alpha;
    b.jacobi = use_mg ? 0 : 1;
    b.r32 = w.r32;
    hipLaunchKernelGGL(cz_update_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
    DOT_TRY_C(fin(CZ_F_RES));
    DOT_TRY_C(precondition());
    DOT_TRY_C(fin(CZ_F_BETA));
    DOT_TRY_C(direction(false));
    ++it;
    if (it % opts->check_every == 0 || it == opts->max_iter) {
      DOT_HIP(hipMemcpyAsync(&n_active, w.n_active, sizeof(int), hipMemcpyDeviceToHost, s));
      DOT_HIP(hipStreamSynchronize(s));
    }
  }
  // x = S^-1 x^, true residual in binary64 with the unscaled operator
  {
    CzArgs b = a;
    b.in0 = w.x;
    b.out0 = x_dev;
    hipLaunchKernelGGL(cz_unscale_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
    b = a;
    b.sx = op->cx;
    b.sy = op->cy;
    b.sz = op->cz;
    b.in0 = x_dev;
    b.in1 = rhs_dev;
    hipLaunchKernelGGL(cz_true_kernel, grid, dim3(CZ_T), 0, s, b);
    DOT_LAUNCH_CHECK();
    hipLaunchKernelGGL(cz_true_fin_kernel, dim3(k), dim3(256), 0, s, k, nblk, w.partial, st);
    DOT_LAUNCH_CHECK();
  }
  std::vector<double> rel(k);
  std::vector<int> its(k), flg(k);
  DOT_HIP(hipMemcpyAsync(rel.data(), w.relres, k * sizeof(double), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipMemcpyAsync(its.data(), w.iters, k * sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipMemcpyAsync(flg.data(), w.flags, k * sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  int imax = 0, bad = 0, nonfin = 0;
  bool conv = true;
  for (int j = 0; j < k; ++j) {
    imax = std::max(imax, its[j]);
    if (flg[j] & 1) bad = 1;
    if ((flg[j] & 2) || !std::isfinite(rel[j])) nonfin = 1;
    // the recursive residual decided the stop; the true one may exceed it
    // by rounding
    if (!(rel[j] <= opts->rtol * 1.01)) conv = false;
  }
  if (info) {
    info->iters_max = imax;
    info->outer = 0;
    if (info->iters_host)
      for (int j = 0; j < k; ++j) info->iters_host[j] = its[j];
    if (info->relres_host)
      for (int j = 0; j < k; ++j) info->relres_host[j] = rel[j];
  }
  if (nonfin) DOT_FAIL(DOT_ENONFINITE, "non-finite value in the complex solve");
  if (bad) DOT_FAIL(DOT_EBREAKDOWN, "COCG breakdown (p^T A p or r^T z vanished)");
  return conv ? DOT_OK : DOT_NOT_CONVERGED;
}

}  // extern "C"
