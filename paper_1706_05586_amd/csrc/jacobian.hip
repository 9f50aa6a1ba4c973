// Sampled Jacobian and adjoint gradient over the PaLS parameters.
//
// Section 3.3, eq. (Jacobian kth column) with the sign of eq. (Jacobiancomp):
//   Js[j + l_d i, k] = - y_j^T (dA/dp_k) z_i = - sum_c Z[c,j] U[c,i] G[c,k],
//   G[c,k] = h^d d mu_c / d p_k = h^d (mu_in - mu_out) delta_eps(phi_c - cut)
//            d phi_c / d p_k,
// visiting only the cells where dA/dp_k is nonzero (the last paragraph of
// Section 3.3): for RBF m these are the cells of its support that lie in
// the Heaviside band, listed by dot_pals_mua in increasing cell order and
// cut into chunks.  One block per chunk contracts the chunk's cells into a
// partial (l_s x l_d x n_act) block; a second kernel sums the partials of
// each RBF in chunk order (deterministic, no atomics).
//
// Gradient (eq. UnbiasedGrad, sampled): g = Js^T vec(Rs) evaluated as
// g_k = - sum_c G[c,k] s_c with s_c = sum_i U[c,i] (Z Rs)[c,i].
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "dot_internal.h"

namespace dot {

struct JacParams {
  int64_t N;
  double h, hd;
  int dim, stride;
  double dmu, cutoff, eps, gamma;
  unsigned active;
  int n_act;
};

// d phi / d theta_a for the active parameters of one RBF at cell centre x.
__device__ __forceinline__ int rbf_dphi(const JacParams& P, const double* th, double x0, double x1,
                                        double x2, double* out) {
  const double alpha = th[0], beta = th[1];
  const double e0 = x0 - th[2], e1 = x1 - th[3];
  const double e2 = P.dim == 3 ? x2 - th[4] : 0.0;
  double rho2 = e0 * e0 + e1 * e1;
  if (P.dim == 3) rho2 += e2 * e2;
  const double r = sqrt(beta * beta * rho2 + P.gamma * P.gamma);
  int q = 0;
  if (r >= 1.0) {
    for (int a = 0; a < P.n_act; ++a) out[a] = 0.0;
    return P.n_act;
  }
  const double o = 1.0 - r;
  const double o3 = o * o * o;
  if (P.active & DOT_ACT_ALPHA) out[q++] = o3 * o * (4.0 * r + 1.0);
  if (P.active & DOT_ACT_BETA) out[q++] = -20.0 * alpha * beta * rho2 * o3;
  if (P.active & DOT_ACT_CHI) {
    const double s = 20.0 * alpha * beta * beta;
    out[q++] = s * e0 * o3;
    out[q++] = s * e1 * o3;
    if (P.dim == 3) out[q++] = s * e2 * o3;
  }
  return q;
}

__device__ __forceinline__ double band_weight(const JacParams& P, double phi) {
  const double s = phi - P.cutoff;
  if (fabs(s) > P.eps) return 0.0;
  return P.dmu * ((1.0 + cos(M_PI * s / P.eps)) / (2.0 * P.eps));
}

__device__ __forceinline__ void cell_xyz(const GridDims& g, int64_t c, double* x0, double* x1,
                                         double* x2) {
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / g.nxy);
  *x0 = (x + 0.5) * g.h;
  *x1 = (y + 0.5) * g.h;
  *x2 = (z + 0.5) * g.h;
}

// ----------------------------------------------------------------------
// Directional derivative of A(p) applied to fields:
//     Y[c, j] = h^d (mu_in - mu_out) delta_eps(phi_c - cutoff)
//               sum_m sum_a Theta[m n_act + a, j] d phi_c / d p_{m,a}  X[c, j],
// i.e. (sum_k Theta[k, j] dA/dp_k) X[:, j] with dA/dp_k = h^d diag(d mu / d p_k).
// One block of 256 threads per cell tile (8 x 8 x 4 in 3D, 16 x 16 in 2D);
// the RBFs whose support reaches the tile are listed in RBF order and summed
// in that order at every cell (deterministic), DIRK columns at a time.
constexpr int DIRK = 8;

__global__ __launch_bounds__(256) void dA_dir_kernel(GridDims g, JacParams P,
                                                     const double* __restrict__ theta,
                                                     const double* __restrict__ phi, int m0,
                                                     int k, const double* __restrict__ Th,
                                                     int n_p, const double* __restrict__ X,
                                                     double* __restrict__ Y) {
  __shared__ int s_wave[4];
  __shared__ int s_list[256];
  const bool d3 = g.dim == 3;
  const int TX = d3 ? 8 : 16, TY = d3 ? 8 : 16, TZ = d3 ? 4 : 1;
  const int tiles_x = (g.nx + TX - 1) / TX, tiles_y = (g.ny + TY - 1) / TY;
  const int tile = blockIdx.x;
  const int bx = tile % tiles_x, by = (tile / tiles_x) % tiles_y, bz = tile / (tiles_x * tiles_y);
  const int t = threadIdx.x;
  const int lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
  const int x = bx * TX + lx, y = by * TY + ly, z = bz * TZ + lz;
  const bool inside = x < g.nx && y < g.ny && z < g.nz;
  const double h = g.h;
  const double xc0 = (x + 0.5) * h, xc1 = (y + 0.5) * h, xc2 = (z + 0.5) * h;
  const double lo0 = (bx * TX + 0.5) * h, hi0 = (min(g.nx, bx * TX + TX) - 0.5) * h;
  const double lo1 = (by * TY + 0.5) * h, hi1 = (min(g.ny, by * TY + TY) - 0.5) * h;
  const double lo2 = (bz * TZ + 0.5) * h, hi2 = (min(g.nz, bz * TZ + TZ) - 0.5) * h;
  const double g2 = P.gamma * P.gamma;
  const int64_t c = inside ? x + (int64_t)g.nx * (y + (int64_t)g.ny * z) : 0;
  const double w = inside ? P.hd * band_weight(P, phi[c]) : 0.0;
  const int na = P.n_act;
  for (int j0 = 0; j0 < k; j0 += DIRK) {
    double acc[DIRK];
#pragma unroll
    for (int q = 0; q < DIRK; ++q) acc[q] = 0.0;
    for (int base = 0; base < m0; base += 256) {
      const int m = base + t;
      int flag = 0;
      if (m < m0) {
        const double* th = theta + (int64_t)m * P.stride;
        const double beta = th[1];
        const double d0 = fmax(0.0, fmax(lo0 - th[2], th[2] - hi0));
        const double d1 = fmax(0.0, fmax(lo1 - th[3], th[3] - hi1));
        double dist2 = d0 * d0 + d1 * d1;
        if (d3) {
          const double dd = fmax(0.0, fmax(lo2 - th[4], th[4] - hi2));
          dist2 += dd * dd;
        }
        flag = (beta * beta * dist2 + g2 < 1.0) ? 1 : 0;
      }
      int total;
      const int pos = block_scan_flag256(flag, s_wave, &total);
      if (flag) s_list[pos] = m;
      __syncthreads();
      if (inside && w != 0.0) {
        for (int q = 0; q < total; ++q) {
          const int mm = s_list[q];
          double d[5];
          rbf_dphi(P, theta + (int64_t)mm * P.stride, xc0, xc1, xc2, d);
          const double* tk = Th + (int64_t)mm * na;
#pragma unroll
          for (int jj = 0; jj < DIRK; ++jj) {
            if (j0 + jj < k) {
              const double* tc = tk + (int64_t)n_p * (j0 + jj);
              double s = 0.0;
              for (int a = 0; a < na; ++a) s += d[a] * tc[a];
              acc[jj] += s;
            }
          }
        }
      }
      __syncthreads();
    }
    if (inside) {
#pragma unroll
      for (int jj = 0; jj < DIRK; ++jj)
        if (j0 + jj < k) {
          const int64_t e = c + P.N * (int64_t)(j0 + jj);
          Y[e] = w == 0.0 ? 0.0 : w * acc[jj] * X[e];
        }
    }
  }
}

// ----------------------------------------------------------------------
// Preparation, run by dot_pals_mua once the pair lists exist:
//   pair_g[p * na + a] = h^d d mu / d p_a at the pair's cell, for its RBF;
//   band rows: every cell of any pair list, numbered in cell order, so the
//   contraction can read the U and Z values of a pair as one packed row.
__global__ __launch_bounds__(256) void pair_g_kernel(GridDims g, JacParams P,
                                                     const double* __restrict__ theta,
                                                     const double* __restrict__ phi,
                                                     const int64_t* __restrict__ rbf_start,
                                                     const int32_t* __restrict__ pair_cell,
                                                     double* __restrict__ pair_g,
                                                     float* __restrict__ pair_g32) {
  // blocks (m, y): RBF m's pairs, split over gridDim.y blocks
  const int m = blockIdx.x;
  const double* th = theta + (int64_t)m * P.stride;
  const int na = P.n_act;
  for (int64_t p = rbf_start[m] + blockIdx.y * 256 + threadIdx.x; p < rbf_start[m + 1];
       p += 256 * (int64_t)gridDim.y) {
    const int64_t c = pair_cell[p];
    double x0, x1, x2, d[5];
    cell_xyz(g, c, &x0, &x1, &x2);
    rbf_dphi(P, th, x0, x1, x2, d);
    const double w = band_weight(P, phi[c]);
    for (int a = 0; a < na; ++a) {
      const double v = P.hd * (w * d[a]);
      pair_g[p * na + a] = v;
      pair_g32[p * na + a] = (float)v;
    }
  }
}

__global__ void fill_double_kernel(double* __restrict__ a, int n, double v) {
  const int i = threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void fill_float_kernel(float* __restrict__ a, int n, float v) {
  const int i = threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void fill_int_kernel(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void band_mark_kernel(int64_t n_pairs, const int32_t* __restrict__ pair_cell,
                                 int32_t* __restrict__ flag) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n_pairs) flag[pair_cell[p]] = 1;
}

constexpr int BAND_BLK = 2048;   // cells per block: 256 threads x 8 consecutive cells

// Exclusive scan of one int per thread over the block (nwaves waves).
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* s_wave, int nwaves, T* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  T woff = 0, tot = 0;
  for (int w = 0; w < nwaves; ++w) {
    if (w < wave) woff += s_wave[w];
    tot += s_wave[w];
  }
  *total = tot;
  return woff + x - v;
}

__global__ __launch_bounds__(256) void band_count_kernel(int64_t N, const int32_t* __restrict__ flag,
                                                         int64_t* __restrict__ cnt) {
  __shared__ int s_wave[4];
  const int64_t c0 = (int64_t)blockIdx.x * BAND_BLK + threadIdx.x * 8;
  int n = 0;
  for (int q = 0; q < 8; ++q)
    if (c0 + q < N) n += flag[c0 + q] != 0 ? 1 : 0;
  int tot;
  block_excl_scan<int>(n, s_wave, 4, &tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

// One block: part[b] = band cells in blocks before b, part[nb] = all of them.
__global__ __launch_bounds__(1024) void band_scan_kernel(int nb, const int64_t* __restrict__ cnt,
                                                         int64_t* __restrict__ part) {
  __shared__ long long s_wave[16];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
  long long loc = 0;
  for (int b = b0; b < b1; ++b) loc += cnt[b];
  long long tot;
  long long run = block_excl_scan<long long>(loc, s_wave, 16, &tot);
  for (int b = b0; b < b1; ++b) {
    part[b] = run;
    run += cnt[b];
  }
  if (t == 0) part[nb] = tot;
}

// flags -> band rows (-1 off the band) and the cell of each band row
__global__ __launch_bounds__(256) void band_fill_kernel(int64_t N, const int64_t* __restrict__ part,
                                                        int32_t* __restrict__ idx,
                                                        int32_t* __restrict__ cells) {
  __shared__ int s_wave[4];
  const int64_t c0 = (int64_t)blockIdx.x * BAND_BLK + threadIdx.x * 8;
  int f[8], n = 0;
  for (int q = 0; q < 8; ++q) {
    f[q] = (c0 + q < N && idx[c0 + q] != 0) ? 1 : 0;
    n += f[q];
  }
  int tot;
  const int off = block_excl_scan<int>(n, s_wave, 4, &tot);
  int64_t r = part[blockIdx.x] + off;
  for (int q = 0; q < 8; ++q) {
    if (c0 + q >= N) break;
    if (f[q]) {
      idx[c0 + q] = (int32_t)r;
      cells[r] = (int32_t)(c0 + q);
      ++r;
    } else {
      idx[c0 + q] = -1;
    }
  }
}

__global__ void pair_band_kernel(int64_t n_pairs, const int32_t* __restrict__ pair_cell,
                                 const int32_t* __restrict__ idx, int32_t* __restrict__ pair_band) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n_pairs) pair_band[p] = idx[pair_cell[p]];
}

// Diffusion mode (dot_pals_mua_diffusion): dA/dp_k also has the face terms
// sum_f dT_f/dp_k (e_c - e_c')(e_c - e_c')^T + boundary faces, with
// dT_f/dp_k = dT_f/dD_c dD_c/dp_k + dT_f/dD_c' dD_c'/dp_k and
// dD_c/dp_k = s_c h^d d mu_c / d p_k, s_c = -3 D_c^2 (1 + (mus_in - mus_out) /
// (mu_in - mu_out)) / h^d.  Each half of a face term belongs to one cell, so
// per (RBF, cell) pair the contraction gains 2 dim rows beside the cell's own:
// row 1 + f (face f = 2 axis + side: -x, +x, -y, +y, -z, +z) is
// (U_c - U_c', w (Z_c - Z_c')) across an interior face and (U_c, w Z_c) on a
// boundary face, w = s_c dT_f/dD_c, all under the same pair weight
// h^d d mu / d p_k:
//   interior   dT/dD_c = h^(d-2) 2 D_c'^2 / (D_c + D_c')^2
//   Dirichlet  dT/dD_c = h^(d-2) 2
//   Robin      dT/dD_c = h^(d-1) 2 h / (h + 4 D_c)^2
struct Faces6 {
  int bc[6];
};

__global__ __launch_bounds__(256) void vrow_kernel(GridDims g, Faces6 fb, int64_t n_band,
                                                   const int32_t* __restrict__ band_cells,
                                                   const double* __restrict__ D, double ratio,
                                                   int R, int32_t* __restrict__ rcell,
                                                   int32_t* __restrict__ rnbr,
                                                   double* __restrict__ rw) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n_band * R) return;
  const int64_t b = q / R;
  const int r = (int)(q - b * R);
  const int64_t c = band_cells[b];
  rcell[q] = (int32_t)c;
  if (r == 0) {
    rnbr[q] = -1;
    rw[q] = 1.0;
    return;
  }
  const int f = r - 1, axis = f >> 1, side = f & 1;
  const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / g.nxy);
  const int pos[3] = {x, y, z};
  const int n[3] = {g.nx, g.ny, g.nz};
  const int64_t stride[3] = {1, g.nx, g.nxy};
  const double h = g.h;
  const double hd2 = g.dim == 3 ? h : 1.0, hd1 = g.dim == 3 ? h * h : h;
  const double Dc = D[c];
  const double sc = -3.0 * Dc * Dc * ratio / g.hd;
  const bool interior = side == 0 ? pos[axis] > 0 : pos[axis] + 1 < n[axis];
  if (interior) {
    const int64_t cn = side == 0 ? c - stride[axis] : c + stride[axis];
    const double Dn = D[cn];
    const double s2 = Dc + Dn;
    rnbr[q] = (int32_t)cn;
    rw[q] = sc * hd2 * 2.0 * Dn * Dn / (s2 * s2);
  } else {
    const int code = fb.bc[f];
    const double t = code == DOT_BC_DIRICHLET ? hd2 * 2.0
                                              : hd1 * 2.0 * h / ((h + 4.0 * Dc) * (h + 4.0 * Dc));
    rnbr[q] = -1;
    rw[q] = sc * t;
  }
}

// virtual pair p R + r: band row of pair p times R plus r, its weights
__global__ __launch_bounds__(256) void vpair_kernel(int64_t n_pairs, int R, int na,
                                                    const int32_t* __restrict__ pair_band,
                                                    const double* __restrict__ pair_g,
                                                    int32_t* __restrict__ vband,
                                                    double* __restrict__ vg,
                                                    float* __restrict__ vg32) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n_pairs * R) return;
  const int64_t p = q / R;
  const int r = (int)(q - p * R);
  vband[q] = pair_band[p] * R + r;
  for (int a = 0; a < na; ++a) {
    const double v = pair_g[p * na + a];
    vg[q * na + a] = v;
    vg32[q * na + a] = (float)v;
  }
}

// Packed rows: packed[b * L + i] = U[c_b, i] (i < l_s) or Z[c_b, i - l_s],
// L = l_s + l_d, through a 64-row x 64-column LDS tile so that both the
// column reads and the row writes are contiguous.
// FACE (diffusion mode): row b is (U_c - U_nbr, w (Z_c - Z_nbr)) with the
// neighbour rnbr[b] (-1: none, the plain values) and weight rw[b].
template <typename T, bool FACE>
__global__ __launch_bounds__(256) void pack_rows_kernel(int64_t N, int64_t n_band,
                                                        const int32_t* __restrict__ band_cells,
                                                        const int32_t* __restrict__ rnbr,
                                                        const double* __restrict__ rw,
                                                        int l_s, const double* __restrict__ U,
                                                        int l_d, const double* __restrict__ Z,
                                                        T* __restrict__ packed) {
  __shared__ T tile[64][65];
  const int L = l_s + l_d;
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  const int i0 = blockIdx.y * 64;
  const int t = threadIdx.x, bl = t & 63;
  const int64_t b = b0 + bl;
  const int64_t c = b < n_band ? band_cells[b] : 0;
  const int64_t cn = (FACE && b < n_band) ? rnbr[b] : -1;
  const double wz = (FACE && b < n_band) ? rw[b] : 1.0;
#pragma unroll 4
  for (int r = 0; r < 16; ++r) {
    const int il = (t >> 6) + 4 * r;
    const int i = i0 + il;
    T v = T(0);
    if (b < n_band && i < L) {
      const double* src = i < l_s ? U + N * (int64_t)i : Z + N * (int64_t)(i - l_s);
      double val = src[c];
      if (FACE) {
        if (cn >= 0) val -= src[cn];
        if (i >= l_s) val *= wz;
      }
      v = (T)val;
    }
    tile[bl][il] = v;
  }
  __syncthreads();
#pragma unroll 4
  for (int r = 0; r < 16; ++r) {
    const int e = t + 256 * r;
    const int bb = e >> 6, ii = e & 63;
    const int64_t ob = b0 + bb;
    const int oi = i0 + ii;
    if (ob < n_band && oi < L) packed[ob * L + oi] = tile[bb][ii];
  }
}

// ----------------------------------------------------------------------
// Binary64 matrix-core contraction of one chunk (the pairs of one RBF, or a
// piece of them).  Per chunk it is a dense product
//     P[i, n] = sum_p U[c_p, i] B[p, n],  B[p, j + l_d a] = Z[c_p, j] G[p, a],
// i < l_s, n < l_d na, over the chunk's pairs in K-steps of 32.  A thread
// stages the values i = t % 16 + 16 r of pair t / 16 of a step from its packed
// row (one contiguous row per pair) into LDS: U as the A operand, Z times the
// pair's G as the B operand.  The next step's rows are loaded while the
// matrix cores work on the current one (band rows two steps ahead).  The
// products run on v_mfma_f64_16x16x4f64 with binary64 accumulation.
// Output tiles of 16 x 16 are dealt to the 8 waves round-robin: tile
// t = wave + 8 q covers rows 16 (t % MT) .. +15 and columns 16 (t / MT) .. +15,
// zero-padded beyond l_s rows and l_d na columns.  Lane layout: A row l % 16,
// B column l % 16, k = l / 16 + 4 s; result column l % 16, rows l / 16 + 4 e.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int JK = 32;            // pairs per K-step
constexpr int JKP64 = JK + 1;     // padded binary64 LDS row
constexpr int JTHREADS = 512;     // 8 waves; 16 threads per pair of a step
constexpr int JRMAX = 8;          // values per thread and step: l_s + l_d <= 128
constexpr int JFLUSH = 16;        // K-steps per binary32 run of the split forms
constexpr int JSLOT = JK * JFLUSH;                                    // pairs per run
constexpr int JSPC = (int)((DOT_PAIR_CHUNK + JSLOT - 1) / JSLOT);     // runs per chunk

template <int TERMS>
__device__ __forceinline__ void split_bf16(float x, __bf16* parts) {
  const __bf16 hi = (__bf16)x;
  float rem = x - (float)hi;
  parts[0] = hi;
  if constexpr (TERMS == 2) {
    parts[1] = (__bf16)rem;
  } else {
    const __bf16 mid = (__bf16)rem;
    parts[1] = mid;
    parts[2] = (__bf16)(rem - (float)mid);
  }
}

// A rows, B columns, and one discard row for the stores of lanes that hold
// no operand value (their stores are unconditional)
__host__ __device__ inline size_t jac_lds_bytes(int rows, int ncp) {
  return (size_t)(rows + ncp + 1) * JKP64 * sizeof(double);
}

template <int QMAX>
__global__ __launch_bounds__(JTHREADS) void jac_mfma_kernel(
    const int32_t* __restrict__ pair_band, const double* __restrict__ pair_g, int64_t n_pairs,
    const int64_t* __restrict__ chunk_begin, int l_s, int l_d, int na,
    const double* __restrict__ packed, double* __restrict__ partial, int ncp) {
  extern __shared__ __attribute__((aligned(16))) unsigned char jsm[];
  const int ch = blockIdx.x;
  const int64_t b0 = chunk_begin[ch], b1 = chunk_begin[ch + 1];
  const int L = l_s + l_d;
  const int lsld = l_s * l_d;
  const int ncol = l_d * na;
  const int MT = (l_s + 15) / 16;
  const int rows = MT * 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* out = partial + (int64_t)ch * lsld * na;
  double* dA = reinterpret_cast<double*>(jsm);   // [rows][JKP64]
  double* dB = dA + rows * JKP64;                // [ncp][JKP64]
  {  // rows >= l_s and columns >= ncol are never written: clear once
    const int words = (int)(jac_lds_bytes(rows, ncp) / 4);
    for (int e = threadIdx.x; e < words; e += JTHREADS) reinterpret_cast<int*>(jsm)[e] = 0;
  }

  // per tile t = wave + 8 q: operand rows/columns of this lane and the output
  // offset of its result rows l / 16 + 4 e
  int arow[QMAX], bcol[QMAX], ooff[QMAX], orow[QMAX], ocol[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int t = wave + 8 * q;
    const int mt = t % MT, nt = t / MT;
    arow[q] = mt * 16 + (lane & 15);
    bcol[q] = nt * 16 + (lane & 15);
    const int i0 = mt * 16 + (lane >> 4);
    const int n = bcol[q];
    orow[q] = i0;
    ocol[q] = n;
    ooff[q] = n < ncol ? (n % l_d) + l_d * i0 + lsld * (n / l_d) : 0;
  }
  f64x4 acc64[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) acc64[q] = f64x4{0.0, 0.0, 0.0, 0.0};

  // staging: thread t holds values i = qv + 16 r of pair pb of a step, in two
  // register slots: the rows of step s + 2 are loaded while step s is staged
  // and multiplied, so a load has two steps to arrive
  const int pb = threadIdx.x >> 4, qv = threadIdx.x & 15;
  const int nr = (L + 15) / 16;
  double val[2][JRMAX];
  double gv[2][5];
  // Loads are unconditional, from clamped (always valid) addresses, and no
  // loaded value is selected on afterwards (a select lets the compiler sink
  // the load into a branch that then waits for it): a pair beyond the chunk
  // reads band row 0 and the zero G entries past the last pair (n_pairs),
  // so its B entries vanish and its A entries multiply zeros; a value index
  // beyond L is clamped and its stores go to the discard row.
  auto band_row = [&](int64_t base) -> int {
    return pair_band[base + pb < b1 ? base + pb : b1 - 1];
  };
  auto load_step = [&](auto slot_c, int64_t base, int bi) {
    constexpr int S = decltype(slot_c)::value;
    const bool valid = base + pb < b1;
    const double* row = packed + (int64_t)(valid ? bi : 0) * L;
#pragma unroll
    for (int r = 0; r < JRMAX; ++r) {
      if (r >= nr) break;
      const int i = qv + 16 * r;
      val[S][r] = row[i < L ? i : L - 1];
    }
    const double* gp = pair_g + (valid ? base + pb : n_pairs) * na;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      if (a >= na) break;
      gv[S][a] = gp[a];
    }
  };
  // every lane stores every slot; a value that is not an A entry (or not a
  // B entry) goes to the discard row instead, so the stores need no branches
  const int discard = rows + ncp;
  auto store_step = [&](auto slot_c) {
    constexpr int S = decltype(slot_c)::value;
#pragma unroll
    for (int r = 0; r < JRMAX; ++r) {
      if (r >= nr) break;
      const int i = qv + 16 * r;
      const bool isA = i < l_s, isB = i >= l_s && i < L;
      const int arow_s = isA ? i : discard;
      const int j = isB ? i - l_s : 0;
      dA[arow_s * JKP64 + pb] = val[S][r];
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        if (a >= na) break;
        const int n = isB ? rows + j + l_d * a : discard;   // row of B within the LDS block
        dA[n * JKP64 + pb] = val[S][r] * gv[S][a];
      }
    }
  };
  auto multiply = [&]() {
    const int kl = lane >> 4;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
#pragma unroll
      for (int ks = 0; ks < JK / 4; ++ks) {
        const double a = dA[arow[q] * JKP64 + 4 * ks + kl];
        const double b = dB[bcol[q] * JKP64 + 4 * ks + kl];
        acc64[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc64[q], 0, 0, 0);
      }
    }
  };

  // prologue: rows of steps 0 and 1 in flight, band rows of steps 2 and 3
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  load_step(S0{}, b0, band_row(b0));
  load_step(S1{}, b0 + JK, band_row(b0 + JK));
  int biA = band_row(b0 + 2 * JK), biB = band_row(b0 + 3 * JK);
  __syncthreads();  // LDS cleared before the first store
  // one K-step from register slot S: stage, multiply, refill the slot with
  // the rows of the step two ahead
  auto step = [&](auto slot_c, int64_t base) {
    const int bnext = band_row(base + 4 * JK);   // used four steps on
    store_step(slot_c);
    __syncthreads();
    if (base + 2 * JK < b1) load_step(slot_c, base + 2 * JK, biA);
    multiply();
    __syncthreads();  // operand reads done before the next store
    biA = biB;
    biB = bnext;
  };
  for (int64_t base = b0; base < b1; base += 2 * JK) {
    step(S0{}, base);
    if (base + JK < b1) step(S1{}, base + JK);
  }
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (orow[q] + 4 * e < l_s && ocol[q] < ncol) out[ooff[q] + l_d * 4 * e] = acc64[q][e];
  }
}

// ----------------------------------------------------------------------
// Split-bfloat16 contraction with operands split once.
//
// pack_split_kernel writes, per band row b (cell c_b), the bfloat16 parts of
// U[c_b, i] rounded to binary32 (i < MT 16, zero for i >= l_s) as one word
// per value (hi | lo << 16 for two parts; {hi | mid << 16, lo} for three)
// and Z[c_b, j] in binary32.  jac_split_kernel then runs one block of four
// waves per chunk, in K-steps of 32 pairs: the 16 threads of a pair couple
// (k, k + 1) copy the A parts of both pairs into LDS as [part][i][k] and
// form the B values Z[c_k, j] G[k, a] for their columns j = q + 16 r,
// splitting each product once and storing its parts as [part][n][k],
// n = j + l_d a; the next step's rows and G are loaded while the waves
// multiply.  Wave w owns the column tiles nt = w + 4 q with every row tile;
// per (row tile, column tile) it issues the part products of total order at
// most TERMS - 1 on v_mfma_f32_16x16x32_bf16, accumulates in binary32 and
// flushes into the binary64 partial block every JFLUSH K-steps.
template <int TERMS>
struct SplitWord {
  using type = uint32_t;
};
template <>
struct SplitWord<3> {
  using type = uint2;
};

__device__ __forceinline__ unsigned short bf16_bits(__bf16 v) {
  return __builtin_bit_cast(unsigned short, v);
}

template <int TERMS>
__device__ __forceinline__ typename SplitWord<TERMS>::type split_word(float x) {
  __bf16 p[TERMS];
  split_bf16<TERMS>(x, p);
  if constexpr (TERMS == 2) {
    return (uint32_t)bf16_bits(p[0]) | ((uint32_t)bf16_bits(p[1]) << 16);
  } else {
    return uint2{(uint32_t)bf16_bits(p[0]) | ((uint32_t)bf16_bits(p[1]) << 16),
                 (uint32_t)bf16_bits(p[2])};
  }
}

// the parts of x0 and x1 (two pairs of one column) packed two to a word:
// word p = part p of x0 | part p of x1 << 16, one two-way conversion per part
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

template <int TERMS>
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t* w) {
  f32x2 r = f32x2{x0, x1};
#pragma unroll
  for (int p = 0; p < TERMS; ++p) {
    const uint32_t b = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
    w[p] = b;
    if (p + 1 < TERMS) {
      r.x -= __builtin_bit_cast(float, b << 16);
      r.y -= __builtin_bit_cast(float, b & 0xffff0000u);
    }
  }
}

// part p of a split word
template <int TERMS>
__device__ __forceinline__ uint32_t word_part(const typename SplitWord<TERMS>::type& w, int p) {
  if constexpr (TERMS == 2) {
    return p == 0 ? (w & 0xffffu) : (w >> 16);
  } else {
    return p == 0 ? (w.x & 0xffffu) : p == 1 ? (w.x >> 16) : (w.y & 0xffffu);
  }
}

template <int TERMS, bool FACE>
__global__ __launch_bounds__(256) void pack_split_kernel(int64_t N, int64_t n_band,
                                                         const int32_t* __restrict__ band_cells,
                                                         const int32_t* __restrict__ rnbr,
                                                         const double* __restrict__ rw,
                                                         int l_s, const double* __restrict__ U,
                                                         int l_d, const double* __restrict__ Z,
                                                         int mt16, int ldj,
                                                         typename SplitWord<TERMS>::type* __restrict__ pu,
                                                         float* __restrict__ pz) {
  extern __shared__ float ptile[];  // [64][L + 1]
  const int L = l_s + l_d, LP = L + 1;
  const int64_t b0 = (int64_t)blockIdx.x * 64;
  const int t = threadIdx.x, bl = t & 63;
  const int64_t b = b0 + bl;
  const int64_t c = b < n_band ? band_cells[b] : 0;
  // FACE: the neighbour's values are subtracted (clamped to the cell itself
  // and multiplied by zero where there is none) and Z is weighted
  const int64_t cr = (FACE && b < n_band) ? rnbr[b] : -1;
  const int64_t cn = cr >= 0 ? cr : c;
  const double fl = cr >= 0 ? 1.0 : 0.0;
  const double wz = (FACE && b < n_band) ? rw[b] : 1.0;
  // columns i = t / 64 + 4 k, eight loads in flight per thread (a row of
  // band cells is a gather: latency, not bandwidth, bounds one load at a
  // time).  Loads and stores are unconditional (a guarded load is waited
  // for inside its branch): rows past n_band read cell 0 and are never
  // written out, columns past L are clamped and land in the pad column L.
  for (int i0 = t >> 6; i0 < L; i0 += 32) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = min(i0 + 4 * k, L - 1);
      const double* src = i < l_s ? U + N * (int64_t)i : Z + N * (int64_t)(i - l_s);
      v[k] = src[c];
      if (FACE) v[k] = (v[k] - fl * src[cn]) * (i < l_s ? 1.0 : wz);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) ptile[bl * LP + min(i0 + 4 * k, L)] = (float)v[k];
  }
  __syncthreads();
  const int rows = (int)(n_band - b0 < 64 ? n_band - b0 : 64);
  for (int e = t; e < rows * mt16; e += 256) {
    const int r = e / mt16, i = e - r * mt16;
    pu[(b0 + r) * mt16 + i] = split_word<TERMS>(i < l_s ? ptile[r * LP + i] : 0.f);
  }
  for (int e = t; e < rows * ldj; e += 256) {
    const int r = e / ldj, j = e - r * ldj;
    pz[(b0 + r) * ldj + j] = j < l_d ? ptile[r * LP + l_s + j] : 0.f;
  }
}

constexpr int JS_THREADS = 256;   // 4 waves; 16 threads per pair couple of a K-step
constexpr int JS_KP = 40;         // LDS row of one operand value over a K-step: 32 pairs + 8 pad (80 B)

// A: [TERMS][MT 16][JS_KP]; B: [TERMS][na JR 16][JS_KP] (column n = a JR 16 + j)
__host__ __device__ inline size_t jac_split_lds_bytes(int terms, int mt, int jr, int na) {
  return (size_t)terms * (mt + na * jr) * 16 * JS_KP * sizeof(unsigned short);
}

// MT row tiles (l_s <= 16 MT), JR detector-sample tiles per parameter
// (l_d <= 16 JR); the B columns of parameter a start at a 16 JR, so every
// LDS offset of a staging thread is a constant from one base address.
// Column tiles: na JR, at most 5 JR; wave w owns tiles w + 4 q, q < NTW.
template <int TERMS, int MT, int JR>
__global__ __launch_bounds__(JS_THREADS) void jac_split_kernel(
    const int32_t* __restrict__ pair_band, const float* __restrict__ pair_g, int64_t n_pairs,
    const int64_t* __restrict__ chunk_begin, int l_s, int l_d, int na,
    const typename SplitWord<TERMS>::type* __restrict__ pu, const float* __restrict__ pz,
    float* __restrict__ partial) {
  using SW = typename SplitWord<TERMS>::type;
  constexpr int MT16 = MT * 16;
  constexpr int LDJ = JR * 16;
  constexpr int NTW = (5 * JR + 3) / 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char jsm[];
  unsigned short* sA = reinterpret_cast<unsigned short*>(jsm);  // [TERMS][MT16][JS_KP]
  unsigned short* sB = sA + TERMS * MT16 * JS_KP;                // [TERMS][na LDJ][JS_KP]
  const int ch = blockIdx.x;
  const int64_t b0 = chunk_begin[ch], b1 = chunk_begin[ch + 1];
  const int lsld = l_s * l_d;
  const int nt = na * JR;
  const int brows = na * LDJ;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* out = partial + (int64_t)ch * JSPC * lsld * na;

  f32x4 acc[NTW][MT];
#pragma unroll
  for (int q = 0; q < NTW; ++q)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[q][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  // the binary32 block of run `slot` (JFLUSH K-steps) is stored, not added:
  // no load waits in the K loop; the reduce sums the runs in binary64
  auto flush = [&](int slot) {
    // an opaque copy of the lane index keeps the output addresses from being
    // computed once before the K loop and held in registers throughout
    int lo = lane;
    asm volatile("" : "+v"(lo));
    float* o_s = out + (int64_t)slot * lsld * na;
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
      const int n = (wave + 4 * q) * 16 + (lo & 15);
      const int a = n / LDJ, j = n - a * LDJ;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int i0 = mt * 16 + 4 * (lo >> 4);
        if (a < na && j < l_d) {
          float* o = o_s + j + l_d * i0 + lsld * a;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (i0 + e < l_s) o[l_d * e] = acc[q][mt][e];
        }
        acc[q][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };

  // staging roles: pair couple cp (pairs 2 cp, 2 cp + 1 of a step), value
  // index qv: A rows i = qv + 16 r (r < MT), B detector samples j = qv + 16 r
  // (r < JR; the packed Z rows are zero past l_d)
  const int cp = threadIdx.x >> 4, qv = threadIdx.x & 15;
  SW ua[MT][2];
  float zv[JR][2];
  float gv[5][2];
  // Loads are unconditional from clamped addresses: a pair beyond the chunk
  // reads band row 0 and the zero G record past the last pair (n_pairs), so
  // its B values vanish.
  auto band_rows = [&](int64_t base, int* r) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t p = base + 2 * cp + h;
      r[h] = p < b1 ? pair_band[p] : 0;
    }
  };
  auto load_step = [&](int64_t base, const int* brow) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t p = base + 2 * cp + h;
      const SW* ur = pu + (int64_t)brow[h] * MT16 + qv;
#pragma unroll
      for (int r = 0; r < MT; ++r) ua[r][h] = ur[16 * r];
      const float* zr = pz + (int64_t)brow[h] * LDJ + qv;
#pragma unroll
      for (int r = 0; r < JR; ++r) zv[r][h] = zr[16 * r];
      const float* gp = pair_g + (p < b1 ? p : n_pairs) * na;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        if (a >= na) break;
        gv[a][h] = gp[a];
      }
    }
  };
  // this thread's LDS words: pairs 2 cp, 2 cp + 1 of row qv (+ constants)
  uint32_t* const wA = reinterpret_cast<uint32_t*>(sA + qv * JS_KP + 2 * cp);
  uint32_t* const wB = reinterpret_cast<uint32_t*>(sB + qv * JS_KP + 2 * cp);
  const int partB = brows * JS_KP / 2;  // words between parts of B
  auto store_step = [&]() {
#pragma unroll
    for (int r = 0; r < MT; ++r)
#pragma unroll
      for (int p = 0; p < TERMS; ++p)
        wA[(p * MT16 + 16 * r) * (JS_KP / 2)] =
            word_part<TERMS>(ua[r][0], p) | (word_part<TERMS>(ua[r][1], p) << 16);
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      if (a >= na) break;
#pragma unroll
      for (int r = 0; r < JR; ++r) {
        uint32_t w[TERMS];
        split_pair<TERMS>(zv[r][0] * gv[a][0], zv[r][1] * gv[a][1], w);
#pragma unroll
        for (int p = 0; p < TERMS; ++p) wB[p * partB + (a * LDJ + 16 * r) * (JS_KP / 2)] = w[p];
      }
    }
  };
  auto multiply = [&]() {
    const int kofs = 8 * (lane >> 4);
    bf16x8 fa[MT][TERMS];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int p = 0; p < TERMS; ++p)
        fa[mt][p] = *reinterpret_cast<const bf16x8*>(sA + (p * MT16 + mt * 16 + (lane & 15)) * JS_KP + kofs);
    // a wave with fewer than NTW column tiles repeats its last valid tile
    // into the spare accumulators (never flushed): no branch around the
    // matrix-core instructions
#pragma unroll
    for (int q = 0; q < NTW; ++q) {
      const int ntq = min(wave + 4 * q, nt - 1);
      bf16x8 fb[TERMS];
#pragma unroll
      for (int p = 0; p < TERMS; ++p)
        fb[p] = *reinterpret_cast<const bf16x8*>(sB + (p * brows + ntq * 16 + (lane & 15)) * JS_KP + kofs);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int pa = 0; pa < TERMS; ++pa)
#pragma unroll
          for (int pb = 0; pb < TERMS; ++pb)
            if (pa + pb <= TERMS - 1)
              acc[q][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[mt][pa], fb[pb], acc[q][mt], 0, 0, 0);
    }
  };

  int brow[2], bnext[2];
  band_rows(b0, brow);
  load_step(b0, brow);
  band_rows(b0 + JK, bnext);
  int kstep = 0;
  for (int64_t base = b0; base < b1; base += JK) {
    store_step();
    __syncthreads();
    if (base + JK < b1) {
      brow[0] = bnext[0];
      brow[1] = bnext[1];
      load_step(base + JK, brow);
      band_rows(base + 2 * JK, bnext);
    }
    multiply();
    if ((kstep + 1) % JFLUSH == 0) flush(kstep / JFLUSH);
    __syncthreads();  // operand reads done before the next store
    ++kstep;
  }
  if (kstep % JFLUSH != 0) flush(kstep / JFLUSH);
}

// Where a tile of t_i sources x t_j detectors lands in J_s: the tile's row
// j + t_j i (detector fastest) and column k go to
// Js[base + j + ldi i + ldk k], so a tile at sources i0.., detectors j0.. of
// an l_s x l_d sample has base j0 + l_d i0, ldi = l_d, ldk = l_s l_d.
struct JacOut {
  int tj;
  int64_t base, ldi, ldk;
  __device__ __forceinline__ int64_t at(int row, int k) const {
    return base + (row % tj) + ldi * (row / tj) + ldk * (int64_t)k;
  }
};

// J_s entry (j, i, m na + a) of the tile = - sum over the chunks of RBF m
// and their runs of JFLUSH K-steps (binary32 blocks), in order, in binary64.
__global__ void jac_reduce_runs_kernel(int m0, const int32_t* __restrict__ rbf_chunk0,
                                       const int64_t* __restrict__ chunk_begin, int lsld, int na,
                                       const float* __restrict__ partial, JacOut o,
                                       double* __restrict__ Js) {
  const int m = blockIdx.y;
  const int nout = lsld * na;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= m0 || e >= nout) return;
  const int c0 = rbf_chunk0[m], c1 = rbf_chunk0[m + 1];
  double s = 0.0;
  if (JSPC == 1) {
    // one run per chunk: four loads in flight as in jac_reduce_kernel
    for (int ch = c0; ch < c1; ch += 4) {
      float v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = partial[(int64_t)min(ch + k, c1 - 1) * nout + e];
#pragma unroll
      for (int k = 0; k < 4; ++k) s += (double)v[k] * (double)(ch + k < c1);
    }
  } else {
    for (int ch = c0; ch < c1; ++ch) {
      const int64_t len = chunk_begin[ch + 1] - chunk_begin[ch];
      const int runs = (int)((len + JSLOT - 1) / JSLOT);
      const float* p = partial + (int64_t)ch * JSPC * nout + e;
      for (int r = 0; r < runs; ++r) s += (double)p[(int64_t)r * nout];
    }
  }
  const int a = e / lsld, row = e % lsld;
  Js[o.at(row, m * na + a)] = -s;
}

// J_s entry (j, i, m na + a) of the tile = - sum over chunks of RBF m.
__global__ void jac_reduce_kernel(int m0, const int32_t* __restrict__ rbf_chunk0, int lsld, int na,
                                  const double* __restrict__ partial, JacOut o,
                                  double* __restrict__ Js) {
  const int m = blockIdx.y;
  const int nout = lsld * na;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= m0 || e >= nout) return;
  const int c0 = rbf_chunk0[m], c1 = rbf_chunk0[m + 1];
  double s = 0.0;
  // four loads in flight, from clamped chunks whose surplus terms are
  // multiplied by zero (the summation order is the chunk order)
  for (int ch = c0; ch < c1; ch += 4) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = partial[(int64_t)min(ch + k, c1 - 1) * nout + e];
#pragma unroll
    for (int k = 0; k < 4; ++k) s += v[k] * (double)(ch + k < c1);
  }
  const int a = e / lsld, row = e % lsld;
  Js[o.at(row, m * na + a)] = -s;
}

// s_c = sum_i U[c,i] sum_j Z[c,j] Rs[j,i] on band cells, 0 elsewhere.
__global__ __launch_bounds__(256) void grad_cell_kernel(GridDims g, JacParams P,
                                                        const double* __restrict__ phi, int l_s,
                                                        const double* __restrict__ U, int l_d,
                                                        const double* __restrict__ Z,
                                                        const double* __restrict__ Rs,
                                                        double* __restrict__ sc) {
  extern __shared__ double sR[];  // l_d x l_s
  for (int t = threadIdx.x; t < l_d * l_s; t += blockDim.x) sR[t] = Rs[t];
  __syncthreads();
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  if (fabs(phi[c] - P.cutoff) > P.eps) {
    sc[c] = 0.0;
    return;
  }
  double s = 0.0;
  for (int i = 0; i < l_s; ++i) {
    double lam = 0.0;
    for (int j = 0; j < l_d; ++j) lam += Z[c + P.N * j] * sR[j + l_d * i];
    s += U[c + P.N * i] * lam;
  }
  sc[c] = s;
}

// The same sums with each Z[c, j] loaded once (l_s <= MAXS): lam[i] is
// accumulated over j in the same order, so the result is identical.
template <int MAXS>
__global__ __launch_bounds__(256) void grad_cell_small_kernel(GridDims g, JacParams P,
                                                              const double* __restrict__ phi,
                                                              int l_s, const double* __restrict__ U,
                                                              int l_d, const double* __restrict__ Z,
                                                              const double* __restrict__ Rs,
                                                              double* __restrict__ sc) {
  extern __shared__ double sR[];  // l_d x l_s
  for (int t = threadIdx.x; t < l_d * l_s; t += blockDim.x) sR[t] = Rs[t];
  __syncthreads();
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  if (fabs(phi[c] - P.cutoff) > P.eps) {
    sc[c] = 0.0;
    return;
  }
  double lam[MAXS];
#pragma unroll
  for (int i = 0; i < MAXS; ++i) lam[i] = 0.0;
  for (int j = 0; j < l_d; ++j) {
    const double zj = Z[c + P.N * j];
#pragma unroll
    for (int i = 0; i < MAXS; ++i)
      if (i < l_s) lam[i] += zj * sR[j + l_d * i];
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < MAXS; ++i)
    if (i < l_s) s += U[c + P.N * i] * lam[i];
  sc[c] = s;
}

// Diffusion mode: Lambda = Z R_s (N x l_s), then per face row q (cell c,
// neighbour c', weight w) e_q = sum_i (U_ci - U_c'i) w (Lambda_ci - Lambda_c'i)
// (the plain values where there is no neighbour), which the virtual pairs
// weight by h^d d mu / d p like the cell sums of the absorption-only mode.
__global__ __launch_bounds__(256) void lambda_kernel(int64_t N, int l_s, int l_d,
                                                     const double* __restrict__ Z,
                                                     const double* __restrict__ Rs,
                                                     double* __restrict__ Lam) {
  extern __shared__ double sR[];  // l_d x l_s
  for (int t = threadIdx.x; t < l_d * l_s; t += blockDim.x) sR[t] = Rs[t];
  __syncthreads();
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= N) return;
  for (int i = 0; i < l_s; ++i) {
    double v = 0.0;
    for (int j = 0; j < l_d; ++j) v += Z[c + N * j] * sR[j + l_d * i];
    Lam[c + N * i] = v;
  }
}

__global__ __launch_bounds__(256) void grad_vrow_kernel(int64_t N, int64_t n_rows, int l_s,
                                                        const int32_t* __restrict__ rcell,
                                                        const int32_t* __restrict__ rnbr,
                                                        const double* __restrict__ rw,
                                                        const double* __restrict__ U,
                                                        const double* __restrict__ Lam,
                                                        double* __restrict__ e) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n_rows) return;
  const int64_t c = rcell[q], cn = rnbr[q];
  double s = 0.0;
  for (int i = 0; i < l_s; ++i) {
    double du = U[c + N * i], dl = Lam[c + N * i];
    if (cn >= 0) {
      du -= U[cn + N * i];
      dl -= Lam[cn + N * i];
    }
    s += du * dl;
  }
  e[q] = rw[q] * s;
}

__global__ __launch_bounds__(256) void grad_chunk_kernel(int na, const int32_t* __restrict__ pair_cell,
                                                         const double* __restrict__ pair_g,
                                                         const int64_t* __restrict__ chunk_begin,
                                                         const double* __restrict__ sc,
                                                         double* __restrict__ partial) {
  __shared__ double red[5][256];
  const int ch = blockIdx.x;
  const int64_t b0 = chunk_begin[ch], b1 = chunk_begin[ch + 1];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t p = b0 + threadIdx.x; p < b1; p += 256) {
    const double s = sc[pair_cell[p]];
    for (int a = 0; a < na; ++a) acc[a] += pair_g[p * na + a] * s;
  }
  for (int a = 0; a < na; ++a) red[a][threadIdx.x] = acc[a];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int a = 0; a < na; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < na) partial[(int64_t)ch * na + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void grad_reduce_kernel(int m0, const int32_t* __restrict__ rbf_chunk0, int na,
                                   const double* __restrict__ partial, double* __restrict__ gout) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m0 * na) return;
  const int m = k / na, a = k % na;
  double s = 0.0;
  for (int ch = rbf_chunk0[m]; ch < rbf_chunk0[m + 1]; ++ch) s += partial[(int64_t)ch * na + a];
  gout[k] = -s;
}

#define DOT_TRY_J(...)             \
  do {                             \
    int rc_ = (__VA_ARGS__);       \
    if (rc_ != DOT_OK) return rc_; \
  } while (0)

static int n_active_bits(unsigned act, int dim) {
  return ((act & DOT_ACT_ALPHA) ? 1 : 0) + ((act & DOT_ACT_BETA) ? 1 : 0) +
         ((act & DOT_ACT_CHI) ? dim : 0);
}

static JacParams make_params(const dot_op* op) {
  JacParams P;
  P.N = op->g.N;
  P.h = op->g.h;
  P.hd = op->g.hd;
  P.dim = op->g.dim;
  P.stride = 2 + op->g.dim;
  P.dmu = op->pals.mu_in - op->pals.mu_out;
  P.cutoff = op->pals.cutoff;
  P.eps = op->pals.eps;
  P.gamma = op->pals.gamma;
  P.active = op->pals.active;
  P.n_act = n_active_bits(op->pals.active, op->g.dim);
  return P;
}

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of dot_jacobian / dot_grad_misfit: per-chunk partial blocks, then
// the packed band rows (binary64, which also holds the binary32 packing).
// binary64 per chunk, or binary32 per run of JSLOT pairs (JSPC per chunk)
// The rows and pairs the contraction runs over: the band cells and the
// (RBF, cell) pairs, or in diffusion mode the face rows and virtual pairs.
struct JacTables {
  int64_t n_rows;
  const int32_t* row_cell;
  const int32_t* row_nbr;    // diffusion mode only
  const double* row_w;       // diffusion mode only
  const int32_t* pair_band;
  const double* pair_g;
  const float* pair_g32;
  int64_t n_pairs;
  const int64_t* chunk_begin;
  int64_t n_chunks;
  const int32_t* rbf_chunk0;
  bool face;
};

static JacTables jac_tables(const dot_op* op) {
  JacTables t;
  t.face = op->diff_mode;
  if (!t.face) {
    t.n_rows = band_count(const_cast<dot_op*>(op));
    t.row_cell = op->band_cells;
    t.row_nbr = nullptr;
    t.row_w = nullptr;
    t.pair_band = op->pair_band;
    t.pair_g = op->pair_g;
    t.pair_g32 = op->pair_g32;
    t.n_pairs = op->n_pairs;
    t.chunk_begin = op->chunk_begin;
    t.n_chunks = op->n_chunks;
    t.rbf_chunk0 = op->rbf_chunk0;
  } else {
    t.n_rows = op->n_vrows;
    t.row_cell = op->vrow_cell;
    t.row_nbr = op->vrow_nbr;
    t.row_w = op->vrow_w;
    t.pair_band = op->vpair_band;
    t.pair_g = op->vpair_g;
    t.pair_g32 = op->vpair_g32;
    t.n_pairs = op->n_vpairs;
    t.chunk_begin = op->vchunk_begin;
    t.n_chunks = op->n_vchunks;
    t.rbf_chunk0 = op->vrbf_chunk0;
  }
  return t;
}

// binary64 per chunk, or binary32 per run of JSLOT pairs (JSPC per chunk)
static size_t jac_partial_bytes(const dot_op* op, int l_s, int l_d) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  return al256((size_t)std::max<int64_t>(jac_tables(op).n_chunks, 1) * l_s * l_d * na *
               std::max(sizeof(double), JSPC * sizeof(float)));
}

// packed rows: binary64 rows of l_s + l_d values, or for the split forms the
// split words of U (at most 8 bytes, l_s rounded up to 16 per row) followed
// by binary32 rows of Z (l_d rounded up to 16)
static size_t packed_split_u_bytes(const dot_op* op, int l_s) {
  return al256((size_t)std::max<int64_t>(jac_tables(op).n_rows, 1) * ((l_s + 15) / 16) * 16 * 8);
}

// Source x detector tile of one contraction pass: the whole sample when the
// matrix-core kernels hold it (binary64: at most 64 output tiles of 16 x 16
// over 8 waves, l_s + l_d <= 16 JRMAX and the LDS staging within 160 KB;
// split forms: l_s, l_d <= 64),
// otherwise tiles of at most 64 sources and as many detectors as fit.
static void jac_tile_shape(int precision, int l_s, int l_d, int na, int* ts, int* td) {
  if (precision == DOT_JAC_FP64) {
    // at most 8 output tiles per wave, JRMAX staged values per thread, and
    // the staged operands within the 160 KB of LDS
    auto fits = [na](int a, int b) {
      const int mt = (a + 15) / 16, tiles = mt * ((b * na + 15) / 16);
      if (tiles > 64 || a + b > 16 * JRMAX) return false;
      const int ncp = ((8 * ((tiles + 7) / 8) - 1) / mt + 1) * 16;
      return jac_lds_bytes(mt * 16, ncp) <= (size_t)160 * 1024;
    };
    if (fits(l_s, l_d)) {
      *ts = l_s;
      *td = l_d;
      return;
    }
    const int a = std::min(l_s, 64);
    int b = std::min(l_d, 16 * JRMAX - a);
    while (b > 1 && !fits(a, b)) --b;
    *ts = a;
    *td = b;
  } else {
    *ts = std::min(l_s, 64);
    *td = std::min(l_d, 64);
  }
}

static size_t jac_tile_bytes(const dot_op* op, int l_s, int l_d) {
  const size_t nb = (size_t)std::max<int64_t>(jac_tables(op).n_rows, 1);
  const size_t packed = std::max(al256(nb * (l_s + l_d) * sizeof(double)),
                                 packed_split_u_bytes(op, l_s) +
                                     al256(nb * ((l_d + 15) / 16) * 16 * sizeof(float)));
  return jac_partial_bytes(op, l_s, l_d) + packed;
}

// gradient scratch in diffusion mode: Lambda = Z R_s (N x l_s), one value
// per face row, one partial per (chunk, active parameter)
static size_t grad_face_bytes(const dot_op* op, int l_s) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  return al256((size_t)op->g.N * l_s * sizeof(double)) +
         al256((size_t)std::max<int64_t>(op->n_vrows, 1) * sizeof(double)) +
         al256((size_t)std::max<int64_t>(op->n_vchunks, 1) * na * sizeof(double));
}

static size_t jac_bytes(const dot_op* op, int l_s, int l_d) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  int a = 0, b = 0, c = 0, d = 0;
  jac_tile_shape(DOT_JAC_FP64, l_s, l_d, na, &a, &b);
  jac_tile_shape(DOT_JAC_SPLIT_BF16, l_s, l_d, na, &c, &d);
  const size_t jac = std::max(jac_tile_bytes(op, a, b), jac_tile_bytes(op, c, d));
  size_t grad = (size_t)op->g.N * sizeof(double) +
                (size_t)std::max<int64_t>(op->n_chunks, 1) * na * sizeof(double) + 256;
  if (op->diff_mode) grad = std::max(grad, grad_face_bytes(op, l_s));
  return al256(std::max(jac, grad));
}

template <typename T>
static int grow(T** p, int64_t* cap, int64_t need) {
  if (need <= *cap) return DOT_OK;
  if (*p) DOT_HIP(hipFree(*p));
  *p = nullptr;
  *cap = 0;
  const int64_t n = std::max<int64_t>(need + need / 8, 1024);
  DOT_HIP(hipMalloc(p, (size_t)n * sizeof(T)));
  *cap = n;
  return DOT_OK;
}

int jac_prepare(dot_op* op, hipStream_t s) {
  const JacParams P = make_params(op);
  const int na = P.n_act;
  const int64_t N = op->g.N, np = op->n_pairs;
  const int m0 = op->pals.m0;
  // one zero G record past the last pair (read by absent pairs of a K-step)
  int rc = grow(&op->pair_g, &op->pair_g_cap, (np + 1) * na + 8);
  if (rc) return rc;
  hipLaunchKernelGGL(fill_double_kernel, dim3(1), dim3(64), 0, s, op->pair_g + np * na, 8, 0.0);
  DOT_LAUNCH_CHECK();
  rc = grow(&op->pair_g32, &op->pair_g32_cap, (np + 1) * na + 8);
  if (rc) return rc;
  hipLaunchKernelGGL(fill_float_kernel, dim3(1), dim3(64), 0, s, op->pair_g32 + np * na, 8, 0.f);
  DOT_LAUNCH_CHECK();
  rc = grow(&op->pair_band, &op->pair_band_cap, std::max<int64_t>(np, 1));
  if (rc) return rc;
  if (!op->band_idx) DOT_HIP(hipMalloc(&op->band_idx, (size_t)N * sizeof(int32_t)));
  const int64_t nb = (N + BAND_BLK - 1) / BAND_BLK;
  rc = grow(&op->band_part, &op->band_part_cap, 2 * (nb + 1));
  if (rc) return rc;
  int64_t* cnt = op->band_part + (nb + 1);
  if (np > 0) {
    // about four blocks per compute unit over all RBFs
    const unsigned split = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, 1024 / std::max(m0, 1)));
    hipLaunchKernelGGL(pair_g_kernel, dim3(m0, split), dim3(256), 0, s, op->g, P, op->theta, op->phi,
                       op->rbf_start, op->pair_cell, op->pair_g, op->pair_g32);
    DOT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                     op->band_idx, N, 0);
  DOT_LAUNCH_CHECK();
  if (np > 0) {
    hipLaunchKernelGGL(band_mark_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np,
                       op->pair_cell, op->band_idx);
    DOT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(band_count_kernel, dim3((unsigned)nb), dim3(256), 0, s, N, op->band_idx, cnt);
  DOT_LAUNCH_CHECK();
  hipLaunchKernelGGL(band_scan_kernel, dim3(1), dim3(1024), 0, s, (int)nb, cnt, op->band_part);
  DOT_LAUNCH_CHECK();
  // the band holds at most min(N, pairs) cells: band_cells is sized by that
  // bound, and the count itself comes back through pinned memory, read
  // when it is first needed (band_count), so nothing here waits for the GPU
  if (op->band_pending) DOT_HIP(hipEventSynchronize(op->band_ev));
  DOT_HIP(hipMemcpyAsync(op->pinned_band, op->band_part + nb, sizeof(int64_t),
                         hipMemcpyDeviceToHost, s));
  DOT_HIP(hipEventRecord(op->band_ev, s));
  op->band_pending = true;
  op->n_band = -1;
  rc = grow(&op->band_cells, &op->band_cap, std::max<int64_t>(std::min<int64_t>(N, np), 1));
  if (rc) return rc;
  hipLaunchKernelGGL(band_fill_kernel, dim3((unsigned)nb), dim3(256), 0, s, N, op->band_part,
                     op->band_idx, op->band_cells);
  DOT_LAUNCH_CHECK();
  if (np > 0) {
    hipLaunchKernelGGL(pair_band_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np,
                       op->pair_cell, op->band_idx, op->pair_band);
    DOT_LAUNCH_CHECK();
  }
  return DOT_OK;
}

int64_t band_count(dot_op* op) {
  if (op->band_pending) {
    if (hipEventSynchronize(op->band_ev) != hipSuccess) return -1;
    op->n_band = *op->pinned_band;
    op->band_pending = false;
  }
  return op->n_band;
}

int jac_prepare_faces(dot_op* op, hipStream_t s) {
  const GridDims& g = op->g;
  const int R = 1 + 2 * g.dim;
  const int na = n_active_bits(op->pals.active, g.dim);
  const int m0 = op->pals.m0;
  const int64_t nr = band_count(op) * R, nv = op->n_pairs * R;
  // the three row arrays share one capacity
  const int64_t old_cap = op->vrow_cap;
  int rc = grow(&op->vrow_cell, &op->vrow_cap, std::max<int64_t>(nr, 1));
  if (rc) return rc;
  if (op->vrow_nbr == nullptr || op->vrow_cap != old_cap) {
    if (op->vrow_nbr) DOT_HIP(hipFree(op->vrow_nbr));
    if (op->vrow_w) DOT_HIP(hipFree(op->vrow_w));
    op->vrow_nbr = nullptr;
    op->vrow_w = nullptr;
    DOT_HIP(hipMalloc(&op->vrow_nbr, (size_t)op->vrow_cap * sizeof(int32_t)));
    DOT_HIP(hipMalloc(&op->vrow_w, (size_t)op->vrow_cap * sizeof(double)));
  }
  Faces6 fb;
  for (int f = 0; f < 6; ++f) fb.bc[f] = op->bc[f];
  const double ratio = 1.0 + (op->mus_in - op->mus_out) / (op->pals.mu_in - op->pals.mu_out);
  if (nr > 0) {
    hipLaunchKernelGGL(vrow_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s, g, fb,
                       band_count(op), op->band_cells, op->D0, ratio, R, op->vrow_cell, op->vrow_nbr,
                       op->vrow_w);
    DOT_LAUNCH_CHECK();
  }
  // virtual pairs (with one zero weight record past the last, as for pairs)
  int64_t cap = op->vpair_cap;
  rc = grow(&op->vpair_band, &cap, std::max<int64_t>(nv, 1));
  if (rc) return rc;
  if (cap != op->vpair_cap || !op->vpair_g) {
    if (op->vpair_g) DOT_HIP(hipFree(op->vpair_g));
    if (op->vpair_g32) DOT_HIP(hipFree(op->vpair_g32));
    op->vpair_g = nullptr;
    op->vpair_g32 = nullptr;
    DOT_HIP(hipMalloc(&op->vpair_g, (size_t)((cap + 1) * na + 8) * sizeof(double)));
    DOT_HIP(hipMalloc(&op->vpair_g32, (size_t)((cap + 1) * na + 8) * sizeof(float)));
    op->vpair_cap = cap;
  }
  hipLaunchKernelGGL(fill_double_kernel, dim3(1), dim3(64), 0, s, op->vpair_g + nv * na, 8, 0.0);
  DOT_LAUNCH_CHECK();
  hipLaunchKernelGGL(fill_float_kernel, dim3(1), dim3(64), 0, s, op->vpair_g32 + nv * na, 8, 0.f);
  DOT_LAUNCH_CHECK();
  if (nv > 0) {
    hipLaunchKernelGGL(vpair_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s,
                       op->n_pairs, R, na, op->pair_band, op->pair_g, op->vpair_band, op->vpair_g,
                       op->vpair_g32);
    DOT_LAUNCH_CHECK();
  }
  // chunks of at most DOT_PAIR_CHUNK virtual pairs within each RBF
  std::vector<int64_t> start(m0 + 1);
  DOT_HIP(hipMemcpyAsync(start.data(), op->rbf_start, (size_t)(m0 + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> vbegin;
  std::vector<int32_t> vrc(m0 + 1, 0);
  for (int m = 0; m < m0; ++m) {
    vrc[m] = (int32_t)vbegin.size();
    for (int64_t b = start[m] * R; b < start[m + 1] * R; b += DOT_PAIR_CHUNK) vbegin.push_back(b);
  }
  vrc[m0] = (int32_t)vbegin.size();
  const int64_t nch = (int64_t)vbegin.size();
  vbegin.push_back(nv);
  rc = grow(&op->vchunk_begin, &op->vchunk_cap, nch + 1);
  if (rc) return rc;
  if (op->vrbf_cap < m0 + 1) {
    if (op->vrbf_chunk0) DOT_HIP(hipFree(op->vrbf_chunk0));
    op->vrbf_chunk0 = nullptr;
    DOT_HIP(hipMalloc(&op->vrbf_chunk0, (size_t)(m0 + 1) * sizeof(int32_t)));
    op->vrbf_cap = m0 + 1;
  }
  DOT_HIP(hipMemcpyAsync(op->vchunk_begin, vbegin.data(), (size_t)(nch + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  DOT_HIP(hipMemcpyAsync(op->vrbf_chunk0, vrc.data(), (size_t)(m0 + 1) * sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
  DOT_HIP(hipStreamSynchronize(s));
  op->n_vrows = nr;
  op->n_vpairs = nv;
  op->n_vchunks = nch;
  return DOT_OK;
}

// One tile of the contraction: t_s sources (U columns) x t_d detectors (Z
// columns) that the matrix-core kernels hold (see jac_tile_shape), reduced
// into J_s at the tile's place.
static int jac_tile(dot_op* op, const JacParams& P, int precision, int l_s, const double* U_dev,
                    int l_d, const double* Z_dev, double* partial, char* packed, const JacOut& o,
                    double* Js_dev, hipStream_t s) {
  const int na = P.n_act;
  const int m0 = op->pals.m0;
  const int lsld = l_s * l_d;
  const int L = l_s + l_d;
  const int MT = (l_s + 15) / 16, NT = (l_d * na + 15) / 16;
  const int tiles = MT * NT;
  const int JRs = (l_d + 15) / 16;
  if (precision == DOT_JAC_FP64 ? !(tiles <= 64 && L <= 16 * JRMAX) : !(MT <= 4 && JRs <= 4))
    DOT_FAIL(DOT_EINVAL, "internal: contraction tile %d x %d does not fit the kernels", l_s, l_d);
  const JacTables tab = jac_tables(op);
  if (tab.n_chunks > 0 && precision == DOT_JAC_FP64) {
    const dim3 pgrid((unsigned)((tab.n_rows + 63) / 64), (unsigned)((L + 63) / 64));
    if (tab.face)
      hipLaunchKernelGGL((pack_rows_kernel<double, true>), pgrid, dim3(256), 0, s, op->g.N,
                         tab.n_rows, tab.row_cell, tab.row_nbr, tab.row_w, l_s, U_dev, l_d, Z_dev,
                         (double*)packed);
    else
      hipLaunchKernelGGL((pack_rows_kernel<double, false>), pgrid, dim3(256), 0, s, op->g.N,
                         tab.n_rows, tab.row_cell, tab.row_nbr, tab.row_w, l_s, U_dev, l_d, Z_dev,
                         (double*)packed);
    DOT_LAUNCH_CHECK();
    // tiles per wave, and the columns the padded tiles reach
    const int qmax = (tiles + 7) / 8;
    const int ncp = ((8 * qmax - 1) / MT + 1) * 16;
    const size_t shm = jac_lds_bytes(MT * 16, ncp);
    int rc = DOT_EINVAL;
#define DOT_JAC_F64(Q)                                                                           \
  case Q: {                                                                                      \
    auto kern = jac_mfma_kernel<Q>;                                                              \
    DOT_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                                (int)shm));                                                      \
    hipLaunchKernelGGL(kern, dim3((unsigned)tab.n_chunks), dim3(JTHREADS), shm, s, tab.pair_band,   \
                       tab.pair_g, tab.n_pairs, tab.chunk_begin, l_s, l_d, na,                         \
                       (const double*)packed, partial, ncp);                                     \
    DOT_LAUNCH_CHECK();                                                                          \
    rc = DOT_OK;                                                                                 \
  } break;
    switch (qmax) {
      DOT_JAC_F64(1) DOT_JAC_F64(2) DOT_JAC_F64(3) DOT_JAC_F64(4)
      DOT_JAC_F64(5) DOT_JAC_F64(6) DOT_JAC_F64(7) DOT_JAC_F64(8)
    }
#undef DOT_JAC_F64
    if (rc) return rc;
  } else if (tab.n_chunks > 0) {
    const int terms = precision == DOT_JAC_SPLIT_BF16 ? 2 : 3;
    char* pu = packed;
    float* pz = reinterpret_cast<float*>(packed + packed_split_u_bytes(op, l_s));
    const size_t pshm = (size_t)64 * (L + 1) * sizeof(float);
    const unsigned pblocks = (unsigned)((tab.n_rows + 63) / 64);
#define DOT_PACK_SPLIT(TT, FF, W)                                                                \
  hipLaunchKernelGGL((pack_split_kernel<TT, FF>), dim3(pblocks), dim3(256), pshm, s, op->g.N,   \
                     tab.n_rows, tab.row_cell, tab.row_nbr, tab.row_w, l_s, U_dev, l_d, Z_dev, MT * 16, \
                     JRs * 16, reinterpret_cast<W*>(pu), pz)
    if (terms == 2) {
      if (tab.face)
        DOT_PACK_SPLIT(2, true, uint32_t);
      else
        DOT_PACK_SPLIT(2, false, uint32_t);
    } else {
      if (tab.face)
        DOT_PACK_SPLIT(3, true, uint2);
      else
        DOT_PACK_SPLIT(3, false, uint2);
    }
#undef DOT_PACK_SPLIT
    DOT_LAUNCH_CHECK();
    const size_t shm = jac_split_lds_bytes(terms, MT, JRs, na);
    int rc = DOT_EINVAL;
#define DOT_JS_LAUNCH(T, M, J)                                                                   \
  if (terms == T && MT == M && JRs == J) {                                                       \
    auto kern = jac_split_kernel<T, M, J>;                                                       \
    DOT_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                                (int)shm));                                                      \
    hipLaunchKernelGGL(kern, dim3((unsigned)tab.n_chunks), dim3(JS_THREADS), shm, s,              \
                       tab.pair_band, tab.pair_g32, tab.n_pairs, tab.chunk_begin, l_s, l_d, na,          \
                       reinterpret_cast<const typename SplitWord<T>::type*>(pu), pz,             \
                       reinterpret_cast<float*>(partial));                                       \
    DOT_LAUNCH_CHECK();                                                                          \
    rc = DOT_OK;                                                                                 \
  }
#define DOT_JS_MT(T)                                                                             \
  DOT_JS_LAUNCH(T, 1, 1) DOT_JS_LAUNCH(T, 1, 2) DOT_JS_LAUNCH(T, 1, 3) DOT_JS_LAUNCH(T, 1, 4)    \
  DOT_JS_LAUNCH(T, 2, 1) DOT_JS_LAUNCH(T, 2, 2) DOT_JS_LAUNCH(T, 2, 3) DOT_JS_LAUNCH(T, 2, 4)    \
  DOT_JS_LAUNCH(T, 3, 1) DOT_JS_LAUNCH(T, 3, 2) DOT_JS_LAUNCH(T, 3, 3) DOT_JS_LAUNCH(T, 3, 4)    \
  DOT_JS_LAUNCH(T, 4, 1) DOT_JS_LAUNCH(T, 4, 2) DOT_JS_LAUNCH(T, 4, 3) DOT_JS_LAUNCH(T, 4, 4)
    DOT_JS_MT(2)
    DOT_JS_MT(3)
#undef DOT_JS_MT
#undef DOT_JS_LAUNCH
    if (rc) return rc;
  }
  dim3 grid((lsld * na + 255) / 256, m0);
  if (precision != DOT_JAC_FP64 && tab.n_chunks > 0) {
    hipLaunchKernelGGL(jac_reduce_runs_kernel, grid, dim3(256), 0, s, m0, tab.rbf_chunk0,
                       tab.chunk_begin, lsld, na, reinterpret_cast<const float*>(partial), o,
                       Js_dev);
  } else {
    hipLaunchKernelGGL(jac_reduce_kernel, grid, dim3(256), 0, s, m0, tab.rbf_chunk0, lsld, na,
                       partial, o, Js_dev);
  }
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

}  // namespace dot

using namespace dot;

extern "C" {

size_t dot_jacobian_workspace_bytes(const dot_op* op, int l_s, int l_d) {
  if (!op || !op->have_pals || l_s < 1 || l_d < 1) return 0;
  return jac_bytes(op, l_s, l_d);
}

int dot_jacobian(dot_op* op, int l_s, const double* U_dev, int l_d, const double* Z_dev,
                 int precision, double* Js_dev, void* work_dev, size_t work_bytes, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (!op->have_pals) DOT_FAIL(DOT_EINVAL, "dot_pals_mua has not been called on this handle");
  if (l_s < 1 || l_d < 1) DOT_FAIL(DOT_EINVAL, "l_s and l_d must be >= 1");
  if (!U_dev || !Z_dev || !Js_dev) DOT_FAIL(DOT_EINVAL, "NULL argument");
  if (precision != DOT_JAC_FP64 && precision != DOT_JAC_SPLIT_BF16 &&
      precision != DOT_JAC_SPLIT_BF16X3)
    DOT_FAIL(DOT_EINVAL, "precision must be DOT_JAC_FP64, DOT_JAC_SPLIT_BF16 or _BF16X3");
  if (l_s > DOT_MAX_COLUMNS || l_d > DOT_MAX_COLUMNS)
    DOT_FAIL(DOT_EINVAL, "l_s and l_d must be <= %d", DOT_MAX_COLUMNS);
  const size_t need = jac_bytes(op, l_s, l_d);
  if (!work_dev || work_bytes < need)
    DOT_FAIL(DOT_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
  hipStream_t s = as_stream(stream);
  const JacParams P = make_params(op);
  int ts = 0, td = 0;
  jac_tile_shape(precision, l_s, l_d, P.n_act, &ts, &td);
  double* partial = (double*)work_dev;
  char* packed = (char*)work_dev + jac_partial_bytes(op, ts, td);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  unsigned long long* cols = nullptr;
  DOT_TRY_J(profile_begin(op, DOT_PROF_JACOBIAN, s, &e0, &e1, &cols));
  for (int i0 = 0; i0 < l_s; i0 += ts)
    for (int j0 = 0; j0 < l_d; j0 += td) {
      const int ti = std::min(ts, l_s - i0), tj = std::min(td, l_d - j0);
      JacOut o;
      o.tj = tj;
      o.base = j0 + (int64_t)l_d * i0;
      o.ldi = l_d;
      o.ldk = (int64_t)l_s * l_d;
      DOT_TRY_J(jac_tile(op, P, precision, ti, U_dev + op->g.N * (int64_t)i0, tj,
                         Z_dev + op->g.N * (int64_t)j0, partial, packed, o, Js_dev, s));
    }
  return profile_end(op, DOT_PROF_JACOBIAN, s, e0, e1);
}

}  // extern "C"

namespace dot {

static int grad_check_args(const dot_op* op, int l_s, int l_d, const double* U_dev,
                           const double* Z_dev, const double* Rs_dev, const double* g_dev) {
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (!op->have_pals) DOT_FAIL(DOT_EINVAL, "dot_pals_mua has not been called on this handle");
  if (l_s < 1 || l_d < 1) DOT_FAIL(DOT_EINVAL, "l_s and l_d must be >= 1");
  if (!U_dev || !Z_dev || !Rs_dev || !g_dev) DOT_FAIL(DOT_EINVAL, "NULL argument");
  if ((size_t)l_s * l_d * sizeof(double) > 48 * 1024)
    DOT_FAIL(DOT_EINVAL, "l_s * l_d too large for the gradient kernel");
  return DOT_OK;
}

// doubles of gradient scratch: per-cell sums s_c (N, padded to 32), then one
// partial per (chunk, active parameter)
static int64_t grad_scratch_doubles(const dot_op* op) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  return ((op->g.N + 31) / 32) * 32 + std::max<int64_t>(op->n_chunks, 1) * na;
}

// The gradient's launches on scratch memory sc of at least grad_scratch_doubles.
static int grad_run(dot_op* op, int l_s, const double* U_dev, int l_d, const double* Z_dev,
                    const double* Rs_dev, double* g_dev, double* sc, hipStream_t s) {
  const JacParams P = make_params(op);
  const int na = P.n_act;
  const int m0 = op->pals.m0;
  if (op->diff_mode) {
    double* lam = sc;
    double* e = lam + al256((size_t)op->g.N * l_s * sizeof(double)) / sizeof(double);
    double* partial =
        e + al256((size_t)std::max<int64_t>(op->n_vrows, 1) * sizeof(double)) / sizeof(double);
    hipLaunchKernelGGL(lambda_kernel, dim3((unsigned)((op->g.N + 255) / 256)), dim3(256),
                       (size_t)l_s * l_d * sizeof(double), s, op->g.N, l_s, l_d, Z_dev, Rs_dev,
                       lam);
    DOT_LAUNCH_CHECK();
    if (op->n_vrows > 0) {
      hipLaunchKernelGGL(grad_vrow_kernel, dim3((unsigned)((op->n_vrows + 255) / 256)), dim3(256),
                         0, s, op->g.N, op->n_vrows, l_s, op->vrow_cell, op->vrow_nbr, op->vrow_w,
                         U_dev, lam, e);
      DOT_LAUNCH_CHECK();
    }
    if (op->n_vchunks > 0) {
      hipLaunchKernelGGL(grad_chunk_kernel, dim3((unsigned)op->n_vchunks), dim3(256), 0, s, na,
                         op->vpair_band, op->vpair_g, op->vchunk_begin, e, partial);
      DOT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((m0 * na + 255) / 256), dim3(256), 0, s, m0,
                       op->vrbf_chunk0, na, partial, g_dev);
    DOT_LAUNCH_CHECK();
    return DOT_OK;
  }
  double* partial = sc + ((op->g.N + 31) / 32) * 32;
  if (l_s <= 32)
    hipLaunchKernelGGL(grad_cell_small_kernel<32>, dim3((unsigned)((op->g.N + 255) / 256)), dim3(256),
                       (size_t)l_s * l_d * sizeof(double), s, op->g, P, op->phi, l_s, U_dev, l_d,
                       Z_dev, Rs_dev, sc);
  else
    hipLaunchKernelGGL(grad_cell_kernel, dim3((unsigned)((op->g.N + 255) / 256)), dim3(256),
                       (size_t)l_s * l_d * sizeof(double), s, op->g, P, op->phi, l_s, U_dev, l_d,
                       Z_dev, Rs_dev, sc);
  DOT_LAUNCH_CHECK();
  if (op->n_chunks > 0) {
    hipLaunchKernelGGL(grad_chunk_kernel, dim3((unsigned)op->n_chunks), dim3(256), 0, s, na,
                       op->pair_cell, op->pair_g, op->chunk_begin, sc, partial);
    DOT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((m0 * na + 255) / 256), dim3(256), 0, s, m0,
                     op->rbf_chunk0, na, partial, g_dev);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

// Fixed scratch of dot_grad_misfit_noalloc, one copy per GPU for the life of
// the process.  In host code `scratch` names a host-side stand-in; kernels
// get the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device and kept in scratch_dev.
static __device__ __align__(256) double scratch[DOT_NOALLOC_SCRATCH_DOUBLES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static double* scratch_dev[SCRATCH_MAX_DEVICES];
static std::mutex scratch_mu;

static int scratch_address(double** out) {
  int dev = -1;
  DOT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    DOT_FAIL(DOT_EINVAL, "device %d beyond the %d devices the fixed scratch supports", dev,
             SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      DOT_FAIL(DOT_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
               hipGetErrorString(e));
    scratch_dev[dev] = (double*)p;
  }
  *out = scratch_dev[dev];
  return DOT_OK;
}

}  // namespace dot

extern "C" {

int dot_dadp_apply(dot_op* op, int k, const double* Theta_dev, const double* X_dev, double* Y_dev,
                 void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (!op->have_pals) DOT_FAIL(DOT_EINVAL, "dot_pals_mua has not been called on this handle");
  if (k < 1 || k > DOT_MAX_COLUMNS) DOT_FAIL(DOT_EINVAL, "k must be in [1, %d]", DOT_MAX_COLUMNS);
  if (!Theta_dev || !X_dev || !Y_dev) DOT_FAIL(DOT_EINVAL, "NULL argument");
  if (X_dev == Y_dev) DOT_FAIL(DOT_EINVAL, "X_dev and Y_dev must not overlap");
  if (op->diff_mode)
    DOT_FAIL(DOT_EINVAL, "dot_dadp_apply covers the absorption-only model (dot_pals_mua)");
  const JacParams P = make_params(op);
  const int n_p = op->pals.m0 * P.n_act;
  const GridDims& g = op->g;
  int64_t tiles;
  if (g.dim == 3)
    tiles = (int64_t)((g.nx + 7) / 8) * ((g.ny + 7) / 8) * ((g.nz + 3) / 4);
  else
    tiles = (int64_t)((g.nx + 15) / 16) * ((g.ny + 15) / 16);
  hipLaunchKernelGGL(dA_dir_kernel, dim3((unsigned)tiles), dim3(256), 0, as_stream(stream), g, P,
                     op->theta, op->phi, op->pals.m0, k, Theta_dev, n_p, X_dev, Y_dev);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

int dot_grad_misfit(dot_op* op, int l_s, const double* U_dev, int l_d, const double* Z_dev,
                    const double* Rs_dev, double* g_dev, void* work_dev, size_t work_bytes,
                    void* stream) {
  clear_error();
  DOT_TRY_J(grad_check_args(op, l_s, l_d, U_dev, Z_dev, Rs_dev, g_dev));
  const size_t need = jac_bytes(op, l_s, l_d);
  if (!work_dev || work_bytes < need)
    DOT_FAIL(DOT_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
  return grad_run(op, l_s, U_dev, l_d, Z_dev, Rs_dev, g_dev, (double*)work_dev,
                  as_stream(stream));
}

int dot_grad_misfit_noalloc(dot_op* op, int l_s, const double* U_dev, int l_d,
                            const double* Z_dev, const double* Rs_dev, double* g_dev,
                            void* stream) {
  clear_error();
  DOT_TRY_J(grad_check_args(op, l_s, l_d, U_dev, Z_dev, Rs_dev, g_dev));
  if (op->diff_mode)
    DOT_FAIL(DOT_EINVAL, "the fixed-scratch gradient covers the absorption-only model "
                         "(dot_pals_mua), not diffusion mode");
  const int64_t need = grad_scratch_doubles(op);
  if (need > (int64_t)DOT_NOALLOC_SCRATCH_DOUBLES)
    DOT_FAIL(DOT_EINVAL,
             "grid too large for the fixed gradient scratch: needs %lld doubles (N = %lld cells "
             "plus %lld chunk partials), the maximum is %lld",
             (long long)need, (long long)op->g.N, (long long)(need - ((op->g.N + 31) / 32) * 32),
             (long long)DOT_NOALLOC_SCRATCH_DOUBLES);
  double* sc = nullptr;
  DOT_TRY_J(scratch_address(&sc));
  return grad_run(op, l_s, U_dev, l_d, Z_dev, Rs_dev, g_dev, sc, as_stream(stream));
}

}  // extern "C"
