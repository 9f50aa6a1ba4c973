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

constexpr int JB = 32;     // cells staged per batch
constexpr int JOUT = 32;   // outputs per thread per output pass
constexpr int JT = 256;    // threads

// Partial contraction of one chunk, binary64.  Output element e of the
// chunk's block is (i, j, a) with e = (j + l_d i) + l_s l_d a.
__global__ __launch_bounds__(JT) void jac_chunk_fp64_kernel(
    GridDims g, JacParams P, const double* __restrict__ theta, const double* __restrict__ phi,
    const int32_t* __restrict__ pair_cell, const int64_t* __restrict__ chunk_begin,
    const int32_t* __restrict__ chunk_rbf, int l_s, const double* __restrict__ U, int l_d,
    const double* __restrict__ Z, double* __restrict__ partial) {
  extern __shared__ double smem[];
  const int ch = blockIdx.x;
  const int64_t b0 = chunk_begin[ch], b1 = chunk_begin[ch + 1];
  const int m = chunk_rbf[ch];
  const double* th = theta + (int64_t)m * P.stride;
  const int na = P.n_act;
  double* Us = smem;                   // [JB][l_s]
  double* Zs = Us + JB * l_s;          // [JB][l_d]
  double* Gs = Zs + JB * l_d;          // [JB][na]
  const int nout = l_s * l_d * na;
  const int lsld = l_s * l_d;
  double* out = partial + (int64_t)ch * nout;
  for (int ob = 0; ob < nout; ob += JT * JOUT) {
    double acc[JOUT];
#pragma unroll
    for (int q = 0; q < JOUT; ++q) acc[q] = 0.0;
    for (int64_t cb = b0; cb < b1; cb += JB) {
      const int nb = (int)min<int64_t>(JB, b1 - cb);
      __syncthreads();
      for (int t = threadIdx.x; t < nb * l_s; t += JT) {
        const int cc = t % nb, i = t / nb;
        Us[cc * l_s + i] = U[pair_cell[cb + cc] + P.N * i];
      }
      for (int t = threadIdx.x; t < nb * l_d; t += JT) {
        const int cc = t % nb, j = t / nb;
        Zs[cc * l_d + j] = Z[pair_cell[cb + cc] + P.N * j];
      }
      if (threadIdx.x < nb) {
        const int64_t c = pair_cell[cb + threadIdx.x];
        double x0, x1, x2, d[5];
        cell_xyz(g, c, &x0, &x1, &x2);
        rbf_dphi(P, th, x0, x1, x2, d);
        const double w = band_weight(P, phi[c]);
        for (int a = 0; a < na; ++a) Gs[threadIdx.x * na + a] = P.hd * (w * d[a]);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < JOUT; ++q) {
        const int e = ob + q * JT + threadIdx.x;
        if (e < nout) {
          const int a = e / lsld, rem = e % lsld;
          const int j = rem % l_d, i = rem / l_d;
          double s = acc[q];
          for (int cc = 0; cc < nb; ++cc) s += Us[cc * l_s + i] * Zs[cc * l_d + j] * Gs[cc * na + a];
          acc[q] = s;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < JOUT; ++q) {
      const int e = ob + q * JT + threadIdx.x;
      if (e < nout) out[e] = acc[q];
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
  const int m = blockIdx.x;
  const double* th = theta + (int64_t)m * P.stride;
  const int na = P.n_act;
  for (int64_t p = rbf_start[m] + threadIdx.x; p < rbf_start[m + 1]; p += 256) {
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

// Packed rows: packed[b * L + i] = U[c_b, i] (i < l_s) or Z[c_b, i - l_s],
// L = l_s + l_d, through a 64-row x 64-column LDS tile so that both the
// column reads and the row writes are contiguous.
template <typename T>
__global__ __launch_bounds__(256) void pack_rows_kernel(int64_t N, int64_t n_band,
                                                        const int32_t* __restrict__ band_cells,
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
#pragma unroll 4
  for (int r = 0; r < 16; ++r) {
    const int il = (t >> 6) + 4 * r;
    const int i = i0 + il;
    T v = T(0);
    if (b < n_band && i < L) v = (T)(i < l_s ? U[c + N * (int64_t)i] : Z[c + N * (int64_t)(i - l_s)]);
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

template <int TERMS>
__global__ __launch_bounds__(256) void pack_split_kernel(int64_t N, int64_t n_band,
                                                         const int32_t* __restrict__ band_cells,
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

// Js[(j + l_d i) + l_s l_d (m na + a)] = - sum over the chunks of RBF m and
// their runs of JFLUSH K-steps (binary32 blocks), in order, in binary64.
__global__ void jac_reduce_runs_kernel(int m0, const int32_t* __restrict__ rbf_chunk0,
                                       const int64_t* __restrict__ chunk_begin, int lsld, int na,
                                       const float* __restrict__ partial, double* __restrict__ Js) {
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
  Js[row + (int64_t)lsld * (m * na + a)] = -s;
}

// Js[(j + l_d i) + l_s l_d (m na + a)] = - sum over chunks of RBF m.
__global__ void jac_reduce_kernel(int m0, const int32_t* __restrict__ rbf_chunk0, int lsld, int na,
                                  const double* __restrict__ partial, double* __restrict__ Js) {
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
  Js[row + (int64_t)lsld * (m * na + a)] = -s;
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
static size_t jac_partial_bytes(const dot_op* op, int l_s, int l_d) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  return al256((size_t)std::max<int64_t>(op->n_chunks, 1) * l_s * l_d * na *
               std::max(sizeof(double), JSPC * sizeof(float)));
}

// packed band rows: binary64 rows of l_s + l_d values, or for the split
// forms the split words of U (at most 8 bytes, l_s rounded up to 16 per row)
// followed by binary32 rows of Z (l_d rounded up to 16)
static size_t packed_split_u_bytes(const dot_op* op, int l_s) {
  return al256((size_t)std::max<int64_t>(op->n_band, 1) * ((l_s + 15) / 16) * 16 * 8);
}

static size_t jac_bytes(const dot_op* op, int l_s, int l_d) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  const size_t nb = (size_t)std::max<int64_t>(op->n_band, 1);
  const size_t packed = std::max(al256(nb * (l_s + l_d) * sizeof(double)),
                                 packed_split_u_bytes(op, l_s) +
                                     al256(nb * ((l_d + 15) / 16) * 16 * sizeof(float)));
  const size_t jac = jac_partial_bytes(op, l_s, l_d) + packed;
  const size_t grad = (size_t)op->g.N * sizeof(double) +
                      (size_t)std::max<int64_t>(op->n_chunks, 1) * na * sizeof(double) + 256;
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
    hipLaunchKernelGGL(pair_g_kernel, dim3(m0), dim3(256), 0, s, op->g, P, op->theta, op->phi,
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
  int64_t n_band = 0;
  DOT_HIP(hipMemcpyAsync(&n_band, op->band_part + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  rc = grow(&op->band_cells, &op->band_cap, std::max<int64_t>(n_band, 1));
  if (rc) return rc;
  hipLaunchKernelGGL(band_fill_kernel, dim3((unsigned)nb), dim3(256), 0, s, N, op->band_part,
                     op->band_idx, op->band_cells);
  DOT_LAUNCH_CHECK();
  if (np > 0) {
    hipLaunchKernelGGL(pair_band_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np,
                       op->pair_cell, op->band_idx, op->pair_band);
    DOT_LAUNCH_CHECK();
  }
  op->n_band = n_band;
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
  if (l_s > 1024) DOT_FAIL(DOT_EINVAL, "l_s must be <= 1024");
  const size_t need = jac_bytes(op, l_s, l_d);
  if (!work_dev || work_bytes < need)
    DOT_FAIL(DOT_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
  hipStream_t s = as_stream(stream);
  const JacParams P = make_params(op);
  const int na = P.n_act;
  const int m0 = op->pals.m0;
  const int lsld = l_s * l_d;
  const int L = l_s + l_d;
  const int MT = (l_s + 15) / 16, NT = (l_d * na + 15) / 16;
  const int tiles = MT * NT;
  // binary64: at most 8 tiles per wave and JRMAX staged values per thread,
  // beyond that the plain kernel.  Split forms: l_s <= 64 and l_d <= 64.
  const int JRs = (l_d + 15) / 16;
  const bool mfma_fits = precision == DOT_JAC_FP64 ? tiles <= 64 && L <= 16 * JRMAX
                                                   : MT <= 4 && JRs <= 4;
  if (precision != DOT_JAC_FP64 && !mfma_fits)
    DOT_FAIL(DOT_EINVAL, "l_s, l_d and n_act too large for the split-bf16 kernel");
  if (precision == DOT_JAC_FP64 && !mfma_fits &&
      (size_t)JB * (l_s + l_d + 5) * sizeof(double) > 64 * 1024)
    DOT_FAIL(DOT_EINVAL, "l_s + l_d too large for the contraction kernel");
  double* partial = (double*)work_dev;
  char* packed = (char*)work_dev + jac_partial_bytes(op, l_s, l_d);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  unsigned long long* cols = nullptr;
  DOT_TRY_J(profile_begin(op, DOT_PROF_JACOBIAN, s, &e0, &e1, &cols));
  if (op->n_chunks > 0 && !mfma_fits) {
    const size_t shm = (size_t)JB * (l_s + l_d + na) * sizeof(double);
    hipLaunchKernelGGL(jac_chunk_fp64_kernel, dim3((unsigned)op->n_chunks), dim3(JT), shm, s, op->g,
                       P, op->theta, op->phi, op->pair_cell, op->chunk_begin, op->chunk_rbf, l_s,
                       U_dev, l_d, Z_dev, partial);
    DOT_LAUNCH_CHECK();
  } else if (op->n_chunks > 0 && precision == DOT_JAC_FP64) {
    const dim3 pgrid((unsigned)((op->n_band + 63) / 64), (unsigned)((L + 63) / 64));
    hipLaunchKernelGGL(pack_rows_kernel<double>, pgrid, dim3(256), 0, s, op->g.N, op->n_band,
                       op->band_cells, l_s, U_dev, l_d, Z_dev, (double*)packed);
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
    hipLaunchKernelGGL(kern, dim3((unsigned)op->n_chunks), dim3(JTHREADS), shm, s, op->pair_band, \
                       op->pair_g, op->n_pairs, op->chunk_begin, l_s, l_d, na,                   \
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
  } else if (op->n_chunks > 0) {
    const int terms = precision == DOT_JAC_SPLIT_BF16 ? 2 : 3;
    char* pu = packed;
    float* pz = reinterpret_cast<float*>(packed + packed_split_u_bytes(op, l_s));
    const size_t pshm = (size_t)64 * (L + 1) * sizeof(float);
    const unsigned pblocks = (unsigned)((op->n_band + 63) / 64);
    if (terms == 2) {
      hipLaunchKernelGGL(pack_split_kernel<2>, dim3(pblocks), dim3(256), pshm, s, op->g.N,
                         op->n_band, op->band_cells, l_s, U_dev, l_d, Z_dev, MT * 16, JRs * 16,
                         reinterpret_cast<uint32_t*>(pu), pz);
    } else {
      hipLaunchKernelGGL(pack_split_kernel<3>, dim3(pblocks), dim3(256), pshm, s, op->g.N,
                         op->n_band, op->band_cells, l_s, U_dev, l_d, Z_dev, MT * 16, JRs * 16,
                         reinterpret_cast<uint2*>(pu), pz);
    }
    DOT_LAUNCH_CHECK();
    const size_t shm = jac_split_lds_bytes(terms, MT, JRs, na);
    int rc = DOT_EINVAL;
#define DOT_JS_LAUNCH(T, M, J)                                                                   \
  if (terms == T && MT == M && JRs == J) {                                                       \
    auto kern = jac_split_kernel<T, M, J>;                                                       \
    DOT_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,   \
                                (int)shm));                                                      \
    hipLaunchKernelGGL(kern, dim3((unsigned)op->n_chunks), dim3(JS_THREADS), shm, s,             \
                       op->pair_band, op->pair_g32, op->n_pairs, op->chunk_begin, l_s, l_d, na,  \
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
  if (precision != DOT_JAC_FP64 && op->n_chunks > 0) {
    hipLaunchKernelGGL(jac_reduce_runs_kernel, grid, dim3(256), 0, s, m0, op->rbf_chunk0,
                       op->chunk_begin, lsld, na, reinterpret_cast<const float*>(partial), Js_dev);
  } else {
    hipLaunchKernelGGL(jac_reduce_kernel, grid, dim3(256), 0, s, m0, op->rbf_chunk0, lsld, na,
                       partial, Js_dev);
  }
  DOT_LAUNCH_CHECK();
  return profile_end(op, DOT_PROF_JACOBIAN, s, e0, e1);
}

int dot_grad_misfit(dot_op* op, int l_s, const double* U_dev, int l_d, const double* Z_dev,
                    const double* Rs_dev, double* g_dev, void* work_dev, size_t work_bytes,
                    void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (!op->have_pals) DOT_FAIL(DOT_EINVAL, "dot_pals_mua has not been called on this handle");
  if (l_s < 1 || l_d < 1) DOT_FAIL(DOT_EINVAL, "l_s and l_d must be >= 1");
  if (!U_dev || !Z_dev || !Rs_dev || !g_dev) DOT_FAIL(DOT_EINVAL, "NULL argument");
  if ((size_t)l_s * l_d * sizeof(double) > 48 * 1024)
    DOT_FAIL(DOT_EINVAL, "l_s * l_d too large for the gradient kernel");
  const size_t need = jac_bytes(op, l_s, l_d);
  if (!work_dev || work_bytes < need)
    DOT_FAIL(DOT_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
  hipStream_t s = as_stream(stream);
  const JacParams P = make_params(op);
  const int na = P.n_act;
  const int m0 = op->pals.m0;
  double* sc = (double*)work_dev;
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

}  // extern "C"
