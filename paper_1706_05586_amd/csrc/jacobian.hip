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
                                                     double* __restrict__ pair_g) {
  const int m = blockIdx.x;
  const double* th = theta + (int64_t)m * P.stride;
  const int na = P.n_act;
  for (int64_t p = rbf_start[m] + threadIdx.x; p < rbf_start[m + 1]; p += 256) {
    const int64_t c = pair_cell[p];
    double x0, x1, x2, d[5];
    cell_xyz(g, c, &x0, &x1, &x2);
    rbf_dphi(P, th, x0, x1, x2, d);
    const double w = band_weight(P, phi[c]);
    for (int a = 0; a < na; ++a) pair_g[p * na + a] = P.hd * (w * d[a]);
  }
}

__global__ void fill_double_kernel(double* __restrict__ a, int n, double v) {
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
// Matrix-core contraction of one chunk (the pairs of one RBF, or a piece of
// them).  Per chunk it is a dense product
//     P[i, n] = sum_p U[c_p, i] B[p, n],  B[p, j + l_d a] = Z[c_p, j] G[p, a],
// i < l_s, n < l_d na, over the chunk's pairs in K-steps of 32.  A thread
// stages the values i = t % 16 + 16 r of pair t / 16 of a step from its packed
// row (one contiguous row per pair) into LDS: U as the A operand, Z times the
// pair's G as the B operand.  The next step's rows are loaded while the
// matrix cores work on the current one (band rows two steps ahead).
// MODE 0: binary64 operands, v_mfma_f64_16x16x4f64, binary64 accumulation.
// MODE 2 / 3: operands rounded to binary32 and split into 2 / 3 bfloat16
// parts (x = hi + lo, or hi + mid + lo); the part products of total order at
// most MODE - 1 are issued as v_mfma_f32_16x16x32_bf16 (3 products for two
// parts, 6 for three), accumulated in binary32 and flushed into the binary64
// partial block every JFLUSH K-steps (512 pairs).
// Output tiles of 16 x 16 are dealt to the 8 waves round-robin: tile
// t = wave + 8 q covers rows 16 (t % MT) .. +15 and columns 16 (t / MT) .. +15,
// zero-padded beyond l_s rows and l_d na columns.  Lane layout of both
// instructions: A row l % 16, B column l % 16, k in groups by l / 16; result
// column l % 16, rows 4 (l / 16) + e for the bfloat16 form and l / 16 + 4 e
// for the binary64 form (e < 4).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int JK = 32;            // pairs per K-step
constexpr int JKP32 = JK + 4;     // padded binary32 LDS row (144 bytes)
constexpr int JKP64 = JK + 1;     // padded binary64 LDS row
constexpr int JTHREADS = 512;     // 8 waves; 16 threads per pair of a step
constexpr int JRMAX = 8;          // values per thread and step: l_s + l_d <= 128
constexpr int JFLUSH = 16;        // K-steps between binary64 flushes

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

template <int MODE>
struct JacPack {
  using type = float;
};
template <>
struct JacPack<0> {
  using type = double;
};

// A rows, B columns, and one discard row for the stores of lanes that hold
// no operand value (their stores are unconditional)
__host__ __device__ inline size_t jac_lds_bytes(int mode, int rows, int ncp) {
  return mode == 0 ? (size_t)(rows + ncp + 1) * JKP64 * sizeof(double)
                   : (size_t)(rows + ncp + 1) * JKP32 * sizeof(float);
}

// MTC: the row-tile count ceil(l_s / 16) as a constant (split forms), or 0
// (binary64, which takes it at run time)
template <int MODE, int QMAX, int MTC>
__global__ __launch_bounds__(JTHREADS) void jac_mfma_kernel(
    const int32_t* __restrict__ pair_band, const double* __restrict__ pair_g, int64_t n_pairs,
    const int64_t* __restrict__ chunk_begin, int l_s, int l_d, int na,
    const typename JacPack<MODE>::type* __restrict__ packed, double* __restrict__ partial,
    int ncp) {
  using PT = typename JacPack<MODE>::type;
  constexpr int TERMS = MODE == 0 ? 1 : MODE;
  extern __shared__ __attribute__((aligned(16))) unsigned char jsm[];
  const int ch = blockIdx.x;
  const int64_t b0 = chunk_begin[ch], b1 = chunk_begin[ch + 1];
  const int L = l_s + l_d;
  const int lsld = l_s * l_d;
  const int ncol = l_d * na;
  const int MT = MTC > 0 ? MTC : (l_s + 15) / 16;
  const int rows = MT * 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* out = partial + (int64_t)ch * lsld * na;
  float* fA = reinterpret_cast<float*>(jsm);     // [rows][JKP32]
  float* fB = fA + rows * JKP32;                 // [ncp][JKP32]
  double* dA = reinterpret_cast<double*>(jsm);   // [rows][JKP64]
  double* dB = dA + rows * JKP64;                // [ncp][JKP64]
  {  // rows >= l_s and columns >= ncol are never written: clear once
    const int words = (int)(jac_lds_bytes(MODE, rows, ncp) / 4);
    for (int e = threadIdx.x; e < words; e += JTHREADS) reinterpret_cast<int*>(jsm)[e] = 0;
  }

  // per tile: operand rows/columns of this lane and the output offset.
  // Binary64: tiles t = wave + 8 q round-robin.  Split bfloat16: wave w owns
  // the column tiles nt = w + 8 c (c < QMAX / MT) with every row tile mt,
  // tile q = c MT + mt, so a wave splits each A fragment once per K-step and
  // each B fragment once (the splitting, not the matrix cores, bounds that
  // form).
  int arow[QMAX], bcol[QMAX], ooff[QMAX], orow[QMAX], ocol[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    int mt, nt;
    if constexpr (MODE == 0) {
      const int t = wave + 8 * q;
      mt = t % MT;
      nt = t / MT;
    } else {
      mt = q % MT;
      nt = wave + 8 * (q / MT);
    }
    arow[q] = mt * 16 + (lane & 15);
    bcol[q] = nt * 16 + (lane & 15);
    // result element e of this lane: row i0 + rstep e (binary32 form: rows
    // 4 (l / 16) + e; binary64 form: rows l / 16 + 4 e), column bcol
    const int i0 = MODE == 0 ? mt * 16 + (lane >> 4) : mt * 16 + 4 * (lane >> 4);
    const int n = bcol[q];
    orow[q] = i0;
    ocol[q] = n;
    ooff[q] = n < ncol ? (n % l_d) + l_d * i0 + lsld * (n / l_d) : 0;
  }
  constexpr int rstep = MODE == 0 ? 4 : 1;
  f32x4 acc[QMAX];
  f64x4 acc64[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    acc64[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  bool first = true;
  auto flush = [&]() {
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (orow[q] + e < l_s && ocol[q] < ncol) {
          double* o = out + ooff[q] + l_d * e;
          *o = first ? (double)acc[q][e] : *o + (double)acc[q][e];
        }
      }
      acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    first = false;
  };

  // staging: thread t holds values i = qv + 16 r of pair pb of a step, in two
  // register slots: the rows of step s + 2 are loaded while step s is staged
  // and multiplied, so a load has two steps to arrive
  const int pb = threadIdx.x >> 4, qv = threadIdx.x & 15;
  const int nr = (L + 15) / 16;
  // G in binary32 for the split forms: it only scales the binary32 B operand
  using GT = typename std::conditional<MODE == 0, double, float>::type;
  PT val[2][JRMAX];
  GT gv[2][5];
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
    const PT* row = packed + (int64_t)(valid ? bi : 0) * L;
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
      gv[S][a] = (GT)gp[a];
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
      if constexpr (MODE == 0) {
        dA[arow_s * JKP64 + pb] = val[S][r];
      } else {
        fA[arow_s * JKP32 + pb] = val[S][r];
      }
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        if (a >= na) break;
        const int n = isB ? rows + j + l_d * a : discard;   // row of B within the LDS block
        if constexpr (MODE == 0) {
          dA[n * JKP64 + pb] = val[S][r] * gv[S][a];
        } else {
          fA[n * JKP32 + pb] = val[S][r] * gv[S][a];
        }
      }
    }
  };
  auto multiply = [&]() {
    if constexpr (MODE == 0) {
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
    } else {
      // binary32 operands staged in LDS, split into bfloat16 parts while the
      // fragments are built (8 consecutive k per lane): the MT row fragments
      // once, then per owned column tile its fragment and MT products
      const int kofs = 8 * (lane >> 4);
      auto build = [&](const float* src, bf16x8* f) {
        const float4* p4 = reinterpret_cast<const float4*>(src);
        const float4 x0 = p4[0], x1 = p4[1];
        const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 xp[TERMS];
          split_bf16<TERMS>(xv[e], xp);
#pragma unroll
          for (int p = 0; p < TERMS; ++p) f[p][e] = xp[p];
        }
      };
      constexpr int MTS = MTC > 0 ? MTC : 1;
      bf16x8 fa[MTS][TERMS];
#pragma unroll
      for (int mt = 0; mt < MTS; ++mt) build(&fA[(mt * 16 + (lane & 15)) * JKP32 + kofs], fa[mt]);
      bf16x8 fbc[TERMS];
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int mt = q % MTS;
        if (mt == 0) build(&fB[(wave + 8 * (q / MTS)) * 16 * JKP32 + (lane & 15) * JKP32 + kofs], fbc);
#pragma unroll
        for (int pa = 0; pa < TERMS; ++pa)
#pragma unroll
          for (int pq = 0; pq < TERMS; ++pq)
            if (pa + pq <= TERMS - 1)
              acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[mt][pa], fbc[pq], acc[q], 0, 0, 0);
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
  int kstep = 0;
  // one K-step from register slot S: stage, multiply, refill the slot with
  // the rows of the step two ahead
  auto step = [&](auto slot_c, int64_t base) {
    const int bnext = band_row(base + 4 * JK);   // used four steps on
    store_step(slot_c);
    __syncthreads();
    if (base + 2 * JK < b1) load_step(slot_c, base + 2 * JK, biA);
    multiply();
    if constexpr (MODE != 0) {
      if ((kstep + 1) % JFLUSH == 0) flush();
    }
    __syncthreads();  // operand reads done before the next store
    biA = biB;
    biB = bnext;
    ++kstep;
  };
  for (int64_t base = b0; base < b1; base += 2 * JK) {
    step(S0{}, base);
    if (base + JK < b1) step(S1{}, base + JK);
  }
  if constexpr (MODE == 0) {
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (orow[q] + rstep * e < l_s && ocol[q] < ncol) out[ooff[q] + l_d * rstep * e] = acc64[q][e];
    }
  } else {
    if (first || kstep % JFLUSH != 0) flush();
  }
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
  for (int ch = c0; ch < c1; ++ch) s += partial[(int64_t)ch * nout + e];
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
static size_t jac_partial_bytes(const dot_op* op, int l_s, int l_d) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  return al256((size_t)std::max<int64_t>(op->n_chunks, 1) * l_s * l_d * na * sizeof(double));
}

static size_t jac_bytes(const dot_op* op, int l_s, int l_d) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  const size_t jac = jac_partial_bytes(op, l_s, l_d) +
                     al256((size_t)std::max<int64_t>(op->n_band, 1) * (l_s + l_d) * sizeof(double));
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
  rc = grow(&op->pair_band, &op->pair_band_cap, std::max<int64_t>(np, 1));
  if (rc) return rc;
  if (!op->band_idx) DOT_HIP(hipMalloc(&op->band_idx, (size_t)N * sizeof(int32_t)));
  const int64_t nb = (N + BAND_BLK - 1) / BAND_BLK;
  rc = grow(&op->band_part, &op->band_part_cap, 2 * (nb + 1));
  if (rc) return rc;
  int64_t* cnt = op->band_part + (nb + 1);
  if (np > 0) {
    hipLaunchKernelGGL(pair_g_kernel, dim3(m0), dim3(256), 0, s, op->g, P, op->theta, op->phi,
                       op->rbf_start, op->pair_cell, op->pair_g);
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
  // the matrix-core kernels hold at most 8 tiles per wave and JRMAX staged
  // values per thread (the split form: every row tile of its column tiles,
  // MT <= 4); binary64 beyond that runs the plain kernel
  const int qn_split = (NT + 7) / 8;
  const bool mfma_fits = precision == DOT_JAC_FP64
                             ? tiles <= 64 && L <= 16 * JRMAX
                             : MT <= 4 && MT * qn_split <= 8 && L <= 16 * JRMAX;
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
  } else if (op->n_chunks > 0) {
    const int mode = precision == DOT_JAC_FP64 ? 0 : precision == DOT_JAC_SPLIT_BF16 ? 2 : 3;
    const dim3 pgrid((unsigned)((op->n_band + 63) / 64), (unsigned)((L + 63) / 64));
    if (mode == 0) {
      hipLaunchKernelGGL(pack_rows_kernel<double>, pgrid, dim3(256), 0, s, op->g.N, op->n_band,
                         op->band_cells, l_s, U_dev, l_d, Z_dev, (double*)packed);
    } else {
      hipLaunchKernelGGL(pack_rows_kernel<float>, pgrid, dim3(256), 0, s, op->g.N, op->n_band,
                         op->band_cells, l_s, U_dev, l_d, Z_dev, (float*)packed);
    }
    DOT_LAUNCH_CHECK();
    // tiles per wave, and the columns the padded tiles reach
    const int qmax = mode == 0 ? (tiles + 7) / 8 : MT * qn_split;
    const int ncp = mode == 0 ? ((8 * qmax - 1) / MT + 1) * 16 : 8 * qn_split * 16;
    const size_t shm = jac_lds_bytes(mode, MT * 16, ncp);
    int rc = DOT_EINVAL;
#define DOT_JAC_LAUNCH(M, Q, MTV)                                                              \
  {                                                                                            \
    auto kern = jac_mfma_kernel<M, Q, MTV>;                                                    \
    DOT_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                (int)shm));                                                    \
    hipLaunchKernelGGL(kern, dim3((unsigned)op->n_chunks), dim3(JTHREADS), shm, s,             \
                       op->pair_band, op->pair_g, op->n_pairs, op->chunk_begin, l_s, l_d, na,  \
                       reinterpret_cast<const typename JacPack<M>::type*>(packed), partial,    \
                       ncp);                                                                   \
    DOT_LAUNCH_CHECK();                                                                        \
    rc = DOT_OK;                                                                               \
  }
#define DOT_JAC_F64(Q) \
  case Q:              \
    DOT_JAC_LAUNCH(0, Q, 0) break;
// split forms: qmax = MT * QN, dispatched on (MT, QN)
#define DOT_JAC_SPLIT(M, MTV, QNV)       \
  if (MT == MTV && qn_split == QNV) {    \
    DOT_JAC_LAUNCH(M, (MTV) * (QNV), MTV) \
  }
#define DOT_JAC_SPLIT_ALL(M)                                                                     \
  DOT_JAC_SPLIT(M, 1, 1) DOT_JAC_SPLIT(M, 1, 2) DOT_JAC_SPLIT(M, 1, 3) DOT_JAC_SPLIT(M, 1, 4)    \
  DOT_JAC_SPLIT(M, 1, 5) DOT_JAC_SPLIT(M, 1, 6) DOT_JAC_SPLIT(M, 1, 7) DOT_JAC_SPLIT(M, 1, 8)    \
  DOT_JAC_SPLIT(M, 2, 1) DOT_JAC_SPLIT(M, 2, 2) DOT_JAC_SPLIT(M, 2, 3) DOT_JAC_SPLIT(M, 2, 4)    \
  DOT_JAC_SPLIT(M, 3, 1) DOT_JAC_SPLIT(M, 3, 2) DOT_JAC_SPLIT(M, 4, 1) DOT_JAC_SPLIT(M, 4, 2)
    if (mode == 0) {
      switch (qmax) {
        DOT_JAC_F64(1) DOT_JAC_F64(2) DOT_JAC_F64(3) DOT_JAC_F64(4)
        DOT_JAC_F64(5) DOT_JAC_F64(6) DOT_JAC_F64(7) DOT_JAC_F64(8)
      }
    } else if (mode == 2) {
      DOT_JAC_SPLIT_ALL(2)
    } else {
      DOT_JAC_SPLIT_ALL(3)
    }
#undef DOT_JAC_SPLIT_ALL
#undef DOT_JAC_SPLIT
#undef DOT_JAC_F64
#undef DOT_JAC_LAUNCH
    if (rc) return rc;
  }
  dim3 grid((lsld * na + 255) / 256, m0);
  hipLaunchKernelGGL(jac_reduce_kernel, grid, dim3(256), 0, s, m0, op->rbf_chunk0, lsld, na,
                     partial, Js_dev);
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
