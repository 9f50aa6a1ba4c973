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
// Split-bfloat16 MFMA contraction of one chunk.
//
// Per chunk the contraction is a dense GEMM:  P[i, n] = sum_c U[c,i] B[c,n],
// B[c, j + l_d a] = Z[c,j] G[c,a],  i < l_s, n < l_d na, c over the chunk.
// Operands are rounded to binary32 and split into TERMS bfloat16 parts
// (x = hi + lo, or hi + mid + lo); the part products of total order at most
// TERMS - 1 are issued as v_mfma_f32_16x16x32_bf16 (3 products for two parts,
// 6 for three; the dropped ones are below the representation error), accumulated in binary32 inside the MFMA and flushed
// into binary64 registers every JFLUSH K-steps of 32 cells.  Block = 8
// waves; output tiles of 16 x 16 are dealt round-robin to the waves.
// Operand layout of the instruction (lane l): A row l%16 with 8 consecutive
// k, B column l%16 with the same 8 k, result rows 4(l/16)..+3, column l%16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MK = 32;          // cells per MFMA K-step
constexpr int MKP = MK + 8;     // padded LDS row (bf16 elements), 80 bytes
constexpr int MT_THREADS = 512;
constexpr int JFLUSH = 8;       // K-steps between binary64 flushes (256 cells)

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

template <int TERMS, int QMAX>
__global__ __launch_bounds__(MT_THREADS) void jac_chunk_mfma_kernel(
    GridDims g, JacParams P, const double* __restrict__ theta, const double* __restrict__ phi,
    const int32_t* __restrict__ pair_cell, const int64_t* __restrict__ chunk_begin,
    const int32_t* __restrict__ chunk_rbf, int l_s, const double* __restrict__ U, int l_d,
    const double* __restrict__ Z, double* __restrict__ partial, int ncp) {
  // ncp: B columns held in LDS (a multiple of 16, >= the padded tile span);
  // tiles t = wave + 8 q (q < QMAX) cover rows mt = t % MT and columns
  // 16 (t / MT) .. +15, zero-padded beyond l_s rows / l_d na columns
  extern __shared__ __attribute__((aligned(16))) unsigned char jsm[];
  const int ch = blockIdx.x;
  const int64_t b0 = chunk_begin[ch], b1 = chunk_begin[ch + 1];
  const double* th = theta + (int64_t)chunk_rbf[ch] * P.stride;
  const int na = P.n_act;
  const int lsld = l_s * l_d;
  const int ncol = l_d * na;
  const int MT = (l_s + 15) / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __bf16* sA = reinterpret_cast<__bf16*>(jsm);            // [TERMS][MT*16][MKP]
  __bf16* sB = sA + TERMS * MT * 16 * MKP;                // [TERMS][ncp][MKP]
  double* sZ = reinterpret_cast<double*>(sB + TERMS * ncp * MKP);  // [MK][l_d]
  double* sG = sZ + MK * l_d;                             // [MK][na]
  double* out = partial + (int64_t)ch * lsld * na;

  // per tile: LDS fragment offsets and the output offset of element e = 0
  int aoff[QMAX], boff[QMAX], ooff[QMAX], orow[QMAX], ocol[QMAX];
  const int kofs = 8 * (lane >> 4);
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int t = wave + 8 * q;
    const int mt = t % MT, nt = t / MT;
    aoff[q] = (mt * 16 + (lane & 15)) * MKP + kofs;
    boff[q] = (nt * 16 + (lane & 15)) * MKP + kofs;
    const int i0 = mt * 16 + 4 * (lane >> 4);
    const int n = nt * 16 + (lane & 15);
    orow[q] = i0;
    ocol[q] = n;
    ooff[q] = n < ncol ? (n % l_d) + l_d * i0 + lsld * (n / l_d) : 0;
  }
  f32x4 acc[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
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

  int kstep = 0;
  for (int64_t cb = b0; cb < b1; cb += MK, ++kstep) {
    const int nb = (int)min<int64_t>(MK, b1 - cb);
    __syncthreads();  // previous K-step's MFMA reads are done
    // U -> A parts (rows beyond l_s and cells beyond nb are zero)
    for (int t = threadIdx.x; t < MT * 16 * MK; t += MT_THREADS) {
      const int cc = t % MK, i = t / MK;
      float v = 0.f;
      if (cc < nb && i < l_s) v = (float)U[pair_cell[cb + cc] + P.N * (int64_t)i];
      __bf16 parts[TERMS];
      split_bf16<TERMS>(v, parts);
#pragma unroll
      for (int q = 0; q < TERMS; ++q) sA[(q * MT * 16 + i) * MKP + cc] = parts[q];
    }
    // Z staging (binary64) and G of each cell
    for (int t = threadIdx.x; t < MK * l_d; t += MT_THREADS) {
      const int cc = t % MK, j = t / MK;
      sZ[cc * l_d + j] = cc < nb ? Z[pair_cell[cb + cc] + P.N * (int64_t)j] : 0.0;
    }
    if (threadIdx.x < MK) {
      double d[5] = {0, 0, 0, 0, 0};
      double w = 0.0;
      if ((int)threadIdx.x < nb) {
        const int64_t c = pair_cell[cb + threadIdx.x];
        double x0, x1, x2;
        cell_xyz(g, c, &x0, &x1, &x2);
        rbf_dphi(P, th, x0, x1, x2, d);
        w = band_weight(P, phi[c]);
      }
      for (int a = 0; a < na; ++a) sG[threadIdx.x * na + a] = P.hd * (w * d[a]);
    }
    __syncthreads();
    // B parts: B[c, n] = Z[c, j] G[c, a] for n < ncol, zero up to ncp
    for (int t = threadIdx.x; t < ncp * MK; t += MT_THREADS) {
      const int cc = t % MK, n = t / MK;
      float v = 0.f;
      if (n < ncol) {
        const int j = n % l_d, a = n / l_d;
        v = (float)(sZ[cc * l_d + j] * sG[cc * na + a]);
      }
      __bf16 parts[TERMS];
      split_bf16<TERMS>(v, parts);
#pragma unroll
      for (int q = 0; q < TERMS; ++q) sB[(q * ncp + n) * MKP + cc] = parts[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      bf16x8 fa[TERMS], fb[TERMS];
#pragma unroll
      for (int p = 0; p < TERMS; ++p) {
        fa[p] = *reinterpret_cast<const bf16x8*>(&sA[p * MT * 16 * MKP + aoff[q]]);
        fb[p] = *reinterpret_cast<const bf16x8*>(&sB[p * ncp * MKP + boff[q]]);
      }
#pragma unroll
      for (int pa = 0; pa < TERMS; ++pa)
#pragma unroll
        for (int pb = 0; pb < TERMS; ++pb)
          if (pa + pb <= TERMS - 1)
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[pa], fb[pb], acc[q], 0, 0, 0);
    }
    if ((kstep + 1) % JFLUSH == 0) flush();
  }
  if (first || kstep % JFLUSH != 0) flush();
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

__global__ __launch_bounds__(256) void grad_chunk_kernel(GridDims g, JacParams P,
                                                         const double* __restrict__ theta,
                                                         const double* __restrict__ phi,
                                                         const int32_t* __restrict__ pair_cell,
                                                         const int64_t* __restrict__ chunk_begin,
                                                         const int32_t* __restrict__ chunk_rbf,
                                                         const double* __restrict__ sc,
                                                         double* __restrict__ partial) {
  __shared__ double red[5][256];
  const int ch = blockIdx.x;
  const int64_t b0 = chunk_begin[ch], b1 = chunk_begin[ch + 1];
  const double* th = theta + (int64_t)chunk_rbf[ch] * P.stride;
  const int na = P.n_act;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t p = b0 + threadIdx.x; p < b1; p += 256) {
    const int64_t c = pair_cell[p];
    double x0, x1, x2, d[5];
    cell_xyz(g, c, &x0, &x1, &x2);
    rbf_dphi(P, th, x0, x1, x2, d);
    const double w = band_weight(P, phi[c]);
    const double s = sc[c];
    for (int a = 0; a < na; ++a) acc[a] += (P.hd * (w * d[a])) * s;
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

static size_t jac_bytes(const dot_op* op, int l_s, int l_d) {
  const int na = n_active_bits(op->pals.active, op->g.dim);
  const size_t jac = (size_t)std::max<int64_t>(op->n_chunks, 1) * l_s * l_d * na * sizeof(double);
  const size_t grad = (size_t)op->g.N * sizeof(double) +
                      (size_t)std::max<int64_t>(op->n_chunks, 1) * na * sizeof(double) + 256;
  return ((std::max(jac, grad) + 255) / 256) * 256;
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
  if ((size_t)JB * (l_s + l_d + 5) * sizeof(double) > 64 * 1024)
    DOT_FAIL(DOT_EINVAL, "l_s + l_d too large for the contraction kernel");
  hipStream_t s = as_stream(stream);
  const JacParams P = make_params(op);
  const int na = P.n_act;
  const int m0 = op->pals.m0;
  const int lsld = l_s * l_d;
  double* partial = (double*)work_dev;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  unsigned long long* cols = nullptr;
  DOT_TRY_J(profile_begin(op, DOT_PROF_JACOBIAN, s, &e0, &e1, &cols));
  if (op->n_chunks > 0 && precision == DOT_JAC_FP64) {
    const size_t shm = (size_t)JB * (l_s + l_d + na) * sizeof(double);
    hipLaunchKernelGGL(jac_chunk_fp64_kernel, dim3((unsigned)op->n_chunks), dim3(JT), shm, s, op->g,
                       P, op->theta, op->phi, op->pair_cell, op->chunk_begin, op->chunk_rbf, l_s,
                       U_dev, l_d, Z_dev, partial);
    DOT_LAUNCH_CHECK();
  } else if (op->n_chunks > 0) {
    const int terms = precision == DOT_JAC_SPLIT_BF16 ? 2 : 3;
    const int MT = (l_s + 15) / 16, NT = (l_d * na + 15) / 16;
    const int tiles = MT * NT;
    if (tiles > 64) DOT_FAIL(DOT_EINVAL, "l_s * l_d * n_act too large for the split-bf16 kernel");
    const int qmax = (tiles + 7) / 8;
    // columns reached by the padded tiles t < 8 qmax
    const int ncp = ((8 * qmax - 1) / MT + 1) * 16;
    const size_t shm = (size_t)terms * (MT * 16 + ncp) * MKP * 2 +
                       (size_t)MK * l_d * sizeof(double) + (size_t)MK * na * sizeof(double);
    auto launch = [&](auto kern) -> int {
      DOT_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shm));
      hipLaunchKernelGGL(kern, dim3((unsigned)op->n_chunks), dim3(MT_THREADS), shm, s, op->g, P,
                         op->theta, op->phi, op->pair_cell, op->chunk_begin, op->chunk_rbf, l_s,
                         U_dev, l_d, Z_dev, partial, ncp);
      DOT_LAUNCH_CHECK();
      return DOT_OK;
    };
    int rc = DOT_EINVAL;
#define DOT_JAC_CASE(T, Q) \
  case Q:                  \
    rc = launch(jac_chunk_mfma_kernel<T, Q>); \
    break;
    if (terms == 2) {
      switch (qmax) {
        DOT_JAC_CASE(2, 1) DOT_JAC_CASE(2, 2) DOT_JAC_CASE(2, 3) DOT_JAC_CASE(2, 4)
        DOT_JAC_CASE(2, 5) DOT_JAC_CASE(2, 6) DOT_JAC_CASE(2, 7) DOT_JAC_CASE(2, 8)
      }
    } else {
      switch (qmax) {
        DOT_JAC_CASE(3, 1) DOT_JAC_CASE(3, 2) DOT_JAC_CASE(3, 3) DOT_JAC_CASE(3, 4)
        DOT_JAC_CASE(3, 5) DOT_JAC_CASE(3, 6) DOT_JAC_CASE(3, 7) DOT_JAC_CASE(3, 8)
      }
    }
#undef DOT_JAC_CASE
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
    hipLaunchKernelGGL(grad_chunk_kernel, dim3((unsigned)op->n_chunks), dim3(256), 0, s, op->g, P,
                       op->theta, op->phi, op->pair_cell, op->chunk_begin, op->chunk_rbf, sc,
                       partial);
    DOT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((m0 * na + 255) / 256), dim3(256), 0, s, m0,
                     op->rbf_chunk0, na, partial, g_dev);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

}  // extern "C"
