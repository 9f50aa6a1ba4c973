// Simultaneous right-hand sides, sampled misfit, small dense products.
//
// Section 3.1 (eq. Rw: one solve per simultaneous source B w), Section 3.3
// (eq. EsTResidual: the sampled residual V^T C^T z_i - V^T D w_i for
// i = 1..l_s) and Thm 3.1 (its squared Frobenius norm estimates ||R||_F^2).
#include <vector>

#include "dot_internal.h"

namespace dot {

__global__ void fill_zero_kernel(double* __restrict__ y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) y[i] = 0.0;
}

// One thread per column; the points of a column are added in order, so
// repeated cells accumulate deterministically.
// One thread per (distinct cell, column): the weights of the points at that
// cell summed in the points' order (the sum a sequential scatter would
// form), written into the zeroed block.
__global__ void scatter_rhs_kernel(int64_t N, int n_pts, int n_u, const int32_t* __restrict__ perm,
                                   const int32_t* __restrict__ ucell,
                                   const int32_t* __restrict__ ustart, int k,
                                   const double* __restrict__ w, double* __restrict__ rhs) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_u * k) return;
  const int u = (int)(e % n_u), l = (int)(e / n_u);
  double s = 0.0;
  for (int i = ustart[u]; i < ustart[u + 1]; ++i) s += w[perm[i] + (int64_t)n_pts * l];
  rhs[ucell[u] + N * l] = s;
}

// Rs[j, i] = sum_a V[a, j] (U[det[a], i] - DW[a, i]);  f = 1/2 sum Rs^2.
__global__ __launch_bounds__(256) void misfit_kernel(int64_t N, int n_d, const int32_t* __restrict__ det,
                                                     int l_s, const double* __restrict__ U, int l_d,
                                                     const double* __restrict__ V,
                                                     const double* __restrict__ DW,
                                                     double* __restrict__ Rs, double* __restrict__ f) {
  __shared__ double red[256];
  double part = 0.0;
  const int total = l_s * l_d;
  for (int e = threadIdx.x; e < total; e += 256) {
    const int j = e % l_d, i = e / l_d;
    double s = 0.0;
    for (int a = 0; a < n_d; ++a) {
      const double t = U[det[a] + N * i] - DW[a + (int64_t)n_d * i];
      s += V[a + (int64_t)n_d * j] * t;
    }
    Rs[j + (int64_t)l_d * i] = s;
    part += s * s;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) f[0] = 0.5 * red[0];
}

// C = alpha op(A) op(B) + beta C.  16x16 output tiles, operands staged through
// LDS in 16-deep slices; each output is a fixed-order sum.
__global__ __launch_bounds__(256) void gemm_kernel(int ta, int tb, int m, int n, int kd, double alpha,
                                                   const double* __restrict__ A, int lda,
                                                   const double* __restrict__ B, int ldb, double beta,
                                                   double* __restrict__ C, int ldc) {
  __shared__ double sa[16][17];
  __shared__ double sb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = blockIdx.y * 16 + tx;  // row of C
  const int colc = blockIdx.x * 16 + ty; // column of C
  double acc = 0.0;
  for (int k0 = 0; k0 < kd; k0 += 16) {
    // sa[kk][r] = op(A)[blockrow + r, k0 + kk]
    {
      const int r = tx, kk = ty;
      const int gi = blockIdx.y * 16 + r, gk = k0 + kk;
      double v = 0.0;
      if (gi < m && gk < kd) v = ta ? A[gk + (int64_t)lda * gi] : A[gi + (int64_t)lda * gk];
      sa[kk][r] = v;
    }
    // sb[kk][cc] = op(B)[k0 + kk, blockcol + cc]
    {
      const int kk = tx, cc = ty;
      const int gk = k0 + kk, gj = blockIdx.x * 16 + cc;
      double v = 0.0;
      if (gk < kd && gj < n) v = tb ? B[gj + (int64_t)ldb * gk] : B[gk + (int64_t)ldb * gj];
      sb[kk][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc += sa[kk][tx] * sb[kk][ty];
    __syncthreads();
  }
  if (row < m && colc < n) {
    double* cp = C + row + (int64_t)ldc * colc;
    *cp = beta == 0.0 ? alpha * acc : alpha * acc + beta * *cp;
  }
}

int gemm_launch(int transa, int transb, int m, int n, int kdim, double alpha, const double* A,
                int lda, const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  if (m == 0 || n == 0) return DOT_OK;
  dim3 grid((n + 15) / 16, (m + 15) / 16);
  hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, transa, transb, m, n, kdim, alpha, A, lda, B,
                     ldb, beta, C, ldc);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

}  // namespace dot

using namespace dot;

extern "C" {

int dot_form_rhs(dot_op* op, int n_pts, const int32_t* cells_host, int k,
                 const double* weights_dev, double* rhs_dev, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (n_pts < 0 || k < 1) DOT_FAIL(DOT_EINVAL, "n_pts must be >= 0 and k >= 1");
  if (!rhs_dev) DOT_FAIL(DOT_EINVAL, "rhs_dev is NULL");
  if (n_pts > 0 && (!cells_host || !weights_dev)) DOT_FAIL(DOT_EINVAL, "cells/weights NULL");
  for (int i = 0; i < n_pts; ++i)
    if (cells_host[i] < 0 || cells_host[i] >= op->g.N)
      DOT_FAIL(DOT_EINVAL, "cell %d of point %d outside [0, %lld)", cells_host[i], i,
               (long long)op->g.N);
  hipStream_t s = as_stream(stream);
  const int64_t n = op->g.N * (int64_t)k;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, rhs_dev, n);
  DOT_LAUNCH_CHECK();
  if (n_pts == 0) return DOT_OK;
  const dot_op::CellList* cl = nullptr;
  int rc = cells_on_device(op, n_pts, cells_host, s, &cl);
  if (rc) return rc;
  const int32_t* perm = cl->dev + n_pts;
  const int32_t* ucell = perm + n_pts;
  const int32_t* ustart = ucell + cl->n_u;
  const int64_t work = (int64_t)cl->n_u * k;
  hipLaunchKernelGGL(scatter_rhs_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, op->g.N,
                     n_pts, cl->n_u, perm, ucell, ustart, k, weights_dev, rhs_dev);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

int dot_sampled_misfit(dot_op* op, int n_d, const int32_t* det_host, int l_s, const double* U_dev,
                       int l_d, const double* V_dev, const double* DW_dev, double* Rs_dev,
                       double* f_host, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (n_d < 1 || l_s < 1 || l_d < 1) DOT_FAIL(DOT_EINVAL, "n_d, l_s, l_d must be >= 1");
  if (!det_host || !U_dev || !V_dev || !DW_dev || !Rs_dev || !f_host)
    DOT_FAIL(DOT_EINVAL, "NULL argument");
  for (int a = 0; a < n_d; ++a)
    if (det_host[a] < 0 || det_host[a] >= op->g.N)
      DOT_FAIL(DOT_EINVAL, "detector cell %d outside the grid", det_host[a]);
  hipStream_t s = as_stream(stream);
  const dot_op::CellList* cl = nullptr;
  int rc = cells_on_device(op, n_d, det_host, s, &cl);
  if (rc) return rc;
  hipLaunchKernelGGL(misfit_kernel, dim3(1), dim3(256), 0, s, op->g.N, n_d, cl->dev, l_s,
                     U_dev, l_d, V_dev, DW_dev, Rs_dev, op->small_dev);
  DOT_LAUNCH_CHECK();
  DOT_HIP(hipMemcpyAsync(op->pinned_d, op->small_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  *f_host = op->pinned_d[0];
  return DOT_OK;
}

int dot_gemm(int transa, int transb, int m, int n, int kdim, double alpha, const double* A_dev,
             int lda, const double* B_dev, int ldb, double beta, double* C_dev, int ldc,
             void* stream) {
  clear_error();
  if (m < 0 || n < 0 || kdim < 0) DOT_FAIL(DOT_EINVAL, "negative dimension");
  if (m == 0 || n == 0) return DOT_OK;
  if (!C_dev || (kdim > 0 && (!A_dev || !B_dev))) DOT_FAIL(DOT_EINVAL, "NULL argument");
  const int arows = transa ? kdim : m, brows = transb ? n : kdim;
  if (lda < std::max(1, arows) || ldb < std::max(1, brows) || ldc < std::max(1, m))
    DOT_FAIL(DOT_EINVAL, "leading dimension too small");
  if ((int64_t)(n + 15) / 16 > 2147483647 || (m + 15) / 16 > 65535)
    DOT_FAIL(DOT_EINVAL, "matrix too large for dot_gemm");
  return gemm_launch(transa, transb, m, n, kdim, alpha, A_dev, lda, B_dev, ldb, beta, C_dev, ldc,
                     as_stream(stream));
}

}  // extern "C"
