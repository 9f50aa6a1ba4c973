// Operator construction, PaLS absorption, right-hand sides.
//
// Section 2 (eq. PDE, PaLS definition, eq. absorption const) and Section 3.1
// (eq. Rw).  The finite-volume coefficients, the smoothed Heaviside and the
// frozen diffusion follow the readings stated in include/dotpath.h.
#include <algorithm>
#include <cstring>
#include <vector>

#include "dot_internal.h"

namespace dot {

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
void clear_error() { g_err[0] = '\0'; }

int validate_grid(const dot_grid* g, GridDims* out, const char** why) {
  if (!g) {
    *why = "grid is NULL";
    return DOT_EINVAL;
  }
  if (g->dim != 2 && g->dim != 3) {
    *why = "grid.dim must be 2 or 3";
    return DOT_EINVAL;
  }
  const int nz = g->dim == 3 ? g->n[2] : 1;
  if (g->n[0] < 1 || g->n[1] < 1 || nz < 1) {
    *why = "grid.n must be positive";
    return DOT_EINVAL;
  }
  if (g->n[0] > (1 << 20) || g->n[1] > (1 << 20) || nz > (1 << 20)) {
    *why = "grid.n too large";
    return DOT_EINVAL;
  }
  const int64_t N = (int64_t)g->n[0] * g->n[1] * nz;
  // the stencil sweeps address a column with 32-bit byte offsets, so a
  // binary64 column of N cells must span less than 4 GiB
  if (N > ((int64_t)1 << 29)) {
    *why = "grid has more than 2^29 cells";
    return DOT_EINVAL;
  }
  for (int f = 0; f < 2 * g->dim; ++f) {
    if (g->bc[f] != DOT_BC_DIRICHLET && g->bc[f] != DOT_BC_ROBIN) {
      *why = "grid.bc entries must be DOT_BC_DIRICHLET or DOT_BC_ROBIN";
      return DOT_EINVAL;
    }
  }
  if (out) {
    out->dim = g->dim;
    out->nx = g->n[0];
    out->ny = g->n[1];
    out->nz = nz;
    out->nxy = (int64_t)g->n[0] * g->n[1];
    out->N = N;
    out->h = 1.0 / g->n[0];
    out->hd = g->dim == 3 ? out->h * out->h * out->h : out->h * out->h;
  }
  return DOT_OK;
}

static int validate_pals(const dot_pals* p, int dim) {
  if (!p) DOT_FAIL(DOT_EINVAL, "pals is NULL");
  if (p->m0 < 1 || p->m0 > (1 << 20)) DOT_FAIL(DOT_EINVAL, "pals.m0 must be in [1, 2^20]");
  if ((p->active & ~7u) != 0 || p->active == 0)
    DOT_FAIL(DOT_EINVAL, "pals.active must be a nonzero combination of DOT_ACT_* bits");
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) DOT_FAIL(DOT_EINVAL, "pals.eps must be > 0");
  if (!(p->gamma >= 0.0) || !(p->gamma < 1.0)) DOT_FAIL(DOT_EINVAL, "pals.gamma must be in [0, 1)");
  if (!std::isfinite(p->mu_in) || !std::isfinite(p->mu_out) || !std::isfinite(p->cutoff))
    DOT_FAIL(DOT_EINVAL, "pals constants must be finite");
  (void)dim;
  return DOT_OK;
}

int cells_on_device(dot_op* op, int n, const int32_t* cells_host, hipStream_t s,
                    const dot_op::CellList** out) {
  ++op->cell_clock;
  dot_op::CellList* hit = nullptr;
  dot_op::CellList* lru = &op->cell_lists[0];
  for (auto& e : op->cell_lists) {
    if (e.dev && e.n == n && std::equal(cells_host, cells_host + n, e.key.begin())) hit = &e;
    if (e.used < lru->used) lru = &e;
  }
  if (!hit) {
    // replace the least recently used list; kernels still queued on this
    // stream may read it
    hit = lru;
    DOT_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int a, int b) { return cells_host[a] < cells_host[b]; });
    std::vector<int32_t> ucell, ustart;
    for (int i = 0; i < n; ++i) {
      if (i == 0 || cells_host[perm[i]] != cells_host[perm[i - 1]]) {
        ucell.push_back(cells_host[perm[i]]);
        ustart.push_back(i);
      }
    }
    ustart.push_back(n);
    const int n_u = (int)ucell.size();
    std::vector<int32_t> buf;
    buf.reserve((size_t)2 * n + 2 * n_u + 1);
    buf.insert(buf.end(), cells_host, cells_host + n);
    buf.insert(buf.end(), perm.begin(), perm.end());
    buf.insert(buf.end(), ucell.begin(), ucell.end());
    buf.insert(buf.end(), ustart.begin(), ustart.end());
    if ((int64_t)buf.size() > hit->cap) {
      if (hit->dev) DOT_HIP(hipFree(hit->dev));
      hit->dev = nullptr;
      hit->cap = 0;
      const int64_t cap = std::max<int64_t>((int64_t)buf.size(), 1024);
      DOT_HIP(hipMalloc(&hit->dev, (size_t)cap * sizeof(int32_t)));
      hit->cap = cap;
    }
    DOT_HIP(hipMemcpyAsync(hit->dev, buf.data(), buf.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    // the copy reads buf asynchronously
    DOT_HIP(hipStreamSynchronize(s));
    hit->key.assign(cells_host, cells_host + n);
    hit->n = n;
    hit->n_u = n_u;
  }
  hit->used = op->cell_clock;
  *out = hit;
  return DOT_OK;
}

// ------------------------------------------------------------------ PaLS
struct PalsK {
  double mu_in, mu_out, cutoff, eps, gamma;
  int m0, dim, stride;  // stride = 2 + dim
};

__device__ __forceinline__ double wendland(double r) {
  if (r >= 1.0) return 0.0;
  const double o = 1.0 - r;
  const double o2 = o * o;
  return o2 * o2 * (4.0 * r + 1.0);
}

__device__ __forceinline__ double heaviside_eps(double s, double eps) {
  if (s < -eps) return 0.0;
  if (s > eps) return 1.0;
  return 0.5 * (1.0 + s / eps + sin(M_PI * s / eps) / M_PI);
}

// One block of 256 threads per cell tile (8x8x4 in 3D, 16x16 in 2D).  RBFs are
// culled against the tile's bounding box in chunks of 256, compacted in RBF
// order, and summed in that order at each cell centre.
__global__ __launch_bounds__(256) void pals_field_kernel(GridDims g, PalsK p,
                                                         const double* __restrict__ theta,
                                                         double mus_prime, double* __restrict__ mua,
                                                         double* __restrict__ diff,
                                                         double* __restrict__ phi_out) {
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
  // tile bounding box of cell centres
  const double lo0 = (bx * TX + 0.5) * h, hi0 = (min(g.nx, bx * TX + TX) - 0.5) * h;
  const double lo1 = (by * TY + 0.5) * h, hi1 = (min(g.ny, by * TY + TY) - 0.5) * h;
  const double lo2 = (bz * TZ + 0.5) * h, hi2 = (min(g.nz, bz * TZ + TZ) - 0.5) * h;
  const double g2 = p.gamma * p.gamma;
  double phi = 0.0;
  for (int base = 0; base < p.m0; base += 256) {
    const int j = base + t;
    int flag = 0;
    if (j < p.m0) {
      const double* th = theta + (int64_t)j * p.stride;
      const double beta = th[1];
      double d0 = fmax(0.0, fmax(lo0 - th[2], th[2] - hi0));
      double d1 = fmax(0.0, fmax(lo1 - th[3], th[3] - hi1));
      double dist2 = d0 * d0 + d1 * d1;
      if (d3) {
        double d2 = fmax(0.0, fmax(lo2 - th[4], th[4] - hi2));
        dist2 += d2 * d2;
      }
      // conservative: every cell in the box has rho >= dist
      flag = (beta * beta * dist2 + g2 < 1.0) ? 1 : 0;
    }
    int total;
    const int pos = block_scan_flag256(flag, s_wave, &total);
    if (flag) s_list[pos] = j;
    __syncthreads();
    if (inside) {
      for (int q = 0; q < total; ++q) {
        const double* th = theta + (int64_t)s_list[q] * p.stride;
        const double alpha = th[0], beta = th[1];
        const double e0 = xc0 - th[2], e1 = xc1 - th[3];
        double rho2 = e0 * e0 + e1 * e1;
        if (d3) {
          const double e2 = xc2 - th[4];
          rho2 += e2 * e2;
        }
        const double r = sqrt(beta * beta * rho2 + g2);
        phi += alpha * wendland(r);
      }
    }
    __syncthreads();
  }
  if (!inside) return;
  const int64_t c = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
  const double H = heaviside_eps(phi - p.cutoff, p.eps);
  const double mu = p.mu_in * H + p.mu_out * (1.0 - H);
  if (mua) mua[c] = mu;
  if (diff) diff[c] = 1.0 / (3.0 * (mu + mus_prime));
  if (phi_out) phi_out[c] = phi;
}

static int launch_pals(const GridDims& g, const dot_pals* pals, const double* theta,
                       double mus_prime, double* mua, double* diff, double* phi, hipStream_t s) {
  PalsK p{pals->mu_in, pals->mu_out, pals->cutoff, pals->eps, pals->gamma, pals->m0, g.dim,
          2 + g.dim};
  int64_t tiles;
  if (g.dim == 3)
    tiles = (int64_t)((g.nx + 7) / 8) * ((g.ny + 7) / 8) * ((g.nz + 3) / 4);
  else
    tiles = (int64_t)((g.nx + 15) / 16) * ((g.ny + 15) / 16);
  hipLaunchKernelGGL(pals_field_kernel, dim3((unsigned)tiles), dim3(256), 0, s, g, p, theta,
                     mus_prime, mua, diff, phi);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

// ------------------------------------------------------------------ operator
__device__ __forceinline__ double bdry_T(int code, double Dc, double h, int d) {
  const double hd2 = d == 3 ? h : 1.0;       // h^(d-2)
  const double hd1 = d == 3 ? h * h : h;     // h^(d-1)
  if (code == DOT_BC_DIRICHLET) return hd2 * 2.0 * Dc;
  return hd1 * 2.0 * Dc / (h + 4.0 * Dc);
}

struct BC6 {
  int f[6];
};

__global__ void build_coef_kernel(GridDims g, BC6 bc, const double* __restrict__ D,
                                  double* __restrict__ cx, double* __restrict__ cy,
                                  double* __restrict__ cz, double* __restrict__ b0) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / g.nxy);
  const int d = g.dim;
  const double hd2 = d == 3 ? g.h : 1.0;
  const double Dc = D[c];
  double tx = 0.0, ty = 0.0, tz = 0.0;
  if (x + 1 < g.nx) {
    const double Dn = D[c + 1];
    tx = hd2 * 2.0 * Dc * Dn / (Dc + Dn);
  }
  if (y + 1 < g.ny) {
    const double Dn = D[c + g.nx];
    ty = hd2 * 2.0 * Dc * Dn / (Dc + Dn);
  }
  if (d == 3 && z + 1 < g.nz) {
    const double Dn = D[c + g.nxy];
    tz = hd2 * 2.0 * Dc * Dn / (Dc + Dn);
  }
  double bb = 0.0;
  if (x == 0) bb += bdry_T(bc.f[0], Dc, g.h, d);
  if (x == g.nx - 1) bb += bdry_T(bc.f[1], Dc, g.h, d);
  if (y == 0) bb += bdry_T(bc.f[2], Dc, g.h, d);
  if (y == g.ny - 1) bb += bdry_T(bc.f[3], Dc, g.h, d);
  if (d == 3) {
    if (z == 0) bb += bdry_T(bc.f[4], Dc, g.h, d);
    if (z == g.nz - 1) bb += bdry_T(bc.f[5], Dc, g.h, d);
  }
  cx[c] = tx;
  cy[c] = ty;
  cz[c] = tz;
  b0[c] = bb;
}

// diag = b0 + sum of the face coefficients + h^d mu;  sd = sqrt(diag)
__global__ void diag_kernel(GridDims g, const double* __restrict__ cx, const double* __restrict__ cy,
                            const double* __restrict__ cz, const double* __restrict__ b0,
                            const double* __restrict__ mua, double* __restrict__ diag,
                            double* __restrict__ sd) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / g.nxy);
  double s = b0[c] + (mua ? g.hd * mua[c] : 0.0);
  s += cx[c];
  if (x > 0) s += cx[c - 1];
  s += cy[c];
  if (y > 0) s += cy[c - g.nx];
  if (g.dim == 3) {
    s += cz[c];
    if (z > 0) s += cz[c - g.nxy];
  }
  diag[c] = s;
  sd[c] = sqrt(s);
}

__global__ void scale_kernel(GridDims g, const double* __restrict__ cx, const double* __restrict__ cy,
                             const double* __restrict__ cz, const double* __restrict__ sd,
                             double* __restrict__ sx, double* __restrict__ sy,
                             double* __restrict__ sz, float* __restrict__ sx32,
                             float* __restrict__ sy32, float* __restrict__ sz32) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / g.nxy);
  const double s0 = sd[c];
  const double vx = (x + 1 < g.nx) ? cx[c] / (s0 * sd[c + 1]) : 0.0;
  const double vy = (y + 1 < g.ny) ? cy[c] / (s0 * sd[c + g.nx]) : 0.0;
  const double vz = (g.dim == 3 && z + 1 < g.nz) ? cz[c] / (s0 * sd[c + g.nxy]) : 0.0;
  sx[c] = vx;
  sy[c] = vy;
  sz[c] = vz;
  sx32[c] = (float)vx;
  sy32[c] = (float)vy;
  sz32[c] = (float)vz;
}

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// D = 1 / (3 (mu + mu_s)) with both optical properties from the level set:
// mu = mu_out + (mu_in - mu_out) H, mu_s = mus_out + (mus_in - mus_out) H,
// H = H_eps(phi - cutoff).
__global__ void diff_from_phi_kernel(GridDims g, PalsK p, double mus_in, double mus_out,
                                     const double* __restrict__ phi, double* __restrict__ D) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const double H = heaviside_eps(phi[c] - p.cutoff, p.eps);
  const double mu = p.mu_in * H + p.mu_out * (1.0 - H);
  const double ms = mus_in * H + mus_out * (1.0 - H);
  D[c] = 1.0 / (3.0 * (mu + ms));
}

// face coefficients and boundary diagonal from the diffusion field in D0
static int rebuild_coefficients(dot_op* op, hipStream_t s) {
  BC6 bc;
  for (int f = 0; f < 6; ++f) bc.f[f] = op->bc[f];
  hipLaunchKernelGGL(build_coef_kernel, dim3(nblk(op->g.N, 256)), dim3(256), 0, s, op->g, bc,
                     op->D0, op->cx, op->cy, op->cz, op->b0);
  DOT_LAUNCH_CHECK();
  return DOT_OK;
}

// back to the diffusion given at build time (absorption-only calls)
static int leave_diffusion_mode(dot_op* op, hipStream_t s) {
  if (!op->diff_mode) return DOT_OK;
  DOT_HIP(hipMemcpyAsync(op->D0, op->Dbuild, (size_t)op->g.N * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  op->diff_mode = false;
  return rebuild_coefficients(op, s);
}

// ------------------------------------------------------------------ multigrid setup
// coarse D and mu: means over the children of the aggregate (2 x 2 x 2, or
// 2 x 2 in 2D; fewer in the last aggregate of an odd side)
__global__ void mg_coarsen_kernel(GridDims gf, GridDims gc, const double* __restrict__ Df,
                                  const double* __restrict__ muf, double* __restrict__ Dc,
                                  double* __restrict__ muc) {
  const int64_t C = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (C >= gc.N) return;
  const int X = (int)(C % gc.nx);
  const int Y = (int)((C / gc.nx) % gc.ny);
  const int Z = (int)(C / gc.nxy);
  double sD = 0.0, sm = 0.0;
  int cnt = 0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int x = 2 * X + dx, y = 2 * Y + dy, z = 2 * Z + dz;
        if (x >= gf.nx || y >= gf.ny || z >= gf.nz) continue;
        const int64_t c = x + gf.nx * ((int64_t)y + gf.ny * (int64_t)z);
        sD += Df[c];
        sm += muf[c];
        ++cnt;
      }
  Dc[C] = sD / cnt;
  muc[C] = sm / cnt;
}

// prolongation weight sd(c) / sd_coarse(parent(c))
__global__ void mg_q_kernel(GridDims gf, GridDims gc, const double* __restrict__ sdf,
                            const double* __restrict__ sdc, double* __restrict__ q,
                            float* __restrict__ q32) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= gf.N) return;
  const int x = (int)(c % gf.nx);
  const int y = (int)((c / gf.nx) % gf.ny);
  const int z = (int)(c / gf.nxy);
  const int64_t P = (x >> 1) + gc.nx * ((int64_t)(y >> 1) + gc.ny * (int64_t)(z >> 1));
  const double v = sdf[c] / sdc[P];
  q[c] = v;
  q32[c] = (float)v;
}

// v rounded to binary32
__global__ void mg_round_kernel(int64_t N, const double* __restrict__ v, float* __restrict__ v32) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c < N) v32[c] = (float)v[c];
}

// flag = 1 if some diagonal entry is not positive (or not finite)
__global__ void mg_check_kernel(int64_t N, const double* __restrict__ diag, int* __restrict__ flag) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c < N && !(diag[c] > 0.0 && diag[c] < INFINITY)) flag[0] = 1;
}

__global__ void mg_flag_clear_kernel(int* __restrict__ flag) { flag[0] = 0; }

// Level l + 1 halves every side of level l, rounding up (the last aggregate
// of an odd side has one cell along it; 2D grids keep n_z = 1), while every
// coarse side keeps at least MG_MIN_SIDE cells.  A coarse level is the same
// discretization with h = 1 / n_x, like the finest.
constexpr int MG_MIN_SIDE = 3;

int mg_levels_for(const GridDims& g, GridDims* lv) {
  if (g.dim != 2 && g.dim != 3) return 0;
  auto coarse_ok = [&](const GridDims& c) {
    return (c.nx + 1) / 2 >= MG_MIN_SIDE && (c.ny + 1) / 2 >= MG_MIN_SIDE &&
           (c.dim == 2 || (c.nz + 1) / 2 >= MG_MIN_SIDE);
  };
  int n = 0;
  GridDims cur = g;
  lv[n++] = cur;
  while (n < DOT_MG_MAXLEV && coarse_ok(cur)) {
    GridDims c = cur;
    c.nx = (cur.nx + 1) / 2;
    c.ny = (cur.ny + 1) / 2;
    c.nz = cur.dim == 3 ? (cur.nz + 1) / 2 : 1;
    c.nxy = (int64_t)c.nx * c.ny;
    c.N = c.nxy * c.nz;
    c.h = 1.0 / c.nx;
    c.hd = cur.dim == 3 ? c.h * c.h * c.h : c.h * c.h;
    lv[n++] = c;
    cur = c;
  }
  return n;
}

void mg_free(dot_op* op) {
  for (int l = 0; l < op->mg_nlev; ++l) {
    MgLevel& L = op->mg[l];
    if (l > 0) {
      void* ptrs[] = {L.D, L.mu, L.cx, L.cy, L.cz, L.b0, L.diag, L.sd, L.sx, L.sy, L.sz,
                      L.sx32, L.sy32, L.sz32};
      for (void* p : ptrs)
        if (p) (void)hipFree(p);
    }
    if (L.sd32) (void)hipFree(L.sd32);
    if (L.q) (void)hipFree(L.q);
    if (L.q32) (void)hipFree(L.q32);
    L = MgLevel{};
  }
  if (op->mg_flag) (void)hipFree(op->mg_flag);
  op->mg_flag = nullptr;
  op->mg_nlev = 0;
  op->mg_ok = false;
}

// (Re)build the hierarchy from the operator's current diagonal.
int mg_refresh(dot_op* op, hipStream_t s) {
  GridDims lv[DOT_MG_MAXLEV];
  const int n = op->D0 ? mg_levels_for(op->g, lv) : 0;
  if (n < 2) return DOT_OK;
  if (op->mg_nlev != n) {
    mg_free(op);
    MgLevel& L0 = op->mg[0];
    L0.g = lv[0];
    L0.D = op->D0;
    L0.mu = op->mu0;
    L0.cx = op->cx;
    L0.cy = op->cy;
    L0.cz = op->cz;
    L0.b0 = op->b0;
    L0.diag = op->diag;
    L0.sd = op->sd;
    L0.sx = op->sx;
    L0.sy = op->sy;
    L0.sz = op->sz;
    L0.sx32 = op->sx32;
    L0.sy32 = op->sy32;
    L0.sz32 = op->sz32;
    op->mg_nlev = n;  // from here mg_free releases whatever was allocated
    for (int l = 1; l < n; ++l) {
      MgLevel& L = op->mg[l];
      L.g = lv[l];
      const size_t n8 = (size_t)lv[l].N * sizeof(double), n4 = (size_t)lv[l].N * sizeof(float);
      double** d64[] = {&L.D, &L.mu, &L.cx, &L.cy, &L.cz, &L.b0, &L.diag, &L.sd, &L.sx, &L.sy,
                        &L.sz};
      float** d32[] = {&L.sx32, &L.sy32, &L.sz32};
      for (double** p : d64) DOT_HIP(hipMalloc(p, n8));
      for (float** p : d32) DOT_HIP(hipMalloc(p, n4));
    }
    for (int l = 0; l < n; ++l)
      DOT_HIP(hipMalloc(&op->mg[l].sd32, (size_t)lv[l].N * sizeof(float)));
    for (int l = 0; l + 1 < n; ++l) {
      DOT_HIP(hipMalloc(&op->mg[l].q, (size_t)lv[l].N * sizeof(double)));
      DOT_HIP(hipMalloc(&op->mg[l].q32, (size_t)lv[l].N * sizeof(float)));
    }
    DOT_HIP(hipMalloc(&op->mg_flag, sizeof(int)));
  }
  BC6 bc;
  for (int f = 0; f < 6; ++f) bc.f[f] = op->bc[f];
  for (int l = 1; l < n; ++l) {
    MgLevel& F = op->mg[l - 1];
    MgLevel& L = op->mg[l];
    const GridDims& gc = L.g;
    hipLaunchKernelGGL(mg_coarsen_kernel, dim3(nblk(gc.N, 256)), dim3(256), 0, s, F.g, gc, F.D,
                       F.mu, L.D, L.mu);
    DOT_LAUNCH_CHECK();
    hipLaunchKernelGGL(build_coef_kernel, dim3(nblk(gc.N, 256)), dim3(256), 0, s, gc, bc, L.D,
                       L.cx, L.cy, L.cz, L.b0);
    DOT_LAUNCH_CHECK();
    hipLaunchKernelGGL(diag_kernel, dim3(nblk(gc.N, 256)), dim3(256), 0, s, gc, L.cx, L.cy, L.cz,
                       L.b0, L.mu, L.diag, L.sd);
    DOT_LAUNCH_CHECK();
    hipLaunchKernelGGL(scale_kernel, dim3(nblk(gc.N, 256)), dim3(256), 0, s, gc, L.cx, L.cy,
                       L.cz, L.sd, L.sx, L.sy, L.sz, L.sx32, L.sy32, L.sz32);
    DOT_LAUNCH_CHECK();
    hipLaunchKernelGGL(mg_q_kernel, dim3(nblk(F.g.N, 256)), dim3(256), 0, s, F.g, gc, F.sd, L.sd,
                       F.q, F.q32);
    DOT_LAUNCH_CHECK();
  }
  for (int l = 0; l < n; ++l) {
    const MgLevel& L = op->mg[l];
    hipLaunchKernelGGL(mg_round_kernel, dim3(nblk(L.g.N, 256)), dim3(256), 0, s, L.g.N, L.sd,
                       L.sd32);
    DOT_LAUNCH_CHECK();
  }
  // the V-cycle is a valid (positive definite) preconditioner only if every
  // level's diagonal is positive; otherwise the solver falls back to Jacobi
  hipLaunchKernelGGL(mg_flag_clear_kernel, dim3(1), dim3(1), 0, s, op->mg_flag);
  DOT_LAUNCH_CHECK();
  for (int l = 0; l < n; ++l) {
    hipLaunchKernelGGL(mg_check_kernel, dim3(nblk(lv[l].N, 256)), dim3(256), 0, s, lv[l].N,
                       op->mg[l].diag, op->mg_flag);
    DOT_LAUNCH_CHECK();
  }
  DOT_HIP(hipMemcpyAsync(op->pinned, op->mg_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  op->mg_ok = op->pinned[0] == 0;
  return DOT_OK;
}

static int refresh_diag(dot_op* op, const double* mua, hipStream_t s) {
  const GridDims& g = op->g;
  hipLaunchKernelGGL(diag_kernel, dim3(nblk(g.N, 256)), dim3(256), 0, s, g, op->cx, op->cy,
                     op->cz, op->b0, mua, op->diag, op->sd);
  DOT_LAUNCH_CHECK();
  hipLaunchKernelGGL(scale_kernel, dim3(nblk(g.N, 256)), dim3(256), 0, s, g, op->cx, op->cy,
                     op->cz, op->sd, op->sx, op->sy, op->sz, op->sx32, op->sy32, op->sz32);
  DOT_LAUNCH_CHECK();
  // the absorption the diagonal was formed with, for the coarse levels
  if (mua) {
    if (mua != op->mu0)
      DOT_HIP(hipMemcpyAsync(op->mu0, mua, (size_t)g.N * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    DOT_HIP(hipMemsetAsync(op->mu0, 0, (size_t)g.N * sizeof(double), s));
  }
  return mg_refresh(op, s);
}

// ------------------------------------------------------------------ RBF cell lists
// For RBF m, the cells inside its support (r < 1) and inside the Heaviside band
// (|phi - c| <= eps): exactly the cells where some d mu / d p_k of that RBF can
// be nonzero.  Enumerated over the support's bounding box in increasing cell
// index, one block per RBF.
struct BoxK {
  int lo[3], ext[3];
};

__device__ __forceinline__ void rbf_box(const GridDims& g, const double* th, double gamma, int* lo,
                                        int* ext) {
  // the support depends on beta^2 only, so its radius uses |beta| (beta = 0
  // gives an infinite radius: the whole grid)
  const double beta = fabs(th[1]);
  const double R = sqrt(fmax(0.0, 1.0 - gamma * gamma)) / beta;
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    if (a >= g.dim) {
      lo[a] = 0;
      ext[a] = 1;
      continue;
    }
    double a0 = (th[2 + a] - R) / g.h - 0.5;
    double a1 = (th[2 + a] + R) / g.h - 0.5;
    int i0 = (int)ceil(fmax(a0, -1.0));
    int i1 = (int)floor(fmin(a1, (double)n[a]));
    i0 = max(i0, 0);
    i1 = min(i1, n[a] - 1);
    lo[a] = i0;
    ext[a] = max(0, i1 - i0 + 1);
  }
}

// RBF m's bounding box is scanned by kRbfSplit blocks, each a contiguous
// range of the box's cells in increasing cell order: a counting pass, then,
// at offsets from the prefix sums over (RBF, range), a filling pass, so each
// RBF's list comes out in increasing cell order.
constexpr int kRbfSplit = 16;

__device__ __forceinline__ void rbf_range(int64_t box, int s, int64_t* q0, int64_t* q1) {
  int64_t per = (box + kRbfSplit - 1) / kRbfSplit;
  per = (per + 255) / 256 * 256;
  *q0 = std::min<int64_t>(box, per * s);
  *q1 = std::min<int64_t>(box, per * (s + 1));
}

template <bool kFill>
__global__ __launch_bounds__(256) void rbf_cells_kernel(GridDims g, PalsK p,
                                                        const double* __restrict__ theta,
                                                        const double* __restrict__ phi,
                                                        int64_t* __restrict__ counts,
                                                        const int64_t* __restrict__ start,
                                                        int32_t* __restrict__ cells) {
  __shared__ int s_wave[4];
  const int m = blockIdx.x / kRbfSplit, part = blockIdx.x % kRbfSplit;
  const double* th = theta + (int64_t)m * p.stride;
  int lo[3], ext[3];
  rbf_box(g, th, p.gamma, lo, ext);
  const int64_t box = (int64_t)ext[0] * ext[1] * ext[2];
  int64_t q0, q1;
  rbf_range(box, part, &q0, &q1);
  const double beta = th[1], g2 = p.gamma * p.gamma;
  int64_t total = 0;
  int64_t out = kFill ? start[blockIdx.x] : 0;
  for (int64_t base = q0; base < q1; base += 256) {
    const int64_t q = base + threadIdx.x;
    int flag = 0;
    int64_t c = 0;
    if (q < q1) {
      const int ix = (int)(q % ext[0]);
      const int iy = (int)((q / ext[0]) % ext[1]);
      const int iz = (int)(q / ((int64_t)ext[0] * ext[1]));
      const int x = lo[0] + ix, y = lo[1] + iy, z = lo[2] + iz;
      c = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
      const double e0 = (x + 0.5) * g.h - th[2], e1 = (y + 0.5) * g.h - th[3];
      double rho2 = e0 * e0 + e1 * e1;
      if (g.dim == 3) {
        const double e2 = (z + 0.5) * g.h - th[4];
        rho2 += e2 * e2;
      }
      const double r = sqrt(beta * beta * rho2 + g2);
      const double s = phi[c] - p.cutoff;
      flag = (r < 1.0 && fabs(s) <= p.eps) ? 1 : 0;
    }
    int tot;
    const int pos = block_scan_flag256(flag, s_wave, &tot);
    if (kFill && flag) cells[out + pos] = (int32_t)c;
    out += tot;
    total += tot;
    __syncthreads();
  }
  if (!kFill && threadIdx.x == 0) counts[blockIdx.x] = total;
}

}  // namespace dot

using namespace dot;

// ====================================================================== ABI
extern "C" {

int dot_abi_version(void) { return DOT_ABI_VERSION; }

const char* dot_last_error(void) { return dot::g_err; }

int64_t dot_grid_cells(const dot_grid* grid) {
  GridDims g;
  const char* why = "";
  if (validate_grid(grid, &g, &why) != DOT_OK) return -1;
  return g.N;
}

int dot_pals_field(const dot_grid* grid, const dot_pals* pals, const double* theta_dev,
                   double mus_prime, double* mua_dev, double* diff_dev, void* stream) {
  clear_error();
  GridDims g;
  const char* why = "";
  if (validate_grid(grid, &g, &why) != DOT_OK) DOT_FAIL(DOT_EINVAL, "%s", why);
  int rc = validate_pals(pals, g.dim);
  if (rc) return rc;
  if (!theta_dev) DOT_FAIL(DOT_EINVAL, "theta_dev is NULL");
  if (!mua_dev) DOT_FAIL(DOT_EINVAL, "mua_dev is NULL");
  if (diff_dev && !(mus_prime >= 0.0)) DOT_FAIL(DOT_EINVAL, "mus_prime must be >= 0");
  return launch_pals(g, pals, theta_dev, mus_prime, mua_dev, diff_dev, nullptr,
                     as_stream(stream));
}

int dot_build_operator(const dot_grid* grid, const double* D_dev, void* stream, dot_op** out) {
  clear_error();
  GridDims g;
  const char* why = "";
  if (validate_grid(grid, &g, &why) != DOT_OK) DOT_FAIL(DOT_EINVAL, "%s", why);
  if (!D_dev) DOT_FAIL(DOT_EINVAL, "D_dev is NULL");
  if (!out) DOT_FAIL(DOT_EINVAL, "out is NULL");
  *out = nullptr;
  hipStream_t s = as_stream(stream);
  dot_op* op = new dot_op();
  op->g = g;
  for (int f = 0; f < 6; ++f) op->bc[f] = (f < 2 * g.dim) ? grid->bc[f] : DOT_BC_DIRICHLET;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  op->device = dev;
  const size_t n8 = (size_t)g.N * sizeof(double), n4 = (size_t)g.N * sizeof(float);
  double** d64[] = {&op->cx, &op->cy, &op->cz, &op->b0, &op->diag, &op->sd,
                    &op->sx, &op->sy, &op->sz, &op->phi, &op->D0, &op->mu0};
  float** d32[] = {&op->sx32, &op->sy32, &op->sz32};
  for (double** p : d64)
    if (e == hipSuccess) e = hipMalloc(p, n8);
  for (float** p : d32)
    if (e == hipSuccess) e = hipMalloc(p, n4);
  if (e == hipSuccess) e = hipMalloc(&op->small_dev, 64 * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc(&op->pinned, kPinnedInts * sizeof(int32_t), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc(&op->pinned_d, 64 * sizeof(double), hipHostMallocDefault);
  for (int i = 0; i < 2; ++i)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&op->poll_ev[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&op->band_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&op->lists_ev, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&op->pinned_band, sizeof(int64_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error("device allocation failed: %s", hipGetErrorString(e));
    dot_destroy_operator(op);
    return e == hipErrorOutOfMemory ? DOT_ENOMEM : DOT_EHIP;
  }
  BC6 bc;
  for (int f = 0; f < 6; ++f) bc.f[f] = op->bc[f];
  hipLaunchKernelGGL(build_coef_kernel, dim3(nblk(g.N, 256)), dim3(256), 0, s, g, bc, D_dev,
                     op->cx, op->cy, op->cz, op->b0);
  int rc = DOT_OK;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(op->D0, D_dev, n8, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) rc = refresh_diag(op, nullptr, s);
  if (e != hipSuccess || rc != DOT_OK) {
    if (e != hipSuccess) set_error("build_coef_kernel: %s", hipGetErrorString(e));
    dot_destroy_operator(op);
    return DOT_EHIP;
  }
  *out = op;
  return DOT_OK;
}

int dot_destroy_operator(dot_op* op) {
  if (!op) return DOT_OK;
  (void)hipDeviceSynchronize();
  destroy_profile(op);
  void* ptrs[] = {op->cx,        op->cy,         op->cz,          op->b0,        op->diag,
                  op->sd,        op->sx,         op->sy,          op->sz,        op->sx32,
                  op->sy32,      op->sz32,       op->phi,         op->theta,     op->pair_cell,
                  op->rbf_start, op->chunk_rbf,  op->chunk_begin, op->rbf_chunk0, op->small_dev,
                  op->pair_g,    op->pair_g32,   op->pair_band,   op->band_idx,   op->band_cells,
                  op->band_part, op->D0,         op->mu0,         op->rbf_sub,
                  op->Dbuild,    op->vrow_cell,  op->vrow_nbr,    op->vrow_w,    op->vpair_band,
                  op->vpair_g,   op->vpair_g32,  op->vchunk_begin, op->vrbf_chunk0};
  for (auto& e : op->cell_lists)
    if (e.dev) (void)hipFree(e.dev);
  mg_free(op);
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (op->pinned) (void)hipHostFree(op->pinned);
  if (op->pinned_band) (void)hipHostFree(op->pinned_band);
  if (op->stage) (void)hipHostFree(op->stage);
  if (op->band_ev) (void)hipEventDestroy(op->band_ev);
  if (op->lists_ev) (void)hipEventDestroy(op->lists_ev);
  if (op->pinned_d) (void)hipHostFree(op->pinned_d);
  for (hipEvent_t ev : op->poll_ev)
    if (ev) (void)hipEventDestroy(ev);
  delete op;
  return DOT_OK;
}

int64_t dot_operator_cells(const dot_op* op) { return op ? op->g.N : -1; }

int64_t dot_pals_pairs(const dot_op* op) { return (op && op->have_pals) ? op->n_pairs : -1; }

int64_t dot_pals_band_cells(const dot_op* op) {
  return (op && op->have_pals) ? band_count(const_cast<dot_op*>(op)) : -1;
}

int dot_set_mua(dot_op* op, const double* mua_dev, void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  if (!mua_dev) DOT_FAIL(DOT_EINVAL, "mua_dev is NULL");
  op->have_pals = false;
  const int rc = leave_diffusion_mode(op, as_stream(stream));
  if (rc) return rc;
  return refresh_diag(op, mua_dev, as_stream(stream));
}

}  // extern "C"

static int pals_state(dot_op* op, const dot_pals* pals, const double* theta_dev, double* mua_dev,
                      bool diffusion, double mus_in, double mus_out, double* diff_dev,
                      hipStream_t s);

extern "C" {

int dot_pals_mua(dot_op* op, const dot_pals* pals, const double* theta_dev, double* mua_dev,
                 void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  int rc = validate_pals(pals, op->g.dim);
  if (rc) return rc;
  if (!theta_dev) DOT_FAIL(DOT_EINVAL, "theta_dev is NULL");
  return pals_state(op, pals, theta_dev, mua_dev, false, 0.0, 0.0, nullptr, as_stream(stream));
}

int dot_pals_mua_diffusion(dot_op* op, const dot_pals* pals, double mus_in, double mus_out,
                           const double* theta_dev, double* mua_dev, double* diff_dev,
                           void* stream) {
  clear_error();
  if (!op) DOT_FAIL(DOT_EINVAL, "op is NULL");
  int rc = validate_pals(pals, op->g.dim);
  if (rc) return rc;
  if (!theta_dev) DOT_FAIL(DOT_EINVAL, "theta_dev is NULL");
  if (!(pals->mu_in != pals->mu_out))
    DOT_FAIL(DOT_EINVAL, "diffusion mode needs an absorption contrast (mu_in != mu_out)");
  if (!std::isfinite(mus_in) || !std::isfinite(mus_out) || mus_in < 0.0 || mus_out < 0.0)
    DOT_FAIL(DOT_EINVAL, "mus_in and mus_out must be finite and >= 0");
  if (!(pals->mu_in + mus_in > 0.0) || !(pals->mu_out + mus_out > 0.0))
    DOT_FAIL(DOT_EINVAL, "mu + mu_s must be positive inside and outside");
  return pals_state(op, pals, theta_dev, mua_dev, true, mus_in, mus_out, diff_dev,
                    as_stream(stream));
}

}  // extern "C"

static int pals_state(dot_op* op, const dot_pals* pals, const double* theta_dev, double* mua_dev,
                      bool diffusion, double mus_in, double mus_out, double* diff_dev,
                      hipStream_t s) {
  int rc = DOT_OK;
  const GridDims& g = op->g;
  const int m0 = pals->m0, stride = 2 + g.dim;
  // keep a copy of theta
  if ((int64_t)m0 * stride > op->theta_cap) {
    if (op->theta) DOT_HIP(hipFree(op->theta));
    op->theta = nullptr;
    op->theta_cap = 0;
    DOT_HIP(hipMalloc(&op->theta, (size_t)m0 * stride * sizeof(double)));
    op->theta_cap = (int64_t)m0 * stride;
  }
  DOT_HIP(hipMemcpyAsync(op->theta, theta_dev, (size_t)m0 * stride * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  // mu and phi, then (diffusion mode) D(theta) and the face coefficients,
  // then the diagonal.  Without a caller buffer, mu is written into the
  // handle's absorption array (kept for the multigrid levels).
  double* tmp_mu = mua_dev ? mua_dev : op->mu0;
  rc = launch_pals(g, pals, op->theta, 0.0, tmp_mu, nullptr, op->phi, s);
  if (rc) return rc;
  if (diffusion) {
    if (!op->Dbuild) {
      DOT_HIP(hipMalloc(&op->Dbuild, (size_t)g.N * sizeof(double)));
      DOT_HIP(hipMemcpyAsync(op->Dbuild, op->D0, (size_t)g.N * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    } else if (!op->diff_mode) {
      DOT_HIP(hipMemcpyAsync(op->Dbuild, op->D0, (size_t)g.N * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    }
    PalsK pk{pals->mu_in, pals->mu_out, pals->cutoff, pals->eps, pals->gamma, m0, g.dim, stride};
    hipLaunchKernelGGL(diff_from_phi_kernel, dim3(nblk(g.N, 256)), dim3(256), 0, s, g, pk, mus_in,
                       mus_out, op->phi, op->D0);
    DOT_LAUNCH_CHECK();
    op->diff_mode = true;
    op->mus_in = mus_in;
    op->mus_out = mus_out;
    rc = rebuild_coefficients(op, s);
    if (rc) return rc;
    if (diff_dev)
      DOT_HIP(hipMemcpyAsync(diff_dev, op->D0, (size_t)g.N * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
  } else {
    rc = leave_diffusion_mode(op, s);
    if (rc) return rc;
  }
  rc = refresh_diag(op, tmp_mu, s);
  if (rc) return rc;
  // per-RBF cell lists
  if (m0 + 1 > op->rbf_cap) {
    if (op->rbf_start) DOT_HIP(hipFree(op->rbf_start));
    if (op->rbf_chunk0) DOT_HIP(hipFree(op->rbf_chunk0));
    op->rbf_start = nullptr;
    op->rbf_chunk0 = nullptr;
    op->rbf_cap = 0;
    DOT_HIP(hipMalloc(&op->rbf_start, (size_t)(m0 + 1) * sizeof(int64_t)));
    DOT_HIP(hipMalloc(&op->rbf_chunk0, (size_t)(m0 + 1) * sizeof(int32_t)));
    op->rbf_cap = m0 + 1;
  }
  PalsK p{pals->mu_in, pals->mu_out, pals->cutoff, pals->eps, pals->gamma, m0, g.dim, stride};
  const int64_t nsub = (int64_t)m0 * kRbfSplit;
  if (nsub > op->rbf_sub_cap) {
    if (op->rbf_sub) DOT_HIP(hipFree(op->rbf_sub));
    op->rbf_sub = nullptr;
    op->rbf_sub_cap = 0;
    DOT_HIP(hipMalloc(&op->rbf_sub, (size_t)nsub * sizeof(int64_t)));
    op->rbf_sub_cap = nsub;
  }
  hipLaunchKernelGGL(rbf_cells_kernel<false>, dim3((unsigned)nsub), dim3(256), 0, s, g, p, op->theta,
                     op->phi, op->rbf_sub, nullptr, nullptr);
  DOT_LAUNCH_CHECK();
  std::vector<int64_t> sub(nsub, 0);
  DOT_HIP(hipMemcpyAsync(sub.data(), op->rbf_sub, (size_t)nsub * sizeof(int64_t),
                         hipMemcpyDeviceToHost, s));
  DOT_HIP(hipStreamSynchronize(s));
  // RBF starts, and each range's start, in (RBF, range) order
  std::vector<int64_t> start(m0 + 1, 0), sub_start(nsub, 0);
  for (int m = 0; m < m0; ++m) {
    int64_t at = start[m];
    for (int r = 0; r < kRbfSplit; ++r) {
      sub_start[(int64_t)m * kRbfSplit + r] = at;
      at += sub[(int64_t)m * kRbfSplit + r];
    }
    start[m + 1] = at;
  }
  const int64_t total = start[m0];
  // chunk table: each RBF's list split into chunks of at most DOT_PAIR_CHUNK cells
  const int64_t kPairChunk = DOT_PAIR_CHUNK;
  std::vector<int32_t> chunk_rbf;
  std::vector<int64_t> chunk_begin;
  std::vector<int32_t> rbf_chunk0(m0 + 1, 0);
  for (int m = 0; m < m0; ++m) {
    rbf_chunk0[m] = (int32_t)chunk_rbf.size();
    for (int64_t b = start[m]; b < start[m + 1]; b += kPairChunk) {
      chunk_rbf.push_back(m);
      chunk_begin.push_back(b);
    }
  }
  rbf_chunk0[m0] = (int32_t)chunk_rbf.size();
  const int64_t nch = (int64_t)chunk_rbf.size();
  if (std::max<int64_t>(total, 1) > op->pair_cap) {
    if (op->pair_cell) DOT_HIP(hipFree(op->pair_cell));
    op->pair_cell = nullptr;
    op->pair_cap = 0;
    const int64_t cap = std::max<int64_t>(total + total / 8, 1024);
    DOT_HIP(hipMalloc(&op->pair_cell, (size_t)cap * sizeof(int32_t)));
    op->pair_cap = cap;
  }
  if (std::max<int64_t>(nch, 1) > op->chunk_cap) {
    if (op->chunk_rbf) DOT_HIP(hipFree(op->chunk_rbf));
    if (op->chunk_begin) DOT_HIP(hipFree(op->chunk_begin));
    op->chunk_rbf = nullptr;
    op->chunk_begin = nullptr;
    op->chunk_cap = 0;
    const int64_t cap = std::max<int64_t>(nch + nch / 8, 256);
    DOT_HIP(hipMalloc(&op->chunk_rbf, (size_t)cap * sizeof(int32_t)));
    DOT_HIP(hipMalloc(&op->chunk_begin, (size_t)(cap + 1) * sizeof(int64_t)));
    op->chunk_cap = cap;
  }
  chunk_begin.push_back(total);
  // the tables go up through the pinned staging buffer: the copies do not
  // wait for the host, and the call returns without waiting for them
  if (op->lists_pending) DOT_HIP(hipEventSynchronize(op->lists_ev));
  op->lists_pending = false;
  size_t sz[5] = {(size_t)(m0 + 1) * sizeof(int64_t), (size_t)(m0 + 1) * sizeof(int32_t),
                  (size_t)nch * sizeof(int32_t), (size_t)(nch + 1) * sizeof(int64_t),
                  (size_t)nsub * sizeof(int64_t)};
  const void* src[5] = {start.data(), rbf_chunk0.data(), chunk_rbf.data(), chunk_begin.data(),
                        sub_start.data()};
  void* dst[5] = {op->rbf_start, op->rbf_chunk0, op->chunk_rbf, op->chunk_begin, op->rbf_sub};
  size_t at[5], need = 0;
  for (int i = 0; i < 5; ++i) {
    at[i] = need;
    need += (sz[i] + 255) & ~(size_t)255;
  }
  if (need > op->stage_cap) {
    if (op->stage) DOT_HIP(hipHostFree(op->stage));
    op->stage = nullptr;
    op->stage_cap = 0;
    const size_t cap = std::max<size_t>(need + need / 4, (size_t)1 << 16);
    DOT_HIP(hipHostMalloc((void**)&op->stage, cap, hipHostMallocDefault));
    op->stage_cap = cap;
  }
  for (int i = 0; i < 5; ++i) {
    if (sz[i] == 0) continue;
    std::memcpy(op->stage + at[i], src[i], sz[i]);
    DOT_HIP(hipMemcpyAsync(dst[i], op->stage + at[i], sz[i], hipMemcpyHostToDevice, s));
  }
  DOT_HIP(hipEventRecord(op->lists_ev, s));
  op->lists_pending = true;
  hipLaunchKernelGGL(rbf_cells_kernel<true>, dim3((unsigned)nsub), dim3(256), 0, s, g, p, op->theta,
                     op->phi, nullptr, op->rbf_sub, op->pair_cell);
  DOT_LAUNCH_CHECK();
  op->n_pairs = total;
  op->n_chunks = nch;
  op->pals = *pals;
  rc = jac_prepare(op, s);
  if (rc) return rc;
  if (op->diff_mode) {
    rc = jac_prepare_faces(op, s);
    if (rc) return rc;
  }
  op->have_pals = true;
  return DOT_OK;
}
