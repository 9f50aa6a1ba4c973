/*
 * dotpath: C ABI of the MI355X (gfx950) library for the hot path of randomized
 * nonlinear inversion in diffuse optical tomography with random and optimized
 * simultaneous sources and detectors (Aslan, de Sturler, Kilmer).
 *
 * Model (Section 2, eq. PDE at zero frequency):
 *     -div(D grad eta) + mu(x; p) eta = g  on a box,
 *     eta = 0 on Dirichlet faces, 0.25 eta + (D/2) d eta/d xi = 0 on Robin faces,
 * discretized by a symmetric cell-centred finite-volume scheme on a uniform
 * grid of spacing h = 1 / n_x (cells are cubes):
 *     interior face       T = h^(d-2) 2 D_c D_c' / (D_c + D_c')
 *     Dirichlet face      T = h^(d-2) 2 D_c
 *     Robin face          T = h^(d-1) 2 D_c / (h + 4 D_c)
 *     (A eta)_c = sum_faces T (eta_c - eta_nbr) + sum_bdry T eta_c + h^d mu_c eta_c.
 * A is symmetric positive definite, so A^T = A.  Cells are numbered
 * c = i + n_x (j + n_y k).  Absorption mu comes from the parametric level set
 * (PaLS) phi = sum_j alpha_j psi(sqrt(beta_j^2 |x - chi_j|^2 + gamma^2)) with
 * the Wendland psi_{2,1}(r) = (1-r)^4 (4r+1) and
 * mu = mu_out + (mu_in - mu_out) H_eps(phi - c), where
 * H_eps(s) = (1 + s/eps + sin(pi s/eps)/pi)/2 on |s| <= eps (0 below, 1 above).
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers (hipMalloc'd or torch tensors),
 *     pointers named *_host are host pointers.  Multi-column arrays are
 *     column-major with leading dimension equal to the row count (an N x k
 *     field block has element (c, j) at c + N j).  All floating point data is
 *     IEEE binary64 unless stated.
 *   - The caller owns every data buffer.  The library allocates device memory
 *     only inside dot_build_operator (coefficients, level set, small state)
 *     and dot_pals_mua (per-RBF cell lists and per-pair data); dot_solve_multi_rhs,
 *     dot_jacobian and dot_grad_misfit use the caller's workspace.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it; calls that return host values synchronize it.
 *   - Arguments are validated on the host before any HIP call; on error the
 *     call returns a negative code and dot_last_error() explains it.  Outputs
 *     are undefined after an error.
 *   - A handle is not thread-safe; separate handles are independent.
 */
#ifndef DOTPATH_H
#define DOTPATH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DOT_ABI_VERSION 2

/* return codes */
#define DOT_OK 0
#define DOT_NOT_CONVERGED 1   /* solve hit max_iter; outputs valid, info.relres filled */
#define DOT_EINVAL (-1)       /* invalid argument */
#define DOT_ENOMEM (-2)       /* workspace too small or device allocation failed */
#define DOT_EHIP (-3)         /* HIP runtime error */
#define DOT_EBREAKDOWN (-4)   /* CG breakdown: p^T A p <= 0 or r^T M^-1 r <= 0 (not SPD) */
#define DOT_ENONFINITE (-5)   /* NaN or Inf in the data */

/* boundary codes per face */
#define DOT_BC_DIRICHLET 0
#define DOT_BC_ROBIN 1

/* solve precision */
#define DOT_FP64 0    /* PCG in binary64 */
#define DOT_MIXED 1   /* binary32 PCG inside binary64 iterative refinement */

/* solve preconditioner */
#define DOT_PRECOND_AUTO 0    /* multigrid where the grid has a hierarchy, else Jacobi */
#define DOT_PRECOND_JACOBI 1  /* Jacobi (the symmetric diagonal scaling alone) */
#define DOT_PRECOND_MG 2      /* geometric multigrid V-cycle (DOT_EINVAL without a hierarchy) */
#define DOT_PRECOND_MG_F32 3  /* the same; with DOT_MIXED its work vectors are kept in binary32
                                 instead of bfloat16 (AUTO and MG), for comparison */

/* Jacobian precision */
#define DOT_JAC_FP64 0        /* binary64 products and sums */
#define DOT_JAC_SPLIT_BF16 1  /* hi/lo bfloat16 operands, 3 MFMA products, fp32 accumulate:
                                 each product carries a relative error up to about 2^-16,
                                 so J_s is within 2e-5 relative Frobenius error of binary64
                                 (a faster option, not within the 1e-6 bound) */
#define DOT_JAC_SPLIT_BF16X3 2  /* hi/mid/lo bfloat16 operands, 6 MFMA products: binary32-level
                                 operands, within 1e-6 relative Frobenius error of binary64 */

/* PaLS parameter activity bits */
#define DOT_ACT_ALPHA 1u
#define DOT_ACT_BETA 2u
#define DOT_ACT_CHI 4u

typedef struct dot_grid {
  int dim;     /* 2 or 3 */
  int n[3];    /* cells per axis (n[2] ignored when dim == 2) */
  int bc[6];   /* faces -x,+x,-y,+y,-z,+z: DOT_BC_DIRICHLET or DOT_BC_ROBIN (z ignored in 2D) */
} dot_grid;

typedef struct dot_pals {
  int m0;            /* number of RBFs; theta is m0 x (2 + dim), RBF-major [alpha, beta, chi] */
  unsigned active;   /* DOT_ACT_* bits: which per-RBF parameters are unknowns */
  double mu_in, mu_out, cutoff, eps, gamma;
} dot_pals;

/* most columns one solve call accepts */
#define DOT_MAX_COLUMNS 4096

typedef struct dot_solve_opts {
  double rtol;        /* per-column target ||b - A x||_2 / ||b||_2 */
  int max_iter;       /* CG iterations (binary32 iterations for DOT_MIXED) */
  int precision;      /* DOT_FP64 or DOT_MIXED */
  double inner_rtol;  /* DOT_MIXED: factor by which the binary32 residual of a column must
                         drop before its correction is folded into x in binary64 and its
                         residual is replaced by the binary64 b - A x (e.g. 0.1) */
  int check_every;    /* iterations between host polls of the column flags (>= 1) */
  int precond;        /* DOT_PRECOND_AUTO, _JACOBI, _MG or _MG_F32 */
} dot_solve_opts;

typedef struct dot_solve_info {
  int iters_max;      /* out: max over columns of CG iterations */
  int outer;          /* out: binary64 residual updates (DOT_MIXED), 0 for DOT_FP64 */
  int32_t* iters_host;   /* in: NULL or host array [k]; out: iterations per column */
  double* relres_host;   /* in: NULL or host array [k]; out: final true relative residual
                            ||b - A x|| / ||b|| per column, recomputed in binary64 */
} dot_solve_info;

typedef struct dot_op dot_op;

/* ABI version (DOT_ABI_VERSION). */
int dot_abi_version(void);

/* Thread-local description of the last error ("" if none). */
const char* dot_last_error(void);

/* Number of cells N of a grid descriptor, or -1 if it is invalid (at most
 * 2^29 cells: the solver addresses one binary64 column with 32-bit offsets). */
int64_t dot_grid_cells(const dot_grid* grid);

/*
 * PaLS field on a grid, without an operator (Section 2, PaLS definition and
 * eq. absorption const): mua_dev[c] = mu(x_c; theta) at cell centres
 * x_c = ((i + 1/2) h, ...).  If diff_dev is not NULL it also receives the
 * diffusion coefficient D = 1 / (3 (mu + mus_prime)) of the diffusion
 * approximation.  theta_dev: m0 x (2 + dim) device array, RBF-major.
 */
int dot_pals_field(const dot_grid* grid, const dot_pals* pals, const double* theta_dev,
                   double mus_prime, double* mua_dev, double* diff_dev, void* stream);

/*
 * Build the frozen part of A from the diffusion coefficient D_dev[N] (the
 * face coefficients T and the boundary diagonal).  The absorption starts at
 * zero; set it with dot_pals_mua or dot_set_mua.  *out receives a handle that
 * owns its device arrays; free it with dot_destroy_operator.
 */
int dot_build_operator(const dot_grid* grid, const double* D_dev, void* stream, dot_op** out);

/* Free a handle (NULL is accepted).  Synchronizes the device. */
int dot_destroy_operator(dot_op* op);

/* Number of cells of the operator's grid. */
int64_t dot_operator_cells(const dot_op* op);

/* Set the absorption of A from an explicit field mua_dev[N] (diagonal h^d mu). */
int dot_set_mua(dot_op* op, const double* mua_dev, void* stream);

/*
 * Set A(theta): evaluate the PaLS absorption at every cell, update the
 * diagonal, and keep on the handle what dot_jacobian and dot_grad_misfit
 * need at this theta (a copy of theta and the descriptor, the level set phi,
 * per-RBF lists of cells where d mu / d p is nonzero, h^d d mu / d p of each
 * (RBF, cell) pair, and the numbering of all listed cells in cell order,
 * which the contraction uses to read the fields as packed rows).  Allocates
 * device memory for these when they grow.  If mua_dev is not NULL it
 * receives mu.  Synchronizes the stream.
 */
int dot_pals_mua(dot_op* op, const dot_pals* pals, const double* theta_dev, double* mua_dev,
                 void* stream);

/*
 * Set A(theta) with the diffusion coefficient an unknown as well (Section
 * 3.3, last paragraph: dA/dp_k then has 5 (2D) or 7 (3D) diagonals).  The
 * level set describes an anomaly in both optical properties:
 * mu = mu_out + (mu_in - mu_out) H, mu_s = mus_out + (mus_in - mus_out) H with
 * H = H_eps(phi - cutoff), and D = 1 / (3 (mu + mu_s)) (the diffusion
 * approximation) replaces the D given to dot_build_operator.  The face
 * coefficients, diagonal and multigrid hierarchy are rebuilt; dot_jacobian
 * and dot_grad_misfit then contract with the full dA/dp_k (the face terms
 * dT_f/dp_k (z_c - z_c')(u_c - u_c') through dD/dp_k = -3 D^2 (mu_in - mu_out +
 * mus_in - mus_out) delta_eps(phi - cutoff) d phi / d p_k, besides the diagonal
 * h^d d mu / d p_k), with the same parameters and band lists.  Needs
 * mu_in != mu_out.  mua_dev and diff_dev (may be NULL) receive mu and D.
 * dot_pals_mua and dot_set_mua return to the diffusion given at build time;
 * dot_dadp_apply and dot_grad_misfit_noalloc cover the absorption-only model
 * and return DOT_EINVAL in this mode.  Synchronizes the stream.
 */
int dot_pals_mua_diffusion(dot_op* op, const dot_pals* pals, double mus_in, double mus_out,
                           const double* theta_dev, double* mua_dev, double* diff_dev,
                           void* stream);

/* Number of (RBF, cell) pairs in the band lists of the last dot_pals_mua call:
 * the nonzeros of G = h^d d mu / d p per active parameter kind, i.e. the cells
 * the contraction visits summed over RBFs (-1 if no PaLS state). */
int64_t dot_pals_pairs(const dot_op* op);

/* Number of distinct cells in the band lists of the last dot_pals_mua call:
 * the rows of U and Z the contraction reads (-1 if no PaLS state). */
int64_t dot_pals_band_cells(const dot_op* op);

/* Y = A X for k columns (X_dev and Y_dev are N x k and must not overlap). */
int dot_apply(dot_op* op, int k, const double* X_dev, double* Y_dev, void* stream);

/*
 * Simultaneous sources (Section 3.1, eq. Rw; Section 3.3): rhs_dev (N x k) =
 * B W, i.e. column l is sum_i weights_dev[i + n_pts l] e_{cells_host[i]}.
 * cells_host: n_pts cell indices in [0, N) (host array, read before the
 * call returns; repeated cells add, in the order given).  The handle keeps
 * device copies of the last few distinct cell lists, so a list seen before
 * costs no copy and the call returns without waiting for the GPU; a new list
 * is copied after the stream's pending work.  Used for C V with the detector
 * cells and V.
 */
int dot_form_rhs(dot_op* op, int n_pts, const int32_t* cells_host, int k,
                 const double* weights_dev, double* rhs_dev, void* stream);

/* Workspace bytes for dot_solve_multi_rhs with k columns at the given precision. */
size_t dot_solve_workspace_bytes(const dot_op* op, int k, int precision);

/*
 * Multi-right-hand-side solve A X = RHS (trans = 0) or A^T X = RHS (trans =
 * 1; identical here since A is symmetric), Section 3.3: the forward fields
 * z_i of A z_i = B w_i and the adjoint fields y_j of A^T y_j = C v_j.
 * Preconditioned CG from x0 = 0 per column until ||b - A x||_2 <= rtol
 * ||b||_2, on the symmetrically Jacobi-scaled system.  Preconditioner
 * (opts.precond): a geometric multigrid V-cycle on 2D and 3D grids whose
 * sides all have at least 5 cells (2 x 2 x 2 aggregation, 2 x 2 in 2D, each
 * side halved rounding up while every coarse side keeps at least 3 cells;
 * the same finite-volume operator on every level, h = 1 / n_x, with D and
 * mu averaged over the children of an aggregate, damped
 * Jacobi smoothing with w = 0.85, 2 steps each way on the finest level, 3 on
 * the next and 5 below, piecewise-constant transfers, 8 damped Jacobi steps
 * on the coarsest level), or the Jacobi scaling alone.  The
 * hierarchy is rebuilt by dot_build_operator, dot_set_mua and dot_pals_mua.
 * DOT_MIXED runs the CG recurrences (stencil,
 * vectors) in binary32 inside binary64 iterative refinement: the binary32
 * correction is folded into x in binary64, and the residual b - A x is
 * recomputed in binary64 and replaces the binary32 one whenever the latter
 * has dropped by inner_rtol (the search direction is kept); convergence is
 * decided on the binary64 residual; the V-cycle then runs in binary32
 * arithmetic with its work vectors (every level's iterates, the coarse
 * right-hand sides and corrections) stored in bfloat16, rounded to nearest
 * even (DOT_PRECOND_MG_F32: stored in binary32); its input r and output z
 * stay binary32.  The preconditioner only steers CG: the accuracy is that
 * of the binary64 residual test.
 * The host reads the column flags every check_every iterations, one such
 * poll late: iterations launched after the last column converged run with
 * every column masked off.
 * rhs_dev, x_dev: N x k, must not overlap.  work_dev: >= the size from
 * dot_solve_workspace_bytes, 256-byte aligned.  Synchronizes the stream.
 * Returns DOT_OK, DOT_NOT_CONVERGED (outputs valid), or an error.
 */
int dot_solve_multi_rhs(dot_op* op, int trans, int k, const double* rhs_dev, double* x_dev,
                        const dot_solve_opts* opts, void* work_dev, size_t work_bytes,
                        dot_solve_info* info, void* stream);

/*
 * Frequency-domain multi-right-hand-side solve (Section 2, eq. PDE with
 * omega > 0, and eq. compmeas): (A + i kappa E) X = RHS with kappa =
 * omega / nu and E = h^d I, the cell volumes (every unknown of the
 * cell-centred scheme is a cell average, so no row of E is zero; the zero
 * rows of the paper's E belong to the boundary nodes of its vertex-centred
 * scheme).  A + i kappa E is complex symmetric, so the adjoint solves of
 * Section 3.3 use the same call.  Conjugate orthogonal CG (COCG) from x0 = 0
 * on the symmetrically scaled system, preconditioned by the real multigrid
 * V-cycle of dot_solve_multi_rhs applied to the real and imaginary parts (or
 * the Jacobi scaling alone), per column until ||b - A_w x||_2 <= rtol
 * ||b||_2 (conjugated norms).  Complex N x k blocks are N x 2k binary64
 * arrays: real parts in columns 0 .. k-1, imaginary parts in k .. 2k-1.
 * opts: rtol, max_iter, check_every and precond as for dot_solve_multi_rhs.
 * opts.precision: DOT_FP64, or DOT_MIXED, which runs the V-cycle in
 * binary32 (binary32 work vectors) on a binary32 copy of r / ||b||; COCG
 * itself and the convergence test stay binary64 either way, and with Jacobi
 * preconditioning the two are the same.
 * The workspace size covers both.  info.relres_host (k values) receives the true
 * relative residual recomputed in binary64; DOT_NOT_CONVERGED when one
 * exceeds 1.01 rtol.  kappa = 0 solves the real system.  k <= 2048.
 * Synchronizes the stream.
 */
size_t dot_solve_complex_workspace_bytes(const dot_op* op, int k, int precond);
int dot_solve_complex(dot_op* op, double kappa, int k, const double* rhs_dev, double* x_dev,
                      const dot_solve_opts* opts, void* work_dev, size_t work_bytes,
                      dot_solve_info* info, void* stream);

/* Levels of the multigrid hierarchy the solver uses for this operator, or 0
 * when it preconditions with Jacobi (a side shorter than 5 cells, or a level
 * whose diagonal is not positive). */
int dot_multigrid_levels(const dot_op* op);

/* Algorithmic HBM bytes per column of one V-cycle of the solver's
 * preconditioner in the given precision (DOT_FP64: binary64 vectors,
 * DOT_MIXED: binary32 input and output, bfloat16 work vectors): every vector
 * each level's kernels must read or write
 * once (right-hand sides, iterates, coarse values, results), the operator's
 * coefficients not counted; 0 without a hierarchy.  For roofline figures. */
double dot_multigrid_cycle_bytes(const dot_op* op, int precision);

/* Workspace bytes for dot_multigrid_apply with k columns (0 without a hierarchy). */
size_t dot_multigrid_workspace_bytes(const dot_op* op, int k);

/*
 * One binary64 V-cycle of the solver's preconditioner as an approximate
 * inverse of A: Z_dev = S^-1 V(S^-1 R_dev), S = diag(A)^(1/2), V the V-cycle on
 * the scaled system (symmetric positive definite).  R_dev, Z_dev: N x k.
 * DOT_EINVAL without a hierarchy.
 */
int dot_multigrid_apply(dot_op* op, int k, const double* R_dev, double* Z_dev, void* work_dev,
                        size_t work_bytes, void* stream);

/*
 * Sampled residual and misfit (Section 3.3, eq. EsTResidual; Thm 3.1):
 * Rs_dev (l_d x l_s) = V^T (C^T U - DW), f = 1/2 ||Rs||_F^2 written to *f_host.
 * det_host: n_d detector cells; U_dev: N x l_s forward fields; V_dev: n_d x l_d;
 * DW_dev: n_d x l_s (data times W).  Synchronizes the stream.
 */
int dot_sampled_misfit(dot_op* op, int n_d, const int32_t* det_host, int l_s, const double* U_dev,
                       int l_d, const double* V_dev, const double* DW_dev, double* Rs_dev,
                       double* f_host, void* stream);

/* Workspace bytes for dot_jacobian / dot_grad_misfit (after dot_pals_mua). */
size_t dot_jacobian_workspace_bytes(const dot_op* op, int l_s, int l_d);

/*
 * Sampled Jacobian (Section 3.3, eq. Jacobian kth column, sign of eq.
 * Jacobiancomp): Js_dev[(j + l_d i) + (l_s l_d) k] = -sum_c Z[c,j] U[c,i]
 * h^d d mu_c / d p_k, for the parameters of the last dot_pals_mua call
 * (n_p = m0 x number of active bits; parameter k = rbf * n_act + local
 * index in the order alpha, beta, chi_1..chi_d).  Only cells where
 * d mu / d p_k is nonzero are visited.  precision: DOT_JAC_FP64 (binary64
 * throughout, on the binary64 matrix cores), DOT_JAC_SPLIT_BF16 or
 * DOT_JAC_SPLIT_BF16X3 (operands rounded to binary32 and split into 2 or 3
 * bfloat16 parts, products on the matrix cores with binary32 accumulation
 * over 512-cell runs, binary64 sums across runs and chunks).  U_dev: N x l_s,
 * Z_dev: N x l_d, l_s, l_d <= DOT_MAX_COLUMNS.  Samples larger than the
 * matrix-core kernels hold in one pass (binary64: ceil(l_s / 16)
 * ceil(l_d n_act / 16) <= 64 and l_s + l_d <= 128; split forms: l_s, l_d <=
 * 64) run as tiles of at most 64 sources and as many detectors as fit, each
 * written into its rows of Js_dev; with l_s = n_s and l_d = n_d (W, V
 * identities) this is the full Jacobian J of eq. Jtensor.  The workspace
 * holds one tile's per-chunk partial blocks and packed rows of U and Z at
 * the listed cells (for the split forms U already split into its bfloat16
 * parts).
 */
int dot_jacobian(dot_op* op, int l_s, const double* U_dev, int l_d, const double* Z_dev,
                 int precision, double* Js_dev, void* work_dev, size_t work_bytes, void* stream);

/*
 * Derivative of A(p) along parameter directions, applied to fields (Section
 * 3.3: with the absorption the unknown, dA/dp_k = h^d diag(d mu / d p_k)):
 * Y_dev[:, j] = (sum_k Theta_dev[k, j] dA/dp_k) X_dev[:, j] for j < k, at the
 * parameters of the last dot_pals_mua call.  Theta_dev: n_p x k column-major
 * (one direction per column, parameter order as in dot_jacobian); X_dev,
 * Y_dev: N x k, must not overlap; Y is zero outside the level-set band.
 * This is the matrix-free product with the Jacobian: for u = A^-1 b and
 * z = A^-T c, c^T A^-1 (dA/d theta) A^-1 b = z^T Y(theta, u), so a sketch
 * J (w kron theta) needs one forward and one adjoint solve.
 */
int dot_dadp_apply(dot_op* op, int k, const double* Theta_dev, const double* X_dev, double* Y_dev,
                 void* stream);

/*
 * Gradient of f = 1/2 ||Rs||_F^2 (Section 3.1, eq. UnbiasedGrad):
 * g_dev[k] = sum_{i,j} Rs[j,i] Js[j + l_d i, k]
 *          = -sum_c h^d d mu_c/d p_k sum_i U[c,i] (Z Rs)[c,i],
 * without forming Js.  Rs_dev: l_d x l_s.
 */
int dot_grad_misfit(dot_op* op, int l_s, const double* U_dev, int l_d, const double* Z_dev,
                    const double* Rs_dev, double* g_dev, void* work_dev, size_t work_bytes,
                    void* stream);

/*
 * dot_grad_misfit for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, bit for bit, with the scratch (the
 * per-cell sums and the per-chunk partials) in a fixed device array of
 * DOT_NOALLOC_SCRATCH_DOUBLES binary64 values (32 MiB) that the library
 * holds on every GPU it runs on until the process ends.  The call allocates
 * nothing and does not synchronize; the caller passes the inputs and g_dev.
 * The scratch needed is N rounded up to 32 plus (band chunks) x (active
 * parameters per RBF) values: grids up to about 4.1 million cells (128^3 with
 * 1000 RBFs fits); larger ones return DOT_EINVAL.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (on different
 * streams or host threads) race and must be serialized by the caller.
 */
#define DOT_NOALLOC_SCRATCH_DOUBLES (1u << 22)
int dot_grad_misfit_noalloc(dot_op* op, int l_s, const double* U_dev, int l_d,
                            const double* Z_dev, const double* Rs_dev, double* g_dev,
                            void* stream);

/*
 * Kernel timing with HIP events on the caller's stream (off by default).
 * dot_profile_enable(op, 1) resets and starts timing of the solver sweeps
 * and the contraction; dot_profile_read returns, for one kernel kind, the
 * summed event time (ms), the number of launches and the sum over launches
 * of the number of active columns each launch processed (a contraction
 * launch counts 1).  Solver launches that found no active column (those
 * queued after convergence) are left out of all three.  Reading
 * synchronizes the device.
 */
#define DOT_PROF_PCG1_FP64 0   /* CG pass 1 (p = r + beta p, A p, p.Ap), binary64 */
#define DOT_PROF_PCG2_FP64 1   /* CG pass 2 (A p, x += alpha p, r -= alpha A p, norms) */
#define DOT_PROF_PCG1_FP32 2
#define DOT_PROF_PCG2_FP32 3
#define DOT_PROF_RESID 4       /* binary64 residual of the refinement */
#define DOT_PROF_JACOBIAN 5    /* Jacobian contraction */
#define DOT_PROF_VCYCLE_FP64 6 /* multigrid V-cycle (all levels), binary64 */
#define DOT_PROF_VCYCLE_FP32 7 /* multigrid V-cycle (all levels), binary32 */
#define DOT_PROF_KINDS 8
int dot_profile_enable(dot_op* op, int enable);
/* Time only the kinds whose bit (1u << DOT_PROF_*) is set in mask (after
 * dot_profile_enable, which selects every kind).  Each timed launch is
 * bracketed by two event records, which keep the next kernel from starting
 * early (about 5 us per boundary on MI355X), so a caller timing a whole
 * workload selects only the kinds it reports.  DOT_EINVAL before the first
 * dot_profile_enable. */
int dot_profile_kinds(dot_op* op, unsigned mask);
int dot_profile_read(dot_op* op, int kind, double* ms_total, int64_t* launches,
                     int64_t* column_sweeps);

/*
 * Small dense binary64 helpers on the device, for the optimized
 * sources/detectors (Section 3.2, Alg. 1) and the Gauss-Newton SVD.
 *
 * dot_gemm: C (m x n) = alpha op(A) op(B) + beta C, op = transpose if trans*
 *   is nonzero; column-major with leading dimensions lda, ldb, ldc.
 */
int dot_gemm(int transa, int transb, int m, int n, int kdim, double alpha, const double* A_dev,
             int lda, const double* B_dev, int ldb, double beta, double* C_dev, int ldc,
             void* stream);

/*
 * Gram matrix of a tensor unfolding, without forming the unfolding.  T_dev
 * is a dA x dB x dC tensor (first index fastest).  mode 0: G (dA x dA) =
 * sum_{b,c} T[a,b,c] T[a',b,c]; mode 1: G (dB x dB) = sum_{a,c} T[a,b,c]
 * T[a,b',c].  These are the J~ J~^T, K~ K~^T and L~ L~^T of Section 3.2
 * (eqs. Jtilde, Ktilde, Ltilde): a column permutation of an unfolding does
 * not change its Gram matrix or left singular vectors.
 */
size_t dot_mode_gram_workspace_bytes(int dA, int dB, int dC, int mode);
int dot_mode_gram(int dA, int dB, int dC, const double* T_dev, int mode, double* G_dev,
                  void* work_dev, size_t work_bytes, void* stream);

/*
 * Symmetric eigensolver (cyclic Jacobi; block Jacobi on 16-index blocks
 * for n > 64): A_dev (n x n, lda) is not modified; w_dev receives the
 * eigenvalues in descending order and V_dev (n x n, ldv) the orthonormal
 * eigenvectors in the same order.  *sweeps_host (if not NULL) receives the
 * number of block sweeps (-1 for the one-block n <= 64 path).  n <= 8192.
 * Synchronizes the stream once per sweep when n > 64.
 */
size_t dot_symeig_workspace_bytes(int n);
int dot_symeig(int n, const double* A_dev, int lda, double* w_dev, double* V_dev, int ldv,
               void* work_dev, size_t work_bytes, int* sweeps_host, void* stream);

/*
 * Householder QR of X_dev (n x q, ldx; not modified) with the complete
 * orthogonal factor Q_dev (n x n, ldq): Q(:, 1:q) spans range(X) and
 * Q(:, q+1:n) its orthogonal complement.  Reflectors follow LAPACK's
 * convention, so Q equals LAPACK's (numpy's) complete Q up to rounding.
 * Used for the optimized directions W_hat = orth(W W~) and their complement
 * W_c (Section 3.2, eqs. newW, newV).
 */
size_t dot_qr_workspace_bytes(int n, int q);
int dot_qr_complete(int n, int q, const double* X_dev, int ldx, double* Q_dev, int ldq,
                    void* work_dev, size_t work_bytes, void* stream);

/*
 * Alg. 1 (optimized simultaneous sources and detectors; HOOI / Tucker2):
 * J_dev is the (n_d n_s) x n_p Jacobian with the detector index fastest
 * (eq. Jacobiancomp; the sampled J_s with n_d = l_d, n_s = l_s works the same
 * way).  Step (1) takes the leading q_d left singular vectors of J~, then
 * steps (2)-(3) alternate W~ (leading q_s left singular vectors of K~) and V~
 * (of L~) until the projectors W~ W~^T and V~ V~^T change by less than tol in
 * Frobenius norm, or maxit iterations.  Outputs W_dev (n_s x q_s), V_dev
 * (n_d x q_d), the iteration count and the objective ||(W~^T kron V~^T) J||_F^2.
 * Singular vectors are computed as eigenvectors of the unfoldings' Gram
 * matrices.  Synchronizes the stream.
 */
size_t dot_hooi_workspace_bytes(int n_d, int n_s, int n_p, int q_d, int q_s);
int dot_hooi(int n_d, int n_s, int n_p, const double* J_dev, int q_d, int q_s, double tol,
             int maxit, double* W_dev, double* V_dev, int* iters_host, double* objective_host,
             void* work_dev, size_t work_bytes, void* stream);

/*
 * Thin SVD A = U diag(s) Y^T of A_dev (m x n, lda = m), m <= n (the sampled
 * Jacobian behind the Gauss-Newton model, eq. GN): U and s from the
 * eigendecomposition of A A^T, Y = A^T U diag(1/s) for s > rcut s_max (zero
 * columns otherwise).  U_dev m x m, s_dev m, Y_dev n x m.  For
 * 64 < m <= 512 and m <= n <= 4096, U = Q W with W, s^2 the eigenpairs of
 * R R^T = Q^T A A^T Q, A P = Q R the QR factorization with column pivoting
 * (on this graded matrix the Jacobi sweeps converge in about half as many
 * sweeps as on A A^T); otherwise from A A^T directly.  Synchronizes.
 */
size_t dot_svd_workspace_bytes(int m, int n);
int dot_svd_thin(int m, int n, const double* A_dev, int lda, double* s_dev, double* U_dev,
                 int ldu, double* Y_dev, int ldy, double rcut, void* work_dev, size_t work_bytes,
                 void* stream);

/*
 * Truncated-SVD Gauss-Newton step for min ||J d + r|| (Section 2, eq. GN and
 * Eq:NLLS; its sampled form eq. TREGS J), kept to the t leading singular
 * triplets of J = L diag(s) R^T:  x = -sum_{i < t} (L(:, i)^T r / s_i) R(:, i).
 * L_dev rows x k (ldl), s_dev k (descending, s_i > 0 for i < t), R_dev
 * cols x k (ldr), r_dev rows, x_dev cols (all device).  For the sampled
 * Jacobian J_s (l_s l_d x n_p) either factor order of dot_svd_thin applies:
 * the SVD of J_s^T gives L = Y, R = U.  Deterministic; does not synchronize.
 */
size_t dot_tsvd_step_workspace_bytes(int t);
int dot_tsvd_step(int rows, int cols, int k, const double* L_dev, int ldl, const double* s_dev,
                  const double* R_dev, int ldr, int t, const double* r_dev, double* x_dev,
                  void* work_dev, size_t work_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DOTPATH_H */
