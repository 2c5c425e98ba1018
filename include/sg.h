/*
 * sg.h -- C ABI of the MI355X stochastic-Galerkin diffusion solver.
 *
 * Solves the stochastic Galerkin (SG) system K u = F of
 *     -div(a(x, y) grad u) = f  on the unit square, u = 0 on the boundary,
 * with the shifted lognormal coefficient a = a_min + exp(gamma), gamma a
 * Gaussian field given by a truncated Karhunen-Loeve (KL) expansion
 * (Aulisa, Capodaglio, Ke: Sec. 2, eqs. Strong_PS, aKL, KL_gamma,
 * standard_deviation), discretised by Q1 finite elements in space and an
 * orthonormal Hermite chaos of total degree p in the random variables
 * (Sec. 2.2), K = sum_k G_k (x) A_k with [G_k]_{ij} = E[psi_k psi_i psi_j].
 *
 * Conventions for every entry point:
 *  - Device pointers are FP64, contiguous, and owned by the caller; the
 *    library never frees them.  SG vectors are mode-major: entry
 *    i*N_h + (iy-1)(n-1) + (ix-1) holds mode i at interior grid node
 *    (ix, iy), 1 <= ix, iy <= n-1 (Dirichlet nodes eliminated), modes in the
 *    graded, descending-lexicographic order of the index set J(p).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream unless stated otherwise.
 *  - Return value: SG_OK (0) or a negative SG_ERR_* code; sg_last_error()
 *    then gives a message (thread-local, valid until the next call on the
 *    same thread).  No C++ exception crosses this interface.
 *  - A handle may be used by one host thread at a time.  Calls on one handle
 *    share its workspace: calls that overlap in time on different streams race.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SG_OK = 0,
  SG_ERR_INVALID_ARG = -1,  /* argument outside its documented range        */
  SG_ERR_UNSUPPORTED = -2,  /* valid, but beyond a compiled limit           */
  SG_ERR_HIP = -3,          /* a HIP runtime call failed                    */
  SG_ERR_NOT_BOUND = -4,    /* the handle has no device workspace yet       */
  SG_ERR_WORKSPACE = -5,    /* workspace too small or misaligned            */
  SG_ERR_INTERNAL = -6
};

/* sg_solve_info.status (not errors) */
enum { SG_CONVERGED = 0, SG_NOT_CONVERGED = 1, SG_BREAKDOWN = 2 };

/* covariance of gamma: eq. standard_deviation (L1 exponential) or the squared
 * exponential sigma^2 exp(-sum_i (x_i - x'_i)^2 / L_c^2) */
enum { SG_COV_EXP_L1 = 0, SG_COV_SQEXP = 1 };

/* preconditioners (Sec. 3): none, mean-based (one V(2,2) cycle on the mean
 * stiffness A_0 per mode), field split (forward block Gauss-Seidel over
 * ordered splits of the modes, eqs. P_preconditioner / P_group, with the
 * same V-cycle for every diagonal block) */
enum { SG_PC_NONE = 0, SG_PC_MEAN = 1, SG_PC_FS = 2, SG_PC_LEARNED = 3, SG_PC_MG = 4 };
/* SG_PC_MG: one multigrid V(1,1) cycle on the full SG system K (Sec. 3, the
 * paper's G-M-F-I / G-M-Fg-I family; needs sg_mg_bind): levels n, n/2, ..., 4
 * rediscretised with the KL values at each level's Gauss points, the
 * field-split level iteration of eq. level_solver as the smoother with the
 * bound grouping's splits (each split's diagonal block approximated by its
 * nodal blocks, inverted exactly, damping 8/9), bilinear transfers, and a
 * direct solve on the 4 x 4 grid.                                          */
/* flag OR-ed into SG_PC_MEAN or SG_PC_FS: the V(2,2) cycle of mode i runs on
 * that mode's own diagonal block K_ii = sum_k [G_k]_{ii} A_k (the paper's
 * diagonal blocks of eq. P_preconditioner) instead of the mean stiffness A_0 */
enum { SG_PC_DIAG_KII = 0x100 };
/* flag OR-ed into SG_PC_MEAN or SG_PC_FS for sg_gmres_solve and
 * sg_batch_solve: start with the A_0 cycles and switch to the K_ii cycles of
 * SG_PC_DIAG_KII, at a restart, once a whole cycle has left the true residual
 * above a fifth of its value at the cycle's start (the A_0 diagonal blocks
 * are not a contraction at large sigma); sg_solve_info.fallbacks then
 * counts 1.                                                                */
enum { SG_PC_SWITCH_KII = 0x200 };
/* inner iterations of the diagonal-block solves (the paper's G-F-I: eq.
 * level_solver applied to each diagonal block): pc | (k << SG_PC_INNER_SHIFT)
 * with 2 <= k <= 255 makes every block solve of SG_PC_MEAN, SG_PC_FS (and
 * the field split inside SG_PC_LEARNED) run k Richardson steps
 * x <- x + V(t - B x) from x = 0, V the V(2,2) cycle on the block's operator
 * B (A_0, or K_ii with SG_PC_DIAG_KII); 0 or 1 = one cycle.               */
enum { SG_PC_INNER_SHIFT = 16 };

/* splits of the modes for SG_PC_FS:
 *  KLVAR         split n = modes whose first nonzero index is n; mean in split 1
 *  KLVAR_MEANSEP KLVAR with the mean mode as its own first split
 *  PERMODE       one split per mode (the paper's G-M-F-I splitting)
 *  FG            the paper's leading-digit grouping (Sec. 3, worked example
 *                N=2, p=4 -> splits of 5, 4, 6 modes)
 *  ALL           one split of all modes: with SG_PC_FS the block-diagonal
 *                (mean-based, or K_ii with SG_PC_DIAG_KII) preconditioner;
 *                with SG_PC_MG a smoother that couples every mode at a node,
 *                the counterpart of the paper's G-M-I (Sec. 3, a level
 *                smoother preconditioned by an incomplete factorisation of
 *                the whole K)                                                */
enum {
  SG_GROUP_KLVAR = 0,
  SG_GROUP_KLVAR_MEANSEP = 1,
  SG_GROUP_PERMODE = 2,
  SG_GROUP_FG = 3,
  SG_GROUP_ALL = 4,
  SG_GROUP_COUNT = 5
};

/* form of the operator apply (sg_set_apply):
 *  TRIPLE    sum over the n_a coefficient modes a_k(x_q) with the triple
 *            products [G_k]_{ij} (Sec. 2.2, eqs. dataProjection, K_matrix);
 *            valid for every q
 *  FACTORED  the same matrix through E[a psi_i psi_j] = a_min delta_ij +
 *            exp(mu + |g|^2/2) (T T^T)_ij, T the Hermite translation matrix
 *            of the KL values g_n(x_q); equal to TRIPLE when q >= 2p (the
 *            projection of eq. dataProjection is then exact on every block),
 *            rejected otherwise
 *  AUTO      FACTORED when q >= 2p, else TRIPLE (the default)              */
enum { SG_APPLY_AUTO = 0, SG_APPLY_TRIPLE = 1, SG_APPLY_FACTORED = 2 };

/* Problem statement (Sec. 2, Sec. 2.1, Sec. 2.2):
 *  n         elements per side, power of two, 4 <= n <= 4096
 *  M         KL terms (the paper's N), 1 <= M <= 12
 *  p         chaos degree of u; P = (M+p)!/(M!p!) modes, 1 <= P <= 256
 *  q         chaos degree of the coefficient projection (eq. dataProjection),
 *            0 <= q <= 16; q >= 2p makes K the exact Galerkin matrix
 *  cov       SG_COV_*; mu, sigma >= 0, corr_len > 0, a_min >= 0 as in
 *            eqs. aKL / KL_gamma / standard_deviation                        */
typedef struct {
  int32_t n, M, p, q, cov;
  double mu, sigma, corr_len, a_min;
} sg_problem;

/* GMRES(restart) options (Sec. 3): right preconditioning, CGS2 Arnoldi.
 *  restart 1..200; max_it >= 1 total iterations; pc SG_PC_*; grouping
 *  SG_GROUP_* (used when pc is SG_PC_FS or SG_PC_LEARNED); use_x0 != 0
 *  starts from the content of u; tol > 0 on the true relative residual
 *  ||F-Ku||/||F||.  SG_PC_LEARNED runs flexible GMRES whose preconditioner
 *  stage is z = P_FS^{-1} v + alpha c: c is the attached network's prediction
 *  of the error left in the field-split residual r = v - K P_FS^{-1} v, and
 *  alpha = <r, K c>/||K c||^2 minimises ||v - K z||, so the field split is
 *  both the judge (the stage never has a larger residual) and the fallback
 *  (alpha = 0 when the prediction is not finite; counted in fallbacks).     */
typedef struct {
  int32_t restart, max_it, pc, grouping, use_x0;
  double tol;
} sg_solve_opts;

typedef struct {
  int32_t status;       /* SG_CONVERGED / SG_NOT_CONVERGED / SG_BREAKDOWN   */
  int32_t iterations;   /* Arnoldi steps taken                              */
  int32_t restarts;     /* completed cycles                                 */
  int32_t fallbacks;    /* learned stage: steps that fell back to plain FS  */
  double relres;        /* true ||F - K u|| / ||F|| in FP64 at exit          */
  double relres_est;    /* last rotated residual estimate / ||F||           */
} sg_solve_info;

typedef struct sg_handle sg_handle;

/* Host-side set-up of one instance (Sec. 2.1 and 2.2): index sets J(p), J(q),
 * the triple products G_k, the KL eigenpairs from a 1D Galerkin procedure on
 * the grid (tensor products on the square), the KL modes at the 2x2 Gauss
 * points, and the field-split groupings.  f_nodal: host array of (n+1)^2
 * nodal forcing values (row-major, x fastest), or NULL for f = 1; copied.
 * *out receives a new handle (free with sg_destroy).  No device work.      */
int sg_setup(const sg_problem* prob, const double* f_nodal, sg_handle** out);

/* The same instance on continuous biquadratic (Q2) elements, the paper's
 * spatial space (Sec. 2.2): prob->n (a power of two in [4, 2048]) elements
 * per side, 3 x 3 Gauss points per element (eq. A_q), K = sum_k G_k (x) A_k
 * with A_k the Q2 stiffness of a_k, F = e_0 (x) M f with the consistent Q2
 * mass matrix.  The unknowns of a mode are the (2n-1)^2 interior Q2 nodes,
 * which are the interior vertices of the twice-refined grid, numbered as for
 * Q1 on 2n elements; f_nodal holds (2n+1)^2 values at those vertices (NULL
 * for f = 1).  The KL eigenpairs come from the 1D Galerkin procedure on the
 * refined grid, and g at a Gauss point is their bilinear interpolant.
 * sg_apply, sg_residual, sg_rhs and sg_gmres_solve use the Q2 operator; the
 * preconditioners (SG_PC_MEAN, SG_PC_FS with any grouping and flag,
 * SG_PC_MG) are those of the Q1 operator on the refined grid, which is
 * spectrally equivalent to the Q2 one with constants independent of n.  The
 * apply is the factored form only.  Errors: INVALID_ARG (as sg_setup, or n
 * out of range), UNSUPPORTED (q < 2p, p > 15, or P * 9 n^2 >= 2^31).  A Q2 handle rejects
 * sg_set_apply, sg_apply_noalloc and sg_attach_cnn with UNSUPPORTED;
 * sg_apply_form reports form 3; sg_sizes reports the Q1 refined grid's n_a
 * and nnz_G; sg_export describes the refined grid's Q1 data.               */
int sg_setup_q2(const sg_problem* prob, const double* f_nodal, sg_handle** out);

/* Sizes of the discrete system (Sec. 2.2): P = |J(p)| = (M+p)!/(M!p!) chaos
 * modes of u, N_h = (n-1)^2 unknowns per mode (Q1, Dirichlet nodes
 * eliminated), n_a = |J(q)| coefficient modes of eq. dataProjection, nnz_G
 * nonzero triple products [G_k]_{ij} (eq. K_matrix).  Any pointer may be
 * NULL.  Host only.  Errors: INVALID_ARG (null handle).                    */
int sg_sizes(const sg_handle* h, int64_t* P, int64_t* N_h, int64_t* n_a, int64_t* nnz_G);

/* Device bytes sg_bind needs (coefficient modes a_k at every quadrature
 * point, stencils of all multigrid levels, triple-product tables, scratch). */
size_t sg_workspace_bytes(const sg_handle* h);

/* Binds a caller-owned device workspace (>= sg_workspace_bytes, 256-byte
 * aligned), uploads the set-up tables and computes on the device the
 * coefficient modes a_k(x_q) (eq. dataProjection in closed form), the mean
 * stiffness stencil and its Galerkin coarse stencils.  Synchronises
 * `stream` before returning.  The workspace must outlive the handle's use. */
int sg_bind(sg_handle* h, void* dev_workspace, size_t bytes, void* stream);

/* F = e_0 (x) M_h f_h (Sec. 2.2, right-hand side of eq. stochastic_matrix):
 * writes P*N_h values to the device array F.                               */
int sg_rhs(sg_handle* h, double* F, void* stream);

/* W = K U = sum_k vec(A_k U G_k^T) (Sec. 2.2, definition of K), matrix-free
 * in the form chosen by sg_set_apply.  U, W: device, P*N_h, must not alias. */
int sg_apply(sg_handle* h, const double* U, double* W, void* stream);

/* W = K U exactly as sg_apply (same kernels, same bits), for callers that
 * cannot allocate device memory or touch the handle's scratch while the call
 * runs (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The apply's only scratch, the edge sums of its 4x4
 * element tiles (9 values per tile and mode: 8 * 9 * P * (n/4)^2 bytes), lives
 * in a fixed library-owned device array of 64 MiB per GPU, held from the first
 * call on that GPU until the process ends; this call allocates nothing.
 * Every call on one GPU shares that array, so calls that overlap in time on
 * one GPU (any handles, any streams) race; the array's content is left from
 * the last call and never read before being written.  U, W: device, P*N_h,
 * must not alias.  Errors: INVALID_ARG, NOT_BOUND, UNSUPPORTED (edge sums
 * above 64 MiB, e.g. n = 256 with P > 227), HIP.                          */
int sg_apply_noalloc(sg_handle* h, const double* U, double* W, void* stream);

/* Chooses the apply form used by sg_apply, sg_residual, the field-split
 * preconditioner and sg_gmres_solve.  points_per_batch (FACTORED only): 0
 * selects the register-resident kernel where it is compiled (every M <= 6
 * with p <= 4), else the LDS tile kernel with the planner's sub-batch size;
 * 8, 16, 32 or 64 select the LDS tile kernel with that many Gauss points per
 * sub-batch of a 4x4-element tile.  Re-uploads the plan on `stream` when the handle is bound
 * and synchronises it.  Errors: INVALID_ARG (unknown kind or size),
 * UNSUPPORTED (FACTORED with q < 2p, or a size whose LDS exceeds 160 KB; the
 * previous plan stays in place).                                            */
int sg_set_apply(sg_handle* h, int kind, int points_per_batch, void* stream);

/* The apply form in use (an inspection call for tests and tools): *form = 2
 * for the register-resident factored kernel, 1 for the factored LDS tile
 * kernel (*points_per_batch: its Gauss points per sub-batch), 0 for the
 * triple-product form, 3 for the biquadratic apply of a sg_setup_q2 handle.  Host only.  Errors: INVALID_ARG (null argument).    */
int sg_apply_form(const sg_handle* h, int* form, int* points_per_batch);

/* z = P^{-1} r for pc in {SG_PC_NONE, SG_PC_MEAN, SG_PC_FS} and a grouping
 * (Sec. 3, eqs. P_preconditioner / P_group), optionally with SG_PC_DIAG_KII.
 * pc = SG_PC_LEARNED (| SG_PC_DIAG_KII) applies one learned stage of the
 * attached network (see sg_solve_opts; not part of the paper):
 * z = P_FS^{-1} r + alpha c, c the network's prediction for
 * r1 = r - K P_FS^{-1} r, alpha = <r1, K c>/||K c||^2 (0 when not finite).
 * r, z: device, P*N_h, must not alias.  Errors: INVALID_ARG (unknown pc or
 * grouping; SG_PC_LEARNED without an attached network), NOT_BOUND.       */
int sg_precond_apply(sg_handle* h, int pc, int grouping, const double* r, double* z,
                     void* stream);

/* Multigrid on the full SG system (SG_PC_MG; Sec. 3, eqs. level_solver and
 * P_group).  sg_mg_workspace_bytes: device bytes for `grouping` (the splits
 * of the smoother; SG_GROUP_FG is the paper's G-M-Fg-I, SG_GROUP_PERMODE its
 * G-M-F-I), 0 for a bad argument.  sg_mg_bind builds the hierarchy in a
 * caller-owned, 256-byte aligned workspace on a bound handle: the KL values
 * and coefficient modes a_k (eq. dataProjection) at the Gauss points of every
 * coarser level, so that every level is applied in the handle's current apply
 * form (factored or triple-product), the nodal blocks of every split on every level but
 * the coarsest (K applied to probe vectors, one mode and one of four node
 * colours at a time, then inverted in place), and the coarsest level's K
 * (column by column) inverted on the host.  Synchronises `stream`.  The
 * workspace must outlive the multigrid's use; binding again replaces the
 * hierarchy.  SG_PC_MG calls must pass the bound grouping.  Errors:
 * INVALID_ARG, NOT_BOUND (handle), UNSUPPORTED (a split of more than 128
 * modes), WORKSPACE, HIP.  */
size_t sg_mg_workspace_bytes(const sg_handle* h, int grouping);
int sg_mg_bind(sg_handle* h, int grouping, void* ws, size_t bytes, void* stream);

/* r = F - K u, the residual of the SG system K u = F (Sec. 2.2, eq.
 * stochastic_matrix), with K applied as by sg_apply.  F, u, r: device,
 * P*N_h each; r must not alias F or u.  Errors: NOT_BOUND, INVALID_ARG.   */
int sg_residual(sg_handle* h, const double* F, const double* u, double* r, void* stream);

/* Device bytes of the Krylov workspace sg_gmres_solve needs for `opts`.    */
size_t sg_gmres_workspace_bytes(const sg_handle* h, const sg_solve_opts* opts);

/* Right-preconditioned restarted GMRES for K u = F (Sec. 3).  F: device
 * right-hand side; u: device solution (initial guess if opts->use_x0);
 * krylov_ws: caller-owned device buffer of sg_gmres_workspace_bytes bytes;
 * resid_hist: optional host array receiving the relative residual estimate
 * after every iteration (entry 0 = initial), at most hist_len entries.
 * Synchronises `stream`; fills *info.  Non-convergence is reported in
 * info->status, not as an error.                                          */
int sg_gmres_solve(sg_handle* h, const sg_solve_opts* opts, const double* F, double* u,
                   void* krylov_ws, size_t ws_bytes, double* resid_hist, int32_t hist_len,
                   sg_solve_info* info, void* stream);

/* Copies a set-up table to host memory (for verification against the
 * definitions of Sec. 2.1 and 2.2: the KL eigenpairs of eqs. KL_gamma /
 * standard_deviation, the coefficient modes of eq. dataProjection, the
 * stiffness of eq. A_q, the groupings of eq. P_group):
 *  SG_EXPORT_COEFF  a_k(x_q), n_a x 4n^2 values, q = 4e + 2qy + qx,
 *                   e = ey*n + ex (synchronous)
 *  SG_EXPORT_KL     lambda_1..lambda_M (host table)
 *  SG_EXPORT_GQ     g_m(x_q) = sqrt(lambda_m) b_m(x_q), M x 4n^2 (host table)
 *  SG_EXPORT_STENCIL the 9-point mean stiffness of multigrid level `level`
 *                   (0 = finest), 9 x (n_l - 1)^2 values, entry s*N_l + node,
 *                   s = 3(dy+1) + (dx+1) (synchronous)
 *  SG_EXPORT_GROUPS for grouping `level`: the number of splits, then for
 *                   each split its size followed by its mode indices
 *  SG_EXPORT_BLOCKS for grouping `level` (an inspection for tests): the
 *                   number of splits, then per split the compiled block
 *                   kernel its off-diagonal apply runs in the register form
 *                   (its first KL variable), 0 where the run-time-mask
 *                   kernel runs it, for split 0 and when the register form
 *                   is not in use                                            */
enum { SG_EXPORT_COEFF = 0, SG_EXPORT_KL = 1, SG_EXPORT_GQ = 2, SG_EXPORT_STENCIL = 3,
       SG_EXPORT_GROUPS = 4, SG_EXPORT_BLOCKS = 5 };
int sg_export(sg_handle* h, int what, int level, double* host_out, size_t count);

void sg_destroy(sg_handle* h);
const char* sg_last_error(void);

/* ---------------------------------------------------------------------------
 * Learned preconditioner stage: a mode-channel CNN (3x3 convolutions over four
 * grid levels, widths 32 and 64, BF16 weights and activations with FP32
 * accumulation on the matrix cores, FP32 master weights trained with Adam).
 * Input: a residual field of P modes on the n x n pixel grid of interior
 * nodes plus a constant sigma channel, scaled by sqrt(P N_h)/||r||; output:
 * the error field scaled by kappa sqrt(P N_h)/(||r|| n^2), kappa = 2 pi^2.
 * Not part of the paper.
 * Errors are reported through sg_cnn_last_error().
 * ------------------------------------------------------------------------- */
typedef struct sg_cnn sg_cnn;
/* P in [1, 63] modes, n grid (power of two in [16, 1024]), hidden widths
 * c0 = 32 or 64 (finest level; 64 passes more than 32 modes through the
 * finest level), c1 = 64 (coarser levels), max_batch in [1, 256] samples per
 * training step.                                                            */
int    sg_cnn_create(int32_t P, int32_t n, int32_t c0, int32_t c1, int32_t max_batch, sg_cnn** out);
/* number of weights (layers concatenated, each (9, c_out, c_in), tap =
 * 3(dy+1)+(dx+1)) and of biases                                              */
int    sg_cnn_param_counts(const sg_cnn* c, int64_t* n_weights, int64_t* n_bias);
size_t sg_cnn_workspace_bytes(const sg_cnn* c);
/* binds a caller-owned, 256-byte aligned device workspace (zeroed here)      */
int    sg_cnn_bind(sg_cnn* c, void* dev_workspace, size_t bytes, void* stream);
/* host FP32 weights/biases in, Adam moments reset (synchronous)               */
int    sg_cnn_set_params(sg_cnn* c, const float* w_host, const float* b_host, void* stream);
int    sg_cnn_get_params(sg_cnn* c, float* w_host, float* b_host);
/* Adam's first and second moments of the weights (n_weights floats each) and
 * biases (n_bias each), host arrays: with the parameters and the step number
 * the caller passes to training calls, the whole optimiser state, so that
 * training can be stopped and resumed.  set: after sg_cnn_set_params (which
 * resets them); synchronous.                                                 */
int    sg_cnn_get_adam(sg_cnn* c, float* wm_host, float* wv_host, float* bm_host, float* bv_host);
int    sg_cnn_set_adam(sg_cnn* c, const float* wm_host, const float* wv_host,
                       const float* bm_host, const float* bv_host, void* stream);
/* one training pair from device FP64 SG vectors: residual r = F - K u of an
 * iterate u and the reference solution ustar (error e = ustar - u):
 * R_out = bf16(r s), T_out = bf16(e s kappa / n^2), s = sqrt(P N_h)/||r||, both
 * P*N_h device arrays                                                        */
int    sg_cnn_make_pair(sg_cnn* c, const double* r, const double* ustar, const double* u,
                        uint16_t* R_out, uint16_t* T_out, void* stream);
/* forward (mode 0), + gradients (1), + one Adam step with learning rate lr at
 * step number `step` >= 1 (2) on the stored pairs idx[0..batch) (host array);
 * R, T: npairs x P x N_h bf16 device arrays, sigma: npairs device floats;
 * Y_out (device, nullable): batch x n x n x c_out FP32 outputs; loss (host,
 * nullable): mean relative squared error.  Synchronous when loss != NULL.  */
int    sg_cnn_run(sg_cnn* c, const uint16_t* R, const uint16_t* T, const float* sigma,
                  const int32_t* idx, int32_t batch, int32_t mode, float lr, int32_t step,
                  float* Y_out, double* loss, void* stream);
/* weight and bias gradients of the last sg_cnn_run with mode >= 1, or of the
 * last sg_cnn_backward (host)                                               */
int    sg_cnn_get_grads(sg_cnn* c, float* dw_host, float* db_host);
/* Training on the learned stage's own objective (the stage is z = z0 + alpha
 * c with alpha minimising |r - alpha K c|, so it removes the share
 * (r.Kc)^2 / (|r|^2 |Kc|^2) of the residual's square).  After a forward
 * (sg_cnn_run, mode 0) on pairs idx[0..batch), for each slot: with r the
 * stored residual R[pair] (bf16 npairs x P x N_h device array, the layout of
 * sg_cnn_make_pair) and c the network's output for that slot, writes the
 * output gradient of L = 1 - (r.Kc)^2 / (|r|^2 |Kc|^2), divided by batch, into
 * the network; K is h's operator (the pair's problem; P and n must match the
 * network).  work: device, sg_cnn_stage_work_doubles(h) doubles; loss
 * (host, nullable): L, synchronous when given.  Then sg_cnn_backward takes
 * the gradients of the summed objective and, with adam != 0, one Adam step
 * (learning rate lr, step number >= 1).  Errors: INVALID_ARG, NOT_BOUND.
 * Not part of the paper.                                                    */
size_t sg_cnn_stage_work_doubles(const sg_handle* h);
int    sg_cnn_stage_grad(sg_handle* h, sg_cnn* c, const uint16_t* R, int64_t pair, int32_t slot,
                         int32_t batch, double* work, double* loss, void* stream);
int    sg_cnn_backward(sg_cnn* c, int32_t batch, int32_t adam, float lr, int32_t step,
                       void* stream);
/* c = prediction for the FP64 SG vector v (device, P*N_h), SG units          */
int    sg_cnn_apply(sg_cnn* c, const double* v, double sigma, double* out, void* stream);
void   sg_cnn_destroy(sg_cnn* c);
const char* sg_cnn_last_error(void);
/* attaches a bound network (P and n must match) and the sigma fed to it for
 * SG_PC_LEARNED solves of this handle; NULL detaches                        */
int    sg_attach_cnn(sg_handle* h, sg_cnn* c, double sigma);

/* ---------------------------------------------------------------------------
 * Batched solves: many instances of uneven grid size, KL dimension, degree
 * and sigma solved together.  Each step kernel is one launch over a device
 * work-item table that covers every instance; per-instance Krylov state stays on the device,
 * so one Arnoldi step of all instances (and the restart step) is captured
 * once in a HIP graph and replayed.  Instances advance in lockstep; converged
 * instances are masked.  Not part of the paper.
 * ------------------------------------------------------------------------- */
typedef struct sg_batch sg_batch;
/* count instances; f_nodal: NULL or an array of count host pointers (each
 * NULL or (n_i+1)^2 values).  autotune != 0 picks each problem class's
 * (device, M, p, q) apply form by timing the candidates the batched step
 * kernels can run on the current device (cached on disk; the cache file is
 * $SG_AUTOTUNE_CACHE or ~/.sgfs_autotune.txt): the register-resident
 * factored kernel (code 1), the factored LDS tile kernel with qb Gauss points
 * per sub-batch (100 + qb, qb in 8..64) or the triple-product form with kc
 * coefficient modes per chunk (200 + kc, kc in 16..64).                     */
int    sg_batch_create(int32_t count, const sg_problem* probs, const double* const* f_nodal,
                       int32_t autotune, sg_batch** out);
/* packed vector layout: offsets[0..count] (instance i occupies
 * [offsets[i], offsets[i+1]) of every packed SG vector); form (nullable):
 * the code of each instance's apply form (as chosen by the autotuner)      */
int    sg_batch_layout(const sg_batch* b, int64_t* offsets, int32_t* form);
size_t sg_batch_workspace_bytes(const sg_batch* b, int32_t restart);
/* binds a caller-owned 256-byte aligned workspace for GMRES(restart)      */
int    sg_batch_bind(sg_batch* b, int32_t restart, void* ws, size_t bytes, void* stream);
/* packed right-hand sides                                                  */
int    sg_batch_rhs(sg_batch* b, double* F, void* stream);
/* the bound handle of instance i (for single-instance calls; owned by b)   */
int    sg_batch_handle(sg_batch* b, int32_t i, sg_handle** h);
/* solves every instance from zero with opts (pc SG_PC_MEAN or SG_PC_FS,
 * restart equal to the bound value; SG_PC_SWITCH_KII applies to the
 * one-at-a-time solves below, the lockstep part keeps the A_0 cycles; any
 * grouping whose splits number at most 12 for every lockstep instance, else
 * UNSUPPORTED); F, u packed device vectors; infos: count entries.  Graph
 * capture needs a non-null stream (the null stream runs the same launch
 * sequences eagerly).  On a non-null stream, instances of at least 2^20
 * unknowns (P*N_h) are solved by sg_gmres_solve, up to three at a time
 * (largest first, each from a host thread on a stream of its own), beside
 * the lockstep batch of the others.  At a restart that leaves at most four
 * lockstep instances running, those continue one at a time through
 * sg_gmres_solve from their current iterate; their infos add both parts.
 * The batch workspace reserves the Krylov areas of both.  Synchronous.     */
int    sg_batch_solve(sg_batch* b, const sg_solve_opts* opts, const double* F, double* u,
                      sg_solve_info* infos, void* stream);
void   sg_batch_destroy(sg_batch* b);
/* the autotuner on its own: the code of the fastest apply form for the
 * problem's class and its time per apply (ms) on the tuning grid; the code
 * is recorded in the tuning cache that sg_batch_create reads, replacing any
 * earlier entry for the class                                              */
int    sg_autotune_apply(const sg_problem* prob, int32_t* best_form, float* best_ms);

#ifdef __cplusplus
}
#endif
#endif /* SG_H */
