/*
 * tbs.h -- C ABI of the MI355X (gfx950) tensor B-spline implicit heat-step library.
 *
 * Method: Shulga, Morozov, Roth, Friedrich, Hunziker, "Tensor B-Spline Numerical Methods for
 * PDEs: a High-Performance Alternative to FEM" (arXiv:1904.03057).  The library computes the
 * paper's system operator F(c) (Sec. 2.4, tensor form F(c) = t) for constant coefficients as a
 * cascade of separable, shift-invariant 1-D filters (Sec. 2.4, separable kernel decomposition,
 * Fig. FiltAlg), "on the fly" without assembling a matrix (Sec. 2.5, strategy (c)), and solves
 * the resulting system with conjugate gradients (Sec. 2.5, step 3 of the method overview):
 *
 *     A = Mx (x) My (x) Mz + tau * ( hx^-2 Kx (x) My (x) Mz + hy^-2 Mx (x) Ky (x) Mz
 *                                                          + hz^-2 Mx (x) My (x) Kz )
 *
 * 1-D taps for basis degree n (Sec. 2.3, Table 1, "scalar product" and "derivative" rows):
 *     mass  m_k = b^{2n+1}(k),  stiffness  s_k = -(b^{2n+1})''(k),  |k| <= n.
 * The operator is divided through by hx*hy*hz, so mass rows sum to 1.  One implicit Euler step
 * of du/dt = Lap u + f is  A u^{k+1} = M (u^k + tau f)  (Galerkin load vector, Sec. 2.3, the
 * discrete Ritz-Galerkin system with the source expanded in the same basis).
 *
 * Conventions for every entry point
 *   - Arrays are caller-owned DEVICE pointers, layout c[z][y][x] with x contiguous, N = Nx*Ny*Nz
 *     elements, 256-byte aligned (TBS_E_INVAL otherwise).  Inputs and outputs must not alias
 *     unless stated.
 *   - Every call is enqueued on the stream given to tbs_setup and is asynchronous, except the
 *     calls that return host-side convergence data (documented below), which synchronise it.
 *   - A context is not thread safe; use one context per stream.
 *   - Arguments are validated before any HIP call, so validation errors are reported on a host
 *     without a GPU.  Returns 0 on success, a negative TBS_E_* code on error, or the positive
 *     TBS_W_NOT_CONVERGED when the output was written but the tolerance was not reached.
 *   - Boundary conditions: TBS_BC_PERIODIC = circulant bands (needs every N_d >= 2n+1);
 *     TBS_BC_DIRICHLET = homogeneous Dirichlet read as bands truncated at both ends (coefficients
 *     outside the index box are zero).
 */
#ifndef TBS_H
#define TBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TBS_OK 0
#define TBS_E_INVAL (-1)       /* bad argument: null/misaligned pointer, bad size, degree, tau, h, dtype */
#define TBS_E_NOMEM (-2)       /* no workspace bound, or the bound workspace is too small */
#define TBS_E_HIP (-3)         /* a HIP runtime call failed; tbs_last_error() has the text */
#define TBS_E_BREAKDOWN (-4)   /* CG breakdown: p^T A p <= 0 or a non-finite value */
#define TBS_E_STATE (-5)       /* call out of order (e.g. tbs_cg_step before tbs_cg_begin) */
#define TBS_W_NOT_CONVERGED 1  /* iteration limit reached; outputs and stats are written */

typedef struct tbs_ctx tbs_ctx;
typedef struct tbs_net tbs_net;

typedef enum { TBS_BC_PERIODIC = 0, TBS_BC_DIRICHLET = 1, TBS_BC_ROBIN = 2 /* tbs_setup_robin only */ } tbs_bc;
typedef enum { TBS_F64 = 0, TBS_F32 = 1, TBS_BF16 = 2 } tbs_dtype;
typedef enum {
  TBS_PREC_FP64 = 0,       /* plain FP64 CG */
  TBS_PREC_FP32 = 1,       /* raw FP32 CG (FP64 dot accumulation), no refinement */
  TBS_PREC_MIXED = 2,      /* FP64 outer residual + FP32 inner CG (iterative refinement) */
  TBS_PREC_MIXED_BF16 = 3  /* as MIXED, inner search direction stored in bf16 */
} tbs_prec;

typedef struct {
  int iters;               /* CG iterations (inner iterations summed over refinement sweeps) */
  int sweeps;              /* refinement sweeps (0 for FP64 / FP32) */
  int used_learned_guess;  /* 1 if the network guess was kept by the fallback test */
  int status;              /* return code of the call */
  double rel_res_fp64;     /* ||b - A u_next|| / ||b|| recomputed in FP64 at exit */
  double rel_res0;         /* same for the chosen initial guess */
  double rel_res_plain;    /* same for the plain guess u^k */
  double rel_res_learned;  /* same for the network guess (NaN if no network) */
  int used_coarse_guess;   /* 1 if the coarse-grid guess was kept by the fallback test */
  int coarse_iters;        /* CG iterations of the coarse solve (0 if none) */
  double rel_res_coarse;   /* FP64 relative residual of the coarse-grid guess (NaN if none) */
  int skipped_learned_guess;  /* 1 if a network was passed but not run this step (guess_backoff) */
  double learned_gamma;    /* multiplier of the network output in the guess u^k + gamma du (energy
                              test: the A-norm-optimal one; residual test: 1; 0 if not run) */
  double learned_saved_iters;  /* guess_backoff 2, kept guess: CG iterations it saved, estimated as
                              ln(rel_res_learned / rel_res_plain) / ln(rho), rho the solve's mean
                              residual reduction per iteration; 0 otherwise */
  double learned_cost_iters;   /* guess_backoff 2, network run: the time of the network and its test
                              in units of this step's time per CG iteration (its CG loops' time over
                              their iterations); 0 otherwise */
} tbs_stats;

typedef struct {
  double inner_rtol;       /* refinement: inner relative tolerance (default 1e-6, at least 1e-4 with a
                              bf16-stored direction); a sweep asks for max(inner_rtol, rtol / (2 rel)) */
  int inner_max_iter;      /* refinement: inner iteration cap per sweep (default 500) */
  int max_sweeps;          /* refinement: sweep cap (default 12) */
  int poll_every;          /* CG iterations enqueued between host convergence polls (default 4).
                              0 = tbs_cg_step polls never: it enqueues all n_iters iterations (those
                              after convergence return at once on the device) and the flush, and
                              with NULL rel_res_out and iters_out nothing in tbs_cg_begin +
                              tbs_cg_step waits on the host, so the pair can be captured into a HIP
                              graph and replayed (the other solvers poll every 4 iterations then). */
  int zchunk;              /* z-planes per workgroup of the stencil kernels (0 = automatic); operator
                              outputs do not depend on it (each output sums its terms in the same
                              order); dot products group their terms by workgroup, so it changes
                              them, and the CG iterates, at rounding level */
  int tile_order;          /* stencil tile order: 0 x-tiles fastest (default), 1 y-tiles fastest
                              (same effect on results as zchunk) */
  int nt_store;            /* 1: stencil outputs use non-temporal stores (no effect on results) */
  int fused_cg;            /* CG iteration form (every CG of the library):
                              1 = one kernel per iteration (default): r and p formed while staging,
                              q = A p, and FP64 sums of p.q, r.q, q.q and r.r; alpha = r.r / p.q from
                              the explicit r.r, beta and the stopping test from the one-step
                              prediction r.r - 2 alpha r.q + alpha^2 q.q; 0 = the two-kernel
                              Hestenes-Stiefel iteration (q = A p and p.q, then r -= alpha q and r.r).
                              FP32 (TBS_PREC_FP32, MIXED, MIXED_BF16, tbs_cg_step in F32) and FP64
                              (TBS_PREC_FP64, tbs_cg_step in F64, tbs_transform_interp and the
                              coarse-grid solve) alike. */
  int coarse_guess;        /* 1: tbs_timestep without a network starts from a coarse-grid guess
                              (Sec. 3 leg example: CG started from a reduced-grid solution): the
                              residual of u_prev is restricted to the halved grid, the coarse
                              system (same tau, spacing 2h) is solved by FP64 CG to coarse_rtol,
                              and its solution is prolongated by the two-scale relation and added;
                              kept only if its FP64 residual is smaller than that of u_prev.  Odd
                              degrees only (the coarse space nests in the fine one), periodic
                              grids need even sizes, every coarse size >= 2n+1 (TBS_E_INVAL
                              otherwise).  Enlarges tbs_workspace_bytes (default 0). */
  double coarse_rtol;      /* relative tolerance of the coarse solve (default 1e-2) */
  int guess_backoff;       /* tbs_timestep with a network: 0 = run and test the network guess on
                              every step (default); 1 = after the k-th consecutive rejection, skip
                              the network for the next min(2^(k-1), 64) steps (plain guess, no
                              network cost), then test it again; a kept guess resets k.  2 = cost
                              aware: as 1, but a kept guess resets k only if the iterations it
                              saved (learned_saved_iters) took longer than the network and its test
                              (learned_cost_iters, both timed with events on the stream); otherwise
                              it counts as a rejection and the wait is at least the number of such
                              steps it would take to pay once, min(64, cost / saving); a kept guess
                              that meets rtol without any iteration pays.  The
                              counters live in the context; tbs_set_opts resets them. */
  int guess_test;          /* how tbs_timestep judges the network output du (not in the paper):
                              0 = residual test (default): u^k + du is kept if its FP64 residual is
                              smaller than that of u^k.  1 = energy test: with r0 = b - A u^k, the
                              guess is u^k + gamma du, gamma = r0.du / du.A du (the multiple that
                              minimises the A-norm of the error; one FP32 apply and two dot
                              products), kept if that A-norm drops, i.e. 2 gamma r0.du - gamma^2
                              du.A du > 0; for the backoff a kept guess that does not halve the plain
                              guess's FP64 residual counts as a rejection. */
  int fused_rhs;           /* 1 (default): a source-free (q = NULL) refined tbs_timestep that starts
                              from the plain guess (no network run, no coarse guess) on a periodic or
                              Dirichlet grid forms b = M u^k and the first residual b - A u^k in one
                              pass over u^k (b bit for bit the rhs kernel's); 0: rhs kernel, then
                              residual kernel. */
} tbs_opts;

/* ---------------------------------------------------------------- context ---------------- */

/* Creates a context for an Nx x Ny x Nz grid (grid = {Nx, Ny, Nz}, each >= 2n+1), basis degree
 * 1..5, spacings h = {hx, hy, hz} > 0, time step tau > 0, boundary condition bc, and a HIP
 * stream (hipStream_t passed as void*, NULL = default stream).  Computes the taps of Sec. 2.3
 * in FP64 on the host.  Owns no device memory: see tbs_workspace_bytes. */
int tbs_setup(tbs_ctx** out, const int64_t grid[3], int degree, const double h[3], double tau,
              int bc, void* hip_stream);
void tbs_destroy(tbs_ctx* ctx);

/* Box domain with the Robin / penalty boundary branch (Sec. 2.2: the Robin condition adds half the
 * boundary integral of phi psi to the bilinear form; Sec. 2.3: the branch (1/(2 gamma)) int over
 * the boundary of b_k b_l in the discrete Ritz-Galerkin system, every domain integral restricted
 * to the box; a small gamma imposes phi = 0 weakly, the Dirichlet-by-penalty of the Sec. 3 leg
 * example).  The box is [0, Nc_d h_d] per axis and every B-spline whose support meets it is a basis
 * function: N_d = Nc_d + 1 + 2 floor(n/2) coefficients, index i <-> offset i - floor(n/2).  One
 * implicit step of du/dt = Lap u + f with du/dn + u / (2 gamma) = 0 solves
 *     A_R u^{k+1} = Mx My Mz (u^k + tau f),
 *     A_R = Mx My Mz + tau sum_d (h_d^-2 K_d + h_d^-1 E_d / (2 gamma)) [axis d; M on the others],
 * divided through by hx hy hz like the rest of the library; M_d, K_d are the box integrals (the
 * Toeplitz taps except in the first and last 2 floor(n/2) + 1 rows and columns), E_d the products
 * of the B-splines at the two end points of the axis.  The context then serves tbs_apply, tbs_rhs
 * (the box mass), tbs_residual, tbs_cg_begin / tbs_cg_step and tbs_timestep (all precisions, the
 * network guess with zero padding; not the coarse-grid guess) exactly as for TBS_BC_DIRICHLET.
 * gamma > 0; every N_d >= 4 floor(n/2) + 2 + n (TBS_E_INVAL otherwise). */
int tbs_setup_robin(tbs_ctx** out, const int64_t grid[3], int degree, const double h[3], double tau,
                    double gamma, void* hip_stream);

/* Device scratch needed by the solver entry points for precision mode prec (tbs_prec), or, with
 * prec = -1, by tbs_residual / tbs_dot only (partial sums); tbs_apply and tbs_rhs need none.  The
 * caller allocates it (256-byte aligned) and binds it; the library never allocates device memory.
 * Options that change the layout (tbs_set_opts: z-chunk, coarse guess) drop the binding. */
size_t tbs_workspace_bytes(const tbs_ctx* ctx, int prec);
int tbs_bind_workspace(tbs_ctx* ctx, void* dev_ptr, size_t bytes);

/* The 2(n+1) one-sided taps m_0..m_n, s_0..s_n in FP64 (host arrays of n+1 doubles each). */
int tbs_taps(const tbs_ctx* ctx, double* mass, double* stiff);

/* Options of the solver entry points (NULL restores the defaults). */
int tbs_set_opts(tbs_ctx* ctx, const tbs_opts* opts);

/* ------------------------------------------------------- operator (Sec. 2.4 / 2.5) ------- */

/* y = A u  (the system operator F(c), on-the-fly strategy of Sec. 2.5).
 * in_dtype / out_dtype: (F64,F64), (F32,F32), (BF16,F32), (F32,F64) or (BF16,F64); arithmetic
 * is FP64 when out is F64, FP32 otherwise.  Needs no workspace. */
int tbs_apply(tbs_ctx* ctx, const void* u, int in_dtype, void* y, int out_dtype);

/* Variable coefficients (Sec. 2.3: the diffusion coefficient D and the absorption coefficient
 * mu_a expanded in the solution's basis, D = sum d_m b_m, mu_a = sum m_m b_m; Sec. 2.4: the
 * domain branches of the tensor form F(c) = t with the three-index kernels f^{klm}, w^{klm}):
 *     y_l = sum_k sum_m u_k (m_m f^{klm} + d_m w^{klm}),
 *     f^{klm} = int b_k b_l b_m,  w^{klm} = int grad b_k . grad b_l b_m  (divided by hx hy hz),
 * computed on the fly (Sec. 2.5 strategy (c)) by exact cell-wise Gauss quadrature (ceil((3n+1)/2)
 * points per cell and axis) with sum factorisation.  u, d, m, y: N-element arrays of dtype F64 or
 * F32 (the arithmetic precision), layout [z][y][x]; u is zero beyond a Dirichlet box, d and m
 * continue beyond it by their edge values; periodic grids wrap.  With d = tau and m = 1 everywhere
 * y = A u.  Uses the context's grid, degree, spacings and boundary condition (tau is not used:
 * d carries it); periodic or Dirichlet solver contexts only (TBS_E_STATE otherwise).  Needs no
 * workspace; asynchronous. */
int tbs_apply_varcoef(tbs_ctx* ctx, const void* u, const void* d, const void* m, void* y, int dtype);

/* b = (Mx (x) My (x) Mz)(u_prev + tau q): right-hand side of one implicit Euler step.
 * q may be NULL (f = 0).  dtype F64 or F32 for all three arrays.  Needs no workspace. */
int tbs_rhs(tbs_ctx* ctx, const void* u_prev, const void* q, void* b, int dtype);

/* FP64 residual norms: *rnorm = ||b - A x||_2, *bnorm = ||b||_2 (x, b FP64).  If r != NULL the
 * residual is also written (r_dtype F64 or F32).  Synchronises the stream. */
int tbs_residual(tbs_ctx* ctx, const double* x, const double* b, void* r, int r_dtype,
                 double* rnorm, double* bnorm);

/* For callers that cannot allocate (code under HIP graph capture, allocation-free serving loops,
 * harnesses that forbid hipMalloc): the same FP64 residual as tbs_residual, computed by the same
 * kernels, but with its partial sums in a static device buffer the library owns (one per GPU,
 * held until the process ends; 256 + 2 * 8 * TBS_NOALLOC_MAX_BLOCKS bytes, about 1 MiB) and the
 * norms written to device memory: norms[0] = ||b - A x||_2, norms[1] = ||b||_2 (norms: device
 * pointer to 2 doubles, 8-byte aligned).  r (nullable, r_dtype F64 or F32) as in tbs_residual.
 * Needs no bound workspace, allocates nothing (no device memory, no pinned host memory, no
 * events) and does not synchronise: asynchronous on the context's stream, whose device must be
 * the current one.  TBS_E_INVAL if the residual launch of this grid needs more than
 * TBS_NOALLOC_MAX_BLOCKS workgroups (its launch has ceil(Nx/64) * ceil(Ny/8) * z-chunks of them;
 * roughly an x-y plane above 3e7 points, or a small tbs_opts.zchunk).  Every call on one GPU
 * uses that GPU's one buffer, which keeps the last call's values: calls that overlap in time on
 * one GPU (other streams or threads) race and must be serialised by the caller. */
#define TBS_NOALLOC_MAX_BLOCKS 65536
int tbs_residual_noalloc(tbs_ctx* ctx, const double* x, const double* b, void* r, int r_dtype, double* norms);

/* *out = sum_i a_i b_i with FP64 accumulation in a fixed order (bitwise reproducible).
 * dtype F64 or F32.  Synchronises the stream. */
int tbs_dot(tbs_ctx* ctx, const void* a, const void* b, int dtype, double* out);

/* Element conversion of N values: F64 -> F32 / BF16 (round to nearest even), F32 -> F64 / BF16,
 * BF16 -> F32 / F64. */
int tbs_convert(tbs_ctx* ctx, const void* src, int src_dtype, void* dst, int dst_dtype);

/* Copies `bytes` bytes from src to dst (device, 256-byte aligned, not overlapping) with 16-byte
 * accesses, four in flight per thread: the device-copy bandwidth reference for the kernels above
 * (not part of the method).  Asynchronous. */
int tbs_stream_copy(tbs_ctx* ctx, const void* src, void* dst, size_t bytes);

/* ------------------------------------------------------- CG (Sec. 2.5, step 3) ----------- */

/* Starts CG on A x = b in dtype (F64 or F32): r = b - A x, p = r, with state in the workspace
 * (bound for prec TBS_PREC_FP64 when dtype is F64, TBS_PREC_FP32 when F32).  b and x stay
 * caller-owned and must stay alive until the last tbs_cg_step.  Asynchronous. */
int tbs_cg_begin(tbs_ctx* ctx, const void* b, void* x, int dtype, double rtol);

/* Runs up to n_iters more CG iterations (the form tbs_opts.fused_cg selects: one kernel per
 * iteration, or the two-kernel Hestenes-Stiefel iteration) and stops once ||r|| <= rtol ||b||, r
 * being the recursive residual (one-kernel form: its one-step prediction), leaving x consistent.
 * It polls the device's convergence flag every tbs_opts.poll_every iterations (which synchronises);
 * with poll_every 0 it enqueues all n_iters and never waits.  If rel_res_out is not NULL it receives
 * ||r||/||b|| and iters_out the total iteration count (both synchronise).  Returns
 * TBS_E_BREAKDOWN on p^T A p <= 0 or non-finite values (with polling). */
int tbs_cg_step(tbs_ctx* ctx, int n_iters, double* rel_res_out, int* iters_out);

/* ------------------------------------------------------- implicit time step -------------- */

/* One implicit Euler step: solves A u_next = M (u_prev + tau q) to ||b - A u|| <= rtol ||b||.
 * u_prev, q (nullable), u_next: FP64 device arrays.  prec selects the arithmetic (tbs_prec).
 * net: optional learned initial guess, judged against the plain guess u_prev by the test
 * tbs_opts.guess_test selects (tbs_opts.guess_backoff: whether a rejected network is skipped on
 * the following steps).  u_next is output only (its prior contents are never read);
 * it holds the answer on TBS_OK, TBS_W_NOT_CONVERGED and TBS_E_BREAKDOWN and is unspecified
 * after any other error.  Synchronises; fills *stats if not NULL. */
int tbs_timestep(tbs_ctx* ctx, const double* u_prev, const double* q, double* u_next, int prec,
                 double rtol, int max_iter, tbs_net* net, tbs_stats* stats);

/* ------------------------------------------------------- B-spline transforms ------------- */
/* Table 1 (interpolation row), Sec. 2.3 (Fig. figBspnSignProc) and Sec. 2.5 (method overview,
 * steps 2 and 4): the indirect transform evaluates a spline at the grid nodes,
 * s_k = sum_l c_l b^n(k - l) with the sampled B-spline b^n_k = beta^n(k), tensor product over the
 * three axes; the direct transform inverts it, c = (b^n)^{-1} * s.  Same grid layout and boundary
 * conditions as the operator: periodic = circular convolution, Dirichlet = coefficients outside
 * the box are zero (truncated band).  The paper applies the inverse by recursive filtering; here
 * the direct transform is the FP64 CG solve of E c = s with E applied on the fly (E is SPD with
 * condition number below 8^3 for degrees 2..5), which reaches the same exact solution. */

/* Creates a transform context for an Nx x Ny x Nz grid and spline degree 2..5 (each N_d >=
 * 2 floor(degree/2) + 1), boundary condition bc, HIP stream.  tbs_destroy releases it;
 * tbs_workspace_bytes / tbs_bind_workspace with TBS_PREC_FP64 size its solver workspace;
 * tbs_apply and tbs_rhs on it also apply E; tbs_timestep refuses it (TBS_E_STATE). */
int tbs_transform_setup(tbs_ctx** out, const int64_t grid[3], int degree, int bc, void* hip_stream);

/* Indirect transform: samples = E coef.  dtype TBS_F64 or TBS_F32 for both arrays (device,
 * 256-byte aligned, not aliased).  Asynchronous.  TBS_E_STATE on a solver context. */
int tbs_transform_eval(tbs_ctx* ctx, const void* coef, void* samples, int dtype);

/* Direct transform: solves E coef = samples in FP64 by CG, stopping when the recursive residual
 * satisfies ||r|| <= rtol ||samples||, starting from the values coef holds on entry (a copy of the
 * samples is a good start).  *iters and *rel_res (nullable) receive the CG iterations and the
 * true FP64 relative residual recomputed at exit (near FP64 precision it can exceed rtol
 * slightly).  Synchronises.  Returns TBS_OK, TBS_W_NOT_CONVERGED or TBS_E_BREAKDOWN. */
int tbs_transform_interp(tbs_ctx* ctx, const double* samples, double* coef, double rtol, int max_iter,
                         int* iters, double* rel_res);

/* ------------------------------------------------------- learned initial guess ----------- */
/* Not in the paper (which warm-starts CG from a coarse-grid solution).  A 3-D CNN
 * Conv(2->16) GELU Conv(16->16) GELU Conv(16->16) GELU Conv(16->1), 3x3x3 kernels, "same"
 * padding (zero for Dirichlet, circular for periodic), exact erf GELU, bf16 operands on the
 * matrix cores with FP32 accumulation, predicts u^{k+1} - u^k from (u^k, f).
 * Parameters: 15,169 fp32 master weights, flat order W1 b1 W2 b2 W3 b3 W4 b4, W as
 * [C_out][C_in][3][3][3] over (dz, dy, dx).  Inputs are scaled by their RMS, the output by
 * tau * RMS(u^k) * out_scale. */

#define TBS_NET_PARAMS 15169

/* Creates a network object bound to a HIP stream (no device memory is allocated). */
int tbs_net_create(tbs_net** out, void* hip_stream);
void tbs_net_destroy(tbs_net* net);

/* Device scratch for a grid of Nx x Ny x Nz voxels and a batch: forward only (training = 0)
 * or training; bind before use.  The parameter block (weights, Adam moments) is included. */
size_t tbs_net_workspace_bytes(const int64_t grid[3], int batch, int training);
int tbs_net_bind_workspace(tbs_net* net, const int64_t grid[3], int batch, int training,
                           void* dev_ptr, size_t bytes);

/* Host <-> device parameter copies (n = TBS_NET_PARAMS fp32 values); set also resets Adam. */
int tbs_net_set_weights(tbs_net* net, const float* host, size_t n);
int tbs_net_get_weights(const tbs_net* net, float* host, size_t n);
/* Output multiplier out_scale (default 1) and the Adam learning rate (default 1e-3). */
int tbs_net_set_hparams(tbs_net* net, double out_scale, double lr);

/* du = network guess for one sample: u_k (F64 or F32 per dtype), q (nullable = zero source),
 * du (F32).  periodic selects circular padding. */
int tbs_net_forward(tbs_net* net, const void* u_k, const void* q, int dtype, float* du,
                    int periodic, double tau);

/* One training step on a batch of `batch` samples laid out back to back (F32 arrays of
 * batch x Nx*Ny*Nz): inputs u_k, q (nullable), targets du_target; loss = mean over the batch
 * of mean((net - du_target)^2 / (tau RMS(u_k) out_scale)^2).  Forward, backward (data and
 * weight gradients), Adam.  *loss_out (nullable) receives the loss (synchronises). */
int tbs_net_train_step(tbs_net* net, const float* u_k, const float* q, const float* du_target,
                       int batch, int periodic, double tau, float* loss_out);

/* Kernel-level probes for parity tests, on the bound workspace's grid, with the current weights
 * rounded to bf16.  mode 0: out[voxel][C_out] = conv(x, W_layer) + b (x: bf16 [voxel][C_in]);
 * mode 1: out[voxel][C_in] = transposed conv of g (bf16 [voxel][C_out]) with W_layer;
 * mode 2 (training workspace): out[C_out][C_in][27] then out[C_out] = weight and bias gradients
 * sum_v x[v + offset][ci] g[v][co] and sum_v g[v][co].  periodic selects circular padding. */
int tbs_net_conv_layer(tbs_net* net, int layer, int mode, const uint16_t* x, const uint16_t* g,
                       int periodic, float* out);
/* Gradient (TBS_NET_PARAMS fp32, flat parameter order) accumulated by the last train step. */
int tbs_net_get_grad(const tbs_net* net, float* host, size_t n);

/* ------------------------------------------------------- kernel timing --------------------- */
/* When enabled, the library brackets each launch of its bandwidth kernels with HIP events on
 * the context's stream and accumulates, per kernel kind, the elapsed time, the launches and the
 * algorithmic bytes (the bytes the method must move: each input element read once, each output
 * written once).  CG launches that found the solve already converged are not counted.
 * Kinds: 0 apply f64, 1 apply f32, 2 apply bf16->f32, 3 rhs f64, 4 rhs f32, 5 cg-fused f64,
 * 6 cg-fused f32, 7 cg-fused f32 with bf16 p, 8 residual f64, 9 cg-update f64, 10 cg-update f32,
 * 11 one-kernel CG iteration f32, 12 one-kernel CG iteration f32 with bf16 p, 13 variable-coefficient
 * apply f64, 14 variable-coefficient apply f32 (bytes: u, d, m read and y written once), 15 one-kernel
 * CG iteration f64, 16 fused rhs and residual f64 (u read, b and the FP32 r written). */
#define TBS_PROF_KINDS 17
int tbs_prof_enable(tbs_ctx* ctx, int on);   /* resets the counters */
int tbs_prof_read(tbs_ctx* ctx, int kind, double* total_ms, double* total_bytes, int64_t* launches);

/* ------------------------------------------------------- errors ---------------------------- */
const char* tbs_strerror(int code);
const char* tbs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TBS_H */
