/*
 * slrf.h - C ABI of the MI355X shifted-Laplace rational-filter eigensolver.
 *
 * The library computes eigenpairs of a sparse symmetric-definite pencil
 * A x = lambda B x in an interval (0, gamma] (Eq. (1) of the ParaSLRF paper)
 * by rational-filter subspace iteration (Algorithms 1 and 2).  Its hot path is
 * the filter application of Eq. (2)-(3) with conjugate-pole halving
 * (Section 2):
 *
 *     U = sum_{j=1}^{N} 2 Re( w_j (A - sigma_j B)^{-1} B X ),
 *
 * one complex shifted system per upper-half-plane pole sigma_j and per column
 * of X, each solved by restarted right-preconditioned GCR (Section 3.2) to the
 * relative residual ||f - M y||_2 / ||f||_2 <= tol_lin, or truncated at
 * It_max-linear (Section 4).  All (pole, column) systems of a call run as one
 * batch on one GPU.
 *
 * Conventions shared by every entry point:
 *  - Device pointers are HIP device addresses on the device that was current
 *    when slrf_setup ran; host pointers are ordinary host memory.
 *  - Dense real blocks (X, U, V, ...) are column-major n x ncols FP64 with
 *    leading dimension n, unless stated otherwise.
 *  - Every call is ordered on the stream given to slrf_setup.  Calls that
 *    return host results (statistics, counts, eigenvalues in host memory)
 *    synchronise that stream before returning.
 *  - Status codes are returned; no exception crosses the ABI.  After an error
 *    slrf_last_error(h) returns a message (thread-unsafe per handle).
 *  - A handle must not be used from two host threads at once.
 *  - All device memory is the caller's: inputs, outputs and the workspace
 *    given to slrf_setup (sized by slrf_workspace_size).
 */
#ifndef SLRF_H
#define SLRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slrf_ctx* slrf_handle;

/* ABI-stable complex double (real part first, as in C99 double complex). */
typedef struct {
  double re, im;
} slrf_zd;

typedef enum {
  SLRF_OK = 0,
  SLRF_E_ARG = 1,       /* invalid argument (null pointer, bad size, malformed CSR, ...) */
  SLRF_E_NOMEM = 2,     /* device or host allocation failed / over the memory budget   */
  SLRF_E_HIP = 3,       /* a HIP runtime call failed                                   */
  SLRF_E_BREAKDOWN = 4, /* projected B-Gram not positive definite even after fallback  */
  SLRF_E_NOCONV = 5,    /* iteration cap reached; partial results are written          */
  SLRF_E_NUMERIC = 6,   /* NaN or Inf detected in a residual norm                       */
  SLRF_E_NOGPU = 7      /* no usable gfx950 device                                      */
} slrf_status;

enum { SLRF_PREC_FP64 = 0, SLRF_PREC_MIXED = 1 };
enum { SLRF_PC_NONE = 0, SLRF_PC_JACOBI = 1, SLRF_PC_AMG = 2 };

/*
 * Sparse matrix in CSR form, device memory, owned by the caller.
 * rowptr: int32[n+1], rowptr[0] = 0, nondecreasing, rowptr[n] = nnz.
 * col:    int32[nnz], strictly increasing within each row, 0 <= col < n.
 * val:    double[nnz].
 * A and B passed to slrf_setup must have identical rowptr/col contents (one
 * shared pattern; store explicit zeros where only one matrix has an entry) and
 * every row must hold its diagonal entry.
 */
typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
} slrf_csr;

/*
 * Solver options.  slrf_default_options fills the paper's settings:
 * tol_lin 1e-10 and maxit_lin 10000 (Section 3.2), tol_eig 1e-8 (Section 3.2
 * residual test), max_outer 100 (Section 4), restart 30, FP64, Jacobi.
 */
typedef struct {
  int32_t precision;   /* SLRF_PREC_FP64: complex FP64 Krylov sweeps.
                          SLRF_PREC_MIXED: complex FP32 Krylov sweeps inside an
                          FP64 residual / iterative-refinement loop.           */
  int32_t precond;     /* SLRF_PC_JACOBI: point Jacobi on A - sigma_j B;
                          SLRF_PC_AMG: one V-cycle of a smoothed-aggregation
                          hierarchy built once from A and shared by all poles
                          (levels A_l - sigma_j B_l, damped-Jacobi smoothing,
                          dense coarsest solve); SLRF_PC_NONE                  */
  int32_t restart;     /* GCR restart length m, 1..32                           */
  int32_t maxit_lin;   /* cap on inner iterations per system (10000)            */
  int32_t it_max_lin;  /* Algorithm 2 It_max-linear; 0 = off; -1 = automatic in
                          slrf_solve: the first outer iteration solves to
                          tol_lin, and half the median of its iteration counts
                          (at least 3) caps the later warm-started ones     */
  int32_t max_outer;   /* outer iteration cap for slrf_solve                    */
  int32_t warm_start;  /* slrf_solve: Y_init = v/(theta - sigma) (Algorithm 2)   */
  int32_t lock;        /* slrf_solve: locking + B-orthogonalisation (Alg. 2)    */
  int32_t timing;      /* record per-kernel HIP event timings into the stats    */
  int32_t max_slots;   /* systems resident at once (multiple of 16); 0 = auto   */
  int32_t spmm_variant;/* shifted SpMM kernel: 0 = autotuned at setup (every
                          variant timed on the pencil, fastest kept per
                          precision, cached per shape class), 1 = row-group
                          union format, 2 / 4 / 5 = CSR staged in LDS with
                          8 / 16 / 32 gathers in flight per lane, 3 = CSR
                          read directly, 6 = halo tiles (the gathered operand
                          staged in LDS per tile of rows), 7 = wave-uniform
                          groups of 4 rows (distinct columns of the group
                          once, coefficients through scalar loads)           */
  int32_t reorder;     /* 1 (default): the library keeps a copy of the pencil
                          in a locality row order (nested aggregation of the
                          graph of A) so stencil gathers stay cache-resident;
                          inputs/outputs keep the caller's order.  0: off.    */
  double tol_lin;      /* relative residual target of each shifted solve        */
  double inner_rtol;   /* MIXED: a Krylov cycle stops once its residual fell by
                          this factor (then the FP64 residual is recomputed)    */
  double tol_eig;      /* Ritz pair converged when ||r||_2 < tol_eig             */
  int32_t amg_block;   /* dofs per node for the AMG aggregation and the row
                          order (node-major numbering: dof = block*node + c):
                          0 = detect (3 or 2 when every node's rows share one
                          column list of whole node blocks, else 1), 1 = scalar
                          aggregation, 2..8 = given (n must be a multiple)    */
  const double* node_xyz; /* host, may be NULL: coordinates of the n / block
                          nodes (block values per node, node-major, the caller's
                          numbering) of a 2D / 3D elasticity pencil (block 2
                          or 3).  With SLRF_PC_AMG the hierarchy's tentative
                          prolongator then carries the rigid-body modes
                          (translations and rotations) instead of the
                          translations alone.  Read by slrf_workspace_size
                          and slrf_setup only.                               */
  int32_t amg_setup;   /* where the AMG hierarchy is built (SLRF_PC_AMG only):
                          SLRF_AMG_HOST (default): all of it on the host, by
                          slrf_workspace_size's and slrf_setup's shared
                          analysis; SLRF_AMG_DEVICE: the aggregation and the
                          tentative prolongators on the host, each level's
                          products (rho(D^-1 A) by power steps, A T, the
                          smoothed prolongator P and R = P^T, A P, B P and the
                          Galerkin products P^T A P, P^T B P: the construction
                          phase of the smoothed aggregation the paper's
                          GAMG reuse implies, Section 3.2) on the GPU inside
                          slrf_setup, in the caller's workspace, with values
                          equal to the host build's.  slrf_workspace_size then
                          cannot see the hierarchy and returns a bound; setup
                          fails with SLRF_E_NOMEM (message: the bytes needed)
                          when the workspace is too small, and with SLRF_E_ARG
                          when a product row has more than 1024 distinct
                          columns.  Fixed at setup.                          */
  int32_t amg_coarse_min; /* smallest coarse level of the AMG hierarchy, 0..2048;
                          0 (default): off.  Where an aggregation would leave
                          fewer coarse dofs, the strength threshold is raised
                          (0.01, 0.02, ... 0.64) to the first value that leaves
                          at least this many while still halving the level;
                          failing that, a level small enough for the dense
                          solve becomes the coarsest, and a larger one takes
                          the largest halving coarse space the thresholds gave.  The shifted systems are
                          indefinite on the modes below Re sigma_j, which the
                          smoothing cannot damp and only the coarse correction
                          reaches: a coarsest level of a few times the number
                          of eigenvalues in (0, gamma] keeps the inner
                          iteration counts low (3D Q1, n = 262,144, 102
                          eigenvalues: 512 instead of 125 coarse dofs).
                          Fixed at setup.                                    */
} slrf_options;

enum { SLRF_AMG_HOST = 0, SLRF_AMG_DEVICE = 1 };

/* Per-kernel-class counters (algorithmic bytes, launches, event time). */
enum {
  SLRF_K_APPLY = 0, /* shifted SpMM q = (A - sigma B) z fused with the CGS dots */
  SLRF_K_ORTH = 1,  /* CGS update of q with <q, q> and <q, r>                    */
  SLRF_K_STEP = 2,  /* r -= alpha q, z = P^-1 r, ||r||                            */
  SLRF_K_RESID = 3, /* FP64 residual f - (A - sigma B) y and solution update      */
  SLRF_K_REDUCE = 4,/* second-stage reductions and per-system scalars             */
  SLRF_K_OTHER = 5, /* admission, compaction, filter sum, RHS SpMM, transposes    */
  SLRF_K_PRECOND = 6,/* AMG V-cycle (all levels)                                 */
  SLRF_K_SWEEP = 7,  /* the fine-level operator sweep alone (halo-tile SpMM: the
                        GCR apply without its projections and the V-cycle's
                        level-0 residual and smoothing sweeps); an overlay:
                        these launches are also counted in APPLY / PRECOND    */
  SLRF_K_COUNT = 8
};

typedef struct {
  int64_t nsystems;      /* N * ncols                                             */
  int64_t total_iters;   /* inner GCR iterations summed over systems              */
  int32_t min_iters, max_iters;
  int32_t cycles;        /* Krylov cycles (restart / refinement boundaries)       */
  int32_t converged;     /* systems that met tol_lin                              */
  int32_t capped;        /* systems stopped by it_max_lin or maxit_lin            */
  int32_t max_pole_iters_ratio_x1000; /* 1000 * max/min over poles of the summed
                                         iterations (the single-GPU analogue of
                                         the paper's Ratio, Table 1)           */
  double max_rel_resid;  /* max final FP64 relative residual over systems         */
  double seconds;        /* wall time of the call                                 */
  int64_t launches[SLRF_K_COUNT];
  double bytes[SLRF_K_COUNT]; /* algorithmic HBM bytes                             */
  double ms[SLRF_K_COUNT];    /* summed kernel time (only with options.timing)     */
  int32_t spmm_variant;  /* SpMM kernel used for the Krylov sweeps (the
                            options.spmm_variant codes; 0 = default choice)   */
  double sweep_systems;  /* systems swept, summed over the SWEEP-class launches
                            (flops of those launches = 8 * nnz * sweep_systems) */
  int32_t basis_bf16;    /* 1 when the Krylov cycles kept their Gram-Schmidt basis
                            in complex bfloat16 (mixed precision, halo sweep,
                            restart <= 9, cold start), else 0                  */
  int32_t* sys_iters;    /* optional, caller-owned host int32[N*ncols]: iterations
                            of system (column c, pole j) at index c*N + j          */
} slrf_filter_stats;

typedef struct {
  int32_t outer_iters;
  int32_t nconv;
  int32_t auto_it_max;   /* the cap chosen for it_max_lin = -1 (else 0)           */
  int64_t inner_iters;   /* summed over all filter calls                          */
  double seconds;
  double filter_seconds;
  double rr_seconds;
} slrf_solve_stats;

const char* slrf_status_string(slrf_status s);
const char* slrf_last_error(slrf_handle h);
void slrf_default_options(slrf_options* opt);

/*
 * slrf_workspace_size - device workspace a handle needs (the caller allocates
 * it, e.g. as a torch tensor, and passes it to slrf_setup).
 * A, B: the CSR pencil as for slrf_setup (read and validated here: the host
 * analysis of the pencil is kept and reused by the next slrf_setup on the same
 * contents and options).  L: the widest block a call will be given (subspace
 * width of slrf_solve, columns of slrf_filter / slrf_rayleigh_ritz); npoles:
 * poles of the table; opt: the options of the handle (NULL = defaults).
 * *full_bytes: the pencil's persistent data (permuted copy, sweep formats,
 * FP32 values, AMG hierarchy when opt->precond is SLRF_PC_AMG) plus the
 * buffers of a solve with all npoles * L shifted systems resident at once;
 * *min_bytes (may be NULL): the same with one panel of 16 resident systems
 * (a filter then streams the systems through the panel).  Any size in
 * between works; more resident systems run faster.  Host memory only.
 * Errors: SLRF_E_ARG (null pointers, L < 1, bad options, malformed CSR).
 */
slrf_status slrf_workspace_size(const slrf_csr* A, const slrf_csr* B, int32_t L, int32_t npoles,
                                const slrf_options* opt, size_t* full_bytes, size_t* min_bytes);

/*
 * slrf_setup - bind a pencil, an interval and a pole/weight table.
 * A, B: CSR descriptors (device arrays, caller-owned; must stay valid and
 *   unchanged until slrf_destroy).  Validated on the host (a copy is read).
 * gamma: upper end of the interval (0, gamma], > 0.
 * npoles, poles, weights: the N upper-half-plane poles (Im > 0) and weights,
 *   host arrays; conjugates are implied (Section 2).  1 <= N <= 64.
 * opt: options (NULL = defaults).
 * workspace, ws_bytes: caller-owned device memory (any alignment) that the
 *   handle uses for all its device data until slrf_destroy: setup places the
 *   pencil's persistent data at its start and every later call carves its
 *   buffers from the rest and releases them on return.  The library
 *   allocates no device memory of its own.  Size it with slrf_workspace_size.
 * stream: hipStream_t (NULL = null stream).
 * Errors: SLRF_E_ARG for malformed input, SLRF_E_NOMEM when the workspace
 * cannot hold the persistent data, SLRF_E_NOGPU, SLRF_E_HIP.  A later call
 * whose buffers do not fit the free part of the workspace returns
 * SLRF_E_NOMEM with the missing byte count in slrf_last_error.
 */
slrf_status slrf_setup(slrf_handle* h, const slrf_csr* A, const slrf_csr* B, double gamma,
                       int32_t npoles, const slrf_zd* poles, const slrf_zd* weights,
                       const slrf_options* opt, void* workspace, size_t ws_bytes, void* stream);

/* Frees the handle (host memory; the workspace stays the caller's).  NULL is a no-op. */
void slrf_destroy(slrf_handle h);

/* Replace options after setup (same validation as setup).  reorder and
 * amg_block cannot change, and SLRF_PC_AMG needs a handle set up with it
 * (the hierarchy lives in the workspace): SLRF_E_ARG otherwise. */
slrf_status slrf_set_options(slrf_handle h, const slrf_options* opt);

/*
 * slrf_filter - U = sum_j 2 Re(w_j Y_j), (A - sigma_j B) Y_j = B X
 * (Eq. (2)-(3); Algorithm 1 solve and sum-reduce steps).
 * X: device, n x ncols column-major.  U: device, n x ncols column-major
 * (may not alias X).  theta_warm: device double[ncols] or NULL; when given,
 * the solve of column c for pole j starts from y0 = x_c / (theta_c - sigma_j)
 * and its initial residual is taken from Proposition 4.1 as
 * (A - theta_c B) x_c / (sigma_j - theta_c) (no complex SpMM).
 * stats: host, may be NULL.
 * Returns SLRF_E_NOCONV when some system stopped at maxit_lin without meeting
 * tol_lin (U is still written); it_max_lin truncation is not an error.
 */
slrf_status slrf_filter(slrf_handle h, int32_t ncols, const double* X, const double* theta_warm,
                        double* U, slrf_filter_stats* stats);

/*
 * slrf_rayleigh_ritz - projected problem (U^T A U) s = theta (U^T B U) s
 * (Algorithm 1, Rayleigh-Ritz step), theta ascending, v = U s with
 * ||v||_B = 1, and the residual norms ||(A - theta B) v||_2 / (theta ||v||_B)
 * (Section 3.2).  When nlocked > 0, U is first B-orthogonalised twice against
 * the B-orthonormal locked block Xlocked (Algorithm 2).
 * U: device n x ncols column-major, overwritten by the Ritz vectors V.
 * Xlocked: device n x nlocked column-major or NULL when nlocked == 0.
 * theta, resid: device double[ncols].
 * Returns SLRF_E_BREAKDOWN if U^T B U is numerically singular beyond repair.
 */
slrf_status slrf_rayleigh_ritz(slrf_handle h, int32_t ncols, double* U, int32_t nlocked,
                               const double* Xlocked, double* theta, double* resid);

/*
 * slrf_solve - Algorithm 1 (opt.lock = opt.warm_start = 0, it_max_lin = 0) or
 * Algorithm 2 (locking, warm start, It_max-linear).
 * nev: wanted eigenpairs in (0, gamma]; L >= nev: subspace width.
 * V1: device n x L column-major start block (not modified).
 * theta_out: device double[nev]; X_out: device n x nev column-major
 * (B-orthonormal eigenvectors, ascending eigenvalues); nconv_out: host.
 * Returns SLRF_E_NOCONV with partial results when max_outer is reached.
 */
slrf_status slrf_solve(slrf_handle h, int32_t nev, int32_t L, const double* V1, double* theta_out,
                       double* X_out, int32_t* nconv_out, slrf_solve_stats* stats);

/*
 * slrf_filter_batch / slrf_solve_batch - many independent pencils at once
 * (the batched form of Eq. (2)-(3) and of Algorithm 1 / 2 over uneven-sized
 * problems).  Entry i is exactly slrf_filter / slrf_solve on hs[i] with the
 * i-th arguments; the calls run concurrently from up to nthreads host threads
 * (0 = min(nh, 8)), largest problems first, each on its handle's stream, so
 * the GPU overlaps the kernels of different pencils.  Give every handle its
 * own stream (handles that share a stream still give correct results, run
 * serially on the GPU).  Handles must be distinct.  Per-entry arguments are
 * arrays of length nh (theta_warm, stats, nconv_out may be NULL; their
 * entries may be NULL).  Results are identical to the single calls (each
 * handle's arithmetic does not depend on what runs beside it).  Each handle
 * works in its own workspace (the batch's device memory is the sum of the
 * workspaces the caller gave the handles).  Returns
 * SLRF_OK if every entry succeeded, else the status of the first failing
 * entry in index order (all entries are still attempted; a failing handle's
 * message is in its slrf_last_error).
 */
slrf_status slrf_filter_batch(int32_t nh, const slrf_handle* hs, const int32_t* ncols,
                              const double* const* X, const double* const* theta_warm,
                              double* const* U, slrf_filter_stats* stats, int32_t nthreads);
slrf_status slrf_solve_batch(int32_t nh, const slrf_handle* hs, const int32_t* nev,
                             const int32_t* L, const double* const* V1,
                             double* const* theta_out, double* const* X_out,
                             int32_t* nconv_out, slrf_solve_stats* stats, int32_t nthreads);

/*
 * slrf_shifted_spmm - one sweep of the shifted operator over a batch of
 * complex block vectors, Q_s = (A - sigma_{pole[s]} B) Z_s (Eq. (2) operator).
 * Z, Q: device, "panel layout": systems in panels of 16; element (row i of the
 * internal row order, see slrf_get_row_order, system s) at complex index
 * ((s / 16) * n + i) * 16 + s % 16, interleaved
 * (re, im); nsys is rounded up to a multiple of 16 and padding systems must
 * be allocated.  precision SLRF_PREC_FP64: complex double; SLRF_PREC_MIXED:
 * complex float (with FP32 copies of A and B).  pole: host int32[nsys],
 * indices into the setup pole table.  Exposed for kernel parity tests and
 * bandwidth measurement.
 */
slrf_status slrf_shifted_spmm(slrf_handle h, int32_t nsys, const int32_t* pole, int32_t precision,
                              const void* Z, void* Q, double* ms_out);

/*
 * slrf_shifted_spmm_noalloc - slrf_shifted_spmm for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same sweep, bitwise the same Q, with
 * the per-system pole table kept in a fixed library array of 65536 entries
 * (1 MiB per GPU the library runs on, held until the process ends) instead of
 * library workspace.  The call allocates no device memory; the caller passes
 * Z and Q exactly as for slrf_shifted_spmm (no timing output).  Errors:
 * SLRF_E_ARG when nsys rounded up to 16 exceeds 65536, for a bad pole index or
 * null pointers.  Every call on one GPU shares that GPU's table, which keeps
 * the last call's contents: calls that overlap on one GPU (other host threads,
 * other streams) race and must be serialised by the caller.  Synchronises the
 * stream before returning.
 */
slrf_status slrf_shifted_spmm_noalloc(slrf_handle h, int32_t nsys, const int32_t* pole,
                                      int32_t precision, const void* Z, void* Q);

/*
 * slrf_eig_grad - eigenvalue sensitivities for per-element parameters
 * (the differentiation form).  For B-normalised eigenpairs (lam_i, x_i) and a
 * loss gradient glam_i = dL/dlam_i:
 *     grad[e] = sum_{i<k} glam_i * x_{i,e}^T (dA_e - lam_i dB_e) x_{i,e},
 * the derivative of the Rayleigh quotient, with dA_e = dA/dtheta_e and
 * dB_e = dB/dtheta_e acting on element e's dofs.
 * X: device n x k column-major; lam, glam: device double[k];
 * elem_dofs: device int32[nelem * ndof_e] row-major, -1 = constrained dof
 * (contributes zero), otherwise 0 <= dof < n; ndof_e in {4, 8, 24} (bilinear,
 * trilinear, trilinear elasticity); dA: device double, element e's
 * ndof_e x ndof_e row-major matrix at dA + e * dA_stride (stride 0: one matrix
 * shared by all elements, else stride >= ndof_e^2), dA_len doubles readable at
 * dA; dB, dB_stride, dB_len likewise, or dB NULL (parameter does not enter B);
 * grad: device double[nelem].
 * Errors: SLRF_E_ARG for a dof outside [-1, n), a stride below ndof_e^2 or an
 * element matrix that would end past dA_len / dB_len (checked on the host,
 * elem_dofs is copied there, before any kernel runs).  Synchronises the stream.
 */
slrf_status slrf_eig_grad(slrf_handle h, int32_t k, const double* X, const double* lam,
                          const double* glam, int32_t nelem, int32_t ndof_e,
                          const int32_t* elem_dofs, const double* dA, int32_t dA_stride,
                          int64_t dA_len, const double* dB, int32_t dB_stride, int64_t dB_len,
                          double* grad);

/*
 * slrf_host_check_grad_args - the host checks slrf_eig_grad makes on its
 * element data, on host arrays (no GPU): elem_dofs host int32[nelem * ndof_e];
 * has_dB nonzero when a dB array is passed.  Returns SLRF_OK or SLRF_E_ARG.
 */
int32_t slrf_host_check_grad_args(int32_t n, int32_t nelem, int32_t ndof_e,
                                  const int32_t* elem_dofs, int32_t dA_stride, int64_t dA_len,
                                  int32_t has_dB, int32_t dB_stride, int64_t dB_len);

/* Problem size of a handle (-1 for NULL). */
int32_t slrf_get_n(slrf_handle h);

/*
 * slrf_get_row_order - the library's internal row order: order[new] = old
 * (host int32[n]).  Identity unless options.reorder was set at setup.  Only
 * slrf_shifted_spmm exposes internal-order vectors.
 */
slrf_status slrf_get_row_order(slrf_handle h, int32_t* order);

/*
 * slrf_host_projected_eig - host-only solve of the small projected problem
 * Ah s = theta Bh s (Algorithm 1, Rayleigh-Ritz step) as used inside
 * slrf_rayleigh_ritz: Ah, Bh symmetric n x n row-major host arrays (Bh
 * positive definite; if Cholesky fails, directions of Bh with eigenvalue below
 * 1e-14 of the largest are dropped), theta host double[n] ascending, S host
 * n x n row-major with S^T Bh S = I.  Returns the number of pairs (n, or fewer
 * after truncation, trailing theta = +inf) or -1.  Makes no GPU call.
 */
int32_t slrf_host_projected_eig(int32_t n, const double* Ah, const double* Bh, double* theta,
                                double* S);

#ifdef __cplusplus
}
#endif

#endif /* SLRF_H */
