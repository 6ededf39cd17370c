/*
 * rb.h -- C ABI of the MI355X (gfx950) reduced-basis solver library (librb.so).
 *
 * Method: Nguyen & Chen, "Reduced-basis method for the iterative solution of
 * parametrized symmetric positive-definite linear systems".  The library solves
 * many instances of the parametrized SPD system A(mu) x(mu) = f(mu) (eq. 1) whose
 * operator and right-hand side are affine in the parameters (eq. 12, Sec. 2.3):
 *
 *     A(mu) = sum_{q<Q} Theta_q(mu) A_q,      f(mu) = sum_{r<R} Phi_r(mu) f_r.
 *
 * The caller evaluates Theta_q(mu) and Phi_r(mu) on the host and passes them per
 * query.  Solvers: RB-preconditioned CG (Alg. 3, Sec. 4.1), the stand-alone RB
 * iteration (Alg. 2, Sec. 3.1) and plain CG.  The reduced basis W comes from the
 * adaptive greedy (Alg. 4, Sec. 4.2) or from the caller.
 *
 * Conventions
 *  - Every function returns rb_status.  No C++ exception crosses this ABI.
 *  - On a non-OK return nothing has been written to caller outputs, and
 *    rb_last_error() returns a message (thread-local, valid until the next call on
 *    the same thread).
 *  - Per-query failures (not SPD, no convergence, breakdown) are reported in
 *    rb_query_stats.status; the call still returns RB_OK and other queries are
 *    unaffected.
 *  - Handles are owned by the library and freed with their *_destroy call.
 *  - Host arrays passed in are borrowed for the duration of the call (copied).
 *  - Vectors exchanged with the caller use the natural lexicographic ordering of
 *    the grid (x fastest).  "DEVICE" pointers are HIP device memory owned by the
 *    caller (e.g. a torch tensor's data_ptr()); all others are host memory.
 *  - All work is ordered on the context's HIP stream.  Calls that return host
 *    results (stats, reports) synchronise that stream before returning.
 *  - One rb_ctx per host thread.  Calls that overlap on one context race.
 */
#ifndef RB_H_
#define RB_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RB_OK = 0,
  RB_EINVAL = 1,       /* bad argument (null pointer, size, NaN parameter, ...) */
  RB_ENOMEM = 2,       /* device allocation failed; nothing left allocated */
  RB_EDEVICE = 3,      /* HIP runtime error */
  RB_ENOTSPD = 4,      /* reduced matrix A_N(mu) not SPD (Cholesky breakdown) */
  RB_ENOCONV = 5,      /* maxit reached before the tolerance */
  RB_EBREAKDOWN = 6,   /* p^T A p <= 0 or y^T r <= 0 in CG */
  RB_EDEGENERATE = 7,  /* snapshot already in span(W) (Gram-Schmidt) */
  RB_EUNSUPPORTED = 8, /* valid request this build does not handle */
  RB_EIO = 9           /* file read/write failure */
} rb_status;

typedef enum { RB_PREC_FP64 = 0, RB_PREC_FP32 = 1, RB_PREC_BF16 = 2 } rb_prec;
typedef enum { RB_SOLVER_RBCG = 0, RB_SOLVER_RBI = 1, RB_SOLVER_CG = 2 } rb_solver;
typedef enum { RB_IND_RESIDUAL = 0, RB_IND_L1 = 1 } rb_indicator;
typedef enum {
  RB_SMOOTH_RBGS = 0,     /* one forward red-black Gauss-Seidel sweep, red first */
  RB_SMOOTH_RBGS_SYM = 1, /* forward then backward red-black sweep */
  RB_SMOOTH_JACOBI = 2,   /* one damped Jacobi step, omega = 2/3 */
  RB_SMOOTH_NONE = 3      /* no smoothing (Lemma 2 of Sec. 3.2: RBI stagnates) */
} rb_smoother;

typedef struct rb_ctx rb_ctx;
typedef struct rb_problem rb_problem;
typedef struct rb_basis rb_basis;

/* Context: a device and a HIP stream.  hip_stream == NULL: the library creates its
 * own blocking stream (default priority), which orders after work on the null
 * stream; otherwise the caller's stream is used and must outlive the context.
 * HIP-graph replay (use_graph) needs a stream other than the null stream. */
rb_status rb_ctx_create(int device, void* hip_stream, rb_ctx** out);
rb_status rb_ctx_destroy(rb_ctx* ctx);
const char* rb_last_error(void);
/* Library version string, e.g. "rb 0.1 gfx950". */
const char* rb_version(void);

/* Per-kernel timing: when on, every kernel class launched by the solvers is bracketed
 * by HIP events on the context's stream (not inside captured graphs).  Entries are
 * accumulated per kernel name; rb_profile_get returns entry idx (0-based) and fails
 * with RB_EINVAL past the last one.  name is NUL-terminated, truncated to name_len. */
rb_status rb_profile_enable(rb_ctx* ctx, int on);
rb_status rb_profile_reset(rb_ctx* ctx);
rb_status rb_profile_get(rb_ctx* ctx, int idx, char* name, size_t name_len, double* ms,
                         int64_t* launches);

/* ---- Problems: the affine operator of eq. (12) ------------------------------
 * Matrix-free block diffusion: -div(kappa grad u) = f on the unit square/cube,
 * u = 0 on the boundary, finite differences with n[a] interior nodes per axis
 * (h_a = 1/(n[a]+1)), kappa constant on blocks[0] x blocks[1] x blocks[2]
 * rectangular blocks.  Face coefficients are the mean of kappa over the face's dual
 * cell, so A_q is the operator with kappa = indicator of block q (block number
 * q = bx + blocks[0]*(by + blocks[1]*bz)) and Q = prod(blocks).
 * Requirements: dim in 1..3; (n[a]+1) % blocks[a] == 0; n[0] odd if dim >= 2 and
 * n[1] odd if dim == 3 (red-black colouring by index parity); Q <= 64.
 * Default right-hand side: R = 1, f_1 = 1. */
typedef struct {
  int dim;
  int n[3];
  int blocks[3];
} rb_stencil_desc;
rb_status rb_problem_create_stencil(rb_ctx* ctx, const rb_stencil_desc* desc, rb_problem** out);

/* General sparse affine problem A(theta) = sum_q theta_q A_q (eq. 12, Sec. 2.3) with all Q
 * terms on one pattern: rowptr [N+1] (int64), col [nnz] (int32, strictly increasing within
 * a row, every row holding its diagonal), vals [Q][nnz] (term q's values on the pattern,
 * zeros allowed); host arrays, copied.  The caller guarantees A(theta) SPD for the thetas
 * it solves with (a symmetric pattern and symmetric terms).  The Gauss-Seidel smoother
 * colours the unknowns greedily (first fit in natural order on the symmetrised pattern)
 * and sweeps the colour classes in increasing order; at most 32 classes.  N < 2^30,
 * nnz < 2^31, Q <= 64.  Default right-hand side R = 1, f = 1.  Errors: RB_EINVAL for
 * malformed arrays or non-finite values, RB_EUNSUPPORTED beyond the limits. */
rb_status rb_problem_create_csr(rb_ctx* ctx, int64_t N, int Q, const int64_t* rowptr,
                                const int32_t* col, const double* vals, rb_problem** out);
/* Colour class of every unknown (natural order, [N] host) and the number of classes. */
rb_status rb_problem_colors(const rb_problem* prob, int32_t* color, int* ncolors);
/* Replace the right-hand-side terms f_r: f is [R][N] host, natural ordering. */
rb_status rb_problem_set_rhs(rb_problem* prob, int R, const double* f);
/* Query sizes: any output pointer may be NULL. */
rb_status rb_problem_info(const rb_problem* prob, int64_t* N, int* Q, int* R);
rb_status rb_problem_destroy(rb_problem* prob);

/* ---- Reduced bases -----------------------------------------------------------
 * W: [n][N] host, column j = basis vector w_j (natural ordering), assumed
 * orthonormal.  The library precomputes A_{N,q} = W^T A_q W and f_{N,r} = W^T f_r
 * (eq. 12c) on the device. */
rb_status rb_basis_from_host(rb_ctx* ctx, const rb_problem* prob, int n, const double* W,
                             rb_basis** out);
/* n, and optional copies: W [n][N] natural ordering, AN [Q][n][n], fN [R][n]. */
rb_status rb_basis_info(const rb_basis* basis, int* n, double* W, double* AN, double* fN);
/* Binary file: header, W (FP64), sample indices, A_{N,q}, f_{N,r}. */
rb_status rb_basis_save(const rb_basis* basis, const char* path);
rb_status rb_basis_load(rb_ctx* ctx, const rb_problem* prob, const char* path, rb_basis** out);
rb_status rb_basis_destroy(rb_basis* basis);

/* ---- Online solves (Alg. 3 RBCG, Alg. 2 RBI, plain CG) -----------------------
 * Stopping rule: ||r_k|| <= rtol ||f|| on the recursive residual, confirmed on the
 * true residual f - A x in FP64 (eq. relerr of Sec. 5.1); if the true residual
 * fails, r is replaced by it and CG restarts from p = y.  iters = number of A p
 * products (RBCG/CG) or of RB iterations (RBI).
 * precond_prec: FP64 = everything in FP64; FP32 / BF16 = the preconditioner's
 * contractions W^T r and W e in FP32 / BF16 with FP32 accumulation and the
 * smoother and y in FP32, while x, r, p, every CG dot product, alpha, beta, the
 * true residual and the reduced Cholesky stay FP64.
 * beta_flexible: 0 = the ratio of Alg. 3, y_{k+1}^T r_{k+1} / y_k^T r_k;
 * 1 = y_{k+1}^T (r_{k+1}-r_k) / y_k^T r_k.  use_graph: replay captured HIP graphs of the iteration.
 * fixed_iters > 0: run exactly that many iterations, no stopping test (testing). */
typedef struct {
  size_t struct_size; /* sizeof(rb_solve_opts) */
  rb_solver solver;
  rb_prec precond_prec;
  rb_smoother smoother;
  double rtol;     /* default 1e-10 */
  int maxit;       /* default 2000 */
  int beta_flexible;
  int use_graph;
  int fixed_iters;
  int check_every; /* iterations between host checks of the active count; 0 = auto */
  int autotune;    /* 1: time candidate tiles of the batched kernels the first time a
                      (problem shape, batch, basis size, precision) is solved and keep
                      the fastest in the context (and in the JSON file named by
                      RB_AUTOTUNE_CACHE, if set); 0: cached choice or built-in default */
  int stencil_kind; /* 3D passes A and B and the colour sweeps: 0 = autotuned / default,
                       1 = chunked over storage positions, 2 = marching along z with the
                       plane in LDS (3D only; other grids use 1), 3 = as 2, with both
                       colours of a one-sweep Gauss-Seidel smoother in one launch marching
                       along z (3D grids with n[0] <= 255; else as 2), 4 = as 2, with the
                       tiles of the passes and sweeps twice as tall (four nodes or column
                       pairs per thread, at most two queries per block).  Changes speed and
                       summation order only. */
  double adapt_gamma; /* RBCG only.  > 0: adaptive basis size (Sec. 4.1, last
                         paragraph): query b starts with n_use[b] vectors (1 if n_use is
                         NULL) and uses one more (up to the basis size) for the next
                         preconditioner application whenever its residual fell by less
                         than this factor in an iteration; 0: fixed size.  Use with
                         beta_flexible (the preconditioner changes between iterations). */
  double floor_factor; /* > 0: the true-residual test also accepts ||f - A x|| <= floor_factor
                          * eps * || |A| |x| || (eps = 2^-52), the rounding level of an FP64
                          * residual of x, once the iteration has stalled there (at two
                          * checks in a row the true residual stayed above half of the
                          * previous check's: residual replacements did not pay); such
                          * queries end RB_OK
                          * with at_floor = 1.  0: off.  For problems whose tolerance lies
                          * below what FP64 reaches (strong kappa contrasts on fine grids). */
  int smooth_sweeps;  /* Gauss-Seidel sweeps per smoother application (RBGS: forward sweeps,
                         RBGS_SYM: forward + backward pairs); 0 or 1 = one.  Jacobi and
                         none take one only (RB_EUNSUPPORTED otherwise). */
  int residual_copy;  /* RBCG with an FP32 / BF16 preconditioner on a stencil problem:
                         1 (default) = the CG updates also keep an FP32 copy of r, which the
                         projection W^T r and the Gauss-Seidel sweeps that form no dot
                         product read instead of r.  Both round r to FP32 before using it,
                         so the results are the same, from fewer bytes read; 0 = read r.
                         Ignored elsewhere. */
  int prolong_kind;   /* prolongation W e of a batch of at least 16 queries with an FP32 /
                         BF16 preconditioner: 0 = autotuned / default (MFMA tiles), 1 = MFMA
                         tiles, 2 = vector units (one node per thread, FP32 FMAs).  Changes
                         speed and summation order only. */
  int paired_x_update; /* RBCG and CG on a stencil problem: 1 (default) = the iterate's update
                          x += alpha_k p_k (Alg. 3) of an even iteration k is applied with the
                          next one's, x = (x + alpha_k p_k) + alpha_k+1 p_k+1, in one read and
                          write of x (or at the true-residual check or the end, if they come
                          first): the same operations in the same order, so the same results
                          bit for bit, from fewer bytes moved; 0 = every iteration.  Ignored
                          elsewhere. */
} rb_solve_opts;
void rb_solve_opts_default(rb_solve_opts* opts);

typedef struct {
  int iters;
  double rel_res_true;
  double rel_res_recursive;
  rb_status status;
  int n_used; /* basis vectors used by the last preconditioner application */
  int at_floor; /* 1: accepted at the rounding level (floor_factor), not at rtol */
} rb_query_stats;

/* B queries on one problem and basis, 0 <= B <= 65535 (B = 0: RB_OK, nothing read or
 * written; theta, x and stats may then be NULL).  theta [B][Q] host; phi [B][R] host or
 * NULL (all ones); n_use [B] host or NULL (= basis size): query b uses the leading
 * n_use[b] basis vectors; basis may be NULL for RB_SOLVER_CG.
 * x: [B][N] DEVICE doubles, natural ordering, written with the solutions.
 * stats: [B] host, written. */
rb_status rb_solve_batch(rb_ctx* ctx, const rb_problem* prob, const rb_basis* basis,
                         const rb_solve_opts* opts, int B, const double* theta,
                         const double* phi, const int* n_use, double* x,
                         rb_query_stats* stats);

/* Queries on several problems/bases in one call (uneven batches).  The queries are
 * grouped by (problem, tolerance); every group is one batched solve on its own stream
 * and workspace, and the groups run concurrently.  At most 65535 queries per group;
 * B = 0 returns RB_OK (queries and stats may then be NULL).  Errors as
 * rb_solve_batch. */
typedef struct {
  int problem;          /* index into probs/bases */
  int n_use;            /* <= 0: the whole basis */
  const double* theta;  /* [Q] host */
  const double* phi;    /* [R] host or NULL */
  double* x;            /* [N] DEVICE */
  double rtol;          /* <= 0: opts->rtol; else this query's tolerance */
} rb_query;
rb_status rb_solve_multi(rb_ctx* ctx, int nprob, const rb_problem* const* probs,
                         const rb_basis* const* bases, const rb_solve_opts* opts, int B,
                         const rb_query* queries, rb_query_stats* stats);

/* ---- Single steps of the hot path (diagnostics and parity tests) ------------
 * y_b = A(theta_b) u_b.  u, y: [B][N] DEVICE, natural ordering. */
rb_status rb_apply_batch(rb_ctx* ctx, const rb_problem* prob, int B, const double* theta,
                         const double* u, double* y);
/* y_b = RBI(A(theta_b), r_b, W_{n_use[b]}, 1): one RB iteration from x = 0 (projection
 * W^T r, reduced Cholesky solve, prolongation, one smoother application) as used by
 * RBCG (Alg. 3).  r, y: [B][N] DEVICE FP64, natural ordering. */
rb_status rb_precond_batch(rb_ctx* ctx, const rb_problem* prob, const rb_basis* basis,
                           const rb_solve_opts* opts, int B, const double* theta,
                           const int* n_use, const double* r, double* y);
/* t_b = W^T r_b (eq. 5) with the given precision.  r: [B][N] DEVICE natural
 * ordering; t: [B][n] host. */
rb_status rb_project_batch(rb_ctx* ctx, const rb_problem* prob, const rb_basis* basis,
                           rb_prec prec, int B, const double* r, double* t);
/* L_b = chol(sum_q theta_bq A_{N,q}) (lower, row-major [B][n][n] host, upper part
 * zero), status[b] = RB_OK or RB_ENOTSPD. */
rb_status rb_reduced_factor_batch(rb_ctx* ctx, const rb_basis* basis, int B,
                                  const double* theta, double* L, rb_status* status);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc): rb_reduced_factor_batch with the same arguments and results, except
 * that it allocates nothing.  theta is staged on the device, and L and status are formed
 * there, in one fixed buffer of RB_NOALLOC_SCRATCH_BYTES per GPU that the library holds
 * until the process ends (its address is resolved when the first context on that GPU is
 * created).  Requires 256-byte-rounded sizes B*Q*8 + B*n*n*8 + B*4 to fit in it (e.g.
 * B = 512 queries at n = 40, Q = 8); larger requests fail with RB_EINVAL and a message
 * naming the sizes, before any work.  Every call on one GPU shares that buffer: calls
 * that overlap on one GPU (from several threads or contexts) race.  It synchronises the
 * context's stream before returning, like rb_reduced_factor_batch. */
#define RB_NOALLOC_SCRATCH_BYTES (8u << 20)
rb_status rb_reduced_factor_batch_noalloc(rb_ctx* ctx, const rb_basis* basis, int B,
                                          const double* theta, double* L, rb_status* status);

/* ---- Offline: adaptive greedy (Alg. 4) --------------------------------------
 * Training set Xi_train of M parameters: theta [M][Q] host (and phi [M][R] or
 * NULL).  mu [M][P] host or NULL is used only for the surrogate's features.
 * Snapshot solves x(mu_N) = RBCG(A(mu_N), f, W_{N-1}) (W_0 empty: smoother-only
 * PCG), modified Gram-Schmidt, growth of A_{N,q} and f_{N,r}, and a sweep of the
 * indicator over Xi_train with argmax over the unpicked candidates (lowest index
 * wins ties).  Indicators: RB_IND_L1 = sum_n |a_n(mu)| (Alg. 1 / Alg. 4);
 * RB_IND_RESIDUAL = ||f - A(mu) W a(mu)|| / ||f||.
 * use_surrogate: rank candidates by an MLP (P -> 128 -> 128 -> 1, GELU) trained
 * on the GPU on the indicators already computed; the true indicator is evaluated
 * on the top `topk` plus `explore` random candidates and decides the pick; full
 * sweeps every `full_sweep_every` steps, for the first `warmup_full_sweeps` steps,
 * and whenever the ranking check fails. */
typedef struct {
  size_t struct_size; /* sizeof(rb_greedy_opts) */
  int n_max;
  int64_t seed_index;
  rb_indicator indicator;
  double snapshot_rtol;  /* default 1e-10 */
  int snapshot_maxit;    /* default 5000 */
  int snapshot_flexible; /* default 1 */
  int use_surrogate;
  int topk;              /* default 256 */
  int explore;           /* default 64 */
  int full_sweep_every;  /* default 10 */
  int warmup_full_sweeps;/* default 4 */
  int train_steps;       /* Adam steps per greedy step, default 50 */
  double lr;             /* default 1e-3 */
  double mu_lo, mu_hi;   /* log range of mu for the features */
  uint64_t seed;
  rb_prec snapshot_prec; /* preconditioner of the snapshot solves: RB_PREC_FP64 (default)
                          * or RB_PREC_FP32 (an FP32 copy of the basis grown column by
                          * column; the CG, its stopping test and Gram-Schmidt stay FP64) */
  rb_prec surrogate_prec; /* the network's products: RB_PREC_BF16 (default; BF16 operands,
                           * FP32 accumulation) or RB_PREC_FP32; master weights and Adam
                           * moments are FP32 either way */
  int snapshot_sweeps;   /* Gauss-Seidel sweeps per preconditioner application in the
                          * snapshot solves (default 1) */
} rb_greedy_opts;
void rb_greedy_opts_default(rb_greedy_opts* opts);

typedef struct {
  int n_built;
  int64_t* picks;          /* caller-allocated [n_max] or NULL */
  double* max_indicator;   /* [n_max] or NULL: max indicator after step N */
  int* snapshot_iters;     /* [n_max] or NULL */
  int64_t true_evals;      /* candidates whose true indicator was computed */
  int full_sweeps;
  double seconds;
  double mlp_loss;         /* last training loss (surrogate, standardised targets) */
  int surrogate_fallbacks; /* surrogate steps that fell back to a full sweep */
} rb_greedy_report;

rb_status rb_offline_build(rb_ctx* ctx, const rb_problem* prob, const rb_greedy_opts* opts,
                           int64_t M, int P, const double* mu, const double* theta,
                           const double* phi, rb_basis** out, rb_greedy_report* rep);

/* Snapshot solves and basis updates of Alg. 4 for a given sequence of K <= 80
 * parameters: each snapshot x(theta_k) = RBCG(A(theta_k), f, W_{k-1})
 * (snapshot_rtol, snapshot_maxit, snapshot_flexible of opts; the other fields are
 * ignored) is orthonormalised into the basis; a degenerate snapshot (already in the span) is skipped.  With the picks of a
 * greedy on a coarse grid (rb_greedy_report.picks) this is the multi-fidelity offline
 * build of Sec. 4.2 (last paragraph).  theta [K][Q], phi [K][R] or NULL, host.
 * rep (nullable): n_built, picks = indices k that entered the basis, snapshot_iters,
 * seconds.  A failed snapshot solve returns its status and no basis. */
rb_status rb_basis_from_parameters(rb_ctx* ctx, const rb_problem* prob,
                                   const rb_greedy_opts* opts, int K, const double* theta,
                                   const double* phi, rb_basis** out, rb_greedy_report* rep);

/* ---- MLP surrogate of the greedy indicator (not in the paper) ----------------
 * Diagnostics of the network rb_offline_build trains when use_surrogate is set.
 * Network P -> H -> H -> 1 with exact-erf GELU; params is FP32 packed in the order
 * W1 [H][P], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1] (H*P + H*H + 3H + 1 values).
 * prec: RB_PREC_BF16 = every product on BF16 MFMA with FP32 accumulation (operands
 * rounded to BF16 when loaded); RB_PREC_FP32 = FP32 MFMA.  Requires 1 <= P <= 64 and
 * H a multiple of 16 in [16, 512].  X [m][P], y [m], out [m] host. */
rb_status rb_mlp_forward(rb_ctx* ctx, int P, int H, rb_prec prec, const float* params, int m,
                         const float* X, float* out);
/* MSE loss mean_m (out_m - y_m)^2 and its gradient w.r.t. params (same packing). */
rb_status rb_mlp_loss_grad(rb_ctx* ctx, int P, int H, rb_prec prec, const float* params, int m,
                           const float* X, const float* y, float* loss, float* grad);
/* `steps` full-batch Adam steps (beta 0.9 / 0.999, eps 1e-8, bias-corrected) from
 * params, updated in place; loss = loss after the last step. */
rb_status rb_mlp_train(rb_ctx* ctx, int P, int H, rb_prec prec, float* params, int m,
                       const float* X, const float* y, int steps, double lr, float* loss);
/* One surrogate-ranked greedy step from a given state (the step rb_offline_build takes
 * with use_surrogate after each basis vector), for parity tests of the protocol.  The
 * basis (n >= 1 columns) is the greedy's current W_N; theta [M][Q] and mu [M][P] the
 * training set (R = 1); excluded [M] flags the candidates already picked; params
 * [H*P + H*H + 3H + 1] (H = 128, packing as rb_mlp_forward) the FP32 master weights,
 * overwritten with the weights after the step's training (Adam moments start at zero);
 * the replay buffer holds nbuf entries (candidate buf_index[i], target buf_target[i] =
 * log10 indicator, greedy step buf_step[i]).  Options used: indicator, topk, explore,
 * warmup_full_sweeps, full_sweep_every, train_steps, lr, mu_lo, mu_hi, seed,
 * surrogate_prec.  The step:
 *  - is a full sweep (the plain greedy's sweep and argmax) if step <= warmup_full_sweeps
 *    or step is a multiple of full_sweep_every;
 *  - otherwise ranks every candidate with the network, evaluates the true indicator on
 *    the top-K unpicked candidates (written to topk in increasing index order, ties at
 *    the K-th value to the lower index) and on `explore` further unpicked candidates
 *    drawn uniformly (index floor(u M), u the counter's next value; redrawn when picked
 *    or listed; at most 100 * explore draws; written to explore in draw order); if at
 *    least 3 were explored and the Spearman rank correlation of prediction and
 *    log10(true indicator) over them is below 0.5 it falls back to a full sweep, else
 *    picks the argmax of the true indicator over the short list (ties: lower index);
 *  - appends every evaluated unpicked candidate with a positive finite indicator to
 *    the buffer, keeps the entries of the last two steps, standardises the targets and
 *    runs train_steps Adam steps on minibatches of min(256, size) entries drawn with
 *    replacement (entry floor(u size)).
 * The not-in-the-paper protocol is the library's own; the paper's greedy (Alg. 4,
 * Sec. 4.2) is what its full sweeps compute. */
typedef struct {
  size_t struct_size;  /* sizeof(rb_surrogate_io) */
  int step;            /* in: greedy step k >= 1 (basis vectors added so far) */
  uint64_t counter;    /* in/out: position in the counter sequence of opts->seed (a fresh
                        * surrogate starts at H*P + H*H + H, after its initial weights) */
  int full_sweep;      /* out: 1 if every candidate was evaluated */
  int fallback;        /* out: 1 if the ranking check failed */
  int n_topk, n_explore; /* out: entries written to topk / explore */
  int64_t pick;        /* out: next sample, -1 if no candidate is left */
  double value;        /* out: its true indicator */
  int64_t true_evals;  /* out: true indicator evaluations of this step */
  float loss;          /* out: training loss of the last Adam step (0 if none) */
} rb_surrogate_io;
rb_status rb_surrogate_step(rb_ctx* ctx, const rb_problem* prob, const rb_basis* basis,
                            const rb_greedy_opts* opts, int64_t M, int P, const double* mu,
                            const double* theta, const int32_t* excluded, float* params,
                            int nbuf, const int32_t* buf_index, const float* buf_target,
                            const int32_t* buf_step, int32_t* topk, int32_t* explore,
                            rb_surrogate_io* io);
/* Indices of the K largest v[m] among the entries with excluded[m] == 0 (excluded may be
 * NULL), as a set: ties at the K-th value go to the lowest indices.  out [>= K] host,
 * count = number written (min(K, available)). */
rb_status rb_topk(rb_ctx* ctx, int M, int K, const float* v, const int* excluded, int* out,
                  int* count);

#ifdef __cplusplus
}
#endif
#endif /* RB_H_ */
