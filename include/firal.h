/*
 * firal.h -- C ABI of the MI355X (gfx950) Relax and Round steps of Approx-FIRAL
 * (Chen, Wen & Biros, "A Scalable Algorithm for Active Learning", SC24).
 *
 * The library computes, on one GPU, every step of the fast Relax solve
 * (Algorithm 2): Rademacher probes, the block-diagonal preconditioner of
 * Definition 1 / eq. 12, block-Jacobi preconditioned CG with the matrix-free
 * Hessian product of Lemma 1, the Hutchinson gradient of eq. 11 and the
 * entropic mirror-descent update; and the diagonal Round step (Algorithm 3)
 * that selects the b points from the relaxed weights.
 *
 * Conventions shared by every call
 * --------------------------------
 * Pointers marked "device" are HIP device addresses on the context's device;
 * "host" pointers are ordinary CPU memory.  Every device buffer belongs to
 * the caller unless stated otherwise; the library never frees caller memory.
 * `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *
 * Rows: X is (n_pool + n_lab) x d row-major, pool rows first, then the
 * labeled rows; H (the class probabilities h_i of eq. 1, one row per point)
 * is (n_pool + n_lab) x c row-major in the same row order.
 *
 * Blocks: s vectors of length d*c are stored as a d x s x c row-major array
 * B, element (a, j, k) at a*s*c + j*c + k.  It is entry k*d + a of the
 * paper's j-th vector v_j = vec(V_j) (vec stacks the columns of the d x c
 * matrix V_j; notation table and Lemma 1).
 *
 * Element type: FP64 for FIRAL_F64; FP32 for FIRAL_F32 and FIRAL_BF16X3
 * (X, H, blocks).  Row weights omega, z, w, gradients and the
 * preconditioner factors are always FP64.
 *
 * Return codes: 0 = success, > 0 = warning, < 0 = error (see FIRAL_E*).
 * Argument errors are detected before any device work; conditions found on
 * the device (non-SPD preconditioner block, CG breakdown, no convergence)
 * are reported through firal_info by the calls that take one.  The
 * detail of the last failure on the calling thread is firal_last_error().
 * A context must not be used from two host threads or two streams at once.
 * Calls that run PCG with a tolerance (firal_pcg_solve, firal_relax_step,
 * firal_sampled_objective) read each CG iteration's per-column flags from pinned
 * host memory one iteration behind the GPU: the calling thread spins on them,
 * for at most 1 ms at a time before it waits on the stream instead.
 */
#ifndef FIRAL_H
#define FIRAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct firal_ctx_s* firal_ctx;

typedef enum {
  FIRAL_F64 = 0,     /* FP64 storage, FP64 MFMA */
  FIRAL_F32 = 1,     /* FP32 storage, FP32 MFMA */
  FIRAL_BF16X3 = 2   /* FP32 storage, products as three bf16 MFMA passes (hi*hi + hi*lo + lo*hi) */
} firal_prec;

enum {
  FIRAL_OK = 0,
  FIRAL_WARN_NOT_CONVERGED = 1, /* a PCG column did not reach tol within max_iter */
  FIRAL_EINVAL = -1,            /* bad argument: null pointer, size out of range, s > s_max ... */
  FIRAL_EHIP = -2,              /* HIP runtime failure or no usable device */
  FIRAL_ENOMEM = -3,            /* device allocation failed */
  FIRAL_ENOTSUP = -4,           /* combination not supported */
  FIRAL_EBREAKDOWN = -5,        /* PCG: p_j^T q_j <= 0 on an active column (operator not SPD) */
  FIRAL_ENOTSPD = -6            /* a preconditioner block failed its Cholesky factorisation */
};

/* pcg_solve / relax_step flag: solve in the complement of {1_c (x) u}.
 * With a full softmax h every H_i annihilates that d-dimensional space, so
 * Sigma_z has the eigenvalue lambda there and block-Jacobi cannot reach it;
 * projecting the right-hand sides and the preconditioner (P M^-1 P) removes
 * it without changing H_p Sigma^-1 V, f_hat or the gradient of eq. 11. */
#define FIRAL_PCG_PROJECT 1u

typedef struct {
  int32_t cg_iters[2];  /* iterations of the first / second PCG solve (pcg_solve fills [0]) */
  int32_t converged;    /* 1 if every column of every solve met tol */
  int32_t bad_block;    /* -1, or the first class k whose preconditioner block is not SPD */
  double relres_max;    /* max_j ||r_j|| / ||b_j|| of the recurrence residual at exit */
  double f_hat;         /* (1/s) sum_j <v_j, H_p Sigma_z^-1 v_j>: Hutchinson estimate of f(z) */
  double g_absmax;      /* max_i |g_i| of the gradient estimate */
  double beta;          /* step used: beta0 / g_absmax */
} firal_info;

/* Create a context for one problem.  X and H (device, element type of prec)
 * are borrowed: they must stay valid and unchanged while the context lives.
 * All workspace for blocks of up to s_max probes is allocated here.
 * Errors: EINVAL (n_pool < 1, n_lab < 0, d < 1, c < 2, s_max < 1, null X/H/out,
 * prec unknown), EHIP (no device), ENOMEM. */
int firal_create(firal_ctx* out, int64_t n_pool, int64_t n_lab, int32_t d, int32_t c,
                 int32_t s_max, int32_t prec, const void* X, const void* H, void* stream);

/* Release the context's workspace (synchronises the device first).  NULL is a no-op. */
int firal_destroy(firal_ctx ctx);

/* Matrix-free Hessian product (Lemma 1; aggregated over rows as in the H_p v formula
 * that follows it):
 *   out_j = sum_{i < n_rows} omega_i H_i v_j + shift * v_j,   H_i = Gamma_i (x) x_i x_i^T,
 * for the s blocks of B (eq. 2).  omega: device FP64 [n_rows] or NULL for all ones.
 * n_rows <= n_pool + n_lab selects rows 0..n_rows-1 (n_pool gives H_p).
 * B, out: device blocks d x s x c; out must not alias B.  Asynchronous. */
int firal_hvp(firal_ctx ctx, const double* omega, int64_t n_rows, double shift,
              const void* B, void* out, int32_t s, void* stream);

/* The product of firal_hvp without a context and without allocating, for callers that cannot
 * allocate device memory (code under stream capture, serving loops that forbid hipMalloc):
 *   out_j = sum_{i < n_rows} omega_i H_i v_j + shift * v_j
 * over the n_rows rows of X (device FP32, n_rows x d row-major) and H (device FP32, n_rows x c),
 * B and out device FP32 blocks d x s x c (out must not alias B), omega device FP64 [n_rows] or
 * NULL for all ones.  It runs the fused FP32 kernels of firal_hvp and keeps their per-row-range
 * partial sums in one fixed 64 MiB device array of the library (each device holds its own until
 * the process ends), so it covers FP32 with d <= 128 and the shapes whose partial sums fit that
 * array.  Calls on one device share the array: calls that overlap on a device (two streams, two
 * host threads) race and must not be issued.  No allocation, no host synchronisation;
 * asynchronous.  Errors: EINVAL (null pointer, size out of range, partial sums larger than the
 * array: checked before any device call), ENOTSUP (d > 128, or no single-pass tile plan), EHIP. */
int firal_hvp_noalloc(const float* X, const float* H, int64_t n_rows, int32_t d, int32_t c,
                      const double* omega, double shift, const float* B, float* out, int32_t s,
                      void* stream);

/* Block-diagonal preconditioner (Definition 1, eq. 12):
 *   P_k = shift * I_d + sum_i omega_i h_ik (1 - h_ik) x_i x_i^T,  k = 0..c-1, all rows,
 * factorised in FP64 as P_k = L_k L_k^T.  L (lower, upper part zero) and Pinv = P_k^-1
 * are device FP64 arrays c x d x d; either may be NULL.  omega: device FP64
 * [n_pool + n_lab] or NULL for all ones.  Synchronous; info (host, may be NULL)
 * gets bad_block.  Returns ENOTSPD when a block fails.  The sums over rows are FP32 (FIRAL_F32,
 * FIRAL_BF16X3) or FP64.  A FIRAL_BF16X3 context created with FIRAL_BF3_GRAM=1 in the
 * environment forms them as bf16x3 products instead when c > 64, d is a multiple of 4 and X is
 * 16-byte aligned (about 1e-5 relative error in P_k: a PCG run to a tolerance reaches the same
 * solution, iterates taken at a fixed iteration count move by up to that error times the
 * conditioning). */
int firal_build_precond(firal_ctx ctx, const double* omega, double shift, double* L,
                        double* Pinv, firal_info* info, void* stream);

/* Block-Jacobi preconditioned CG for (sum_i omega_i H_i + shift I) Xsol_j = B_j, all s
 * columns in lock-step from x0 = 0 (the two solves of Algorithm 2).  Pinv: device FP64
 * c x d x d from firal_build_precond.  B, Xsol: device blocks d x s x c that either
 * coincide or do not overlap.  Column j stops once ||r_j|| <= tol ||b_j||; the
 * loop ends when all have stopped or after max_iter iterations (tol = 0: exactly
 * max_iter).  flags: FIRAL_PCG_PROJECT.  Synchronous; returns WARN_NOT_CONVERGED or
 * EBREAKDOWN; info (host, may be NULL) gets cg_iters[0], converged, relres_max. */
int firal_pcg_solve(firal_ctx ctx, const double* omega, double shift, const double* Pinv,
                    const void* B, void* Xsol, int32_t s, double tol, int32_t max_iter,
                    uint32_t flags, firal_info* info, void* stream);

/* Per-point contraction of eq. 11 for every pool row i:
 *   g_i = -(1/s) sum_j u_j^T H_i w_j = -(1/s) sum_j (U_j^T x_i)^T Gamma_i (W_j^T x_i)
 * U, W: device blocks d x s x c; g: device FP64 [n_pool].  Asynchronous. */
int firal_grad_z(firal_ctx ctx, const void* U, const void* W, int32_t s, double* g,
                 void* stream);

/* Rademacher probes of iteration t >= 1 (Algorithm 2, probe line): entry (a, j, k) is -1
 * when the top bit of SplitMix64 output number ((t-1)*s + j)*(d*c) + k*d + a of the
 * stream seeded with `seed` is set, else +1.  V: device block d x s x c.  Asynchronous. */
int firal_probes(firal_ctx ctx, uint64_t seed, int32_t t, int32_t s, void* V, void* stream);

/* One iteration t >= 1 of the fast Relax solve (Algorithm 2) on the simplex weights w:
 *   z = b w; omega = [z; 1]; V = probes(seed, t); P_k = blocks of Sigma_z + lambda I;
 *   W1 = Sigma^-1 V; Y = H_p W1; W2 = Sigma^-1 Y; g = grad_z(V, W2);
 *   beta = beta0 / max|g|;  w_i <- w_i exp(-beta g_i) / sum_l w_l exp(-beta g_l).
 * w: device FP64 [n_pool], in/out (positive, summing to 1).  g_out: device FP64 [n_pool]
 * or NULL.  On a device-side failure (ENOTSPD, EBREAKDOWN) w is left unchanged.
 * Synchronous; info (host, may be NULL) gets every field. */
int firal_relax_step(firal_ctx ctx, double* w, double b, double lambda, double beta0,
                     uint64_t seed, int32_t t, int32_t s, double tol, int32_t max_iter,
                     uint32_t flags, double* g_out, firal_info* info, void* stream);

/* The default mirror-descent step scale for T iterations over n weights: sqrt(2 ln n / T), the
 * textbook step of entropic mirror descent (Algorithm 2 leaves the schedule beta_t open; the
 * step of iteration t is this scale divided by max_i |g_i|).  0 for n < 1. */
double firal_default_beta0(int64_t n, int32_t T);

/* The fast Relax solve (Algorithm 2): up to T iterations of firal_relax_step from the uniform
 * weights w_i = 1/n_pool, then z = b w.  beta0 < 0 selects firal_default_beta0(n_pool, T).
 * stop_rel > 0 adds the termination of the experiments section: after iteration t >= 2 the loop
 * ends when |f_t - f_{t-1}| <= stop_rel |f_{t-1}|, f_t the objective estimate f_hat of iteration
 * t (its weights are kept); stop_rel = 0 runs all T iterations.
 * z: device FP64 [n_pool], written (it holds w while the iterations run).  f_hist (host double
 * [T]), cg_hist (host int32 [2T]: both solves of each iteration) and iters (host, the number of
 * iterations run) may be NULL.  info gets the last iteration's fields, with converged = 1 only if
 * every solve of every iteration converged.  Synchronous.  Returns WARN_NOT_CONVERGED if some
 * solve did not converge; on ENOTSPD or EBREAKDOWN the loop stops at that iteration, whose
 * weights are left unchanged, and z = b w of the iterations before it. */
int firal_relax_solve(firal_ctx ctx, double b, double lambda, double beta0, uint64_t seed,
                      int32_t T, int32_t s, double tol, int32_t max_iter, uint32_t flags,
                      double stop_rel, double* z, double* f_hist, int32_t* cg_hist,
                      int32_t* iters, firal_info* info, void* stream);

/* Sampled objective and its gradient (the objective of eq. 4-5 with the trace replaced by
 * the Hutchinson estimate of eq. 11 for a fixed probe block V):
 *   f_V(z) = (1/s) sum_j v_j^T Sigma_z^-1 H_p v_j,   Sigma_z = H_o + H_z + lambda I (eq. 7),
 *   df_V/dz_i = -(1/s) sum_j (Sigma_z^-1 v_j)^T H_i (Sigma_z^-1 H_p v_j)   (i in the pool),
 * the exact derivative of f_V (dSigma_z/dz_i = H_i): preconditioner at z, U = Sigma^-1 V,
 * Y = H_p V, f from <U, Y>; with g: Y' = Sigma^-1 Y and the eq. 11 contraction of U and Y'.
 * z: device FP64 [n_pool] (any positive weights, not normalised); V: device block d x s x c;
 * f: host double; g: device FP64 [n_pool] or NULL for the objective alone.  PCG as in
 * firal_pcg_solve (tol, max_iter, flags).  Synchronous; info gets cg_iters (solve of V, solve
 * of H_p V), converged, relres_max and f_hat. */
int firal_sampled_objective(firal_ctx ctx, const double* z, double lambda, const void* V,
                            int32_t s, double tol, int32_t max_iter, uint32_t flags, double* f,
                            double* g, firal_info* info, void* stream);

/* Kernels that firal_profile_begin can time (the kernels of the product of Lemma 1 and of the
 * Round step's per-point objective):
 *   FIRAL_PROF_PRODUCT      the product's main kernel: the fused single-pass kernel where it
 *                           applies, else the row-tiled path's first contraction X V with the
 *                           row step of Lemma 1 (one launch per row chunk);
 *   FIRAL_PROF_PRODUCT_T    the row-tiled path's second contraction X^T G' (one launch per chunk);
 *   FIRAL_PROF_ROUND_SCORE  the Round step's scoring kernel (one launch per row chunk and round). */
#define FIRAL_PROF_PRODUCT 0
#define FIRAL_PROF_PRODUCT_T 1
#define FIRAL_PROF_ROUND_SCORE 2

/* Measurement: between firal_profile_begin and firal_profile_end the library attaches a HIP
 * event pair to every launch of the chosen kernel (hipExtLaunchKernel, so each pair spans the
 * kernel's own execution, as a profiler's kernel trace does).  firal_profile_end synchronises
 * the device and returns the summed kernel time in milliseconds (host double) and the number of
 * launches (host int64); either pointer may be NULL.  Recording adds no synchronisation to the
 * timed calls.  Errors: EINVAL (null context, unknown kernel, end without begin). */
int firal_profile_begin(firal_ctx ctx, int32_t kernel);
int firal_profile_end(firal_ctx ctx, double* total_ms, int64_t* launches);

/* Kernel-variant tuner (the tile plan of extension (2); usable on any context).  Times on this
 * context, for s probes, the product's tilings (the fused single pass with one or two 16-column
 * blocks per wave and a target of 256, 512 or 1024 workgroups, which sets the rows each
 * workgroup covers, wherever its plan fits; the row-tiled kernels) and the PCG step forms
 * (column-local, separate kernels), keeps the fastest of each for the context and remembers
 * the choice for the process per bucket (precision, d, c, s, n_pool + n_lab rounded up to a
 * power of two); a bucket already tuned is applied without timing.  The context's work blocks
 * and preconditioner are overwritten.  choice (host, may be NULL) gets bit 0 = row-tiled
 * product (and FP32 gradient), bit 1 = separate-kernel PCG, bit 2 = fused product with two
 * column blocks per wave (else one, the next row chunk fetched ahead), bits 3-4 = code k of
 * the fused workgroup target 256 << k.  Synchronous. */
int firal_autotune(firal_ctx ctx, int32_t s, int32_t* choice, void* stream);

/* Batch of independent Relax problems (extension (2)): one Relax iteration (Algorithm 2) of
 * every problem captured into a single HIP graph, one branch per problem, replayed as a whole.
 * Each problem keeps its own context (created as usual, one per problem, not shared) and its
 * own simplex weights; the branches run concurrently.  In the captured step every PCG solve
 * enqueues exactly max_iter iterations whose kernels return at once after all columns have
 * met tol (the results equal those of firal_relax_step with the same arguments), and the
 * iteration index is kept on the device: replay k runs iteration t0 + k of every problem. */
typedef struct firal_batch_s* firal_batch;
typedef struct {
  firal_ctx ctx;        /* the problem's context */
  double* w;            /* device FP64 [n_pool]: simplex weights, advanced in place */
  double b;             /* budget: z = b w */
  double lambda;        /* regulariser of Sigma_z */
  double beta0;         /* mirror-descent step scale */
  uint64_t seed;        /* probe stream seed */
  int32_t t0;           /* iteration index of the first replay, >= 1 */
  int32_t s;            /* probes, 1..s_max of the context */
  double tol;           /* PCG relative-residual tolerance */
  int32_t max_iter;     /* PCG iterations enqueued per solve */
  uint32_t flags;       /* FIRAL_PCG_PROJECT */
} firal_batch_problem;

/* Tune each problem (firal_autotune), run one uncaptured pass of each problem's captured step
 * (weights and iteration index restored afterwards), then capture and instantiate the graph.
 * probs (host, n entries) is copied.  Errors: EINVAL (null argument, n < 1, a shared context,
 * s outside the context's range, t0 < 1, max_iter < 0, b or lambda not positive), EHIP, ENOMEM.
 * Synchronous. */
int firal_batch_create(firal_batch* out, int32_t n, const firal_batch_problem* probs,
                       void* stream);
/* Replay the graph iters times on stream (asynchronous). */
int firal_batch_run(firal_batch batch, int32_t iters, void* stream);
/* Synchronise stream and report problem i's last iteration (as firal_relax_step's info; the
 * return code carries ENOTSPD, EBREAKDOWN or WARN_NOT_CONVERGED of that iteration). */
int firal_batch_info(firal_batch batch, int32_t i, firal_info* info, void* stream);
/* The iteration index problem i's next replay will run (synchronises the device). */
int firal_batch_next_t(firal_batch batch, int32_t i, int32_t* t);
/* Release the graph, streams and events (the contexts stay with the caller).  NULL is a no-op. */
int firal_batch_destroy(firal_batch batch);

/* Diagonal Round step of Approx-FIRAL (Algorithm 3).  Every Fisher matrix keeps only its c
 * diagonal d x d blocks (Section 3.2), so all state is c blocks of d x d.  Round t selects the
 * unselected pool row i maximising the per-point objective of the Section 3.2 proposition,
 *   sum_k g_ik x_i^T (B_t)_k^-1 (Sigma_o)_k (B_t)_k^-1 x_i / (1 + eta g_ik x_i^T (B_t)_k^-1 x_i),
 * g_ik = h_ik (1 - h_ik) (ties: lowest row index; a row is selected at most once), then
 *   (H)_k += (H_o)_k / b + g_ik x_i x_i^T,
 *   nu_{t+1}: sum_kj (nu + eta lambda_kj)^-2 = 1 over the eigenvalues lambda_kj of
 *             (Sigma_o)_k^-1/2 (H)_k (Sigma_o)_k^-1/2,
 *   B_{t+1} = nu_{t+1} Sigma_o + eta H + (eta / b) H_o,   B_1 = sqrt(dc) Sigma_o + (eta / b) H_o.
 * (Sigma_o)_k = lambda I + (H_o)_k + sum_i z_i g_ik x_i x_i^T over the pool rows (the blocks of
 * Sigma_z at the relaxed weights z); (H_o)_k = sum over the labeled rows of g_ik x_i x_i^T.  The
 * objective's numerator holds Sigma_o itself, as the proposition's proof derives it (the stated
 * objective prints its inverse).  Arithmetic is FP64 (FP32 X and H are read exactly) except
 * the objective in FIRAL_ROUND_FP32 mode.
 * Requires d <= 1024 and c <= 65535.  The state borrows the context (X and H): destroy it first. */
typedef struct firal_round_s* firal_round;

/* firal_round_create flag: evaluate the per-point objective (the two quadratic forms, the class
 * terms and their sum) and take the argmax in FP32, the precision of the paper's
 * implementation (Section 3.3); without it they are FP64.  The block state (Sigma_o factors,
 * eigenvalues, nu, the update) is FP64 either way. */
#define FIRAL_ROUND_FP32 1u

/* Set up rounds of one Round solve on ctx's rows: z (device FP64 [n_pool]) the relaxed
 * weights (read during the call only), lambda >= 0 the regulariser of Sigma_o, eta > 0 the
 * learning rate, b in [1, n_pool] the number of rounds (points to select), flags 0 or
 * FIRAL_ROUND_FP32.  Forms Sigma_o's blocks and Cholesky factors, H_o's blocks and the first round's
 * B^-1.  Synchronous.
 * Errors: EINVAL, ENOTSPD (a Sigma_o block is not positive definite), EHIP, ENOMEM. */
int firal_round_create(firal_round* out, firal_ctx ctx, const double* z, double lambda,
                       double eta, int32_t b, uint32_t flags, void* stream);
/* Enqueue the next `rounds` rounds (asynchronous: nothing is read back and the host does not
 * wait; each round's index is fixed when it is enqueued, so a captured call replays the same
 * rounds).  EINVAL if fewer than `rounds` of the b rounds are left. */
int firal_round_step(firal_round round, int32_t rounds, void* stream);
/* The per-point objective of every pool row at the current round (device FP64 [n_pool];
 * selected rows get -inf).  Asynchronous; changes no state. */
int firal_round_scores(firal_round round, double* scores, void* stream);
/* Synchronise and copy to host buffers (each may be NULL): the t rounds done so far,
 * selected[0..t) (row indices into the pool), nu[0..t] (nu_1 .. nu_{t+1}), score_max[0..t)
 * (the winning objective of each round).  EINVAL if a round found no unselected row with a
 * finite objective. */
int firal_round_result(firal_round round, int64_t* selected, double* nu, double* score_max,
                       int32_t* t, void* stream);
/* min over k of the smallest eigenvalue of (H)_k after the rounds done so far (host *out):
 * the quantity the eta choice of the experiments section maximises.  Synchronous. */
int firal_round_criterion(firal_round round, double* out, void* stream);
/* Release the state (NULL is a no-op). */
int firal_round_destroy(firal_round round);

/* The eta choice of the experiments section: run all b rounds of the Round step for each of the
 * n_eta learning rates etas[] (host array) on ctx's rows with the relaxed weights z (device FP64
 * [n_pool]), lambda and flags as in firal_round_create, and keep the run whose (H)_k maximise
 * min_k lambda_min((H)_k) (firal_round_criterion; the first such eta on ties).  selected (host
 * int64 [b]) gets that run's selections in round order, criteria (host double [n_eta], may be
 * NULL) each run's criterion, best (host, may be NULL) the index of the kept eta.  Synchronous.
 * Errors: EINVAL (null argument, n_eta < 1, b outside [1, n_pool]), and those of the Round calls. */
int firal_round_eta_sweep(firal_ctx ctx, const double* z, double lambda, const double* etas,
                          int32_t n_eta, int32_t b, uint32_t flags, int64_t* selected,
                          double* criteria, int32_t* best, void* stream);

/* Static description of a return code. */
const char* firal_strerror(int code);

/* Detail of the last failing call on this host thread ("" if none). */
const char* firal_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FIRAL_H */
