/*
 * libwlra: the sWLR alternating sweep on one AMD Instinct MI355X (gfx950).
 *
 * Solves problem (5) of Dutta & Li, "A Fast Algorithm for a Weighted Low Rank
 * Approximation" (arXiv 1703.06303):
 *
 *     min over X1, X2 with rank([X1 X2]) <= r of
 *         || (A1 - X1) o W1 ||_F^2 + || A2 - X2 ||_F^2
 *
 * A = [A1 A2] is m x n, A1 its first k columns, W1 (m x k) has entries > 0,
 * and o is the entrywise product.  Each sweep is Algorithm 1 (Section 3): the
 * Golub-Hoffman-Stewart closed form of Theorem 1 gives C_p and
 * D_p = H_{r-k}((I - Q_p Q_p^T) A2) from X1_p = Q_p R_p, and the row update
 * below eq. (9) gives X1_{p+1}(i,:) = E_p(i,:) (diag(W1(i,:)^2) + C_p C_p^T)^-1
 * with E_p = A1 o W1 o W1 + (A2 - D_p) C_p^T.  The stopping rule is the one of
 * Section 4.1: with Error_p = ||X_p - X_{p-1}||_F, stop when Error_p < tol or
 * Error_p / ||X_{p-1}||_F < tol, or after max_sweeps X1 updates.
 *
 * Every call takes plain pointers and sizes.  Matrices are column-major
 * (a video frame is one contiguous column).  Device pointers are HIP device
 * memory on the handle's device; the caller owns every buffer it passes and
 * the library owns only its workspace.  No exception crosses this interface:
 * every entry point returns a status code (wlra_status below).
 */
#ifndef WLRA_H
#define WLRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  0, 1 and 2 mean a result is in the outputs; negative codes
 * mean the outputs are not written (argument and input errors) or must not
 * be used (WLRA_E_ROWSOLVE, WLRA_E_RANK, WLRA_E_EIG: the solve ran). */
enum wlra_status {
  WLRA_OK = 0,            /* converged under the Section 4.1 rule             */
  WLRA_MAX_SWEEPS = 1,    /* max_sweeps X1 updates done; result is X_p        */
  WLRA_INEXACT = 2,       /* a result X_p is returned, but the eigen step of
                             its sweep stopped at its round limit (see
                             WLRA_OPT_EIG_MAXIT) with a wanted Ritz pair still
                             above its residual target: D_p is a rank-(r-k)
                             matrix close to, but not within the stated
                             accuracy of, H_{r-k}(P^perp A2)                 */
  WLRA_E_ARG = -1,        /* bad dimension, leading dimension or pointer      */
  WLRA_E_WEIGHT = -2,     /* a W1 entry is not > 0 or not finite (Theorem 2
                             assumes (W1)_ij > 0)                             */
  WLRA_E_NONFINITE = -3,  /* A or X1_init has a NaN or Inf                     */
  WLRA_E_RANK = -4,       /* X1_p is numerically rank deficient: the paper
                             assumes rank(X1) = k (Section 3)                 */
  WLRA_E_NOMEM = -5,      /* workspace allocation failed                      */
  WLRA_E_HIP = -6,        /* a HIP runtime call failed                        */
  WLRA_E_NODEVICE = -7,   /* no usable gfx950 device                          */
  WLRA_E_ROWSOLVE = -8,   /* a per-row system diag(W1(i,:)^2) + C C^T of the
                             X1 update (row formula below eq. (9)) had a
                             pivot <= 0 in the storage precision (it is SPD in
                             exact arithmetic; this happens when W1^2 is below
                             the rounding of C C^T)                          */
  WLRA_E_EIG = -9,        /* the eigen step for H_{r-k} could not
                             orthonormalise its block                        */
  WLRA_E_SCRATCH = -10    /* wlra_solve_noalloc: the problem needs more
                             workspace than WLRA_NOALLOC_SCRATCH_BYTES        */
};

/* Arithmetic of a handle.  The storage type of A, W1, X1_init, X1_out and
 * X2_out is double for WLRA_FP64 and float otherwise.  Sums over the m rows
 * (the Grams X1^T X1, X1^T A2, A2^T A2 and the objective) and all k x k,
 * k x (n-k), (n-k) x (n-k) steps run in double in every mode. */
typedef enum {
  WLRA_FP64 = 0,
  WLRA_FP32 = 1,
  WLRA_MIXED_BF16 = 2    /* float storage; the validation pass stages A2 in
                            BF16 (round to nearest even).  The sweeps' X1
                            updates take the product with A2 (step 7) from
                            that copy on the BF16 matrix cores, with float
                            accumulation; every other step (the Grams of A2
                            and X1, the small steps, the change) uses A2
                            itself.  This phase runs until the Section 4.1
                            rule holds at max(tol, 1e-5) or max_sweeps - 1
                            updates; then one exact sweep (the refinement)
                            gives the returned X_{p+1}.  The status is that
                            of the first phase.                             */
} wlra_precision;

/* Start X1_0 (Algorithm 1 leaves it open; Section 4.1 recommends a random
 * matrix). */
typedef enum {
  WLRA_INIT_RANDOM = 0,  /* iid N(0,1) from Philox4x32-10 keyed by `seed`     */
  WLRA_INIT_GIVEN = 1,   /* X1_init (device, m x k, ld ldx0)                  */
  WLRA_INIT_A1 = 2,      /* X1_0 = A1                                         */
  WLRA_INIT_LEARNED = 3  /* learned warm start (not in the paper): a network
                            maps a Gaussian sketch of A to an n x r basis Y
                            of the solution's row space, and row i of the
                            start is the weighted least-squares fit of a_i
                            in span(Y^T) (weights W1 on the first k entries,
                            1 on the rest; problem (5) separates over rows
                            once the row space is fixed); X1_0 is its first
                            k columns.  If Y is zero or rank deficient, or a
                            row's solve fails, the random start keyed by
                            `seed` is used instead.  Needs `model` and
                            r <= 32.                                          */
} wlra_init;

typedef struct {
  int64_t m, n, k, r;      /* 0 <= k <= r <= min(m, n); A1 = first k columns    */
  const void *A;           /* device, m x n, column-major                       */
  int64_t lda;             /* >= m                                              */
  const void *W1;          /* device m x k, entries > 0 and finite; NULL means
                              every entry equals w1_const                       */
  int64_t ldw;             /* >= m when W1 != NULL                              */
  double w1_const;         /* > 0, used when W1 == NULL                         */
  double tol;              /* epsilon of Section 4.1 (the paper uses 1e-7);
                              tol <= 0 runs exactly max_sweeps X1 updates        */
  int32_t max_sweeps;      /* >= 0                                              */
  int32_t init;            /* wlra_init                                         */
  uint64_t seed;           /* WLRA_INIT_RANDOM key                              */
  const void *X1_init;     /* device m x k when init == WLRA_INIT_GIVEN         */
  int64_t ldx0;            /* >= m when X1_init is used                         */
  void *X1_out;            /* device m x k, required                            */
  int64_t ldx1;            /* >= m                                              */
  void *X2_out;            /* device m x (n-k) = X1 C + D, optional (NULL)      */
  int64_t ldx2;            /* >= m when X2_out != NULL                          */
  double *trace;           /* host, optional: 2*(max_sweeps+1) doubles; trace[p]
                              = F(X_p), trace[max_sweeps+1+p] = Error_p (p>=1)  */
  double eig_tol;          /* relative residual target of the H_{r-k} eigen
                              step (times ||A2^T A2||_F); <= 0 selects the
                              default: 64 eps for FP64, 1e-10 otherwise       */
  const float *model;      /* device, WLRA_INIT_LEARNED only: the network's
                              wlra_mlp_param_count(n, r) parameters (below)     */
  double *factors_out;     /* device, optional: the returned X_p's factors, in
                              order R (k x k, upper, X1_p^T X1_p = R^T R),
                              C (k x (n-k)), V (n-k x r-k, the top right
                              singular vectors of P_perp A2) and their squared
                              singular values (r-k), all column-major double:
                              X2_p = X1_p C + (A2 - X1_p C) V V^T               */
  /* ---- extensions around problem (5) (zero-filled: not used) ---- */
  const void *W2;          /* device, n - k entries of the storage type, or
                              NULL: one weight per column of the unweighted
                              block, eq. (6) with W2(i, j) = W2[j - k] > 0 and
                              finite (else WLRA_E_WEIGHT).  Column scaling
                              reduces it to problem (5) for [A1, A2 diag(W2)]
                              with X2 diag(W2) in place of X2 (same rank, same
                              objective); the validation pass stages that
                              matrix once in the workspace (m n extra
                              elements) and the sweeps run on it.  X2_out and
                              the mask are of the original problem; objective,
                              Error_p, the trace and factors_out are those of
                              the scaled problem (the objective is the same)  */
  uint8_t *mask_out;       /* device m x n bytes, column-major, optional: 1
                              where |A(i, j) - X(i, j)| > mask_tau for the
                              returned X_p, else 0 -- the foreground left by
                              the background estimate X (Section 4).  Decided
                              in the storage precision                        */
  int64_t ldm;             /* >= m when mask_out != NULL                        */
  double mask_tau;         /* >= 0 and finite when mask_out != NULL            */
  const double *V_init;    /* device, optional: v0_rows x (r - k) column-major
                              (ld ldv0) start of the first eigen step's block
                              for H_{r-k}, such as V from factors_out of a
                              solve on the same frames minus the newest ones;
                              rows v0_rows .. n - k - 1 start at zero.  Only
                              the eigen iteration's start changes, not what
                              it converges to                                 */
  int64_t ldv0;            /* >= v0_rows when V_init != NULL                    */
  int64_t v0_rows;         /* 1 <= v0_rows <= n - k when V_init != NULL         */
} wlra_problem;

typedef struct {
  int32_t status;          /* wlra_status                                       */
  int32_t sweeps;          /* X1 updates done (p of the returned X_p)           */
  double objective;        /* F(X_p) of problem (5), accumulated in double      */
  double abs_change;       /* Error_p = ||X_p - X_{p-1}||_F (0 when p = 0)      */
  double rel_change;       /* Error_p / ||X_{p-1}||_F                           */
  double gap;              /* sigma_{r-k} - sigma_{r-k+1} of P^perp A2, with
                              sigma_{r-k+1} from the first guard Ritz value of
                              the eigen block; +inf when r = k                  */
  float ms;                /* wall time of the call on the handle's stream      */
  int32_t eig_iters;       /* filter rounds of the eigen step, summed            */
  int32_t eig_matvecs;     /* products of M = (P^perp A2)^T P^perp A2 with one
                              vector done by the eigen step, summed             */
} wlra_result;

typedef struct wlra_ctx *wlra_handle;

/* wlra_create flags. */
#define WLRA_FLAG_PROFILE 1u  /* bracket every kernel launch with HIP events on
                                 the handle's stream and keep per-kernel totals
                                 (read with wlra_profile); adds event overhead */

/* Per-kernel timing totals of a profiling handle. */
typedef struct {
  char name[24];           /* kernel name                                       */
  int64_t launches;        /* launches since create or the last reset           */
  double ms;               /* summed device time between the bracketing events  */
  double bytes;            /* summed algorithmic HBM bytes of those launches
                              (each operand read or written once; 0 for the
                              small steps, whose data stay in cache)           */
  double flops;            /* summed algorithmic flops of those launches (0
                              where not tallied)                               */
} wlra_kstat;

/* Create a handle bound to `device` and `hip_stream` (a hipStream_t; NULL is
 * the null stream).  The handle owns a workspace that grows on demand before
 * the kernels of a solve are enqueued; wlra_reserve grows it ahead of time.
 * Returns WLRA_E_NODEVICE when the device is absent or not gfx950. */
int wlra_create(wlra_handle *out, int device, void *hip_stream, int precision,
                uint32_t flags);

/* Grow the workspace for problems up to the given sizes (optional). */
int wlra_reserve(wlra_handle h, int64_t m, int64_t n, int64_t k, int64_t r);

/* Solve one instance of problem (5) with Algorithm 1.  Blocks until the
 * result is on the host.  Writes X1_out (and X2_out when given) with the
 * returned X_p.  Inputs are only read. */
int wlra_solve(wlra_handle h, const wlra_problem *prob, wlra_result *res);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as wlra_solve, with the same kernels and results, but its workspace
 * is a fixed per-device array of WLRA_NOALLOC_SCRATCH_BYTES bytes inside the
 * library (set up by wlra_create for the handle's device and held until the
 * process ends) instead of the handle's growable workspace.  The call
 * allocates nothing: no hipMalloc, hipFree or allocating library routine.
 * Returns WLRA_E_SCRATCH, before any device work, when the problem needs a
 * larger workspace than the array holds (the size wlra_solve would grow the
 * handle's workspace to: about 12 MB for a 19200 x 200 FP32 problem with
 * k = 20, r = 25, and 19 MB in mixed precision, which fit; about 61 MB for
 * a 76800 x 600 one, which does not), and
 * WLRA_E_ARG for a handle created with WLRA_FLAG_PROFILE.  Every call on a
 * device shares that device's array and leaves its contents behind: calls
 * that overlap in time on one device (two streams, two threads, two handles)
 * race and must be ordered by the caller. */
#define WLRA_NOALLOC_SCRATCH_BYTES (32ll << 20)
int wlra_solve_noalloc(wlra_handle h, const wlra_problem *prob, wlra_result *res);

/* Solve `count` independent instances of problem (5) (uneven m, n, k, r
 * allowed; each one as wlra_solve would, with the one-workgroup eigen
 * kernel for every n - k).  The instances advance in lockstep, one sweep per
 * round: the single-workgroup small steps of every active instance (the
 * coefficients, M, the eigen step, the post step, the change pass's basis
 * and the stopping decision) run as one launch each with one workgroup per
 * instance, the streaming passes of each instance go to the batch streams
 * (the handle's stream and wlra_set_batch_lanes - 1 more, round robin), and
 * one read-back of all sweep states per round decides which instances go
 * on.  The batch starts after the work already queued on the handle's
 * stream, and that stream waits for all of it before later work.  Blocks
 * until every result is on the host.  The batch workspace (the sum of the
 * instances' workspaces) is grown before the first kernel of the call.
 * Returns WLRA_E_ARG if any instance fails the argument checks (nothing is
 * run), a negative status if the batch cannot be set up, else 0; the status
 * of each instance is in res[i].status, and res[i].ms is the time from the
 * start of the batch to the round in which that instance's last sweep was
 * decided (its outputs are written at the end of the batch).  Instances
 * must not share output buffers. */
int wlra_solve_batched(wlra_handle h, int32_t count, const wlra_problem *probs,
                       wlra_result *res);

/* Handle options (wlra_set_option).  They apply to later calls on the
 * handle. */
enum wlra_option {
  WLRA_OPT_EIG_MAXIT = 1,   /* filter rounds per eigen step before it stops
                               and reports WLRA_INEXACT (1..100000, default
                               60)                                           */
  WLRA_OPT_EIG_ONE_WG = 2   /* 1: the one-workgroup eigen kernel for every
                               n - k (default 0: a cooperative multi-workgroup
                               kernel for n - k >= 256 in wlra_solve;
                               wlra_solve_batched always uses the
                               one-workgroup kernel)                          */,
  WLRA_OPT_AUTOTUNE = 3     /* 1 (default): the first solve of each shape
                               (m, n - k, k, precision) on the handle times
                               the tall-skinny products X1^T A2 and A2^T A2 at
                               4 workgroup counts (512 .. 4096) on its own
                               operands and keeps the fastest for later
                               solves of that shape (the row sums then run
                               in that split's order: results are
                               reproducible per handle); 0: the default
                               count (2048)                                  */
};

/* Set a handle option; WLRA_E_ARG for an unknown option or a value out of
 * range. */
int wlra_set_option(wlra_handle h, int32_t option, int64_t value);

/* Number of streams used by wlra_solve_batched for the instances' streaming
 * passes (1..16, default 4; 1: the handle's stream only). */
int wlra_set_batch_lanes(wlra_handle h, int32_t lanes);

int wlra_destroy(wlra_handle h);

/* Copy up to `max` per-kernel totals into `out` (host) and return how many
 * kernels have totals (0 when the handle was created without
 * WLRA_FLAG_PROFILE).  reset != 0 clears the totals afterwards. */
int wlra_profile(wlra_handle h, int32_t max, wlra_kstat *out, int32_t reset);

/* Host-only argument check of one problem for a precision (no device access):
 * returns WLRA_OK or WLRA_E_ARG. */
int wlra_validate(const wlra_problem *prob, int precision);

const char *wlra_strerror(int status);

/* ---- Learned warm start (a systems extension; the paper's start is random).
 *
 * Sketch: s = vec(Om^T A Ps) / ||Om^T A Ps||_F (512 floats, s[a + 16 b]) with
 * Om (m x 16) and Ps (n x 32) iid N(0,1) from Philox4x32-10 under two fixed
 * keys (0x5EEDA001, 0x5EEDA002), element (i, c) of Om being draw i + c m.
 * Network: h1 = relu(W1 s + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
 * 512 -> 256 -> 256 -> n r, Y = y as an n x r column-major basis.  Parameter
 * vector (float, device): W1 (256 x 512 row-major), b1, W2 (256 x 256), b2,
 * W3 (n r x 256), b3.
 * Training target of a solved instance: T = [[I_k, C], [0, V^T]]^T (n x r),
 * whose column space is the row space of the solution X_p (from
 * factors_out).  Loss per sample, Q an orthonormal basis of T:
 * ||Y - Q Q^T Y||_F^2 + ||Y^T Y - I||_F^2, averaged over the batch; Adam
 * with beta1 0.9, beta2 0.999, eps 1e-8.  Batched arrays are row-major
 * (sample-major); every pointer below is device memory unless noted. */

/* Number of network parameters for (n, r), or -1 for bad sizes. */
int64_t wlra_mlp_param_count(int64_t n, int64_t r);

/* Fill `params` with a start: W_l = sqrt(2 / fan_in) N(0,1) draws keyed by
 * seed + l (l = 1, 2, 3), biases 0. */
int wlra_mlp_init(wlra_handle h, float *params, int64_t n, int64_t r, uint64_t seed);

/* The 512-float sketch of A (m x n, column-major, the handle's storage type). */
int wlra_sketch(wlra_handle h, int64_t m, int64_t n, const void *A, int64_t lda, float *out);

/* Y (batch x n r) = network(X (batch x 512)). */
int wlra_mlp_forward(wlra_handle h, const float *params, int64_t n, int64_t r, int32_t batch,
                     const float *X, float *Y);

/* One training step on a batch: loss and gradient for sketches X
 * (batch x 512) and targets T (batch x n x r, each column-major), then an
 * Adam update with step number `step` (1, 2, ...) of params, adam_m, adam_v
 * (all of wlra_mlp_param_count floats).  step <= 0 computes the loss and
 * gradient only.  *loss (host) gets the batch-mean loss; grad_out, when not
 * NULL, the gradient.  Returns WLRA_E_RANK if a target basis is singular. */
int wlra_mlp_train_step(wlra_handle h, float *params, float *adam_m, float *adam_v,
                        int32_t step, int64_t n, int64_t r, int32_t batch, const float *X,
                        const float *T, double lr, double *loss, float *grad_out);

/* Library version, major * 10000 + minor * 100 + patch. */
int wlra_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WLRA_H */
