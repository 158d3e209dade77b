/*
 * aapdhg.h -- C ABI of the MI355X AA-PDHG / FAA-PDHG library for linear programs.
 *
 * Problem (Section 2.1, problem LP-O, written with K = [G; A], q = [h; b]):
 *
 *     minimise  c^T x
 *     subject to (K x)_i >= q_i   for rows of type AAPDHG_ROW_GE  (the G x >= h block)
 *                (K x)_i  = q_i   for rows of type AAPDHG_ROW_EQ  (the A x  = b block)
 *                l <= x <= u      (l_j may be -inf, u_j may be +inf)
 *
 * Rows of the two types may be interleaved; the row type picks the dual cone
 * of y_i (y_i >= 0 on GE rows, free on EQ rows; Section 3, the set Y).
 *
 * Method: the PDHG map T of eq. pdhg, accelerated by Anderson mixing with a
 * safeguard (Alg 2, AA-PDHG) or with angle and length filtering (Alg 3-6,
 * FAA-PDHG), terminated on the relative KKT residual of Remark
 * re:constrcution-termi-con.  Vanilla PDHG is the same iteration with the
 * Anderson step switched off.  Options add the primal-weight update of Alg 7
 * (with the D-hat re-blend that follows it and the Iter_AA / c safeguard),
 * the fixed-frequency restarted PDHG that Section 5.2 compares against, and
 * the Ruiz + Pock-Chambolle preconditioning of Section 5.2.
 *
 * Conventions for every entry point:
 *   - Every call returns an aapdhg_status; nothing is thrown across the ABI.
 *     On failure the handle (or, for a NULL handle, the calling thread) keeps
 *     a message readable with aapdhg_last_error().
 *   - "host" arrays are ordinary CPU memory owned by the caller; the library
 *     copies what it needs before returning and never keeps the pointer.
 *     aapdhg_create_device and aapdhg_result_device take caller-owned device
 *     memory instead (for example torch tensors), under the same rule.
 *   - The library's own device memory is owned by it from create to destroy.
 *   - A stream argument is a hipStream_t passed as void*; NULL means the
 *     default stream.  A handle is used by one host thread at a time.
 *   - Not converging is not an error: it is reported in aapdhg_info.term.
 *
 * Library errors: AAPDHG_E_ARG (invalid argument or problem data),
 * AAPDHG_E_NOMEM (device or host allocation failed), AAPDHG_E_HIP (a HIP
 * runtime call failed; the message names it), AAPDHG_E_STATE (call not valid
 * in the handle's current state, e.g. result before solve).
 */
#ifndef AAPDHG_H
#define AAPDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AAPDHG_MAX_MEMORY 16 /* largest Anderson memory m_A supported */

typedef struct aapdhg_problem *aapdhg_t;
typedef struct aapdhg_batch *aapdhg_batch_t;
typedef struct aapdhg_server *aapdhg_server_t;

typedef enum { AAPDHG_ROW_EQ = 0, AAPDHG_ROW_GE = 1 } aapdhg_row_type;

typedef enum {
  AAPDHG_OK = 0,
  AAPDHG_E_ARG = -1,
  AAPDHG_E_NOMEM = -2,
  AAPDHG_E_HIP = -3,
  AAPDHG_E_STATE = -4,
  AAPDHG_PENDING = 1 /* server: the ticket is not finished yet (not an error) */
} aapdhg_status;

typedef enum {
  AAPDHG_CONVERGED = 0,  /* relative KKT <= tol at the returned iterate       */
  AAPDHG_ITER_LIMIT = 1, /* max_iter loop passes done                        */
  AAPDHG_TIME_LIMIT = 2, /* wall-clock limit reached at an epoch boundary     */
  AAPDHG_NUMERICAL = 3,  /* the fixed-point residual became NaN or infinite   */
  AAPDHG_RUNNING = 4     /* not finished (only seen before a solve completes) */
} aapdhg_term;

/* AAPDHG_VARIANT_RPDHG: fixed-frequency restarted PDHG, the comparison method of Section 5.2
 * (its toy example restarts every 75 iterations): PDHG steps, and every restart_period-th
 * iterate u^{eR} is replaced by the average of its epoch u^{(e-1)R+1}, ..., u^{eR} (the
 * restart point of the cited restarted PDHG; the paper does not name one). */
typedef enum {
  AAPDHG_VARIANT_PDHG = 0,
  AAPDHG_VARIANT_AA = 1,
  AAPDHG_VARIANT_FAA = 2,
  AAPDHG_VARIANT_RPDHG = 3
} aapdhg_variant;

typedef struct {
  int32_t variant;    /* aapdhg_variant: PDHG, AA-PDHG (Alg 2), FAA-PDHG (Alg 3) or
                         restarted PDHG                                                   */
  int32_t precision;  /* 0: float32 data and iterates, float64 reductions, Gram, solve
                         and KKT; 1: float64 throughout                                  */
  int32_t memory;     /* Anderson memory m_A, 1..AAPDHG_MAX_MEMORY                        */
  double D;           /* safeguard constant D > 0 (Alg 2, safeguard line)                 */
  double eps_sg;      /* safeguard exponent epsilon > 0                                   */
  double beta;        /* damping beta in (0, 1]                                           */
  double eta;         /* Tikhonov shift eta >= 0 of (dG^T dG + eta I), AA-PDHG only       */
  double cs;          /* angle-filter threshold c_s in (0, 1] (Alg 4), FAA only           */
  double kappa_bar;   /* length-filter bound kappa-bar > 0 (Alg 5), FAA only              */
  double tau, sigma;  /* step sizes; if either is <= 0 both are set to 0.9 / ||K||_2
                         with ||K||_2 estimated by power iteration (Section 5.1; `seed`
                         gives the start vector; a zero estimate for a nonzero K falls
                         back to the Frobenius norm, an upper bound)                      */
  double tol;         /* relative KKT tolerance (Remark re:constrcution-termi-con)        */
  int64_t max_iter;   /* loop passes before AAPDHG_ITER_LIMIT                             */
  double time_limit_s;/* wall-clock limit per solve call, <= 0 for none                   */
  int32_t kkt_every;  /* evaluate the KKT test at iterations k with k % kkt_every == 0    */
  int32_t dhat_mode;  /* D-hat (Remark se:Dhat_construction): 0 identity, 1 the square
                         root of the column/row max-abs of K (literal), 2 its reciprocal */
  int32_t ruiz_iters; /* Ruiz equilibration sweeps applied at create (Section 5.2), 0 off */
  int32_t power_iters;/* power-iteration cap for the step size                            */
  int32_t epoch;      /* iterations per device epoch between host checks of the status    */
  int32_t chunks_per_block; /* work items per workgroup of the SpMV passes, 0 = automatic   */
  int32_t loop_kernel;/* 0: loop passes run in one persistent cooperative launch per epoch
                         when the LPs fit the resident workgroups, else three launches per
                         pass; 1: always three launches per pass                          */
  int32_t wait_limit_us; /* bound (microseconds) of every cross-workgroup wait of the
                         persistent loop kernel; a wait that reaches it stops the LP
                         (AAPDHG_NUMERICAL) and the solve returns AAPDHG_E_HIP;
                         0 = 4 s                                                          */
  /* Primal-weight update (Alg 7 and the remark on the primal-weight form that follows it):
   * at the top of every iteration k > 0 with k % pw_period == 0 the distances
   * dx = ||x^k - x^{k-pw_period}||, dy = ||y^k - y^{k-pw_period}|| (to u^0 for the first
   * check) are measured; if both exceed pw_eps_zero the Anderson memory is reset,
   * omega = exp(theta log(dy/dx) + (1 - theta) log omega), tau = gamma / omega and
   * sigma = gamma * omega with gamma = sqrt(tau_0 sigma_0), and (pw_dhat = 1) D-hat becomes
   * (1 - alpha) diag(1/omega, omega) + alpha diag(D-hat_1 / omega, D-hat_2 omega), alpha = 0.1
   * when rho_k = (||g^{k-1}|| - ||g^k||) / max(||g^{k-1}||, pw_eps_zero) > pw_rho, else 0.9.
   * The difference pair of iteration k is not formed (it would join residuals of two
   * maps): iteration k runs with an empty memory. */
  int32_t pw_period;  /* U_P; 0 = no primal-weight update                                 */
  double pw_theta;    /* smoothing theta in [0, 1] (0.5 in Section 5.2)                   */
  double pw_eps_zero; /* epsilon_zero > 0 of the acceptance test (default 1e-10)          */
  double pw_omega0;   /* omega^0 > 0; <= 0 takes sqrt(sigma / tau) (1 for tau = sigma)     */
  double pw_rho;      /* residual-decrease threshold of the D-hat re-blend (default 0)    */
  double sg_div;      /* c of the Iter_AA / c safeguard (supplement, update-D-hat study):
                         the bound uses (i^k / c + 1); 1 = Alg 2 as printed               */
  int32_t pw_dhat;    /* 1: re-blend D-hat at every accepted weight update, 0: keep it    */
  int32_t restart_period; /* epoch length R of AAPDHG_VARIANT_RPDHG (>= 1; default 75)     */
  int32_t prep_device;    /* where the Ruiz and Pock-Chambolle scaling run: 0 host, 1 device,
                             2 (default) the device from 2^20 entries, else the host.  Ruiz
                             gives the same bits either way                               */
  int32_t pock_chambolle; /* 1: after the Ruiz sweeps, one Pock-Chambolle step with alpha = 1
                             (rows and columns divided by the square roots of their absolute
                             sums), the preconditioning of Section 5.2 together with Ruiz */
  int32_t angle_mode;     /* FAA AngleFilter (Alg 4): 0 (default) judges every column against
                             one factorisation of the reversed history, as printed; 1 judges
                             column i against the columns kept so far (the factor refreshed
                             after each removal), which keeps every column mode 0 keeps   */
  uint64_t seed;          /* start vector of the power iteration for ||K||_2: entry j is 2u - 1,
                             u the top 53 bits of output j of SplitMix64 started at `seed`, as
                             a fraction of 2^53 (a random start; a constant one is orthogonal
                             to the dominant singular vector when the rows of K sum to zero) */
  int32_t length_floor;   /* FAA LengthFilter (Alg 5) when no k passes its test: 0 (default)
                             keeps no column (the count-down loop runs out), 1 keeps the
                             newest column (the loop read as stopping at k = 1)            */
  int32_t graph;          /* 1: the three-launch passes of an epoch are captured once in a HIP
                             graph and replayed (a set uses the graph when any member asks;
                             the persistent kernel is one launch already); 0 (default) off.
                             The same kernels run in the same order: results are unchanged */
  int32_t autotune;       /* 1: the LP's work-table parameters (row weight of the chunking,
                             chunks per workgroup, loop kernel) are chosen at create by timing
                             candidates on the device, or taken from the tuning cache (file
                             AAPDHG_TUNE_CACHE, default ~/.cache/aapdhg/tune.txt) for LPs of
                             the same shape class; 0 (default): the built-in choice        */
  int32_t gram_mode;      /* how Alg 2's Gram matrix of the memory and its right-hand side are
                             formed.  The persistent loop kernel updates them on every pass
                             (dots of the new difference column with the stored ones).  The
                             three launches per pass can instead form them from the stored
                             columns only for Anderson steps, which saves reading the memory
                             on every pass.  0 (default): on demand for an LP that cannot run
                             in the persistent kernel by itself (so it always runs in three
                             launches), every pass otherwise, so an LP's iterates do not
                             depend on the other LPs of its batch or server set; 1: every
                             pass; 2: on demand whenever the LP runs in three launches (an
                             LP that moves between the kernels, such as a batch member or a
                             served request whose set changes, can then differ from its solo
                             run in rounding)                                            */
} aapdhg_options;

typedef struct {
  int32_t term;            /* aapdhg_term                                                  */
  int32_t gram_on_demand;  /* 1: the LP's three-launch passes form the Gram matrix only for
                              Anderson steps (option gram_mode); 0: on every pass          */
  int64_t iters;           /* index k of the returned iterate u^k                          */
  int64_t aa_steps;        /* i^k: Anderson steps taken                                    */
  int64_t pdhg_steps;      /* j^k: plain PDHG steps taken                                  */
  double primal_obj;       /* c^T x  (on the problem as solved, i.e. after any scaling)    */
  double dual_obj;         /* q^T y + l^T lambda+ - u^T lambda-                            */
  double r_gap, r_pri, r_dual, kkt; /* relative KKT pieces and their max               */
  double gnorm;            /* ||g^k|| of the last loop pass                                */
  double g0norm;           /* ||g^0||                                                      */
  double solve_seconds;    /* host wall time of the last solve call; for a batch member, the
                              time until the member was seen stopped (status read once per
                              epoch)                                                       */
  double step_tau, step_sigma; /* step sizes in use (they change with the primal weight) */
  double omega;            /* primal weight (sqrt(step_sigma / step_tau))                  */
  int64_t pw_updates;      /* accepted primal-weight updates                               */
  int64_t faa_empty;       /* FAA steps whose filters left no column (u_AA = u + beta D g) */
} aapdhg_info;

/* Fills *o with the defaults of Section 5.1: AA-PDHG, float32, m_A = 10, D = 10,
 * epsilon = 1, beta = 1, eta = 1e-10, c_s = 0.2, kappa-bar = 1e8, tol = 1e-4,
 * tau = sigma = 0 (power iteration), max_iter = 100000, kkt_every = 64,
 * dhat_mode = 1, no Ruiz, power_iters = 200, epoch = 256. */
void aapdhg_default_options(aapdhg_options *o);

/* Create a solver for one LP.
 *   m, n        rows and columns of K (m >= 1, n >= 1); nnz entries (0 <= nnz < 2^31).
 *   row_ptr     host int64[m+1], CSR row offsets, row_ptr[0] = 0, non-decreasing, row_ptr[m] = nnz.
 *   col_idx     host int32[nnz], column of each entry, in [0, n), no repeats within a row
 *               (any order within a row; the library sorts).
 *   val         host double[nnz], finite.
 *   c           host double[n], finite.         q   host double[m], finite (b and h).
 *   l, u        host double[n], l_j <= u_j, l_j < +inf, u_j > -inf; +-inf allowed.
 *   row_type    host uint8[m], each AAPDHG_ROW_EQ or AAPDHG_ROW_GE.
 *   opt         options (NULL for defaults); copied.
 * The data is copied, validated (E_ARG with a message on any violation), equilibrated if
 * requested, and moved to the current HIP device.  In float32 mode values are rounded to
 * float32.  Step sizes must satisfy tau * sigma * ||K||^2 < 1 (the standing assumption of
 * Section 3); when both are given this is checked against the power-iteration estimate.
 * On success *out owns the device state until aapdhg_destroy. */
aapdhg_status aapdhg_create(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr,
                            const int32_t *col_idx, const double *val, const double *c,
                            const double *q, const double *l, const double *u,
                            const uint8_t *row_type, const aapdhg_options *opt, aapdhg_t *out);

/* Solve from the start point u^0 = (clip(0, l, u), 0) (Alg 2 initialisation): the init step
 * u^1 = T u^0, then loop passes (Alg 2 loop; Alg 3 for FAA-PDHG) until the KKT test of Remark
 * re:constrcution-termi-con passes, max_iter, or time_limit_s.  Asynchronous: the reset and the
 * init step are enqueued on `stream`, and a thread of the handle enqueues the loop passes in
 * epochs of `epoch` passes on the same stream, reading the LP's status (decided on the device
 * by each pass) between epochs; the call returns at once.  aapdhg_result, aapdhg_wait and every
 * other call on the handle wait for the solve first; a failure of the solve (for example a HIP
 * error) is returned by the first of them.  The stream must stay valid until then. */
aapdhg_status aapdhg_solve(aapdhg_t h, void *stream);

/* Wait for a solve started with aapdhg_solve to finish (no-op without one); returns the
 * solve's error, if it had one. */
aapdhg_status aapdhg_wait(aapdhg_t h);

/* Device-memory variants, for callers whose data already lives on the GPU (say in torch
 * tensors).  The LP is the one of Section 2 (the standard form the method solves), stored as
 * for aapdhg_create.
 *
 * aapdhg_create_device: the same arguments, sizes and layouts as aapdhg_create, with every
 * array in device memory of the current device.  It copies them to the host on `stream`
 * (NULL = the default stream), waits for the copies, and then creates exactly as
 * aapdhg_create does: the two give the same problem, bit for bit.  Each array must lie
 * inside one device allocation, checked with hipMemGetAddressRange; a host pointer, or a
 * buffer shorter than m, n and nnz imply, is AAPDHG_E_ARG.  Other errors as aapdhg_create.
 *
 * aapdhg_result_device: waits for the handle's work, runs the evaluation pass at the current
 * iterate (the relative KKT quantities of the termination remark) and enqueues on `stream`,
 * without waiting, a kernel that writes x double[n], y double[m] and lambda double[n] into
 * the caller's device memory, unscaled as aapdhg_result gives them (the same float64 operations, so the same
 * bits).  Any of the three may be NULL; info is host memory (may be NULL), filled before
 * return.  AAPDHG_E_STATE before any solve or iterate.  The caller owns every buffer in
 * both calls. */
aapdhg_status aapdhg_create_device(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr,
                                   const int32_t *col_idx, const double *val, const double *c,
                                   const double *q, const double *l, const double *u,
                                   const uint8_t *row_type, const aapdhg_options *opt, void *stream,
                                   aapdhg_t *out);
aapdhg_status aapdhg_result_device(aapdhg_t h, double *x, double *y, double *lambda, aapdhg_info *info,
                                   void *stream);

/* Enqueue `iters` loop passes on `stream` without waiting (asynchronous): each pass is one
 * iteration of the loop of Alg 2 (Alg 3 for FAA-PDHG; eq. pdhg for the map T), with the KKT
 * test of Remark re:constrcution-termi-con every kkt_every passes.  On a fresh or reset handle
 * the first pass is the init step (Alg 2 initialisation).  Passes after termination do
 * nothing. */
aapdhg_status aapdhg_iterate(aapdhg_t h, void *stream, int64_t iters);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same passes as aapdhg_iterate, with
 * the same results bit for bit, but the passes' scratch (partial-sum records, decision, split
 * and Gram-launch partials and counters, the persistent kernel's barrier counters and
 * published decisions) lives in
 * a static device array of the library instead of the handle's buffers.  The call allocates
 * nothing: it clears the part of the array the LP needs with a fill kernel on `stream` and
 * enqueues the passes (asynchronous, like aapdhg_iterate).  The array holds 2 MiB per GPU
 * (kept until the process ends); an LP whose pass tables need more is AAPDHG_E_ARG with the
 * size in the message.  The need is 384 bytes per workgroup of a pass and per row or column
 * longer than 2048 entries, plus, per 2048 entries of n + m, 16 bytes and 8 (M (M + 1) / 2 + M)
 * bytes of Gram partials (M: m_A rounded up to 4, 8, 10 or 16): about 1.5 MiB for a
 * 1M x 2M LP with 20M entries and m_A = 10 (too much with m_A = 16), 0.2 MiB for a
 * 20k x 50k LP.  Every call on one
 * GPU uses the same array: calls that overlap on one GPU (other streams, other host threads)
 * race and must be serialised by the caller; consecutive calls on one stream are safe. */
aapdhg_status aapdhg_iterate_noalloc(aapdhg_t h, void* stream, int64_t iters);

/* Measurement variant of aapdhg_iterate: `iters` loop passes (after the init step, which is
 * run first and not timed on a fresh or reset handle) with HIP events recorded on `stream`
 * around the launches; waits for completion and fills ms4[0..3]:
 *   persistent loop kernel: {1, duration in ms of its one launch, iters, 1}
 *     (iters <= 65535);
 *   three launches per pass: {0, mean ms of the primal CSC launch, of the dual CSR launch
 *     with the float64 decisions, of the Gram launch and the mix launch}; the events add a
 *     small gap between launches, so use aapdhg_iterate for throughput. */
aapdhg_status aapdhg_iterate_timed(aapdhg_t h, void *stream, int64_t iters, double *ms4);

/* Return to the start point u^0 of Alg 2's initialisation (discard iterate, history and
 * counters); asynchronous on `stream`. */
aapdhg_status aapdhg_reset(aapdhg_t h, void *stream);

/* Wait for the handle's work, evaluate the KKT quantities of Remark re:constrcution-termi-con
 * at the current iterate (primal and dual objectives, relative gap, primal and dual
 * residuals, lambda = P_Lambda(c - K^T y) by the cases of eq. lambda-case), and copy results
 * to host memory: x double[n], y double[m], lambda double[n], each may be NULL.  Values refer to the original (unscaled) problem when Ruiz scaling was
 * used; info (may be NULL) reports the KKT pieces of the problem as solved. */
aapdhg_status aapdhg_result(aapdhg_t h, double *x, double *y, double *lambda, aapdhg_info *info);

/* Copy the full iteration state to host memory (checkpoint): what Alg 2 carries from k to
 * k+1 (the iterate, the previous iterate and residual, the memory Delta G and Delta U, the
 * latter kept as W = Delta U + beta D-hat Delta G, and the counters i, j).  Buffers, all
 * double:
 *   u      [n+m]  current iterate u^k (x then y, scaled problem)
 *   u_prev [n+m]  u^{k-1}            g_prev [n+m]  g^{k-1}
 *   dG     [m_A*(n+m)] history columns by physical slot, W [m_A*(n+m)] = dU + beta D-hat dG
 *   meta   int64[8 + 2*AAPDHG_MAX_MEMORY]: k, status, i, j, nlive, newslot, branch of the last
 *          pass (0 none, 1 PDHG, 2 Anderson), nmix (columns the last Anderson step mixed), the
 *          live slots (oldest first, AAPDHG_MAX_MEMORY entries), then the nmix mixed slots in
 *          the order of gamma (AAPDHG_MAX_MEMORY entries, zero past nmix)
 *   gram   double[AAPDHG_MAX_MEMORY^2 + 3*AAPDHG_MAX_MEMORY + 2]: Gram by slot, rhs, du2, n0,
 *          gnorm, then gamma of the last Anderson step (nmix entries used, zero past them).
 *          The Gram entries of the live slots and rhs (<dG[slot], g^{k-1}>) are current: passes
 *          that leave them stale (three launches per pass form them only for Anderson steps)
 *          are followed by a refresh on the device before they are copied.
 * Any pointer may be NULL to skip it.  aapdhg_set_state reads meta up to the live slots and
 * gram up to gnorm. */
aapdhg_status aapdhg_get_state(aapdhg_t h, double *u, double *u_prev, double *g_prev, double *dG,
                               double *W, int64_t *meta, double *gram);
/* Restore a state written by aapdhg_get_state (same problem and options). */
aapdhg_status aapdhg_set_state(aapdhg_t h, const double *u, const double *u_prev,
                               const double *g_prev, const double *dG, const double *W,
                               const int64_t *meta, const double *gram);

/* Primal-weight state (not part of aapdhg_get_state's checkpoint; aapdhg_set_state resets
 * it to the start values, so restore it with aapdhg_set_weights after aapdhg_set_state).
 *   w       double[AAPDHG_WEIGHT_WORDS]: omega, gamma, tau, sigma, D-hat coefficients
 *           a_x, a_y, b_x, b_y (D-hat in use = a D-hat_0 + b on each part, D-hat_0 that of
 *           the D-hat construction), accepted updates, and 1 when the weight changed at the
 *           last check and the next iteration is the first after the reset (else 0).
 *   anchor  double[n+m]: the iterate of the last check (u^0 before the first); E_STATE
 *           when pw_period = 0.  Either pointer may be NULL (set_weights needs w). */
#define AAPDHG_WEIGHT_WORDS 10
aapdhg_status aapdhg_get_weights(aapdhg_t h, double *anchor, double *w);
aapdhg_status aapdhg_set_weights(aapdhg_t h, const double *anchor, const double *w);

/* Sizes of the created problem and the step sizes it was created with (before any
 * primal-weight update; aapdhg_info holds the ones in use). */
aapdhg_status aapdhg_get_dims(aapdhg_t h, int32_t *m, int32_t *n, int64_t *nnz, double *tau,
                              double *sigma);

/* Ruiz scaling factors in use (d_row[m], d_col[n]); all ones without Ruiz. */
aapdhg_status aapdhg_get_scaling(aapdhg_t h, double *d_row, double *d_col);

aapdhg_status aapdhg_destroy(aapdhg_t h);

/* Text of the last error on the handle (or of the calling thread when h is NULL). */
const char *aapdhg_last_error(aapdhg_t h);

/* ---- batched solves: many LPs of uneven sizes advance in the same kernel launches ----
 * Each member runs its own Alg 2 / Alg 3 loop (the paper solves one LP at a time; batching
 * is how this library fills the device with independent solves).
 * The batch refers to the problems' device state; they must outlive the batch, must share
 * the precision and may not be used on their own while the batch is alive.  Each problem
 * keeps its own options, tiles and reduction order, so its iterates do not depend on the
 * other members of the batch. */
aapdhg_status aapdhg_batch_create(int32_t count, const aapdhg_t *problems, aapdhg_batch_t *out);
/* Solve every member from its start point; returns when all have terminated. */
aapdhg_status aapdhg_batch_solve(aapdhg_batch_t b, void *stream);
/* Enqueue `iters` loop passes for every member (asynchronous).  A member that has not
 * started takes its init step first, in a launch of its own. */
aapdhg_status aapdhg_batch_iterate(aapdhg_batch_t b, void *stream, int64_t iters);
/* Measurement variant of aapdhg_batch_iterate (see aapdhg_iterate_timed). */
aapdhg_status aapdhg_batch_iterate_timed(aapdhg_batch_t b, void *stream, int64_t iters, double *ms4);
/* Result of member i (0 <= i < count, in the order given to aapdhg_batch_create): the same
 * as aapdhg_result on that member's handle (waits for the device; caller-owned host buffers
 * x[n_i], y[m_i], lambda[n_i], any may be NULL).  AAPDHG_E_ARG for an index out of range,
 * with the text on the calling thread (aapdhg_last_error(NULL)). */
aapdhg_status aapdhg_batch_result(aapdhg_batch_t b, int32_t i, double *x, double *y, double *lambda,
                                  aapdhg_info *info);
aapdhg_status aapdhg_batch_destroy(aapdhg_batch_t b);

/* ---- serving: continuous batching of LP requests (not in the paper: a serving form of the
 * batched solves; each request is solved by Alg 2 as aapdhg_solve would) ----
 * An admission thread creates submitted LPs (host tables, uploads, scaling, step sizes, the
 * init step of Alg 2) on `copy_stream` while their estimated device footprint fits in
 * hbm_budget_bytes and fewer than max_slots are admitted; an epoch thread takes the created
 * LPs in at epoch boundaries, advances all resident LPs in shared epochs of loop passes on
 * `compute_stream`, and retires finished ones.  So requests that arrive while others run are
 * set up while the device computes, and then share the device.  opt applies to every request
 * (NULL: defaults).  Streams are hipStream_t passed as void*, distinct, non-blocking
 * (hipStreamNonBlocking) so that neither waits on the default stream; NULL: the server
 * creates its own.  Caller-given streams must outlive aapdhg_server_stop. */
aapdhg_status aapdhg_server_start(size_t hbm_budget_bytes, int32_t max_slots,
                                  const aapdhg_options *opt, void *compute_stream, void *copy_stream,
                                  aapdhg_server_t *out);
/* Submit one LP (arguments as aapdhg_create; copied).  Returns at once with *ticket. */
aapdhg_status aapdhg_server_submit(aapdhg_server_t s, int32_t m, int32_t n, int64_t nnz,
                                   const int64_t *row_ptr, const int32_t *col_idx,
                                   const double *val, const double *c, const double *q,
                                   const double *l, const double *u, const uint8_t *row_type,
                                   uint64_t *ticket);
/* AAPDHG_PENDING while the request is queued or running; AAPDHG_OK once finished, with the
 * results copied out (x[n], y[m], each may be NULL) and the ticket released.  t_admit and
 * t_done (may be NULL) receive the seconds from submission to admission and to completion
 * (t_admit is -1 for a request that failed before admission). */
aapdhg_status aapdhg_server_poll(aapdhg_server_t s, uint64_t ticket, aapdhg_info *info,
                                 double *x, double *y, double *t_admit, double *t_done);
/* Counters: submitted, admitted (taken into the epochs), finished, resident now, epochs run,
 * estimated device bytes of the admitted requests (being created, ready or resident). */
aapdhg_status aapdhg_server_stats(aapdhg_server_t s, int64_t *stats6);
/* Stop the worker (running requests are abandoned) and free everything. */
aapdhg_status aapdhg_server_stop(aapdhg_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* AAPDHG_H */
