/*
 * cakf.h - C ABI of the MI355X computation-aware Kalman filter library (libcakf.so).
 *
 * The library runs the update step of the computation-aware Kalman filter (CAKF) and
 * its smoother (CAKS) of Pfoertner, Wenger, Cockayne and Hennig (arXiv 2405.08971)
 * for the separable spatiotemporal prior with an Ornstein-Uhlenbeck temporal factor
 * (Lemma C.1 with D' = 1):
 *
 *   state   u_k in R^n at the n spatial points X,
 *   prior   Sigma = signal_var * K(X, X)        (Matern(nu) spatial correlation K),
 *   dynamics u_k = a u_{k-1} + q_k,  q_k ~ N(0, (1 - a^2) Sigma),  a = exp(-dt / ell_t),
 *   observations y_k = u_k[idx_k] + eps_k,  eps_k ~ N(0, noise_var I).
 *
 * Covariances are never formed.  The filter state is a mean m (n) and a downdate
 * factor M (n x rank) with covariance Sigma - M M^T (Prop. A.2).  Kernel matrices are
 * evaluated tile by tile inside the kernels and never stored.
 *
 * Conventions for every entry point:
 *  - All device buffers hold FP32 unless stated; "device" means GPU memory of the
 *    device current at cakf_create.  Matrices are row-major unless stated.
 *  - Work is enqueued asynchronously on the configured stream; no entry point
 *    synchronises the host except cakf_diagnostics and cakf_loglik, which say so.
 *  - Argument errors are detected on the host and returned as negative codes before
 *    anything is enqueued.  Numerical events (a dropped action, a non-finite value)
 *    are never errors: they are counted in a device status word (cakf_diagnostics).
 *  - A context is not thread-safe.  Results are deterministic: the same inputs give
 *    bitwise identical outputs (no floating-point atomics are used).
 */
#ifndef CAKF_H
#define CAKF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cakf_ctx cakf_ctx;

/* Status codes. */
#define CAKF_OK        0
#define CAKF_E_ARG    -1   /* invalid argument (null pointer, size out of range)      */
#define CAKF_E_HIP    -2   /* a HIP runtime call failed                                */
#define CAKF_E_NOMEM  -3   /* device allocation failed in cakf_create                  */
#define CAKF_E_STATE  -4   /* call out of order (e.g. truncate with nothing to drop)   */
#define CAKF_E_SOLVER -5   /* rocBLAS / rocSOLVER returned an error                    */
#define CAKF_E_SCRATCH -6  /* the call needs more than the static scratch array holds  */

/* Spatial Matern kernel, identified by 2*nu. */
#define CAKF_MATERN12 1
#define CAKF_MATERN32 3
#define CAKF_MATERN52 5

/* Distance between points: Euclidean (chordal for points on the unit sphere, the
 * extrinsic construction of App. D.2.3) or great-circle (arccos of the dot product of
 * unit vectors). */
#define CAKF_DIST_EUCLID   0
#define CAKF_DIST_GEODESIC 1

/* Arithmetic of the kernel-matrix x block product P^- H^T [W w] (Alg. 2):
 *  FP32   - FP32 kernel tiles, FP32 MFMA contraction of 64 observations at a time, the
 *           chunk sums added in FP64;
 *  BF16   - FP32 kernel tiles rounded to BF16, BF16 MFMA with FP32 accumulation;
 *  BF16X3 - BF16 MFMA on split operands: K = Kh + Kl, B = Bh + Bl (each part BF16),
 *           Y = Kh Bh + Kl Bh + Kh Bl, which restores close to FP32 accuracy.
 * The observation-space loop (actions, Gram matrix) always runs in FP32 with FP64
 * small matrices.  In FP32 mode every kernel entry takes its Euclidean distance from
 * coordinate differences; the BF16 modes form the squared distances of the Euclidean
 * Matern-3/2 and -5/2 kernels on FP32 MFMA from norms and dot products, which is faster
 * but leaves relative errors up to ~1e-5 in single entries. */
#define CAKF_PREC_FP32   0
#define CAKF_PREC_BF16   1
#define CAKF_PREC_BF16X3 2

/* Policy (Sec. 3.3): CG - the current residual is the next action (App. E, the
 * policy of all the paper's experiments); GIVEN - the actions are supplied by the
 * caller (any full-rank S is admissible); BLOCK - block-residual actions, not one of the
 * paper's experiments but admissible in the same sense: actions come in rounds of
 * block_actions, each round splitting the residual at its start over fixed contiguous
 * groups of the observations (group g of b = [floor(g m / b), floor((g + 1) m / b))),
 * so that one kernel-matrix product with b vectors serves the whole round.  The last
 * round takes the actions left (b_t = min(b, actions left)); resid_tol must be 0 with
 * BLOCK and GIVEN (cakf_create returns CAKF_E_ARG otherwise). */
#define CAKF_POLICY_CG    0
#define CAKF_POLICY_GIVEN 1
#define CAKF_POLICY_BLOCK 2

/* Temporal factor of the separable prior (Lemma C.1):
 *   OU        - exponential (Matérn-1/2) kernel exp(-|t - t'| / ell_t): the state is the
 *               value at the n points, A = a I with a = exp(-dt / ell_t) (ou_coeff);
 *   MATERN32  - Matérn-3/2 kernel (1 + lam |tau|) exp(-lam |tau|), lam = sqrt(3) / ell_t:
 *               the state stacks the values (rows 0..n-1) and the time derivatives
 *               scaled by 1/lam (rows n..2n-1), so that its stationary covariance is
 *               I_2 (x) Sigma; with s = lam dt and a = exp(-s) (ou_coeff) one step is
 *               A = a [[1 + s, s], [-s, 1 - s]] (x) I_n.  Observations pick value rows.
 * The state (mean, factor) has n rows (OU) or 2n rows (MATERN32).  MATERN32 supports
 * predict, update (any policy), truncate, step, the state and marginal-variance calls
 * (value rows) and the log-likelihood; the smoother, sampler and derivative workspaces
 * are OU-only (cakf_create returns CAKF_E_ARG). */
#define CAKF_TEMPORAL_OU       0
#define CAKF_TEMPORAL_MATERN32 1

typedef struct {
    int n;                  /* spatial points (state dimension n, or 2n), >= 1       */
    int dim;                /* coordinates per point: 2 or 3                         */
    const float* X;         /* device, n x dim row-major; read once in cakf_create   */
    int kernel;             /* CAKF_MATERN12/32/52                                   */
    int dist;               /* CAKF_DIST_*; GEODESIC needs dim = 3 unit vectors      */
    double lengthscale;     /* spatial lengthscale ell > 0                           */
    double signal_var;      /* sigma_f^2 > 0                                         */
    double noise_var;       /* observation noise variance > 0                        */
    double ou_coeff;        /* a = exp(-dt / ell_t) (OU) or exp(-sqrt(3) dt / ell_t)
                               (MATERN32), 0 < a <= 1                                */
    int temporal;           /* CAKF_TEMPORAL_*                                        */
    int max_obs;            /* largest m passed to cakf_update                       */
    int max_actions;        /* action budget i per update, 1..256 (at most m used)   */
    int max_rank;           /* rank cap r of the truncated factor, 1..1024           */
    int policy;             /* CAKF_POLICY_*                                         */
    int block_actions;      /* actions per round of POLICY_BLOCK, 1..max_actions
                               (ignored by the other policies)                       */
    double resid_tol;       /* stop when ||r|| <= resid_tol * ||r0||; 0 = never;
                               POLICY_CG only (the stop compares the norms of the
                               residual actions; cakf_create returns CAKF_E_ARG for
                               resid_tol != 0 with another policy)                  */
    double pivot_tol;       /* drop action j when its Ghat-orthogonal part keeps no
                               more than pivot_tol of s_j^T Ghat s_j (breakdown);
                               typical 1e-10                                         */
    int prec;               /* CAKF_PREC_* of the block product                      */
    int smoother;           /* nonzero: also allocate the smoother workspace         */
    int sample_paths;       /* largest number of paths per sampler call, 0..256
                               (0: no sampler workspace)                              */
    int gradient;           /* nonzero: also allocate the workspace of
                               cakf_loglik_grad (needs max_actions <= 256)           */
    void* stream;           /* hipStream_t for all work; NULL = the null stream      */
} cakf_config;

/* Optional per-update record, all caller-owned device buffers; any field may be NULL.
 * Sizes use m of the update and i = max_actions; entries beyond the number of kept
 * actions are zero. */
typedef struct {
    float*   S;             /* m x i: the actions used (Ghat-unnormalised residuals
                               for CG, the given columns for GIVEN)                  */
    float*   W_obs;         /* m x i: S L^{-T}, i.e. V of the iterative update in
                               observation coordinates (W = H^T W_obs)              */
    float*   w_obs;         /* m: S (S^T Ghat S)^{-1} S^T r0 (w = H^T w_obs)         */
    double*  chol;          /* i x i: lower Cholesky factor L of S^T Ghat S          */
    double*  chol_inv;      /* i x i: L^{-1} (lower triangular)                      */
    double*  loglik;        /* 1: projected log-likelihood term of this step         */
    int*     n_actions;     /* 1: number of actions kept                             */
} cakf_record;

/* Create a context: copies and pre-scales X, allocates every workspace and the filter
 * state (mean = 0, rank = 0, i.e. the prior N(0, Sigma)).  No later call allocates. */
int cakf_create(const cakf_config* cfg, cakf_ctx** out);

/* Release a context and all its device memory (synchronises its stream). */
void cakf_destroy(cakf_ctx* ctx);

/* Reset the filter state to the prior (mean 0, empty factor). */
int cakf_reset(cakf_ctx* ctx);

/* Device views of the context-owned filter state: mean (N), factor (N x rank,
 * row-major with leading dimension *ld); N = n, or 2n with the Matérn-3/2 temporal
 * factor.  The pointers stay valid until the next
 * cakf_update / cakf_truncate / cakf_step / cakf_set_state / cakf_destroy.  Any output
 * pointer may be NULL.  The views are read-only: after a truncation the context relies on
 * the factor's leading max_rank columns being the orthogonal columns M V_r it wrote (their
 * Gram block is not recomputed), so a state is changed through cakf_set_state only. */
int cakf_state(cakf_ctx* ctx, float** mean, float** factor, int* ld, int* rank);

/* Copy the state out into caller-owned device buffers: mean (N) and factor (N x rank,
 * leading dimension ld >= rank).  Either pointer may be NULL. */
int cakf_copy_state(cakf_ctx* ctx, float* mean, float* factor, int ld);

/* Copy a state in (device buffers: mean N, factor N x rank with leading dimension ld).
 * rank <= max_rank + max_actions: a factor with more than max_rank columns is an
 * untruncated one, which cakf_truncate reduces (cakf_update needs rank <= max_rank and
 * returns CAKF_E_STATE otherwise). */
int cakf_set_state(cakf_ctx* ctx, const float* mean, const float* factor, int ld, int rank);

/* Predict (Alg. 1): m <- a m, M <- a M. */
int cakf_predict(cakf_ctx* ctx);

/* Update (Alg. 2 / the iterative update of App. B) with m observations y (device, m)
 * at the distinct state indices idx (device int32, m, each in [0, n)).
 * actions: device m x i row-major, required for POLICY_GIVEN, ignored for CG.
 * Afterwards the factor has rank + max_actions columns (the untruncated M_k; columns
 * of dropped actions are zero).  m == 0 means no data (the IsMissing branch). */
int cakf_update(cakf_ctx* ctx, const int32_t* idx, const float* y, int m,
                const float* actions, const cakf_record* rec);

/* Truncate (Sec. 3.2): replace M by M V_r, where V_r holds the leading
 * min(max_rank, rank) eigenvectors of M^T M (FP64 Gram and FP64 eigensolver), so that
 * M M^T keeps its best rank-r approximation.  rotation (device FP64, rank x r_new,
 * row-major, nullable) receives V_r.  A factor of at most max_rank columns is left
 * unchanged.  The kept columns are mutually orthogonal with the kept eigenvalues as squared
 * norms, and stay so through OU predictions (scaled by a^2) and updates (which append
 * columns): the next truncation takes that diagonal block of M^T M as known and computes
 * only the products that involve the appended columns. */
int cakf_truncate(cakf_ctx* ctx, double* rotation);

/* One filter step of Alg. 1: predict, update (skipped when m == 0), truncate. */
int cakf_step(cakf_ctx* ctx, const int32_t* idx, const float* y, int m,
              const float* actions, const cakf_record* rec);

/* Marginal variances diag(Sigma - M M^T) of the current state at the state indices
 * rows (device int32, count entries; NULL = all n) into out (device, count): the values
 * at the points (rows < n).  A row index outside [0, n) yields NaN. */
int cakf_marginal_var(cakf_ctx* ctx, const int32_t* rows, int count, float* out);

/* Log marginal likelihood of the data seen since the last reset, as the filter defines
 * it: the sum over updates of the projected prediction-error terms
 *   l_k = -1/2 [ i log 2 pi + log det(S^T Ghat S) - log det(S^T S)
 *                + (S^T r0)^T (S^T Ghat S)^{-1} (S^T r0) ]
 * (the paper leaves evidence maximisation to future work, Sec. 8; for full actions and
 * no truncation the sum is the exact Gaussian-process evidence).  value: host double;
 * steps (nullable): number of updates with data.  Synchronises the stream. */
int cakf_loglik(cakf_ctx* ctx, double* value, int* steps);

/* Device status words since the last reset: actions dropped on breakdown, non-finite
 * pivots, and observation indices outside [0, n) (each read as index 0).  Any output
 * pointer may be NULL.  Synchronises the stream. */
int cakf_diagnostics(cakf_ctx* ctx, int* dropped_actions, int* nonfinite, int* bad_index);

/* One backward step k of the computation-aware RTS smoother (Alg. 3).  Inputs come from
 * the filter run (caller-owned device buffers, read only):
 *   mean        m_k, filter mean after the update of step k (n);
 *   factor      M_k, the untruncated filter factor after the update of step k
 *               (n x rank, row-major, leading dimension ld);
 *   pred_factor M_k^- = a M_{k-1}^+, the predictive factor of step k (n x pred_rank);
 *   idx, w_obs, W_obs, m   the observation indices and the record of step k (w_obs: m,
 *               W_obs: m x max_actions); m = 0 for a step without data.
 * The smoother requires the m indices of a step to be distinct. */
typedef struct {
    const float* mean;
    const float* factor;
    int ld, rank;
    const float* pred_factor;
    int pred_ld, pred_rank;
    const int32_t* idx;
    const float* w_obs;
    const float* W_obs;
    int m;
} cakf_smooth_input;

/* Start the backward pass at the last step T (Alg. 3): ws_T = H_T^T w_obs,
 * Ws_T = H_T^T W_obs from the record of step T (m = 0: no data).  Needs
 * cfg.smoother != 0.  The smoothed moments of step T are the filter's. */
int cakf_smooth_begin(cakf_ctx* ctx, const int32_t* idx, const float* w_obs,
                      const float* W_obs, int m);

/* One backward step k = T-1, ..., 1 (Alg. 3):
 *   smoothed mean   m_k + P_k A^T ws_{k+1}                          -> mean_out (n)
 *   smoothed factor (M_k, P_k A^T Ws_{k+1})                         -> factor_out
 *                   (n x *out_rank, leading dimension ld_out)
 *   marginal variances sigma_f^2 - row sums of the factor squared   -> var_out (n)
 * then advances ws, Ws to step k (truncating Ws to max_rank columns, Sec. 3.2).  Any
 * output may be NULL.  P_k = Sigma - M_k M_k^T uses the untruncated filter factor. */
int cakf_smooth_step(cakf_ctx* ctx, const cakf_smooth_input* in, float* mean_out,
                     float* factor_out, int ld_out, float* var_out, int* out_rank);

/* The whole backward pass (Alg. 3) over T recorded steps: steps[k] holds step k+1's
 * filter output and record as for cakf_smooth_step (steps[T-1] may have pred_factor
 * NULL: it is not read).  Writes the smoothed means and marginal variances of every
 * step, row-major T x n (mean_out[k * n + p], var_out[k * n + p]; either may be NULL);
 * step T's are the filter's.  Equivalent to cakf_smooth_begin with step T's record
 * followed by cakf_smooth_step for k = T-1, ..., 1.  Needs cfg.smoother != 0. */
int cakf_smooth(cakf_ctx* ctx, int T, const cakf_smooth_input* steps, float* mean_out,
                float* var_out);

/* Temporal interpolation (App. C, the corollary on temporal interpolation): the
 * filter's or the smoother's moments at a time t with t_k <= t < t_{k+1}, from step k's
 * filter moments (in->mean = m_k, in->factor = M_k untruncated; the other fields are not
 * read) and, smoothed != 0, the smoother's current messages ws_{k+1}, Ws_{k+1}:
 *   filter    m(t)  = A(t, t_k) m_k,     M(t) = A(t, t_k) M_k,  P(t) = Sigma - M(t) M(t)^T
 *   smoother  ms(t) = m(t) + P(t) A(t_{k+1}, t) ws_{k+1},
 *             Ms(t) = [M(t) | P(t) A(t_{k+1}, t) Ws_{k+1}]
 * a_left = A(t, t_k), a_right = A(t_{k+1}, t), both in (0, 1]; for the OU prior
 * a_left = exp(-(t - t_k) / ell_t) and a_right = exp(-(t_{k+1} - t) / ell_t).  The
 * messages of step k+1 are current between cakf_smooth_step for step k+1 (or
 * cakf_smooth_begin when k + 1 = T) and cakf_smooth_step for step k; interpolation does
 * not advance them.  Before the first step pass m = 0 and rank 0 (the prior); after the
 * last step the smoothed moments are the filter's (smoothed = 0).  Outputs as in
 * cakf_smooth_step; *out_rank = rank (+ the messages' rank when smoothed). */
int cakf_interpolate(cakf_ctx* ctx, const cakf_smooth_input* in, double a_left,
                     double a_right, int smoothed, float* mean_out, float* factor_out,
                     int ld_out, float* var_out, int* out_rank);

/* ------------------------------------------------------------ path sampler (App. C)
 * Joint sample paths of the computation-aware filter and smoother (the CAKF/CAKS
 * sampler): draws from the prior are pushed through the gains of a recorded filter run,
 * in the manner of Matheron's rule.  ns <= cfg.sample_paths paths are the columns of
 * row-major device arrays with leading dimension ns: state arrays n x ns, observation
 * arrays m x ns.  The random draws are inputs, drawn by the caller:
 *   x0  ~ N(0, Sigma)              the first state's stationary prior (x_prev at k = 1),
 *   q_k ~ N(0, (1 - a^2) Sigma)    the process noise of the prediction of step k,
 *   e_k ~ N(0, I_m)                observation noise in units of sigma (the projected
 *                                  noise of the paper is eps_k = S_k^T sigma e_k).
 * Forward, k = 1..T:     x^-_k = a x_{k-1} + q_k,
 *                        w_k   = H_k^T W_obs L^{-1} S^T (y_k - x^-_k[idx] - sigma e_k),
 *                        x_k   = x^-_k + P^-_k w_k        (P^-_k = Sigma - M^-_k M^-_k^T).
 * Backward, k = T-1..1:  ws_T = w_T,  xs_T = x_T,
 *                        xs_k = x_k + P_k a ws_{k+1}      (P_k = Sigma - M_k M_k^T,
 *                                                          M_k untruncated),
 *                        ws_k = w_k + (I - W_k W_k^T P^-_k) a ws_{k+1},  W_k = H^T W_obs.
 * Without truncation, xs_1..xs_T are distributed as the posterior of the projected
 * model (conditioning on S_k^T y_k for every k).  Needs cfg.sample_paths >= ns; the m
 * indices of a step must be distinct.
 *
 * Step k's inputs (caller-owned device buffers from the filter run, read only): idx, y,
 * m (m = 0: a step without data); the record's S (m x max_actions), W_obs
 * (m x max_actions) and chol_inv (L^{-1}, max_actions x max_actions FP64); the
 * predictive factor M^-_k = a M^+_{k-1} (n x pred_rank, leading dimension pred_ld). */
typedef struct {
    const int32_t* idx;
    const float* y;
    int m;
    const float* S;
    const float* W_obs;
    const double* chol_inv;
    const float* pred_factor;
    int pred_ld, pred_rank;
} cakf_sample_input;

/* Forward step k: x_prev = x_{k-1} (x0 at k = 1), q = q_k (n x ns), e = e_k (m x ns;
 * may be NULL when m = 0) -> x_out = x_k (n x ns; may alias x_prev) and w_obs_out (m x ns),
 * the message in observation coordinates (w_k = H^T w_obs_out; not written when m = 0). */
int cakf_sample_forward(cakf_ctx* ctx, int ns, const float* x_prev, const float* q,
                        const float* e, const cakf_sample_input* in, float* x_out,
                        float* w_obs_out);

/* Forward step k as cakf_sample_forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * step's workspace is a file-scope device array of CAKF_STATIC_SCRATCH_BYTES (32 MiB) that
 * each GPU the library runs on holds until the process ends, instead of the context's
 * sampler workspace, so the context may be created with sample_paths = 0.  The call makes
 * no device allocation and no library call that allocates; buffers it must start from
 * zero are cleared by a kernel.  Same arguments, same kernels and the same results as
 * cakf_sample_forward; ns <= CAKF_STATIC_MAX_PATHS.  The layout needs
 * 4 bsp (3 mp + 2 imax + n) + 16 mp bytes, plus 4 bsp (n + pred_rank) when pred_rank > 0
 * (bsp = ns rounded up to 32, mp = m rounded up to 128, imax = max_actions, each segment
 * rounded up to 256 bytes); what is left holds the partial products of a block product
 * split along the observations.  A call that needs more returns CAKF_E_SCRATCH before
 * anything is enqueued.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (several streams or host threads) race
 * and must be serialised by the caller. */
#define CAKF_STATIC_SCRATCH_BYTES (32u << 20)
#define CAKF_STATIC_MAX_PATHS 256
int cakf_sample_forward_static(cakf_ctx* ctx, int ns, const float* x_prev, const float* q,
                               const float* e, const cakf_sample_input* in, float* x_out,
                               float* w_obs_out);

/* ws_out (n x ns) = H^T w_obs: the last step's message, ws_T = w_T (zeros when m = 0). */
int cakf_sample_lift(cakf_ctx* ctx, int ns, const int32_t* idx, const float* w_obs, int m,
                     float* ws_out);

/* Backward step k = T-1..1: x = x_k (n x ns) and factor = M_k (untruncated, n x rank,
 * leading dimension ld) from the forward pass and the filter; in = step k's inputs (y,
 * S and chol_inv are not read); w_obs = step k's forward message (m x ns);
 * ws_next = ws_{k+1} (n x ns) -> xs_out = xs_k and ws_out = ws_k (n x ns each; xs_out
 * may alias x, ws_out may alias ws_next). */
int cakf_sample_backward(cakf_ctx* ctx, int ns, const float* x, const float* factor, int ld,
                         int rank, const cakf_sample_input* in, const float* w_obs,
                         const float* ws_next, float* xs_out, float* ws_out);

/* One filter step as the derivative of the log-likelihood needs it: the step's inputs,
 * its record and the state it passed on, all caller-owned device buffers written by the
 * forward run (read only here).
 *   idx, y, m     the observations of step k (m = 0: no data);
 *   S, W_obs, w_obs, chol, chol_inv, n_actions   the step's cakf_record;
 *   mean          m_k, the filter mean after step k (n);
 *   factor        M_k^+, the factor after the truncation of step k (n x rank, row-major,
 *                 leading dimension ld), i.e. the state the next step predicts from;
 *   rotation      the V_r of the step's cakf_truncate (rank_full x rank, row-major FP64),
 *                 or NULL when the step did not truncate (then rank = rank_full). */
typedef struct {
    const int32_t* idx;
    const float* y;
    int m;
    const float* S;
    const float* W_obs;
    const float* w_obs;
    const double* chol;
    const double* chol_inv;
    const int* n_actions;
    const float* mean;
    const float* factor;
    int ld, rank;
    const double* rotation;
    int rank_full;
} cakf_tape_step;

/* Derivative of the log-likelihood of cakf_loglik over the T steps of tape (a run from
 * the prior with this context's parameters) with respect to
 *   grad[0] the spatial lengthscale,
 *   grad[1] the temporal lengthscale ell_t = -dt / log(a) when dt > 0 (the time step the
 *           OU coefficient a = exp(-dt / ell_t) was formed with), or the OU coefficient a
 *           itself when dt == 0,
 *   grad[2] the signal variance,      grad[3] the noise variance,
 * holding the actions and the truncation rotations fixed at their recorded values (the
 * derivative of the filter as it was run; the paper leaves evidence maximisation to future
 * work, Sec. 8).  Reverse sweep over the steps of Alg. 1 and Alg. 2: kernel tiles are
 * recomputed, nothing of size n x m is stored.  Needs cfg.gradient != 0, the context's
 * max_actions <= 256 and distinct indices within each step; dt < 0 is CAKF_E_ARG.
 * grad: host, 4 doubles.  Synchronises the stream. */
int cakf_loglik_grad(cakf_ctx* ctx, int T, const cakf_tape_step* tape, double dt,
                     double* grad);

/* Phases timed by the profiling hooks (HIP events on the context stream around each
 * launch of the phase). */
#define CAKF_PHASE_SYM_TILES     0   /* one action of the loop: kernel-matrix x action   */
                                     /* matvec, its reduction and the FP64 Cholesky step */
#define CAKF_PHASE_FORM_U        1   /* (no separate launch: part of SYM_TILES)          */
#define CAKF_PHASE_TAIL          2   /* FP64 Cholesky steps of a block-policy round      */
#define CAKF_PHASE_NEXT_ACTION   3   /* CG residual = next action                        */
#define CAKF_PHASE_BLOCK_PRODUCT 4   /* kernel-matrix x [W w] block product               */
#define CAKF_PHASE_GRAM          5   /* FP64 Gram matrix of the factor                   */
#define CAKF_PHASE_EIG           6   /* FP64 symmetric eigensolver                       */
#define CAKF_PHASE_ROTATE        7   /* factor rotation M V_r                            */
#define CAKF_PHASE_PREDICT       8   /* cakf_step: predict                               */
#define CAKF_PHASE_UPDATE        9   /* cakf_step: update                                */
#define CAKF_PHASE_TRUNCATE     10   /* cakf_step: truncate                              */
#define CAKF_PHASES             11

/* Per-phase timing: phases is a bit mask (bit p times phase p; -1 = all phases, 0 =
 * off).  Enabling resets the counters and creates HIP events once (host-side objects,
 * no device memory); at most 2048 launches per phase are timed between reads.  The
 * SYM_TILES phase (one kernel per action) takes the launch's own start and stop
 * timestamps; every other timed phase is bracketed by two events on the stream, which
 * adds a few microseconds per launch: time only the phases needed. */
#define CAKF_PROFILE_ALL (-1)
int cakf_profile_enable(cakf_ctx* ctx, int phases);

/* Time only every `every`-th launch of each timed phase (every >= 1; 1, the default,
 * times every launch).  A sample of the launches keeps the event overhead out of most of
 * a timed run; the counters and the launch count of cakf_profile_read cover the sampled
 * launches only.  Takes effect from the next launch; CAKF_E_ARG for every < 1. */
int cakf_profile_stride(cakf_ctx* ctx, int every);

/* Total milliseconds and number of timed launches per phase since the last enable or
 * read (arrays of CAKF_PHASES entries), then reset the counters.  Synchronises the
 * stream. */
int cakf_profile_read(cakf_ctx* ctx, double* total_ms, int* launches);

/* Issue rates of the current device for the VALU instructions the kernel-matrix products
 * are built from, the peaks their roofline figures are quoted against: lanes_per_s[0..2]
 * = lane operations per second of v_exp_f32, v_sqrt_f32 and v_fma_f32, each measured by
 * a kernel of dependent chains (eight independent chains per lane, every SIMD full; best
 * of three timed launches on the null stream).  A measurement utility, not part of the
 * filter: it allocates and frees a small buffer and synchronises the device.  No context
 * is needed. */
int cakf_profile_rates(double* lanes_per_s);

#ifdef __cplusplus
}
#endif
#endif /* CAKF_H */
