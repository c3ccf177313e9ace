/*
 * smc2.h -- C ABI of the MI355X (gfx950) library for the hot path of Enhanced SMC^2
 * (Rosato, Murphy, Varsi, Horridge & Maskell, 2024: "Enhanced SMC^2: Leveraging Gradient
 * Information from Differentiable Particle Filters Within Langevin Proposals").
 *
 * The hot path, per SMC^2 iteration k and for every parameter sample theta^i of every series s:
 *   1. smc2_langevin_move      -- the first-order (Langevin) proposal SMC1 (Sec. III-D);
 *   2. smc2_pf_loglik_grad     -- the common-random-numbers particle filter (Sec. II) returning
 *                                 the log-likelihood estimate and its gradient (App. A, App. B);
 *   3. smc2_reweight_resample  -- L-kernel reweighting (eq. l_weights, Sec. III-E),
 *                                 normalisation (eq. normalise_smc2), ESS (eq. ess_smc2) and
 *                                 resampling of the samples (Sec. III-B).
 *
 * Conventions for every call:
 *   - Pointers marked "dev" are device (HBM) pointers on the context's GPU; "host" are host
 *     pointers.  The caller owns every buffer passed in; the context owns its scratch
 *     (ancestor indices, checkpoints, segment buffers, work queue, status word), all allocated
 *     by smc2_ctx_reserve and nowhere else.
 *   - Calls enqueue work on `stream` (a hipStream_t passed as void*) and return without
 *     synchronising, so a sequence of them can be captured in a HIP graph.  Iteration numbers
 *     are read from device memory for that reason.
 *   - Host-side argument errors return a status and never abort; the message is available from
 *     smc2_last_error().  Non-finite values are data, not errors: a theta whose filter ends with
 *     every weight zero gets loglik = -inf and gradient 0, and its outer weight becomes zero.
 *   - Arrays are row-major with the last index contiguous.  S = number of independent series,
 *     N = parameter samples per series, M = particles per filter, D = dim theta, d = dim x.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed, counter
 *     (slot, block, s*N + i, (k << 8) | stream), Box-Muller normals and uniforms in (0, 1].
 *     The numbers of a filter depend only on (seed, k, s, i) and the particle slot, which is the
 *     paper's common-random-numbers device (Sec. II-A) with a different seed per sample and
 *     iteration (Sec. I).
 */
#ifndef SMC2_H
#define SMC2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smc2_ctx smc2_ctx; /* opaque; owns all scratch on one device */

typedef enum {
  SMC2_OK = 0,
  SMC2_E_INVALID_ARG = 1,   /* a size, pointer or option is out of its documented range */
  SMC2_E_UNSUPPORTED = 2,   /* valid, but beyond what the built kernels handle (e.g. M too large) */
  SMC2_E_OUT_OF_MEMORY = 3, /* reservation exceeds the scratch budget or device memory */
  SMC2_E_DEVICE = 4,        /* a HIP runtime call failed */
  SMC2_E_NONFINITE = 5      /* device status: every outer weight of some series was zero */
} smc2_status;

/* State-space models (paper eqs. xt and yt).  Parameters are unconstrained:
 *   SMC2_MODEL_LG1D    d=1,  D=3:  theta = (a, log sx, log sy);
 *                      x_t = a x_{t-1} + sx v, y_t = x_t + sy w, x_0 ~ N(0, 1)
 *   SMC2_MODEL_LG_DIAG d=16, D=18: theta = (A_11..A_dd, log sx, log sy);
 *                      x_t = A x_{t-1} + sx v with A diagonal, y_t = x_t + sy w, x_0 ~ N(0, I)
 *                      (the kernels are built for d = 16 only)
 *   SMC2_MODEL_GROWTH  d=1,  D=2:  theta = (log sx, log sy);
 *                      x_t = x/2 + 25 x/(1+x^2) + 8 cos(1.2 t) + sx v, y_t = x_t^2/20 + sy w,
 *                      x_0 ~ N(0, 1)
 *   SMC2_MODEL_SV      d=1,  D=3:  theta = (mu, atanh phi, log s);
 *                      x_t = mu + phi (x_{t-1} - mu) + s v, y_t = exp(x_t/2) w,
 *                      x_0 ~ N(mu, s^2/(1-phi^2))
 *   SMC2_MODEL_LG1D_OPT d=1, D=3:  the LG1D model filtered with the "optimal" proposal of
 *                      Sec. IV-A instead of the bootstrap one: x_t ~ N(rho^2 (y_t/sy^2 +
 *                      a x_{t-1}/sx^2), rho^2) with 1/rho^2 = 1/sx^2 + 1/sy^2, weighted by the
 *                      predictive density N(y_t; a x_{t-1}, sx^2 + sy^2)
 *   SMC2_MODEL_SIR     d_x=2, d_y=1, D=2: theta = (beta, gamma) on their natural scale; the
 *                      discrete-time SIR model of Sec. IV-B with state (S, I):
 *                      S_t = S - beta I S / N_pop + s_e v_1,
 *                      I_t = I + beta I S / N_pop - gamma I - s_e v_1 + s_e v_2,
 *                      y_t = I_t + s_y w, x_0 = (N_pop - I_0, I_0); the constants
 *                      (N_pop, I_0, s_e^2, s_y) default to (763, 1, 0.5, 5).  The paper prints
 *                      the infection term without the division by N_pop and states no
 *                      observation model; these are readings, as is s_e^2 = 0.5 for N(0, 0.5).
 * with v, w ~ N(0, 1).  The prior p(theta) is independent over the parameters: N(prior_mu[p],
 * prior_sd[p]^2), or, where prior_kind[p] = SMC2_PRIOR_UNIFORM, uniform on the closed interval
 * [prior_mu[p], prior_sd[p]] (the SIR model's priors are U(0, 1), Sec. IV-B).  A sample outside
 * a uniform prior's support has posterior zero: its outer weight is zero. */
typedef enum {
  SMC2_MODEL_LG1D = 0,
  SMC2_MODEL_LG_DIAG = 1,
  SMC2_MODEL_GROWTH = 2,
  SMC2_MODEL_SV = 3,
  SMC2_MODEL_LG1D_OPT = 4,
  SMC2_MODEL_SIR = 5
} smc2_model_kind;

typedef enum { SMC2_PRIOR_NORMAL = 0, SMC2_PRIOR_UNIFORM = 1 } smc2_prior_kind;

typedef struct {
  int32_t kind;             /* smc2_model_kind */
  int32_t d_x, d_y, D;      /* state dim, observation dim (d_x, or 1 for SIR), parameter dim */
  const double *prior_mu;   /* host [D]: mean (normal) or lower bound (uniform), finite */
  const double *prior_sd;   /* host [D]: sd > 0 (normal) or upper bound > lower (uniform) */
  const int32_t *prior_kind; /* host [D] smc2_prior_kind, or NULL: every parameter normal */
  const double *constants;  /* host, the model's constants (SIR: 4 values), or NULL for the
                               defaults; ignored by the models that have none.  The values are
                               copied at each call that takes the model. */
} smc2_model;

typedef enum { SMC2_FP64 = 0, SMC2_MIXED = 1 } smc2_precision;
typedef enum { SMC2_SYSTEMATIC = 0, SMC2_MULTINOMIAL = 1 } smc2_resampler;

typedef struct {
  int32_t precision;     /* SMC2_FP64: every operation in FP64.  SMC2_MIXED: propagation,
                            weighting and the ESS test's sum of squared weights in FP32; running
                            log-likelihood, logsumexp, the weight prefix sum that selects
                            ancestors and the gradient sums in FP64 */
  int32_t resampler;     /* SMC2_SYSTEMATIC or SMC2_MULTINOMIAL (App. B) */
  double ess_frac;       /* resample after step t < T iff ESS < ess_frac * M (Sec. II-B: 0.5) */
  int32_t ckpt_interval; /* adjoint checkpoint interval c in steps; 0 = ceil(sqrt(T_max)) */
  int32_t want_grad;     /* 0: log-likelihood only; 1: also the gradient */
  int32_t tile;          /* launch shape: 0 = tuned default, else an index from smc2_tile_info */
  int32_t persistent;    /* 1: persistent grid pulling (s, i) items longest-series-first from an
                            on-device queue; 0: one workgroup per item in the same order */
  int32_t store_noise;   /* 1: the forward sweep stores its reparameterised noise (drawn in
                            advance, eq. reparam_epsilon) and the adjoint reads it back, at
                            (T_max + 1) * d_x * MP values per item of extra scratch; 0: the
                            adjoint regenerates it from the counter-based stream */
} smc2_pf_opts;

/* ---- context ------------------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  *out is NULL on failure. */
smc2_status smc2_ctx_create(smc2_ctx **out, int device);

/* Reserve every device buffer the three calls need for up to S series, N samples, M particles,
 * T_max steps and the given options (precision, resampler and checkpoint interval fix the
 * layout).  Must precede graph capture; calls made with larger sizes than reserved fail with
 * SMC2_E_INVALID_ARG.  scratch_budget_bytes = 0 means no limit beyond device memory; a larger
 * need returns SMC2_E_OUT_OF_MEMORY and allocates nothing.  T_len (host [S]) gives each series'
 * length, used to order work longest first.  SMC2_E_UNSUPPORTED when M is above the largest
 * built tile, when the requested tile is not built for the model and precision, when the series
 * do not fit the kernel's LDS staging, or when one filter's
 * checkpoints or stored noise would take 4 GiB or more (they are addressed with 32-bit
 * offsets). */
smc2_status smc2_ctx_reserve(smc2_ctx *ctx, const smc2_model *model, const smc2_pf_opts *opts,
                             int32_t S, int32_t N, int32_t M, const int32_t *T_len,
                             int32_t T_max, size_t scratch_budget_bytes);

/* Bytes that smc2_ctx_reserve would allocate for these arguments (no allocation). */
smc2_status smc2_ctx_scratch_bytes(const smc2_model *model, const smc2_pf_opts *opts, int32_t S,
                                   int32_t N, int32_t M, int32_t T_max, size_t *bytes);

void smc2_ctx_destroy(smc2_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *smc2_last_error(void);

/* Synchronise `stream`, read and clear the device status word: SMC2_OK, or SMC2_E_NONFINITE if
 * some series had every outer weight zero since the last read. */
smc2_status smc2_ctx_device_status(smc2_ctx *ctx, void *stream);

/* ---- the hot path --------------------------------------------------------------------------- */

/* CRN particle filter with gradient, for every (series s, sample i).
 *
 * Defines: the bootstrap filter of Sec. II (proposal = transition, eq. prior_proposal; weight
 * update eq. priorproposalweight; normalised weights eq. normalisedweights; ESS eq. ess with
 * resampling below ess_frac*M), the likelihood estimate of eq. likelihood_pf_, accumulated as
 * the sum over t of s_t = log sum_j exp(lW_{t-1}^j + log g(y_t | x_t^j)), and its gradient
 * (App. A eqs. dloglik, weightupdate, deriv_loglike, dxk with the reparameterised noise of eq.
 * reparam_epsilon; App. B: resampled weights equal and sum-preserving, eq. weightresample, and
 * particle gradients inherited from the parent).  The gradient is computed in reverse mode: a
 * forward sweep that stores int32 ancestors at resampling steps and (x, log W) checkpoints
 * every ckpt_interval steps, then a backward sweep that recomputes each segment from its
 * checkpoint with the stored ancestors (and the stored noise with store_noise = 1); with
 * ckpt_interval = 1 nothing is recomputed: each step is rebuilt from the state before it.
 *
 *   T_len    host [S]: length of series s (0 <= T_len[s] <= T_max); y rows past it are ignored.
 *   theta    dev  [S][N][D] FP64.
 *   y        dev  [S][T_max][d_y] FP64.
 *   iteration dev scalar uint32: k, part of the random-number key (so a captured graph can
 *            advance it on the device).
 *   loglik   dev  [S][N] FP64 out.
 *   grad     dev  [S][N][D] FP64 out (NULL iff opts->want_grad == 0).
 * Errors: SMC2_E_INVALID_ARG for NULL pointers, sizes < 1 (T_len >= 0), sizes beyond the
 * reservation or T_len[s] > T_max; SMC2_E_UNSUPPORTED for M above the largest built tile
 * (4096 for d_x = 1, 2048 for d_x = 2 and 16) or an unknown model/precision. */
smc2_status smc2_pf_loglik_grad(smc2_ctx *ctx, const smc2_model *model, const smc2_pf_opts *opts,
                                int32_t S, int32_t N, int32_t M, const int32_t *T_len,
                                int32_t T_max, const double *theta, const double *y,
                                uint64_t seed, const uint32_t *iteration, double *loglik,
                                double *grad, void *stream);

/* Langevin move (proposal SMC1 of Sec. III-D, in the velocity form of the one-step dynamics of
 * Sec. III-E): p_{k-1} = gamma * xi with xi ~ N(0, I) from the MOVE stream of iteration k, and
 * theta_new = theta + (gamma^2 / 2) * grad_logpost + p_{k-1}.
 *   theta, grad_logpost dev [S][N][D] FP64 in;  theta_new, p_prev dev [S][N][D] FP64 out.
 *   gamma > 0.  random_walk = 1 drops the gradient term (the SMC0 proposal N(theta, gamma^2 I)).
 * The context must be reserved (it names the device).
 * Errors: SMC2_E_INVALID_ARG for an unreserved context, NULL pointers, sizes < 1, gamma <= 0. */
smc2_status smc2_langevin_move(smc2_ctx *ctx, const smc2_model *model, int32_t S, int32_t N,
                               double gamma, int32_t random_walk, const double *theta,
                               const double *grad_logpost, uint64_t seed,
                               const uint32_t *iteration, double *theta_new, double *p_prev,
                               void *stream);

/* The sample population of one SMC^2 iteration (all dev, FP64). */
typedef struct {
  double *theta;        /* [S][N][D] */
  double *logpost;      /* [S][N]    log pi = log p(theta) + loglik (eq. log_posterior) */
  double *grad_logpost; /* [S][N][D] grad log pi (eq. first_gradientlogposterior) */
  double *loglik;       /* [S][N]    loglik estimate */
  double *logw;         /* [S][N]    unnormalised log weight */
} smc2_population;

/* Reweight, normalise, ESS and resample, one workgroup per series.
 *   On entry cur->theta holds theta_k, cur->loglik the filter's estimate and cur->grad_logpost
 *   the filter's gradient of the log-likelihood.  The call first adds the prior:
 *   logpost = log p(theta) + loglik, grad_logpost += grad log p(theta) (logpost = -inf, so a
 *   weight of zero, outside a uniform prior's support).  Then the weight:
 *     first_iteration = 1: log w = loglik (eq. init_weights with q_1 = prior);
 *     otherwise          : log w = prev->logw + logpost - prev->logpost
 *                          + log N(-p_k; 0, G) - log N(p_{k-1}; 0, G),
 *                          p_k = p_{k-1} + (gamma^2/2)(prev->grad_logpost + grad_logpost)
 *                          (eq. l_weights with the L-kernel of eq. l=q; random_walk = 1 uses
 *                          the symmetric random-walk kernel, ratio 1).
 *   Then ESS = 1 / sum W^2 of the normalised weights (eqs. normalise_smc2, ess_smc2) and, if
 *   ESS < N/2, systematic resampling from the OUTER stream of iteration k: cur's theta,
 *   logpost, grad_logpost and loglik are permuted in place, log w = logsumexp - log N.
 *   Before returning, the device iteration counter is incremented by one when
 *   advance_iteration = 1 (so that one captured graph replays iteration after iteration).
 *   prev   : population of iteration k-1 after its resampling (ignored if first_iteration).
 *   p_prev : dev [S][N][D] from smc2_langevin_move (ignored if first_iteration).
 *   ancestors dev [S][N] int32 out (identity where not resampled), ess dev [S] FP64 out,
 *   resampled dev [S] int32 out; each may be NULL.
 *   estimate dev [S][2][D] FP64 out (may be NULL): the realised estimates of E[theta] and
 *   E[theta^2] (elementwise) under the normalised weights, before resampling (eq.
 *   realised_estimates with eq. normalise_smc2); NaN for a series whose weights are all zero.
 *   recycle dev [S][1 + 4D] FP64 in/out (may be NULL): per series, [0] the running sum over
 *   iterations of l_k = ESS_k (eq. recycling_I), [1, 2D] the running sums of l_k E[theta] and
 *   l_k E[theta^2], and [2D + 1, 4D] the recycled estimates of E[theta] and E[theta^2]
 *   (Sec. III-C: sum_k c_k E_k with the constants c_k = l_k / sum_j l_j of eq.
 *   opt_recycling_constant), rewritten by every call; NaN while every l_k so far is zero.
 *   Iterations whose weights are all zero add nothing.  The caller zeroes it before the first
 *   iteration.
 * A series whose weights are all zero keeps its population and sets the device status word
 * to SMC2_E_NONFINITE (see smc2_ctx_device_status).
 * Errors: SMC2_E_INVALID_ARG for an unreserved context, NULL pointers, N > 4096, sizes < 1,
 * S * N above the reservation, gamma <= 0, or a model whose kind, d_x or D differs from the
 * reservation's (the context's gather scratch is laid out for the reserved D). */
smc2_status smc2_reweight_resample(smc2_ctx *ctx, const smc2_model *model, int32_t S, int32_t N,
                                   double gamma, int32_t random_walk, smc2_population *cur,
                                   const smc2_population *prev, const double *p_prev,
                                   int32_t first_iteration, uint64_t seed,
                                   uint32_t *iteration, int32_t advance_iteration,
                                   int32_t *ancestors, double *ess, int32_t *resampled,
                                   double *estimate, double *recycle, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): smc2_reweight_resample without a context.  It takes
 * the same arguments with the same meaning, layout and ownership, except that the device is the
 * calling thread's current HIP device and the status word is the caller's: status dev int32
 * out (may be NULL), set to SMC2_E_NONFINITE when some series has every weight zero (the caller
 * zeroes it; nothing resets it).  The gather scratch is a fixed array of 2^20 doubles (8 MiB)
 * in the library's device image, which every GPU the library runs on holds until the process
 * ends; the call allocates nothing.  Every call on a GPU shares that GPU's array, so calls that
 * overlap on one GPU (concurrent streams, or threads) race and must be ordered by the caller.
 * The array's contents need no clearing between calls.
 * Errors: those of smc2_reweight_resample without the reservation checks, and
 * SMC2_E_INVALID_ARG when S * N * (2D + 2) exceeds 2^20. */
smc2_status smc2_reweight_resample_noalloc(const smc2_model *model, int32_t S, int32_t N,
                                           double gamma, int32_t random_walk,
                                           smc2_population *cur, const smc2_population *prev,
                                           const double *p_prev, int32_t first_iteration,
                                           uint64_t seed, uint32_t *iteration,
                                           int32_t advance_iteration, int32_t *ancestors,
                                           double *ess, int32_t *resampled, double *estimate,
                                           double *recycle, int32_t *status, void *stream);

/* ---- initialisation and inspection ------------------------------------------------------- */

/* theta_1 ~ prior (eq. init_sample with q_1 = prior): theta[s][i][p] = prior_mu[p] +
 * prior_sd[p] * z with z normal number p of the PRIOR stream of sample s*N+i (iteration 1), or,
 * for a uniform parameter, prior_mu[p] + (prior_sd[p] - prior_mu[p]) * u with u uniform number p
 * of the same stream.  theta dev [S][N][D] out.  The context must be reserved (it names the
 * device).  Errors: SMC2_E_INVALID_ARG for an unreserved context, sizes < 1 or a NULL theta. */
smc2_status smc2_prior_init(smc2_ctx *ctx, const smc2_model *model, int32_t S, int32_t N,
                            uint64_t seed, double *theta, void *stream);

/* Copy the trace of item (s, i) from the last smc2_pf_loglik_grad call made with
 * persistent = 0: flags host [T_len[s]] (1 where the filter resampled after step t), ancestors
 * host [T_len[s]][M] (-1 rows where it did not) and, if steps_s is not NULL, steps_s host
 * [T_len[s]] FP64: the per-step log normalisers s_t = log sum_j W_{t-1}^j g(y_t | x_t^j) with
 * the normalised weights W_{t-1} (eq. likelihood_pf_ taken step by step; their sum over t is
 * the returned log-likelihood).  For a filter whose weights all became zero (loglik = -inf) no
 * entry is written.  Synchronises `stream`.
 * Errors: SMC2_E_INVALID_ARG for an unreserved or persistent context, an item out of range or
 * NULL flags / ancestors. */
smc2_status smc2_pf_trace(smc2_ctx *ctx, int32_t s, int32_t i, uint8_t *flags,
                          int32_t *ancestors, double *steps_s, void *stream);

/* Counter-contract probe: out[r][0..3] = Philox4x32-10 words for counter ctr[r][0..3] under
 * `seed`; normals[r] = normal number n[r] and uniforms[r] = uniform number n[r] of stream
 * (c0 = ctr[r][0], c2 = ctr[r][2], c3 = ctr[r][3]) in FP64, normals32/uniforms32 in FP32.
 * All dev: ctr, n [R] in; out [R][4], normals, uniforms [R] FP64, normals32, uniforms32 [R] FP32
 * out (any output may be NULL). */
smc2_status smc2_philox_probe(int32_t R, const uint32_t *ctr, const uint32_t *n, uint64_t seed,
                              uint32_t *out, double *normals, double *uniforms, float *normals32,
                              float *uniforms32, void *stream);

/* Launch shapes built into the library: for tile index t >= 1, the particles per workgroup,
 * waves per workgroup and particles per lane of a shape built for state dimension d_x in at least
 * one precision; returns SMC2_E_INVALID_ARG past the last or for a shape not built for d_x.  A
 * precision can lack a shape (the 16-dimensional FP64 form has no sixteen waves x two particles
 * per lane), which smc2_ctx_reserve refuses with SMC2_E_UNSUPPORTED. */
smc2_status smc2_tile_info(int32_t tile, int32_t d_x, int32_t *max_particles, int32_t *waves,
                           int32_t *per_lane);

/* Library version string.  0.2: smc2_model carries prior_kind and constants (the SIR model).
 * 0.3: the recycle row of smc2_reweight_resample also holds the recycled estimate, and
 * smc2_pf_trace returns the per-step log normalisers. */
const char *smc2_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SMC2_H */
