/*
 * oracle.h -- C ABI of the serial FP64 CPU oracle for Enhanced SMC^2 (Rosato, Murphy, Varsi,
 * Horridge & Maskell, 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its Python
 * binding) may include, link, load or call this file or liboracle.so.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark use it.  It shares no code, header,
 * constant table or helper with the GPU path: the counter-based generator, the models, the
 * filter and the outer step are written here a second time, from their published definitions.
 *
 * Conventions (both sides implement them independently, see the counter contract in the design
 * notes):
 *   - Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), key = (lo32(seed), hi32(seed)),
 *     counter = (c0, c1, c2 = filter id or series, c3 = (k << 8) | stream).
 *   - Filter noise: element g = j*d + q of step t (t = 0: the initial draw) is normal g % 4 of
 *     block (c0 = g / 4, c1 = t); resampling uniforms of step t: word i % 4 of block
 *     (i / 4, t) per offspring (multinomial), word 0 of block (0xFFFFFFFF, t) (systematic).
 *   - Per-sample streams (prior, move, outer resampling): c0 = 0xFFFFFFFF, normal n in block
 *     n / 4 (c1), uniform m in block m / 4.
 *   - Box-Muller (Box & Muller 1958) on word pairs; uniforms (w + 1) * 2^-32 in (0, 1].
 *   - Arrays are row-major; y is [T][d_y] (d_y = d, or 1 for ORC_SIR); theta is [D];
 *     ancestors are [T][M] int32.
 *   - Prior draws: normal n = p of the prior stream of sample i (normal parameters), uniform
 *     m = p of the same stream (uniform parameters).
 */
#ifndef SMC2_ORACLE_H
#define SMC2_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* model kinds (same numbering as the library's smc2_model_kind, written out again here) */
enum { ORC_LG1D = 0, ORC_LG_DIAG = 1, ORC_GROWTH = 2, ORC_SV = 3, ORC_LG1D_OPT = 4, ORC_SIR = 5 };
/* prior kinds per parameter: N(prior_mu, prior_sd^2), or uniform on (prior_mu, prior_sd) */
enum { ORC_PRIOR_KIND_NORMAL = 0, ORC_PRIOR_KIND_UNIFORM = 1 };
/* random streams of the counter contract */
enum { ORC_INIT_NORMAL = 1, ORC_STEP_NORMAL = 2, ORC_RESAMPLE_UNIFORM = 3, ORC_PRIOR_NORMAL = 4,
       ORC_MOVE_NORMAL = 5, ORC_OUTER_RESAMPLE_UNIFORM = 6 };
enum { ORC_SYSTEMATIC = 0, ORC_MULTINOMIAL = 1 };

/* ORC_SIR: the discrete-time SIR model of Sec. IV-B, state x = (S, I) (R = N_pop - S - I),
 * theta = (beta, gamma) on their natural scale:
 *   S_t = S - beta I S / N_pop + s_e e_b,
 *   I_t = I + beta I S / N_pop - gamma I - s_e e_b + s_e e_g,
 *   y_t = I_t + s_y w  (one observation per step),   x_0 = (N_pop - I_0, I_0),
 * with the model constants (N_pop, I_0, s_e^2, s_y), default (763, 1, 0.5, 5) (C28-C30). */
typedef struct {
  int32_t kind;      /* ORC_* model kind */
  int32_t d;         /* state dimension (1, 2 for ORC_SIR, or 16 for ORC_LG_DIAG) */
  int32_t D;         /* parameter dimension */
  const double *prior_mu, *prior_sd; /* [D] independent priors: mean and sd (normal) or the
                                        lower and upper bound (uniform) */
  const int32_t *prior_kind;         /* [D] ORC_PRIOR_KIND_* or NULL: every parameter normal */
  const double *constants;           /* model constants (ORC_SIR: 4 values) or NULL: defaults */
} orc_model;

typedef struct {
  int32_t resampler; /* ORC_SYSTEMATIC / ORC_MULTINOMIAL */
  double ess_frac;   /* resample iff ESS < ess_frac * M and t < T */
} orc_pf_opts;

/* Philox4x32-10 block function: out = bijection(ctr) under key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* n-th standard normal of the stream (seed, c0, c2, c3) and m-th uniform in (0, 1]. */
double orc_normal(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t n);
double orc_uniform(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t m);
/* bulk helpers for statistics tests: out[i] = normal/uniform index (first + i) */
void orc_normals(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t first,
                 int64_t count, double *out);
void orc_uniforms(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t first,
                  int64_t count, double *out);

/* The filter's noise and resampling uniforms under the contract above. */
double orc_filter_normal(uint64_t seed, uint32_t fid, uint32_t c3, uint32_t t, uint32_t g);
double orc_filter_uniform(uint64_t seed, uint32_t fid, uint32_t c3, uint32_t t, uint32_t c0,
                          uint32_t word);

/* Resampling rule (paper App. B): given unnormalised weights w[M] and positions u[M] in (0, 1],
 * a[i] = first m with P_m >= u[i] * P_{M-1}, P the inclusive prefix sum of w. */
void orc_resample_lower_bound(int32_t M, const double *w, const double *u, int32_t *a);

/* CRN particle filter with forward-mode tangent (paper Sec. II, App. A, App. B).
 * Returns 0 on success, nonzero on bad arguments.
 *   loglik: log-likelihood estimate; grad[D]: its gradient (may be NULL).
 *   ancestors[T][M] (may be NULL): written at resampling steps, -1 elsewhere.
 *   flags[T] (may be NULL): 1 where the filter resampled after weighting step t.
 *   steps_s[T] (may be NULL): the per-step log normaliser s_t.
 * filter_id = s * N + i; k = SMC^2 iteration (PF stream key). */
int orc_pf(const orc_model *mdl, const orc_pf_opts *opt, const double *theta, int32_t T,
           const double *y, int32_t M, uint64_t seed, uint32_t k, uint32_t filter_id,
           double *loglik, double *grad, int32_t *ancestors, uint8_t *flags, double *steps_s);

/* Complex-step derivative of the same filter along direction e_p (Squire & Trapp 1998):
 * runs the filter on theta + i*h*e_p with every decision on real parts; returns Im(l)/h in
 * *dl and Re(l) in *loglik, and the ancestors taken (may be NULL). */
int orc_pf_complex_step(const orc_model *mdl, const orc_pf_opts *opt, const double *theta,
                        int32_t T, const double *y, int32_t M, uint64_t seed, uint32_t k,
                        uint32_t filter_id, int32_t p, double h, double *loglik, double *dl,
                        int32_t *ancestors);

/* Exact log-likelihood of the linear-Gaussian models by the Kalman filter, and its gradient by
 * complex step (ORC_LG1D, ORC_LG_DIAG, ORC_LG1D_OPT). */
int orc_kalman(const orc_model *mdl, const double *theta, int32_t T, const double *y,
               double *loglik, double *grad);

/* Outer-step pieces (paper Sec. III). */
double orc_log_prior(const orc_model *mdl, const double *theta, double *grad /* [D] or NULL */);
/* Langevin move with velocity p_{k-1} = gamma * xi: theta_new = theta + (gamma^2/2) g + p. */
void orc_langevin_move(int32_t D, double gamma, const double *theta, const double *grad_logpost,
                       const double *xi, double *theta_new, double *p_prev);
/* Random-walk move (SMC0) with the same velocity: theta_new = theta + gamma xi, p = gamma xi. */
void orc_random_walk_move(int32_t D, double gamma, const double *theta, const double *xi,
                          double *theta_new, double *p_prev);
/* Incremental log L-kernel/proposal ratio of the Langevin proposal,
 * log N(-p_k; 0, G) - log N(p_{k-1}; 0, G), with p_k = p_{k-1} + F(theta_{k-1}) + F(theta_k). */
double orc_lkernel_log_ratio(int32_t D, double gamma, const double *grad_prev,
                             const double *grad_new, const double *p_prev);

/* Realised estimates of E[theta] and E[theta^2] (elementwise) under the normalised weights of
 * the sample population (eqs. realised_estimates, normalise_smc2); returns the recycling weight
 * l_k = (sum w)^2 / sum w^2 (eq. recycling_I).  logw [N], theta [N][D], mean/second [D] out. */
double orc_realised_estimate(int32_t N, int32_t D, const double *logw, const double *theta,
                             double *mean, double *second);
/* Recycled estimate sum_k c_k est_k with c_k = l_k / sum l (eq. opt_recycling_constant);
 * l [K], est [K][D], out [D]. */
void orc_recycle(int32_t K, int32_t D, const double *l, const double *est, double *out);

/* A full SMC^2 run on one series (paper Sec. III with the CRN-PF of Sec. II).
 * Records, for k = 1..K (index k-1): proposed theta [K][N][D], loglik [K][N],
 * grad_loglik [K][N][D], log weights before resampling [K][N], ESS [K], resampled flag [K],
 * outer ancestors [K][N] (identity when not resampled).  Any record pointer may be NULL.
 * Final population after iteration K: theta_out [N][D], logw_out [N] (may be NULL). */
typedef struct {
  int32_t N, M, K, series;
  double gamma;
  uint64_t seed;
  int32_t proposal;  /* 1 = Langevin (SMC1), 0 = random walk (SMC0) */
} orc_smc2_opts;

int orc_smc2_run(const orc_model *mdl, const orc_pf_opts *pf, const orc_smc2_opts *so,
                 int32_t T, const double *y, double *rec_theta, double *rec_loglik,
                 double *rec_grad, double *rec_logw, double *rec_ess, int32_t *rec_resampled,
                 int32_t *rec_anc, double *theta_out, double *logw_out);

#ifdef __cplusplus
}
#endif
#endif
