/*
 * oracle.cpp -- serial FP64 CPU oracle of the Enhanced SMC^2 hot path (Rosato et al. 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this code.  The product path never does; it shares nothing with it.
 *
 * What it computes, in the paper's order and notation:
 *   - the bootstrap particle filter of Sec. II: proposal = transition (eqs. prior_proposal and
 *     priorproposalweight), likelihood estimate (eq. likelihood_pf_) accumulated as a sum of
 *     per-step log normalisers, normalised weights (eq. normalisedweights), the ESS test
 *     (eq. ess) and CRN resampling (App. B);
 *   - its gradient by forward-mode tangent propagation (App. A: eqs. dloglik, weightupdate,
 *     deriv_loglike, df/partialf/dxk with the reparameterised noise of eq. reparam_epsilon; and
 *     App. B: eqs. weightdiffresample and the almost-sure particle-gradient rule);
 *   - the SMC^2 outer step of Sec. III: prior draws (eqs. init_sample, init_weights), the
 *     Langevin proposal SMC1 of Sec. III-D, the L-kernel weight (eq. l_weights with the kernel of
 *     Sec. III-E), normalisation (eq. normalise_smc2), ESS (eq. ess_smc2) and resampling.
 * Readings where the paper is silent or garbled are listed with the design notes; each is named
 * at the line that takes it (C1..C30 numbering of the design notes).
 *
 * Every loop is serial with the particle index ascending.  No blocking, no fusion.
 */
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <type_traits>
#include <vector>

namespace {

typedef std::complex<double> cplx;
const double kTwoPi = 6.283185307179586476925286766559;
const double kHalfLog2Pi = 0.91893853320467274178032973640562;
const double kNegInf = -std::numeric_limits<double>::infinity();

/* ---------------- counter-based random numbers ---------------------------------------------- */

/* Philox4x32-10: ten rounds of the Philox S-box with the Weyl key schedule (Salmon et al. 2011,
 * Sec. 5).  Round: two 32x32->64 products of words 0 and 2 by the round multipliers; the high
 * halves are xored with the other two words and the round key; the words are permuted. */
void philox(const uint32_t in[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void block_words(uint64_t seed, uint32_t c0, uint32_t blk, uint32_t c2, uint32_t c3,
                 uint32_t w[4]) {
  uint32_t ctr[4] = {c0, blk, c2, c3};
  uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
  philox(ctr, key, w);
}

/* Normal number n: Box-Muller pair p = n/2 lives in block p/2, words 2(p%2) and 2(p%2)+1. */
double normal_n(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t n) {
  uint32_t p = n >> 1;
  uint32_t w[4];
  block_words(seed, c0, p >> 1, c2, c3, w);
  uint32_t wa = w[2 * (p & 1u)], wb = w[2 * (p & 1u) + 1];
  double u1 = ((double)wa + 1.0) * 0x1p-32; /* (0, 1] */
  double u2 = (double)wb * 0x1p-32;         /* [0, 1) */
  double r = std::sqrt(-2.0 * std::log(u1));
  double ang = kTwoPi * u2;
  return (n & 1u) ? r * std::sin(ang) : r * std::cos(ang);
}

/* Uniform number m in (0, 1]: block m/4, word m%4 (the paper draws nu from U((0,1]), App. B). */
double uniform_m(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t m) {
  uint32_t w[4];
  block_words(seed, c0, m >> 2, c2, c3, w);
  return ((double)w[m & 3u] + 1.0) * 0x1p-32;
}

uint32_t c3_of(uint32_t k, uint32_t stream) { return (k << 8) | stream; }

/* Per-filter noise of one step (t >= 1) or of the initial draw (t = 0): element g = j*d + q
 * (slot j, component q) is normal number g % 4 of block (c0 = g / 4, c1 = t), i.e. Box-Muller
 * pair (g % 4) / 2 of that block, cosine branch for even g.  One generator block serves four
 * consecutive elements of the same step. */
double filter_normal(uint64_t seed, uint32_t fid, uint32_t c3, uint32_t t, uint32_t g) {
  uint32_t w[4];
  block_words(seed, g >> 2, t, fid, c3, w);
  uint32_t pr = (g & 3u) >> 1;
  double u1 = ((double)w[2 * pr] + 1.0) * 0x1p-32;
  double u2 = (double)w[2 * pr + 1] * 0x1p-32;
  double r = std::sqrt(-2.0 * std::log(u1));
  double ang = kTwoPi * u2;
  return (g & 1u) ? r * std::sin(ang) : r * std::cos(ang);
}

/* Per-filter resampling uniform of step t: offspring slot i uses word i % 4 of block
 * (c0 = i / 4, c1 = t) (multinomial); the systematic offset uses word 0 of block
 * (c0 = 0xFFFFFFFF, c1 = t). */
double filter_uniform(uint64_t seed, uint32_t fid, uint32_t c3, uint32_t t, uint32_t c0,
                      uint32_t word) {
  uint32_t w[4];
  block_words(seed, c0, t, fid, c3, w);
  return ((double)w[word & 3u] + 1.0) * 0x1p-32;
}

/* ---------------- real/complex helpers ------------------------------------------------------- */

inline double re(double v) { return v; }
inline double re(const cplx &v) { return v.real(); }

/* ---------------- the state-space models (paper eqs. xt, yt; instances in the configs) --------
 * theta layouts:
 *   LG1D    (a, log sx, log sy):      x_t = a x + sx e,  y = x + sy w,  x_0 ~ N(0,1)
 *   LG_DIAG (A_1..A_d, log sx, log sy): x_t,q = A_q x_q + sx e_q,  y_q = x_q + sy w_q,
 *                                     x_0 ~ N(0, I)
 *   GROWTH  (log sx, log sy):         x_t = x/2 + 25x/(1+x^2) + 8 cos(1.2 t) + sx e,
 *                                     y = x^2/20 + sy w,  x_0 ~ N(0,1)   (C17, C18)
 *   SV      (mu, atanh phi, log s):   x_t = mu + phi (x - mu) + s e,  y = exp(x/2) w,
 *                                     x_0 ~ N(mu, s^2/(1-phi^2))         (C16, C17)
 *   LG1D_OPT (a, log sx, log sy): the LG1D model filtered with the "optimal" proposal of
 *                                     Sec. IV-A, q(x_t | x_{t-1}, y_t) = N(rho^2 (y/sy^2 +
 *                                     a x_{t-1}/sx^2), rho^2), 1/rho^2 = 1/sx^2 + 1/sy^2, and
 *                                     incremental weight p(y_t | x_{t-1}) =
 *                                     N(y_t; a x_{t-1}, sx^2 + sy^2) (C24)
 *   SIR     (beta, gamma):            S_t = S - beta I S / N_pop + s_e e_0,
 *                                     I_t = I + beta I S / N_pop - gamma I - s_e e_0 + s_e e_1,
 *                                     y = I_t + s_y w,  x_0 = (N_pop - I_0, I_0)  (C28-C30)
 * The bootstrap proposal q = f is written in reparameterised form x = mu(x) + sqrt(C) e
 * (eq. reparam_epsilon), and the optimal proposal likewise x = m(x, y) + rho e.  Each routine also returns the partial derivatives that the tangent
 * recursion of eqs. df..dxk needs; they are only used by the real instantiation. */

/* SIR constants (N_pop, I_0, s_e^2, s_y): the paper's population, initial infections and noise
 * variance (Sec. IV-B), and the observation sd of C30 */
const double kSirDefaults[4] = {763.0, 1.0, 0.5, 5.0};

int obs_dim(const orc_model *m) { return m->kind == ORC_SIR ? 1 : m->d; }

template <class R>
struct Model {
  int kind, d, D;
  const R *th;
  double np = 0, i0 = 0, se = 0, sy = 0; /* SIR: N_pop, I_0, s_e, s_y */

  void set_constants(const double *c) {
    const double *v = c ? c : kSirDefaults;
    np = v[0];
    i0 = v[1];
    se = std::sqrt(v[2]);
    sy = v[3];
  }

  /* x_0 = m0(theta) + s0(theta) e_0;  dx0[q*D + p] = d x_0,q / d theta_p */
  void init(const double *e0, R *x, double *dx0) const {
    if (kind == ORC_SV) {
      R mu = th[0], s = std::exp(th[2]);
      R sd0 = s * std::cosh(th[1]); /* s / sqrt(1 - tanh^2) */
      x[0] = mu + sd0 * e0[0];
      if (dx0) {
        dx0[0] = 1.0;
        dx0[1] = re(s * std::sinh(th[1])) * e0[0];
        dx0[2] = re(sd0) * e0[0];
      }
      return;
    }
    if (kind == ORC_SIR) { /* deterministic start (Sec. IV-B): no dependence on theta */
      x[0] = R(np - i0);
      x[1] = R(i0);
      if (dx0)
        for (int r = 0; r < 2 * D; ++r) dx0[r] = 0.0;
      return;
    }
    for (int q = 0; q < d; ++q) {
      x[q] = R(e0[q]);
      if (dx0)
        for (int p = 0; p < D; ++p) dx0[q * D + p] = 0.0;
    }
  }

  /* x_t = f(x_{t-1}, theta, e_t, t).  Tangent (eq. dxk): dx_new = F_x dx_old + F_theta.
   * dx is [d][D], updated in place when non-NULL (F_x is diagonal for every model but SIR). */
  void propagate(int t, R *x, const double *e, double *dx) const {
    switch (kind) {
      case ORC_LG1D: {
        R a = th[0], sx = std::exp(th[1]);
        R xo = x[0];
        x[0] = a * xo + sx * e[0];
        if (dx) {
          double ar = re(a), xr = re(xo), sxe = re(sx) * e[0];
          dx[0] = ar * dx[0] + xr;  /* d/da */
          dx[1] = ar * dx[1] + sxe; /* d/dlog sx */
          dx[2] = ar * dx[2];       /* d/dlog sy */
        }
        break;
      }
      case ORC_LG_DIAG: {
        R sx = std::exp(th[d]);
        for (int q = 0; q < d; ++q) {
          R a = th[q], xo = x[q];
          x[q] = a * xo + sx * e[q];
          if (dx) {
            double ar = re(a), xr = re(xo), sxe = re(sx) * e[q];
            double *row = dx + q * D;
            for (int p = 0; p < D; ++p) row[p] *= ar;
            row[q] += xr;
            row[d] += sxe;
          }
        }
        break;
      }
      case ORC_GROWTH: {
        R sx = std::exp(th[0]);
        R xo = x[0];
        x[0] = xo / 2.0 + 25.0 * xo / (1.0 + xo * xo) + 8.0 * std::cos(1.2 * (double)t) +
               sx * e[0];
        if (dx) {
          double xr = re(xo);
          double den = 1.0 + xr * xr;
          double fx = 0.5 + 25.0 * (1.0 - xr * xr) / (den * den);
          dx[0] = fx * dx[0] + re(sx) * e[0];
          dx[1] = fx * dx[1];
        }
        break;
      }
      case ORC_SIR: {
        /* new infections beta I S / N_pop move from S to I; recoveries gamma I leave I */
        R beta = th[0], gam = th[1];
        R So = x[0], Io = x[1];
        R inf = beta * Io * So / np;
        x[0] = So - inf + se * e[0];
        x[1] = Io + inf - gam * Io - se * e[0] + se * e[1];
        if (dx) {
          double br = re(beta), gr = re(gam), sr = re(So), ir = re(Io);
          for (int p = 0; p < D; ++p) {
            double dS = dx[p], dI = dx[D + p];
            /* d inf = (beta I / N) dS + (beta S / N) dI + (I S / N) d beta */
            double dinf = br * ir / np * dS + br * sr / np * dI + (p == 0 ? ir * sr / np : 0.0);
            dx[p] = dS - dinf;
            dx[D + p] = dI + dinf - gr * dI - (p == 1 ? ir : 0.0);
          }
        }
        break;
      }
      case ORC_SV: {
        R mu = th[0], phi = std::tanh(th[1]), s = std::exp(th[2]);
        R xo = x[0];
        x[0] = mu + phi * (xo - mu) + s * e[0];
        if (dx) {
          double ph = re(phi), xr = re(xo), mr = re(mu);
          dx[0] = ph * dx[0] + (1.0 - ph);
          dx[1] = ph * dx[1] + (1.0 - ph * ph) * (xr - mr);
          dx[2] = ph * dx[2] + re(s) * e[0];
        }
        break;
      }
    }
  }

  /* The optimal proposal of the LG1D_OPT model: x_t = m(x_{t-1}, y_t) + rho e_t with
   * m = rho^2 (y / sy^2 + a x / sx^2); tangent dx_new = m_x dx_old + m_theta + rho_theta e
   * (eq. dxk for this proposal). */
  void propagate_opt(R *x, const double *e, const double *y, double *dx) const {
    R a = th[0], isx2 = std::exp(-2.0 * th[1]), isy2 = std::exp(-2.0 * th[2]);
    R rho2 = 1.0 / (isx2 + isy2), rho = std::sqrt(rho2);
    R xo = x[0];
    R m = rho2 * (y[0] * isy2 + a * xo * isx2);
    x[0] = m + rho * e[0];
    if (dx) {
      double ar = re(a), xr = re(xo), r2 = re(rho2), r1 = re(rho), ix = re(isx2), iy = re(isy2);
      double mr = re(m);
      double mx = r2 * ar * ix;                                  /* d m / d x_{t-1} */
      double ma = r2 * xr * ix;                                  /* d m / d a */
      /* d rho^2 / d log sx = 2 rho^4 / sx^2, so d m / d log sx = 2 rho^2 / sx^2 (m - a x) and
       * d rho / d log sx = rho^3 / sx^2; likewise for log sy with y in place of a x */
      double mu = 2.0 * r2 * ix * (mr - ar * xr) + r1 * r2 * ix * e[0];
      double mv = 2.0 * r2 * iy * (mr - y[0]) + r1 * r2 * iy * e[0];
      dx[0] = mx * dx[0] + ma;
      dx[1] = mx * dx[1] + mu;
      dx[2] = mx * dx[2] + mv;
    }
  }

  /* Incremental weight of the optimal proposal, log N(y_t; a x_{t-1}, sx^2 + sy^2), from the
   * state BEFORE the step; partial derivatives dl_dx [1] (w.r.t. x_{t-1}) and dl_dth [3]. */
  R logp_pred(const double *y, const R *x, double *dl_dx, double *dl_dth) const {
    R a = th[0], vx = std::exp(2.0 * th[1]), vy = std::exp(2.0 * th[2]);
    R s2 = vx + vy, r = y[0] - a * x[0];
    if (dl_dx) {
      double rr = re(r), is2 = 1.0 / re(s2), q = rr * rr * is2 - 1.0;
      dl_dx[0] = re(a) * rr * is2;
      dl_dth[0] = re(x[0]) * rr * is2;
      dl_dth[1] = re(vx) * is2 * q;
      dl_dth[2] = re(vy) * is2 * q;
    }
    return -kHalfLog2Pi - 0.5 * std::log(s2) - 0.5 * r * r / s2;
  }

  /* lambda = log g(y_t | x_t, theta).  With dl_dx [d] and dl_dth [D] (eq. deriv_loglike). */
  R logg(const double *y, const R *x, double *dl_dx, double *dl_dth) const {
    switch (kind) {
      case ORC_LG1D:
      case ORC_LG_DIAG: {
        int iy = (kind == ORC_LG1D) ? 2 : d + 1;
        R lsy = th[iy], sy = std::exp(lsy);
        R acc = R(0.0);
        double dsy = 0.0;
        for (int q = 0; q < d; ++q) {
          R r = (y[q] - x[q]) / sy;
          acc += -kHalfLog2Pi - lsy - 0.5 * r * r;
          if (dl_dx) {
            double rr = re(r);
            dl_dx[q] = rr / re(sy);
            dsy += -1.0 + rr * rr;
          }
        }
        if (dl_dth) {
          for (int p = 0; p < D; ++p) dl_dth[p] = 0.0;
          dl_dth[iy] = dsy;
        }
        return acc;
      }
      case ORC_GROWTH: {
        R lsy = th[1], sy = std::exp(lsy);
        R h = x[0] * x[0] / 20.0;
        R r = (y[0] - h) / sy;
        if (dl_dx) {
          double rr = re(r);
          dl_dx[0] = rr / re(sy) * (re(x[0]) / 10.0);
          dl_dth[0] = 0.0;
          dl_dth[1] = -1.0 + rr * rr;
        }
        return -kHalfLog2Pi - lsy - 0.5 * r * r;
      }
      case ORC_SIR: { /* y = I_t + s_y w (C30) */
        R r = (y[0] - x[1]) / sy;
        if (dl_dx) {
          dl_dx[0] = 0.0;
          dl_dx[1] = re(r) / sy;
          dl_dth[0] = dl_dth[1] = 0.0;
        }
        return -kHalfLog2Pi - std::log(sy) - 0.5 * r * r;
      }
      case ORC_SV: {
        R ex = std::exp(-x[0]);
        if (dl_dx) {
          dl_dx[0] = -0.5 + 0.5 * y[0] * y[0] * re(ex);
          dl_dth[0] = dl_dth[1] = dl_dth[2] = 0.0;
        }
        return -kHalfLog2Pi - 0.5 * x[0] - 0.5 * y[0] * y[0] * ex;
      }
    }
    return R(0.0);
  }
};

bool model_ok(const orc_model *m) {
  if (!m) return false;
  switch (m->kind) {
    case ORC_LG1D: return m->d == 1 && m->D == 3;
    case ORC_LG_DIAG: return m->d >= 1 && m->D == m->d + 2;
    case ORC_GROWTH: return m->d == 1 && m->D == 2;
    case ORC_SV: return m->d == 1 && m->D == 3;
    case ORC_LG1D_OPT: return m->d == 1 && m->D == 3;
    case ORC_SIR: return m->d == 2 && m->D == 2;
  }
  return false;
}

/* ---------------- resampling (App. B) -------------------------------------------------------
 * The paper's index kappa_i = sum_j [nu_i > c_j] with c the normalised cumulative weights
 * counts the cumulative weights strictly below nu_i; the sampled particle is kappa_i (1-based),
 * i.e. the first m (0-based) with c_m >= nu_i (C6b, C7).  Here the comparison is made on the
 * unnormalised prefix: P_m >= nu_i * P_{M-1}. */
void lower_bound_ancestors(int M, const double *w, const double *u, int32_t *a) {
  std::vector<double> P(M);
  double acc = 0.0;
  for (int m = 0; m < M; ++m) {
    acc += w[m];
    P[m] = acc;
  }
  double total = P[M - 1];
  for (int i = 0; i < M; ++i) {
    double target = u[i] * total;
    int m = 0;
    while (m < M - 1 && P[m] < target) ++m;
    a[i] = m;
  }
}

/* ---------------- the CRN particle filter ---------------------------------------------------- */

template <class R>
int run_pf(const orc_model *mdl, const orc_pf_opts *opt, const R *theta, int T, const double *y,
           int M, uint64_t seed, uint32_t k, uint32_t fid, R *loglik, double *grad,
           int32_t *anc, uint8_t *flags, double *steps_s) {
  const bool tangent = std::is_same<R, double>::value && grad != nullptr;
  const int d = mdl->d, D = mdl->D;
  Model<R> mod{mdl->kind, d, D, theta};
  mod.set_constants(mdl->constants);
  const int dy = obs_dim(mdl);

  if (anc)
    for (long i = 0; i < (long)T * M; ++i) anc[i] = -1;
  if (flags)
    for (int t = 0; t < T; ++t) flags[t] = 0;
  if (steps_s)
    for (int t = 0; t < T; ++t) steps_s[t] = 0.0;
  if (grad)
    for (int p = 0; p < D; ++p) grad[p] = 0.0;
  *loglik = R(0.0);

  /* a non-finite parameter explains nothing: loglik = -inf, gradient 0 (C21) */
  for (int p = 0; p < D; ++p)
    if (!std::isfinite(re(theta[p]))) {
      *loglik = R(kNegInf);
      return 0;
    }

  std::vector<R> x(M * d), xn(M * d), lW(M), lw(M);
  std::vector<double> dx, dxn, gam, lwd, e(M), u(M);
  std::vector<int32_t> a(M);
  std::vector<R> eR(M);
  if (tangent) {
    dx.assign((size_t)M * d * D, 0.0);
    dxn.assign((size_t)M * d * D, 0.0);
    gam.assign((size_t)M * D, 0.0); /* d lW / d theta */
    lwd.assign((size_t)M * D, 0.0); /* d lw / d theta */
  }
  std::vector<double> eps(d), dl_dx(d), dl_dth(D);

  /* t = 0: draw x_0 from its initial law; unnormalised weights 1 ie normalised lW = -log M (C2) */
  const uint32_t c3_init = c3_of(k, ORC_INIT_NORMAL), c3_step = c3_of(k, ORC_STEP_NORMAL),
                 c3_res = c3_of(k, ORC_RESAMPLE_UNIFORM);
  const double lWeq = -std::log((double)M);
  for (int j = 0; j < M; ++j) {
    for (int q = 0; q < d; ++q) eps[q] = filter_normal(seed, fid, c3_init, 0u, (uint32_t)(j * d + q));
    mod.init(eps.data(), &x[(size_t)j * d], tangent ? &dx[(size_t)j * d * D] : nullptr);
    lW[j] = R(lWeq);
  }

  R ll = R(0.0);
  std::vector<double> lld(D, 0.0);
  for (int t = 1; t <= T; ++t) {
    const double *yt = y + (size_t)(t - 1) * dy;
    /* propagate with the bootstrap proposal and weight by g (eq. priorproposalweight) */
    for (int j = 0; j < M; ++j) {
      for (int q = 0; q < d; ++q)
        eps[q] = filter_normal(seed, fid, c3_step, (uint32_t)t, (uint32_t)(j * d + q));
      double *dxj = tangent ? &dx[(size_t)j * d * D] : nullptr;
      R lam;
      if (mdl->kind == ORC_LG1D_OPT) {
        /* optimal proposal: the weight p(y_t | x_{t-1}) uses the state before the step, so it
         * and its tangent are taken first, then the particle moves */
        lam = mod.logp_pred(yt, &x[(size_t)j * d], tangent ? dl_dx.data() : nullptr,
                            tangent ? dl_dth.data() : nullptr);
        if (tangent)
          for (int p = 0; p < D; ++p)
            lwd[(size_t)j * D + p] = gam[(size_t)j * D + p] + dl_dth[p] + dl_dx[0] * dxj[p];
        mod.propagate_opt(&x[(size_t)j * d], eps.data(), yt, dxj);
      } else {
        mod.propagate(t, &x[(size_t)j * d], eps.data(), dxj);
        lam = mod.logg(yt, &x[(size_t)j * d], tangent ? dl_dx.data() : nullptr,
                       tangent ? dl_dth.data() : nullptr);
        if (tangent) {
          /* d log w_t = d log w_{t-1} + dL/dtheta, dL = dL/dx dx/dtheta + dL/dtheta (eqs.
           * weightupdate, deriv_loglike) */
          for (int p = 0; p < D; ++p) {
            double v = gam[(size_t)j * D + p] + dl_dth[p];
            for (int q = 0; q < d; ++q) v += dl_dx[q] * dxj[q * D + p];
            lwd[(size_t)j * D + p] = v;
          }
        }
      }
      if (std::isnan(re(lam))) lam = R(kNegInf);
      lw[j] = lW[j] + lam;
    }
    /* log normaliser s_t = log sum_j exp(lw_j) (eq. likelihood_pf_ accumulated step-wise, C1) */
    double mx = kNegInf;
    for (int j = 0; j < M; ++j) mx = std::max(mx, re(lw[j]));
    if (mx == kNegInf) { /* no particle explains y_t (C21) */
      *loglik = R(kNegInf);
      if (grad)
        for (int p = 0; p < D; ++p) grad[p] = 0.0;
      return 0;
    }
    R S = R(0.0);
    double Sre = 0.0, Q = 0.0;
    for (int j = 0; j < M; ++j) {
      eR[j] = std::exp(lw[j] - mx);
      e[j] = re(eR[j]);
      S += eR[j];
      Sre += e[j];
      Q += e[j] * e[j];
    }
    R s_t = mx + std::log(S);
    ll += s_t;
    if (steps_s) steps_s[t - 1] = re(s_t);
    for (int j = 0; j < M; ++j) lW[j] = lw[j] - s_t; /* normalised log weights (eq. normalisedweights) */
    if (tangent) {
      /* d s_t = sum_j W_j d lw_j (eq. dloglik, C4); the normalised tangent is d lw - d s_t */
      std::vector<double> ds(D, 0.0);
      for (int j = 0; j < M; ++j) {
        double W = e[j] / Sre;
        /* a particle of exactly zero weight takes no part, even where its state has overflowed
         * and its own tangent is not finite (C32) */
        if (W == 0.0) continue;
        for (int p = 0; p < D; ++p) ds[p] += W * lwd[(size_t)j * D + p];
      }
      for (int p = 0; p < D; ++p) lld[p] += ds[p];
      for (int j = 0; j < M; ++j)
        for (int p = 0; p < D; ++p) gam[(size_t)j * D + p] = lwd[(size_t)j * D + p] - ds[p];
    }
    /* effective sample size 1 / sum W^2 = S^2 / Q (eq. ess); resample below ess_frac M, never at
     * the last step (C5) */
    double ess = Sre * Sre / Q;
    if (t < T && ess < opt->ess_frac * (double)M) {
      if (opt->resampler == ORC_SYSTEMATIC) {
        double nu = filter_uniform(seed, fid, c3_res, (uint32_t)t, 0xFFFFFFFFu, 0u);
        for (int i = 0; i < M; ++i) u[i] = ((double)i + nu) / (double)M;
      } else {
        for (int i = 0; i < M; ++i)
          u[i] = filter_uniform(seed, fid, c3_res, (uint32_t)t, (uint32_t)i >> 2, (uint32_t)i & 3u);
      }
      lower_bound_ancestors(M, e.data(), u.data(), a.data());
      /* x'_i = x_{kappa_i}; dx'_i = dx_{kappa_i} almost surely; equal sum-preserving weights, whose
       * normalised log is -log M with zero tangent (App. B, eq. weightresample; C8) */
      for (int i = 0; i < M; ++i)
        for (int q = 0; q < d; ++q) xn[(size_t)i * d + q] = x[(size_t)a[i] * d + q];
      x.swap(xn);
      if (tangent) {
        for (int i = 0; i < M; ++i)
          for (int r = 0; r < d * D; ++r) dxn[(size_t)i * d * D + r] = dx[(size_t)a[i] * d * D + r];
        dx.swap(dxn);
        std::fill(gam.begin(), gam.end(), 0.0);
      }
      for (int j = 0; j < M; ++j) lW[j] = R(lWeq);
      if (anc)
        for (int i = 0; i < M; ++i) anc[(size_t)(t - 1) * M + i] = a[i];
      if (flags) flags[t - 1] = 1;
    }
  }
  *loglik = ll;
  if (grad)
    for (int p = 0; p < D; ++p) grad[p] = lld[p];
  return 0;
}

/* ---------------- Kalman filter (exact likelihood of the linear-Gaussian models) ------------- */

template <class R>
R kalman_ll(const orc_model *mdl, const R *th, int T, const double *y) {
  const int d = mdl->d;
  R lsx = (mdl->kind == ORC_LG_DIAG) ? th[d] : th[1];
  R lsy = (mdl->kind == ORC_LG_DIAG) ? th[d + 1] : th[2];
  R qv = std::exp(2.0 * lsx), rv = std::exp(2.0 * lsy);
  R ll = R(0.0);
  for (int q = 0; q < d; ++q) { /* LG_DIAG factorises into d independent scalar filters */
    R a = th[q];
    R m = R(0.0), P = R(1.0); /* x_0 ~ N(0, 1) */
    for (int t = 1; t <= T; ++t) {
      R mp = a * m, Pp = a * a * P + qv;
      R v = y[(size_t)(t - 1) * d + q] - mp, Sv = Pp + rv;
      ll += -kHalfLog2Pi - 0.5 * std::log(Sv) - 0.5 * v * v / Sv;
      R K = Pp / Sv;
      m = mp + K * v;
      P = (1.0 - K) * Pp;
    }
  }
  return ll;
}

}  // namespace

/* ======================= C ABI ================================================================ */

extern "C" {

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(ctr, key, out);
}

double orc_normal(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t n) {
  return normal_n(seed, c0, c2, c3, n);
}

double orc_uniform(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t m) {
  return uniform_m(seed, c0, c2, c3, m);
}

void orc_normals(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t first,
                 int64_t count, double *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = normal_n(seed, c0, c2, c3, first + (uint32_t)i);
}

void orc_uniforms(uint64_t seed, uint32_t c0, uint32_t c2, uint32_t c3, uint32_t first,
                  int64_t count, double *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = uniform_m(seed, c0, c2, c3, first + (uint32_t)i);
}

double orc_filter_normal(uint64_t seed, uint32_t fid, uint32_t c3, uint32_t t, uint32_t g) {
  return filter_normal(seed, fid, c3, t, g);
}

double orc_filter_uniform(uint64_t seed, uint32_t fid, uint32_t c3, uint32_t t, uint32_t c0,
                          uint32_t word) {
  return filter_uniform(seed, fid, c3, t, c0, word);
}

void orc_resample_lower_bound(int32_t M, const double *w, const double *u, int32_t *a) {
  lower_bound_ancestors(M, w, u, a);
}

int orc_pf(const orc_model *mdl, const orc_pf_opts *opt, const double *theta, int32_t T,
           const double *y, int32_t M, uint64_t seed, uint32_t k, uint32_t filter_id,
           double *loglik, double *grad, int32_t *ancestors, uint8_t *flags, double *steps_s) {
  if (!model_ok(mdl) || !opt || !theta || !loglik || T < 0 || M < 1 || (T > 0 && !y)) return 1;
  return run_pf<double>(mdl, opt, theta, T, y, M, seed, k, filter_id, loglik, grad, ancestors,
                        flags, steps_s);
}

int orc_pf_complex_step(const orc_model *mdl, const orc_pf_opts *opt, const double *theta,
                        int32_t T, const double *y, int32_t M, uint64_t seed, uint32_t k,
                        uint32_t filter_id, int32_t p, double h, double *loglik, double *dl,
                        int32_t *ancestors) {
  if (!model_ok(mdl) || !opt || !theta || !loglik || !dl || T < 0 || M < 1 || p < 0 ||
      p >= mdl->D || (T > 0 && !y))
    return 1;
  std::vector<cplx> th(mdl->D);
  for (int q = 0; q < mdl->D; ++q) th[q] = cplx(theta[q], q == p ? h : 0.0);
  cplx ll;
  int rc = run_pf<cplx>(mdl, opt, th.data(), T, y, M, seed, k, filter_id, &ll, nullptr,
                        ancestors, nullptr, nullptr);
  *loglik = ll.real();
  *dl = std::isfinite(ll.real()) ? ll.imag() / h : 0.0;
  return rc;
}

int orc_kalman(const orc_model *mdl, const double *theta, int32_t T, const double *y,
               double *loglik, double *grad) {
  if (!model_ok(mdl) ||
      (mdl->kind != ORC_LG1D && mdl->kind != ORC_LG_DIAG && mdl->kind != ORC_LG1D_OPT) || !theta ||
      !loglik || T < 0)
    return 1;
  *loglik = kalman_ll<double>(mdl, theta, T, y);
  if (grad) {
    const double h = 1e-30;
    std::vector<cplx> th(mdl->D);
    for (int p = 0; p < mdl->D; ++p) {
      for (int q = 0; q < mdl->D; ++q) th[q] = cplx(theta[q], q == p ? h : 0.0);
      grad[p] = kalman_ll<cplx>(mdl, th.data(), T, y).imag() / h;
    }
  }
  return 0;
}

double orc_log_prior(const orc_model *mdl, const double *theta, double *grad) {
  double lp = 0.0;
  for (int p = 0; p < mdl->D; ++p) {
    if (mdl->prior_kind && mdl->prior_kind[p] == ORC_PRIOR_KIND_UNIFORM) {
      /* U(lo, hi): constant density on the closed interval, zero outside; the gradient of
       * its log is zero wherever it is finite */
      double lo = mdl->prior_mu[p], hi = mdl->prior_sd[p];
      lp += (theta[p] >= lo && theta[p] <= hi) ? -std::log(hi - lo) : kNegInf;
      if (grad) grad[p] = 0.0;
      continue;
    }
    double sd = mdl->prior_sd[p], z = (theta[p] - mdl->prior_mu[p]) / sd;
    lp += -kHalfLog2Pi - std::log(sd) - 0.5 * z * z;
    if (grad) grad[p] = -z / sd;
  }
  return lp;
}

void orc_langevin_move(int32_t D, double gamma, const double *theta, const double *grad_logpost,
                       const double *xi, double *theta_new, double *p_prev) {
  /* SMC1 proposal N(theta + F(theta), Gamma), F = Gamma grad log pi / 2, Gamma = gamma^2 I
   * (Sec. III-D, C11); written in velocity form p_{k-1} = gamma xi ~ N(0, Gamma) (C12) */
  for (int p = 0; p < D; ++p) {
    p_prev[p] = gamma * xi[p];
    theta_new[p] = theta[p] + 0.5 * gamma * gamma * grad_logpost[p] + p_prev[p];
  }
}

void orc_random_walk_move(int32_t D, double gamma, const double *theta, const double *xi,
                          double *theta_new, double *p_prev) {
  /* SMC0 proposal N(theta, Gamma), Gamma = gamma^2 I (Sec. III-D), with the same velocity
   * p_{k-1} = gamma xi; it uses no gradient, and its kernel is symmetric */
  for (int p = 0; p < D; ++p) {
    p_prev[p] = gamma * xi[p];
    theta_new[p] = theta[p] + p_prev[p];
  }
}

double orc_lkernel_log_ratio(int32_t D, double gamma, const double *grad_prev,
                             const double *grad_new, const double *p_prev) {
  /* L(theta_{k-1} | theta_k) / q(theta_k | theta_{k-1}) for the one-step Langevin dynamics
   * (Sec. III-E, eq. l=q): both Jacobians are 1 for the leapfrog map, so the ratio is
   * N(-p_k; 0, Gamma) / N(p_{k-1}; 0, Gamma) with p_k = p_{k-1} + F(theta_{k-1}) + F(theta_k)
   * (C12). */
  double g2 = gamma * gamma, npk = 0.0, npp = 0.0;
  for (int p = 0; p < D; ++p) {
    double pk = p_prev[p] + 0.5 * g2 * (grad_prev[p] + grad_new[p]);
    npk += pk * pk;
    npp += p_prev[p] * p_prev[p];
  }
  return -(npk - npp) / (2.0 * g2);
}

double orc_realised_estimate(int32_t N, int32_t D, const double *logw, const double *theta,
                             double *mean, double *second) {
  /* Realised estimates of the first two moments (eq. realised_estimates with f(theta) = theta
   * and theta^2 elementwise) under the normalised weights of eq. normalise_smc2, and the
   * iteration's recycling weight l_k = (sum_i w_i)^2 / sum_i w_i^2 (eq. recycling_I).  The
   * weights are taken relative to their maximum, which cancels in every ratio.  Every weight
   * zero: the moments are NaN and l_k = 0. */
  double mx = kNegInf;
  for (int i = 0; i < N; ++i) mx = std::max(mx, logw[i]);
  if (mx == kNegInf) {
    for (int p = 0; p < D; ++p) mean[p] = second[p] = std::nan("");
    return 0.0;
  }
  double S = 0.0, Q = 0.0;
  for (int i = 0; i < N; ++i) {
    double w = std::exp(logw[i] - mx);
    S += w;
    Q += w * w;
  }
  for (int p = 0; p < D; ++p) {
    double m1 = 0.0, m2 = 0.0;
    for (int i = 0; i < N; ++i) {
      double wn = std::exp(logw[i] - mx) / S; /* normalised weight */
      double v = theta[(size_t)i * D + p];
      m1 += wn * v;
      m2 += wn * v * v;
    }
    mean[p] = m1;
    second[p] = m2;
  }
  return S * S / Q;
}

void orc_recycle(int32_t K, int32_t D, const double *l, const double *est, double *out) {
  /* Recycled estimate (Sec. III-C): sum_k c_k f_k with the optimal constants
   * c_k = l_k / sum_k l_k (eq. opt_recycling_constant).  est is [K][D]; iterations with l_k = 0
   * take no part. */
  double L = 0.0;
  for (int k = 0; k < K; ++k) L += l[k];
  for (int p = 0; p < D; ++p) {
    double acc = 0.0;
    for (int k = 0; k < K; ++k)
      if (l[k] > 0.0) acc += (l[k] / L) * est[(size_t)k * D + p];
    out[p] = acc;
  }
}

int orc_smc2_run(const orc_model *mdl, const orc_pf_opts *pf, const orc_smc2_opts *so,
                 int32_t T, const double *y, double *rec_theta, double *rec_loglik,
                 double *rec_grad, double *rec_logw, double *rec_ess, int32_t *rec_resampled,
                 int32_t *rec_anc, double *theta_out, double *logw_out) {
  if (!model_ok(mdl) || !pf || !so || so->N < 1 || so->M < 1 || so->K < 1 || T < 0) return 1;
  const int N = so->N, D = mdl->D, K = so->K;
  const uint64_t seed = so->seed;
  std::vector<double> th(N * D), thn(N * D), lpi(N), lpin(N), gpi(N * D), gpin(N * D), ll(N),
      lln(N), gll(N * D), logw(N), pprev(N * D), xi(D), tmp(N * D), tmp1(N), lprior_g(D);
  std::vector<double> e(N), u(N);
  std::vector<int32_t> a(N);

  for (int k = 1; k <= K; ++k) {
    if (k == 1) {
      /* eq. init_sample: theta_1 ~ q_1 = prior */
      for (int i = 0; i < N; ++i)
        for (int p = 0; p < D; ++p) {
          const uint32_t c2 = (uint32_t)(so->series * N + i), c3 = c3_of(1, ORC_PRIOR_NORMAL);
          if (mdl->prior_kind && mdl->prior_kind[p] == ORC_PRIOR_KIND_UNIFORM) {
            double lo = mdl->prior_mu[p], hi = mdl->prior_sd[p];
            thn[i * D + p] = lo + (hi - lo) * uniform_m(seed, 0xFFFFFFFFu, c2, c3, (uint32_t)p);
          } else {
            thn[i * D + p] = mdl->prior_mu[p] +
                             mdl->prior_sd[p] * normal_n(seed, 0xFFFFFFFFu, c2, c3, (uint32_t)p);
          }
        }
    } else {
      for (int i = 0; i < N; ++i) {
        for (int p = 0; p < D; ++p)
          xi[p] = normal_n(seed, 0xFFFFFFFFu, (uint32_t)(so->series * N + i),
                           c3_of((uint32_t)k, ORC_MOVE_NORMAL), (uint32_t)p);
        if (so->proposal == 1) {
          orc_langevin_move(D, so->gamma, &th[i * D], &gpi[i * D], xi.data(), &thn[i * D],
                            &pprev[i * D]);
        } else {
          orc_random_walk_move(D, so->gamma, &th[i * D], xi.data(), &thn[i * D], &pprev[i * D]);
        }
      }
    }
    /* run the CRN-PF at every proposed theta: a fresh random stream per sample and iteration */
    for (int i = 0; i < N; ++i) {
      orc_pf(mdl, pf, &thn[i * D], T, y, so->M, seed, (uint32_t)k, (uint32_t)(so->series * N + i),
             &lln[i], &gll[i * D], nullptr, nullptr, nullptr);
      /* log posterior and its gradient (eqs. log_posterior, first_gradientlogposterior) */
      double lp = orc_log_prior(mdl, &thn[i * D], lprior_g.data());
      lpin[i] = lp == kNegInf ? kNegInf : lp + lln[i]; /* outside the prior's support: 0 */
      for (int p = 0; p < D; ++p) gpin[i * D + p] = lprior_g[p] + gll[i * D + p];
    }
    /* weights: eq. init_weights at k = 1 (q_1 = prior, so w = likelihood; C13), eq. l_weights
     * with the Langevin L-kernel afterwards */
    for (int i = 0; i < N; ++i) {
      if (k == 1) {
        logw[i] = lln[i];
      } else if (logw[i] == kNegInf || lpin[i] == kNegInf) {
        logw[i] = kNegInf;
      } else {
        double inc = lpin[i] - lpi[i];
        if (so->proposal == 1)
          inc += orc_lkernel_log_ratio(D, so->gamma, &gpi[i * D], &gpin[i * D], &pprev[i * D]);
        logw[i] = logw[i] + inc;
      }
      if (std::isnan(logw[i])) logw[i] = kNegInf;
    }
    th.swap(thn);
    lpi.swap(lpin);
    gpi.swap(gpin);
    ll.swap(lln);
    if (rec_theta) std::memcpy(rec_theta + (size_t)(k - 1) * N * D, th.data(), sizeof(double) * N * D);
    if (rec_loglik) std::memcpy(rec_loglik + (size_t)(k - 1) * N, ll.data(), sizeof(double) * N);
    if (rec_grad) std::memcpy(rec_grad + (size_t)(k - 1) * N * D, gll.data(), sizeof(double) * N * D);
    if (rec_logw) std::memcpy(rec_logw + (size_t)(k - 1) * N, logw.data(), sizeof(double) * N);

    /* normalise (eq. normalise_smc2) and ESS (eq. ess_smc2) */
    double mx = kNegInf;
    for (int i = 0; i < N; ++i) mx = std::max(mx, logw[i]);
    double S = 0.0, Q = 0.0;
    if (mx != kNegInf)
      for (int i = 0; i < N; ++i) {
        e[i] = std::exp(logw[i] - mx);
        S += e[i];
        Q += e[i] * e[i];
      }
    double ess = (mx == kNegInf) ? 0.0 : S * S / Q;
    if (rec_ess) rec_ess[k - 1] = ess;
    int did = 0;
    for (int i = 0; i < N; ++i) a[i] = i;
    if (mx == kNegInf) {
      /* every sample has zero weight: nothing to normalise; reported through ess = 0 */
    } else if (ess < 0.5 * (double)N) { /* resample iff N_eff < N/2 (Sec. III-B, C14) */
      double nu = uniform_m(seed, 0xFFFFFFFFu, (uint32_t)so->series,
                            c3_of((uint32_t)k, ORC_OUTER_RESAMPLE_UNIFORM), 0u);
      for (int i = 0; i < N; ++i) u[i] = ((double)i + nu) / (double)N;
      lower_bound_ancestors(N, e.data(), u.data(), a.data());
      double lse = mx + std::log(S);
      for (int i = 0; i < N; ++i)
        for (int p = 0; p < D; ++p) tmp[i * D + p] = th[a[i] * D + p];
      th.swap(tmp);
      for (int i = 0; i < N; ++i)
        for (int p = 0; p < D; ++p) tmp[i * D + p] = gpi[a[i] * D + p];
      gpi.swap(tmp);
      for (int i = 0; i < N; ++i) tmp1[i] = lpi[a[i]];
      lpi.swap(tmp1);
      for (int i = 0; i < N; ++i) tmp1[i] = ll[a[i]];
      ll.swap(tmp1);
      for (int i = 0; i < N; ++i) logw[i] = lse - std::log((double)N);
      did = 1;
    }
    if (rec_resampled) rec_resampled[k - 1] = did;
    if (rec_anc) std::memcpy(rec_anc + (size_t)(k - 1) * N, a.data(), sizeof(int32_t) * N);
  }
  if (theta_out) std::memcpy(theta_out, th.data(), sizeof(double) * N * D);
  if (logw_out) std::memcpy(logw_out, logw.data(), sizeof(double) * N);
  return 0;
}

}  // extern "C"
