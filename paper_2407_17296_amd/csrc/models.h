// The state-space models of the library (paper eqs. xt and yt), each with the pieces the fused
// filter kernel needs: the initial draw and one filter step, `advance`, which moves a particle
// with its reparameterised noise (eq. reparam_epsilon) and returns the log incremental weight,
// and the transposed (adjoint) form of its derivatives, `advance_adj` (App. A, eqs.
// deriv_loglike and df..dxk, transposed).  With the bootstrap proposal (Sec. II) a step is the
// transition x_t = mu(x_{t-1}, theta) + sqrt(C(theta)) e_t followed by the observation
// log-density log g(y_t | x_t, theta); the optimal proposal of the 1-D LG model (Sec. IV-A)
// moves by q(x_t | x_{t-1}, y_t) and weighs by p(y_t | x_{t-1}).
//
// `setup` receives the parameters (FP64) and the model constants (FP64, only the SIR model has
// any).  DX / DY / NP: state, observation and parameter dimensions.
//
// Every model's noise enters through an invertible map, x_t = m(x_{t-1}, y_t, theta) + C e_t, so
// `noise_of` recovers a step's noise from the states before and after it (up to rounding), and
// `weight_of` gives its log incremental weight from the same two states: a reverse sweep that
// has both states needs neither the random stream nor a rebuilt step.
//
// R is the arithmetic type of propagation and weighting (double in the plain FP64 form, float
// in the mixed form).  Parameters arrive in FP64 and are transformed once in FP64.  Gradient
// contributions are added into accumulators `tb` indexed like theta (type Acc: the kernel
// sums a step's particles in R and carries the total in FP64).  The library is
// compiled without floating-point contraction and every fused multiply-add here is written out,
// so the adjoint's recomputation of a segment reproduces the forward sweep bit for bit.
#pragma once

#include "device_common.h"

namespace smc2 {

// w * v with w = 0 giving 0 even for an infinite v: adjoint terms of particles whose weight or
// state adjoint vanishes must contribute nothing (a select, not a branch).
template <typename R>
__device__ __forceinline__ R mulz(R w, R v) {
  return w == (R)0 ? (R)0 : w * v;
}

// a * b + c rounded once
__device__ __forceinline__ float fmar(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double fmar(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// A bootstrap step from a model's transition (step / step_adj) and observation density
// (logg / logg_adj): advance = step then log g at the new state.
template <class Derived, typename R>
struct Bootstrap {
  // values of theta the model keeps in LDS (one copy per workgroup) instead of registers
  static constexpr int kShared = 0;
  __device__ void bind_shared(R *) {}
  // values of each step that depend on t alone, tabulated once per filter in LDS (kPerStep per
  // step; step_values(t, v) gives those of step t, and the model reads them back from the table
  // bound before the first step)
  static constexpr int kPerStep = 0;
  __device__ static void step_values(int, R *) {}
  __device__ void bind_steps(const R *) {}
  __device__ R advance(R *x, const R *e, const R *y) const {
    const Derived &m = *static_cast<const Derived *>(this);
    m.step(x, e);
    return m.logg(y, x);
  }
  // the log incremental weight of a step from the states before (xp) and after (xn) it
  __device__ R weight_of(const R *y, const R *, const R *xn) const {
    const Derived &m = *static_cast<const Derived *>(this);
    return m.logg(y, xn);
  }
  // xb: adjoint of the state after the step on entry, before it on return; wb: adjoint of
  // the step's log-weight; xp / xn: the state before / after the step
  template <typename Acc>
  __device__ void advance_adj(const R *y, const R *xp, const R *xn, const R *e, R wb, R *xb,
                              Acc *tb) const {
    const Derived &m = *static_cast<const Derived *>(this);
    m.logg_adj(y, xn, wb, xb, tb);
    m.step_adj(xp, e, xb, tb);
  }
};

// x_t = a x + sx e;  y = x + sy w;  theta = (a, log sx, log sy);  x_0 ~ N(0, 1).
template <typename R>
struct ModelLG1D : Bootstrap<ModelLG1D<R>, R> {
  static constexpr int DX = 1, DY = 1, NP = 3;
  R a, sx, c0, isy, isx;  // c0 = -log(2 pi)/2 - log sy
  __device__ void setup(const double *th, const double *) {
    a = (R)th[0];
    sx = (R)exp(th[1]);
    c0 = (R)(-kHalfLog2Pi - th[2]);
    isy = (R)exp(-th[2]);
    isx = (R)exp(-th[1]);
  }
  __device__ void per_step(int) {}
  __device__ void init(const R *e0, R *x) const { x[0] = e0[0]; }
  __device__ void init_adj(const R *, const R *, double *) const {}
  __device__ void step(R *x, const R *e) const { x[0] = fmar(a, x[0], sx * e[0]); }
  __device__ void noise_of(const R *xp, const R *xn, const R *, R *e) const {
    e[0] = (xn[0] - a * xp[0]) * isx;
  }
  // reverse of step: tb += F_theta^T xb;  xb <- F_x^T xb   (xp = state before the step)
  template <typename Acc>
  __device__ void step_adj(const R *xp, const R *e, R *xb, Acc *tb) const {
    tb[0] += (Acc)mulz(xb[0], xp[0]);
    tb[1] += (Acc)mulz(xb[0], sx * e[0]);
    xb[0] = a * xb[0];
  }
  __device__ R logg(const R *y, const R *x) const {
    const R r = (y[0] - x[0]) * isy;
    return fmar((R)-0.5 * r, r, c0);
  }
  // xb += wb d lambda/dx;  tb += wb d lambda/dtheta
  template <typename Acc>
  __device__ void logg_adj(const R *y, const R *x, R wb, R *xb, Acc *tb) const {
    const R r = (y[0] - x[0]) * isy;
    xb[0] += mulz(wb, r * isy);
    tb[2] += (Acc)mulz(wb, fmar(r, r, (R)-1));
  }
};

// x_t,q = A_q x_q + sx e_q;  y_q = x_q + sy w_q;  theta = (A_1..A_d, log sx, log sy);
// x_0 ~ N(0, I).  A is diagonal, so the transition is elementwise.
template <typename R, int D_X>
struct ModelLGDiag : Bootstrap<ModelLGDiag<R, D_X>, R> {
  static constexpr int DX = D_X, DY = D_X, NP = D_X + 2;
  // the diagonal A is the same for every particle of the workgroup: it lives in LDS (bound
  // before setup), where a block of four reads it with one broadcast load
  static constexpr int kShared = D_X;
  R *A;
  R sx, c0, isy;  // c0 = d (-log(2 pi)/2 - log sy)
  __device__ void bind_shared(R *sh) { A = sh; }
  // one thread writes A; the caller makes the writes visible before the first step
  __device__ void setup(const double *th, const double *) {
    if (threadIdx.x == 0)
#pragma unroll
      for (int q = 0; q < D_X; ++q) A[q] = (R)th[q];
    sx = (R)exp(th[D_X]);
    c0 = (R)((double)D_X * (-kHalfLog2Pi - th[D_X + 1]));
    isy = (R)exp(-th[D_X + 1]);
  }
  __device__ void per_step(int) {}
  __device__ void init(const R *e0, R *x) const {
#pragma unroll
    for (int q = 0; q < D_X; ++q) x[q] = e0[q];
  }
  __device__ void init_adj(const R *, const R *, double *) const {}
  __device__ void step(R *x, const R *e) const {
#pragma unroll
    for (int q = 0; q < D_X; ++q) x[q] = fmar(A[q], x[q], sx * e[q]);
  }
  template <typename Acc>
  __device__ void step_adj(const R *xp, const R *e, R *xb, Acc *tb) const {
    R ssx = (R)0;
#pragma unroll
    for (int q = 0; q < D_X; ++q) {
      tb[q] += (Acc)mulz(xb[q], xp[q]);
      ssx += mulz(xb[q], e[q]);
      xb[q] = A[q] * xb[q];
    }
    tb[D_X] += (Acc)(ssx * sx);
  }
  __device__ R logg(const R *y, const R *x) const {
    R s2 = (R)0;
#pragma unroll
    for (int q = 0; q < D_X; ++q) {
      const R r = (y[q] - x[q]) * isy;
      s2 = fmar(r, r, s2);
    }
    return fmar((R)-0.5, s2, c0);
  }
  template <typename Acc>
  __device__ void logg_adj(const R *y, const R *x, R wb, R *xb, Acc *tb) const {
    R s2 = (R)0;
#pragma unroll
    for (int q = 0; q < D_X; ++q) {
      const R r = (y[q] - x[q]) * isy;
      xb[q] += mulz(wb, r * isy);
      s2 = fmar(r, r, s2);
    }
    tb[D_X + 1] += (Acc)mulz(wb, s2 - (R)D_X);
  }

  // Blockwise form, for streaming a particle through a step four components at a time
  // (components 4b .. 4b + 3): given theta the components are independent, and log g couples
  // them only through its sum of squared residuals.  Taking the blocks in order reproduces the
  // sums of step / logg / logg_adj / step_adj bit for bit.
  static constexpr bool kBlocks = true;
  // the start of a block from its noise
  __device__ void init_block(int, const R (&e4)[4], R (&x4)[4]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) x4[i] = e4[i];
  }
  __device__ void step_block(int b, R (&x4)[4], const R (&e4)[4]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) x4[i] = fmar(A[4 * b + i], x4[i], sx * e4[i]);
  }
  // s2 += the block's squared residuals of log g at the state after the step
  __device__ void resid_block(int b, const R *y, const R (&x4)[4], R &s2) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const R r = (y[4 * b + i] - x4[i]) * isy;
      s2 = fmar(r, r, s2);
    }
  }
  __device__ R logg_of(R s2) const { return fmar((R)-0.5, s2, c0); }
  // the transposed step of a block: xb4 holds the block's state adjoint after the step on entry
  // and before it on return; tb4 receives the adjoints of the block's parameters A_{4b..4b+3}
  // (parameter 4b + i of theta); s2 and ssx carry the sums whose adjoints adj_finish adds once
  // all blocks are done
  template <typename Acc>
  __device__ void adj_block(int b, const R *y, const R (&xp4)[4], const R (&xn4)[4],
                            const R (&e4)[4], R wb, R (&xb4)[4], Acc (&tb4)[4], R &s2,
                            R &ssx) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const R r = (y[4 * b + i] - xn4[i]) * isy;
      xb4[i] += mulz(wb, r * isy);
      s2 = fmar(r, r, s2);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      tb4[i] += (Acc)mulz(xb4[i], xp4[i]);
      ssx += mulz(xb4[i], e4[i]);
      xb4[i] = A[4 * b + i] * xb4[i];
    }
  }
  template <typename Acc>
  __device__ void adj_finish(R wb, R s2, R ssx, Acc *tb) const {
    tb[D_X] += (Acc)(ssx * sx);
    tb[D_X + 1] += (Acc)mulz(wb, s2 - (R)D_X);
  }
};

// x_t = x/2 + 25 x/(1+x^2) + 8 cos(1.2 t) + sx e;  y = x^2/20 + sy w;
// theta = (log sx, log sy);  x_0 ~ N(0, 1).
template <typename R>
struct ModelGrowth : Bootstrap<ModelGrowth<R>, R> {
  static constexpr int DX = 1, DY = 1, NP = 2;
  R sx, c0, isy, drive, isx;  // c0 = -log(2 pi)/2 - log sy
  const R *dtab;                // the forcing of steps 1..T (LDS)
  __device__ void setup(const double *th, const double *) {
    sx = (R)exp(th[0]);
    c0 = (R)(-kHalfLog2Pi - th[1]);
    isy = (R)exp(-th[1]);
    isx = (R)exp(-th[0]);
    drive = (R)0;
  }
  // the deterministic forcing of step t, evaluated in FP64 once per filter and step
  static constexpr int kPerStep = 1;
  __device__ static void step_values(int t, R *v) { v[0] = (R)(8.0 * cos(1.2 * (double)t)); }
  __device__ void bind_steps(const R *tab) { dtab = tab; }
  __device__ void per_step(int t) { drive = dtab[t - 1]; }
  __device__ void init(const R *e0, R *x) const { x[0] = e0[0]; }
  __device__ void init_adj(const R *, const R *, double *) const {}
  __device__ void step(R *x, const R *e) const {
    const R v = x[0];
    x[0] = fmar((R)0.5, v, (R)25 * v * frcp(fmar(v, v, (R)1))) + fmar(sx, e[0], drive);
  }
  // per_step(t) sets the forcing first
  __device__ void noise_of(const R *xp, const R *xn, const R *, R *e) const {
    const R v = xp[0];
    e[0] = (xn[0] - fmar((R)0.5, v, (R)25 * v * frcp(fmar(v, v, (R)1))) - drive) * isx;
  }
  template <typename Acc>
  __device__ void step_adj(const R *xp, const R *e, R *xb, Acc *tb) const {
    const R v = xp[0], iden = frcp(fmar(v, v, (R)1));
    const R fx = fmar((R)25 * fmar(-v, v, (R)1), iden * iden, (R)0.5);
    tb[0] += (Acc)mulz(xb[0], sx * e[0]);
    xb[0] = mulz(xb[0], fx);
  }
  __device__ R logg(const R *y, const R *x) const {
    const R r = fmar(-x[0] * x[0], (R)0.05, y[0]) * isy;
    return fmar((R)-0.5 * r, r, c0);
  }
  template <typename Acc>
  __device__ void logg_adj(const R *y, const R *x, R wb, R *xb, Acc *tb) const {
    const R r = fmar(-x[0] * x[0], (R)0.05, y[0]) * isy;
    xb[0] += mulz(wb, r * isy * x[0] * (R)0.1);
    tb[1] += (Acc)mulz(wb, fmar(r, r, (R)-1));
  }
};

// x_t = mu + phi (x - mu) + s e;  y = exp(x/2) w;  theta = (mu, atanh phi, log s);
// x_0 ~ N(mu, s^2 / (1 - phi^2)) = mu + s cosh(theta_1) e_0.
template <typename R>
struct ModelSV : Bootstrap<ModelSV<R>, R> {
  static constexpr int DX = 1, DY = 1, NP = 3;
  R mu, phi, s, sd0, dsd0, is;  // dsd0 = d sd0 / d theta_1 = s sinh(theta_1), is = 1 / s
  __device__ void setup(const double *th, const double *) {
    mu = (R)th[0];
    phi = (R)tanh(th[1]);
    s = (R)exp(th[2]);
    sd0 = (R)(exp(th[2]) * cosh(th[1]));
    dsd0 = (R)(exp(th[2]) * sinh(th[1]));
    is = (R)exp(-th[2]);
  }
  __device__ void per_step(int) {}
  __device__ void init(const R *e0, R *x) const { x[0] = fmar(sd0, e0[0], mu); }
  __device__ void init_adj(const R *e0, const R *xb, double *tb) const {
    tb[0] += (double)xb[0];
    tb[1] += (double)mulz(xb[0], dsd0 * e0[0]);
    tb[2] += (double)mulz(xb[0], sd0 * e0[0]);
  }
  __device__ void step(R *x, const R *e) const {
    x[0] = fmar(phi, x[0] - mu, fmar(s, e[0], mu));
  }
  __device__ void noise_of(const R *xp, const R *xn, const R *, R *e) const {
    e[0] = (xn[0] - fmar(phi, xp[0] - mu, mu)) * is;
  }
  template <typename Acc>
  __device__ void step_adj(const R *xp, const R *e, R *xb, Acc *tb) const {
    tb[0] += (Acc)(xb[0] * ((R)1 - phi));
    tb[1] += (Acc)mulz(xb[0], ((R)1 - phi * phi) * (xp[0] - mu));
    tb[2] += (Acc)mulz(xb[0], s * e[0]);
    xb[0] = phi * xb[0];
  }
  __device__ R logg(const R *y, const R *x) const {
    return fmar((R)-0.5, fmar(y[0] * y[0], fexp(-x[0]), x[0]), (R)(-kHalfLog2Pi));
  }
  template <typename Acc>
  __device__ void logg_adj(const R *y, const R *x, R wb, R *xb, Acc *) const {
    xb[0] += mulz(wb, fmar((R)0.5 * y[0] * y[0], fexp(-x[0]), (R)-0.5));
  }
};

// The 1-D LG model filtered with the optimal proposal of Sec. IV-A:
//   x_t = m + rho e,  m = rho^2 (y_t / sy^2 + a x_{t-1} / sx^2),  1/rho^2 = 1/sx^2 + 1/sy^2,
// weighted by the predictive density log N(y_t; a x_{t-1}, sx^2 + sy^2) of the state before the
// step.  theta = (a, log sx, log sy); x_0 ~ N(0, 1).
template <typename R>
struct ModelLG1DOpt {
  static constexpr int DX = 1, DY = 1, NP = 3;
  static constexpr int kShared = 0, kPerStep = 0;  // as for the bootstrap models: no tables
  __device__ void bind_shared(R *) {}
  __device__ static void step_values(int, R *) {}
  __device__ void bind_steps(const R *) {}
  // kx = dm/dx = rho^2 a / sx^2, ky = rho^2 / sy^2, rx = rho^2 / sx^2, c0 = -log(2 pi)/2 -
  // log(s2)/2 and is2 = 1/s2 with s2 = sx^2 + sy^2, fx / fy = sx^2 / s2, sy^2 / s2
  R a, kx, ky, rx, rho, c0, is2, fx, fy, irho;
  __device__ void setup(const double *th, const double *) {
    const double vx = exp(2.0 * th[1]), vy = exp(2.0 * th[2]);
    const double rho2 = 1.0 / (1.0 / vx + 1.0 / vy), s2 = vx + vy;
    a = (R)th[0];
    kx = (R)(rho2 * th[0] / vx);
    ky = (R)(rho2 / vy);
    rx = (R)(rho2 / vx);
    rho = (R)sqrt(rho2);
    irho = (R)(1.0 / sqrt(rho2));
    c0 = (R)(-kHalfLog2Pi - 0.5 * log(s2));
    is2 = (R)(1.0 / s2);
    fx = (R)(vx / s2);
    fy = (R)(vy / s2);
  }
  __device__ void per_step(int) {}
  __device__ void init(const R *e0, R *x) const { x[0] = e0[0]; }
  __device__ void init_adj(const R *, const R *, double *) const {}
  __device__ R advance(R *x, const R *e, const R *y) const {
    const R xo = x[0], r = fmar(-a, xo, y[0]);
    x[0] = fmar(ky, y[0], fmar(kx, xo, rho * e[0]));
    return fmar((R)-0.5 * r * is2, r, c0);
  }
  // the predictive weight depends on the state before the step only
  __device__ R weight_of(const R *y, const R *xp, const R *) const {
    const R r = fmar(-a, xp[0], y[0]);
    return fmar((R)-0.5 * r * is2, r, c0);
  }
  __device__ void noise_of(const R *xp, const R *xn, const R *y, R *e) const {
    e[0] = (xn[0] - fmar(ky, y[0], kx * xp[0])) * irho;
  }
  template <typename Acc>
  __device__ void advance_adj(const R *y, const R *xp, const R *xn, const R *e, R wb, R *xb,
                              Acc *tb) const {
    const R x = xp[0], r = fmar(-a, x, y[0]), q = fmar(r * is2, r, (R)-1);
    const R m = fmar(-rho, e[0], xn[0]);  // the proposal mean
    const R g = xb[0];
    // the weight's dependence on theta and on x_{t-1}
    tb[0] += (Acc)mulz(wb, x * r * is2);
    tb[1] += (Acc)mulz(wb, fx * q);
    tb[2] += (Acc)mulz(wb, fy * q);
    // the new state's: dm/da = rho^2 x / sx^2; d x_t / d log sx = rho^2 / sx^2 (2 (m - a x) +
    // rho e); d x_t / d log sy = rho^2 / sy^2 (2 (m - y) + rho e)
    tb[0] += (Acc)mulz(g, rx * x);
    tb[1] += (Acc)mulz(g, rx * fmar((R)2, m - a * x, rho * e[0]));
    tb[2] += (Acc)mulz(g, ky * fmar((R)2, m - y[0], rho * e[0]));
    xb[0] = fmar(kx, g, mulz(wb, a * r * is2));
  }
};

// The discrete-time SIR model of Sec. IV-B: state (S, I), R = N_pop - S - I implied,
//   S_t = S - beta I S / N_pop + s_e e_0,
//   I_t = I + beta I S / N_pop - gamma I - s_e e_0 + s_e e_1,
//   y = I_t + s_y w,  x_0 = (N_pop - I_0, I_0);  theta = (beta, gamma) on their natural scale.
// Constants (N_pop, I_0, s_e^2, s_y).  The start is fixed, so init_adj has nothing to add.
template <typename R>
struct ModelSIR : Bootstrap<ModelSIR<R>, R> {
  static constexpr int DX = 2, DY = 1, NP = 2;
  R beta, gam, bn, s0, i0, se, isy, c0;  // bn = beta / N_pop, c0 = -log(2 pi)/2 - log s_y
  R inp;                                 // 1 / N_pop
  __device__ void setup(const double *th, const double *mc) {
    beta = (R)th[0];
    gam = (R)th[1];
    bn = (R)(th[0] / mc[0]);
    inp = (R)(1.0 / mc[0]);
    s0 = (R)(mc[0] - mc[1]);
    i0 = (R)mc[1];
    se = (R)sqrt(mc[2]);
    isy = (R)(1.0 / mc[3]);
    c0 = (R)(-kHalfLog2Pi - log(mc[3]));
  }
  __device__ void per_step(int) {}
  __device__ void init(const R *, R *x) const {
    x[0] = s0;
    x[1] = i0;
  }
  __device__ void init_adj(const R *, const R *, double *) const {}
  __device__ void step(R *x, const R *e) const {
    const R S = x[0], I = x[1];
    const R inf = bn * I * S;  // new infections
    x[0] = fmar(se, e[0], S - inf);
    x[1] = fmar(se, e[1] - e[0], fmar(-gam, I, I) + inf);
  }
  // the noise does not depend on theta, so the adjoint never reads it
  __device__ void noise_of(const R *, const R *, const R *, R *e) const {
    e[0] = (R)0;
    e[1] = (R)0;
  }
  // inf enters S with -1 and I with +1, so its adjoint is xb_I - xb_S
  template <typename Acc>
  __device__ void step_adj(const R *xp, const R *, R *xb, Acc *tb) const {
    const R S = xp[0], I = xp[1], gS = xb[0], gI = xb[1];
    const R d = gI - gS;
    tb[0] += (Acc)mulz(d, I * S * inp);
    tb[1] -= (Acc)mulz(gI, I);
    // a zero adjoint adds nothing, also where the state has overflowed (I or S infinite)
    xb[0] = d == (R)0 ? gS : fmar(bn * I, d, gS);
    xb[1] = d == (R)0 ? fmar(-gam, gI, gI) : fmar(bn * S, d, fmar(-gam, gI, gI));
  }
  __device__ R logg(const R *y, const R *x) const {
    const R r = (y[0] - x[1]) * isy;
    return fmar((R)-0.5 * r, r, c0);
  }
  template <typename Acc>
  __device__ void logg_adj(const R *y, const R *x, R wb, R *xb, Acc *) const {
    xb[1] += mulz(wb, (y[0] - x[1]) * isy * isy);
  }
};

}  // namespace smc2
