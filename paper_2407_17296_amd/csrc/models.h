// The state-space models of the library (paper eqs. xt and yt), each with the pieces the fused
// filter kernel needs: the initial draw, the reparameterised bootstrap transition
// x_t = mu(x_{t-1}, theta) + sqrt(C(theta)) e_t (eq. reparam_epsilon), the observation
// log-density lambda = log g(y_t | x_t, theta), and the transposed (adjoint) forms of their
// derivatives (App. A, eqs. deriv_loglike and df..dxk, transposed).
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

// x_t = a x + sx e;  y = x + sy w;  theta = (a, log sx, log sy);  x_0 ~ N(0, 1).
template <typename R>
struct ModelLG1D {
  static constexpr int DX = 1, NP = 3;
  R a, sx, c0, isy;  // c0 = -log(2 pi)/2 - log sy
  __device__ void setup(const double *th) {
    a = (R)th[0];
    sx = (R)exp(th[1]);
    c0 = (R)(-kHalfLog2Pi - th[2]);
    isy = (R)exp(-th[2]);
  }
  __device__ void per_step(int) {}
  __device__ void init(const R *e0, R *x) const { x[0] = e0[0]; }
  __device__ void init_adj(const R *, const R *, double *) const {}
  __device__ void step(R *x, const R *e) const { x[0] = fmar(a, x[0], sx * e[0]); }
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
struct ModelLGDiag {
  static constexpr int DX = D_X, NP = D_X + 2;
  R A[D_X], sx, c0, isy;  // c0 = d (-log(2 pi)/2 - log sy)
  __device__ void setup(const double *th) {
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
};

// x_t = x/2 + 25 x/(1+x^2) + 8 cos(1.2 t) + sx e;  y = x^2/20 + sy w;
// theta = (log sx, log sy);  x_0 ~ N(0, 1).
template <typename R>
struct ModelGrowth {
  static constexpr int DX = 1, NP = 2;
  R sx, c0, isy, drive;  // c0 = -log(2 pi)/2 - log sy
  __device__ void setup(const double *th) {
    sx = (R)exp(th[0]);
    c0 = (R)(-kHalfLog2Pi - th[1]);
    isy = (R)exp(-th[1]);
    drive = (R)0;
  }
  // the deterministic forcing of step t, evaluated once per step in FP64
  __device__ void per_step(int t) { drive = (R)(8.0 * cos(1.2 * (double)t)); }
  __device__ void init(const R *e0, R *x) const { x[0] = e0[0]; }
  __device__ void init_adj(const R *, const R *, double *) const {}
  __device__ void step(R *x, const R *e) const {
    const R v = x[0];
    x[0] = fmar((R)0.5, v, (R)25 * v * frcp(fmar(v, v, (R)1))) + fmar(sx, e[0], drive);
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
struct ModelSV {
  static constexpr int DX = 1, NP = 3;
  R mu, phi, s, sd0, dsd0;  // dsd0 = d sd0 / d theta_1 = s sinh(theta_1)
  __device__ void setup(const double *th) {
    mu = (R)th[0];
    phi = (R)tanh(th[1]);
    s = (R)exp(th[2]);
    sd0 = (R)(exp(th[2]) * cosh(th[1]));
    dsd0 = (R)(exp(th[2]) * sinh(th[1]));
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

}  // namespace smc2
