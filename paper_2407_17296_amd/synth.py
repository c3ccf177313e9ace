"""Seeded synthetic workloads: sizes, true parameters and simulated observations.

This module only builds inputs.  It holds none of the filter's or the sampler's arithmetic: it
simulates each state-space model forward once, with numpy's own generator, to produce the data
y_{1:T} that both the HIP path and the test oracle consume.

The five workloads follow the paper's problem statement (a state-space model with parameter
theta, observations y_{1:T}, N parameter samples, M particles, K SMC^2 iterations, step size
gamma; Sec. II and Sec. III) at the sizes of the project's benchmark table:

  0  LG1D     x_t = a x + sx v, y = x + sy w, (a, sx, sy) = (0.8, 1, 0.5),   T = 50,  N = 32,
              M = 64,   K = 10
  1  LG1D     (0.9, 0.7, 0.3),                                               T = 250, N = 1024,
              M = 1024, K = 20
  2  LG_DIAG  d = 16, A diagonal with A_qq ~ U(0.5, 0.95), sx = 1, sy = 0.5, T = 100, N = 512,
              M = 2048, K = 10
  3  GROWTH   x_t = x/2 + 25x/(1+x^2) + 8 cos(1.2t) + sx v, y = x^2/20 + sy w,
              (sx, sy) = (sqrt 10, 1),                                       T = 100, N = 4096,
              M = 512,  K = 20
  4  SV       x_t = mu + phi (x - mu) + s v, y = exp(x/2) w, (mu, phi, s) = (-1, 0.95, 0.25),
              S = 64 series with T_s ~ U{50..1000},                          N = 256, M = 256,
              K = 10

Parameters are sampled in unconstrained coordinates (log of scales, atanh of phi) under an
independent N(0, 1) prior.  data_seed = 20240724 + i, run seed = 17296 + i.
"""
from dataclasses import dataclass, field

import numpy as np

LG1D, LG_DIAG, GROWTH, SV = 0, 1, 2, 3
MODEL_NAMES = {LG1D: "lg1d", LG_DIAG: "lg_diag16", GROWTH: "growth", SV: "sv"}


@dataclass
class Workload:
    index: int
    name: str
    kind: int
    d: int
    D: int
    S: int
    N: int
    M: int
    K: int
    gamma: float
    T_len: np.ndarray          # [S] int32
    y: np.ndarray              # [S][T_max][d] float64, zero past T_s
    theta_true: np.ndarray     # [D]
    prior_mu: np.ndarray = field(default=None)
    prior_sd: np.ndarray = field(default=None)
    seed: int = 0
    data_seed: int = 0

    @property
    def T_max(self):
        return int(self.T_len.max()) if len(self.T_len) else 0

    def particle_steps(self):
        """N * M * sum_s T_s: particle-steps of one CRN-PF pass over every (series, sample)."""
        return int(self.N) * int(self.M) * int(np.sum(self.T_len, dtype=np.int64))


def _simulate(kind, theta, T, d, rng):
    """Simulate one series of length T from the model at theta (unconstrained coordinates)."""
    y = np.zeros((T, d))
    if kind == LG1D:
        a, sx, sy = theta[0], np.exp(theta[1]), np.exp(theta[2])
        x = rng.standard_normal()
        for t in range(T):
            x = a * x + sx * rng.standard_normal()
            y[t, 0] = x + sy * rng.standard_normal()
    elif kind == LG_DIAG:
        A, sx, sy = theta[:d], np.exp(theta[d]), np.exp(theta[d + 1])
        x = rng.standard_normal(d)
        for t in range(T):
            x = A * x + sx * rng.standard_normal(d)
            y[t] = x + sy * rng.standard_normal(d)
    elif kind == GROWTH:
        sx, sy = np.exp(theta[0]), np.exp(theta[1])
        x = rng.standard_normal()
        for t in range(1, T + 1):
            x = x / 2 + 25 * x / (1 + x * x) + 8 * np.cos(1.2 * t) + sx * rng.standard_normal()
            y[t - 1, 0] = x * x / 20 + sy * rng.standard_normal()
    elif kind == SV:
        mu, phi, s = theta[0], np.tanh(theta[1]), np.exp(theta[2])
        x = mu + s / np.sqrt(1 - phi * phi) * rng.standard_normal()
        for t in range(T):
            x = mu + phi * (x - mu) + s * rng.standard_normal()
            y[t, 0] = np.exp(x / 2) * rng.standard_normal()
    else:
        raise ValueError(kind)
    return y


def make(index, N=None, M=None, K=None, S=None, T=None):
    """Build workload `index` (0..4).  N, M, K, S, T override the sizes (T caps every T_s)."""
    i = int(index)
    data_seed, seed = 20240724 + i, 17296 + i
    rng = np.random.default_rng(data_seed)
    if i == 0:
        kind, d, D = LG1D, 1, 3
        th = np.array([0.8, np.log(1.0), np.log(0.5)])
        Ss, Ts, Nn, Mm, Kk, gam = 1, [50], 32, 64, 10, 0.085
    elif i == 1:
        kind, d, D = LG1D, 1, 3
        th = np.array([0.9, np.log(0.7), np.log(0.3)])
        Ss, Ts, Nn, Mm, Kk, gam = 1, [250], 1024, 1024, 20, 0.085
    elif i == 2:
        kind, d, D = LG_DIAG, 16, 18
        A = rng.uniform(0.5, 0.95, size=16)
        th = np.concatenate([A, [np.log(1.0), np.log(0.5)]])
        Ss, Ts, Nn, Mm, Kk, gam = 1, [100], 512, 2048, 10, 0.02
    elif i == 3:
        kind, d, D = GROWTH, 1, 2
        th = np.array([np.log(np.sqrt(10.0)), np.log(1.0)])
        Ss, Ts, Nn, Mm, Kk, gam = 1, [100], 4096, 512, 20, 0.05
    elif i == 4:
        kind, d, D = SV, 1, 3
        th = np.array([-1.0, np.arctanh(0.95), np.log(0.25)])
        Ss, Nn, Mm, Kk, gam = 64, 256, 256, 10, 0.05
        Ts = list(rng.integers(50, 1001, size=Ss))
    else:
        raise ValueError("workload index must be 0..4")
    if S is not None:
        Ss = int(S)
        Ts = (list(Ts) * Ss)[:Ss]
    if T is not None:
        Ts = [min(int(t), int(T)) for t in Ts]
    T_len = np.asarray(Ts, dtype=np.int32)
    T_max = int(T_len.max())
    y = np.zeros((Ss, T_max, d))
    for s in range(Ss):
        y[s, :T_len[s]] = _simulate(kind, th, int(T_len[s]), d, rng)
    return Workload(index=i, name=f"config{i}_{MODEL_NAMES[kind]}", kind=kind, d=d, D=D, S=Ss,
                    N=int(N or Nn), M=int(M or Mm), K=int(K or Kk), gamma=float(gam),
                    T_len=T_len, y=y, theta_true=th, prior_mu=np.zeros(D), prior_sd=np.ones(D),
                    seed=seed, data_seed=data_seed)


def prior_draws(w, rng_seed=None, count=None):
    """Independent N(prior_mu, prior_sd) draws [S][N][D] from numpy's generator, for tests that
    want parameters without running the sampler's own prior stream."""
    rng = np.random.default_rng(w.seed if rng_seed is None else rng_seed)
    n = w.N if count is None else int(count)
    return w.prior_mu + w.prior_sd * rng.standard_normal((w.S, n, w.D))
