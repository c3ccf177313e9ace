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
  5  SIR      the discrete SIR model of Sec. IV-B (state (S, I), N_pop = 763, I_0 = 1, noise
              variance 0.5) observed as y = I + 5 w, (beta, gamma) = (0.6, 0.3), T = 35, N = 64,
              M = 250, K = 15: the paper's outbreak experiment with simulated data in place of
              its outbreak record

Workloads 0, 1, 3 and 4 sample parameters in unconstrained coordinates (log of scales, atanh of
phi) under an independent N(0, 1) prior; workload 2 puts N(0.725, 0.13^2) (the centre and the
spread of U(0.5, 0.95)) on each transition entry and N(0, 1) on the log scales, since entries of
N(0, 1) draws beyond one make a 16-dimensional state explode within T = 100 steps; workload 5
samples (beta, gamma) on their natural scale under the paper's independent U(0, 1) priors.  data_seed = 20240724 + i, run seed = 17296 + i.
"""
from dataclasses import dataclass, field

import numpy as np

LG1D, LG_DIAG, GROWTH, SV, SIR = 0, 1, 2, 3, 5
MODEL_NAMES = {LG1D: "lg1d", LG_DIAG: "lg_diag16", GROWTH: "growth", SV: "sv", SIR: "sir"}
PRIOR_KIND_NORMAL, PRIOR_KIND_UNIFORM = 0, 1
# SIR model constants: population, initial infections, process-noise variance, observation sd
SIR_CONSTANTS = (763.0, 1.0, 0.5, 5.0)


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
    dy: int = 0                     # observation dimension (0: equal to d)
    prior_kind: np.ndarray = field(default=None)  # [D] PRIOR_KIND_*, None: all normal
    constants: np.ndarray = field(default=None)   # model constants, None: the defaults

    def __post_init__(self):
        if not self.dy:
            self.dy = self.d

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
    elif kind == SIR:
        beta, gam = theta[0], theta[1]
        npop, i0, var, sy = SIR_CONSTANTS
        se = np.sqrt(var)
        S, I = npop - i0, i0
        for t in range(T):
            e = rng.standard_normal(2)
            inf = beta * I * S / npop
            S, I = S - inf + se * e[0], I + inf - gam * I - se * e[0] + se * e[1]
            y[t, 0] = I + sy * rng.standard_normal()
    else:
        raise ValueError(kind)
    return y


def make(index, N=None, M=None, K=None, S=None, T=None):
    """Build workload `index` (0..5).  N, M, K, S, T override the sizes (T caps every T_s)."""
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
    elif i == 5:
        kind, d, D = SIR, 2, 2
        th = np.array([0.6, 0.3])
        Ss, Ts, Nn, Mm, Kk, gam = 1, [35], 64, 250, 15, 0.006
    else:
        raise ValueError("workload index must be 0..5")
    if S is not None:
        Ss = int(S)
        Ts = (list(Ts) * Ss)[:Ss]
    if T is not None:
        Ts = [min(int(t), int(T)) for t in Ts]
    T_len = np.asarray(Ts, dtype=np.int32)
    T_max = int(T_len.max())
    dy = 1 if kind == SIR else d
    y = np.zeros((Ss, T_max, dy))
    for s in range(Ss):
        y[s, :T_len[s]] = _simulate(kind, th, int(T_len[s]), dy, rng)
    extra = {}
    if kind == LG_DIAG:  # a prior on the transition entries that keeps the dynamics stable
        extra = dict(prior_mu=np.concatenate([np.full(d, 0.725), np.zeros(2)]),
                     prior_sd=np.concatenate([np.full(d, 0.13), np.ones(2)]))
    if kind == SIR:  # U(0, 1) priors: the bounds ride in prior_mu / prior_sd
        extra = dict(prior_mu=np.zeros(D), prior_sd=np.ones(D), dy=1,
                     prior_kind=np.full(D, PRIOR_KIND_UNIFORM, dtype=np.int32),
                     constants=np.array(SIR_CONSTANTS))
    n_, m_ = int(N or Nn), int(M or Mm)
    name = ("sir_outbreak" if kind == SIR else MODEL_NAMES[kind]) + \
        (f"_S{Ss}" if Ss > 1 else "") + f"_T{T_max}_N{n_}_M{m_}"
    return Workload(index=i, name=name, kind=kind, d=d, D=D, S=Ss, N=n_,
                    M=m_, K=int(K or Kk), gamma=float(gam), T_len=T_len, y=y,
                    theta_true=th, seed=seed, data_seed=data_seed,
                    **({"prior_mu": np.zeros(D), "prior_sd": np.ones(D)} | extra))


def prior_draws(w, rng_seed=None, count=None):
    """Independent prior draws [S][N][D] from numpy's generator (normal, or uniform between the
    bounds), for tests that want parameters without running the sampler's own prior stream."""
    rng = np.random.default_rng(w.seed if rng_seed is None else rng_seed)
    n = w.N if count is None else int(count)
    z = w.prior_mu + w.prior_sd * rng.standard_normal((w.S, n, w.D))
    if w.prior_kind is not None:
        u = w.prior_mu + (w.prior_sd - w.prior_mu) * rng.uniform(size=(w.S, n, w.D))
        z = np.where(np.asarray(w.prior_kind) == PRIOR_KIND_UNIFORM, u, z)
    return z
