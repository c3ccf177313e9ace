"""SMC^2 driver over the three hot-path calls (paper Sec. III with the CRN-PF of Sec. II).

Iteration k = 1 draws theta from the prior (eq. init_sample), runs the filter and weights by the
likelihood (eq. init_weights); every later iteration runs the Langevin move (Sec. III-D), the
filter at the moved samples, and the L-kernel reweighting/resampling (eq. l_weights, Sec. III-B).
The iteration counter lives in device memory and is advanced by the reweighting call, so one
captured HIP graph replays iteration after iteration with no host synchronisation.

Torch provides device memory, streams and graph capture only; every arithmetic step is a
library kernel.
"""
from dataclasses import dataclass

import numpy as np
import torch

from . import smc2


@dataclass
class Records:
    theta: np.ndarray      # [K][S][N][D] proposed theta (before outer resampling)
    loglik: np.ndarray     # [K][S][N]
    grad: np.ndarray       # [K][S][N][D] gradient of the log-likelihood estimate
    logw: np.ndarray       # [K][S][N] log weights after the iteration's resampling step
    ess: np.ndarray        # [K][S]
    resampled: np.ndarray  # [K][S]
    anc: np.ndarray        # [K][S][N]
    prev_theta: np.ndarray         # [K][S][N][D] population the move started from
    estimate: np.ndarray   # [K][S][2][D] realised E[theta], E[theta^2] before resampling
    prev_logpost: np.ndarray       # [K][S][N]
    prev_grad_logpost: np.ndarray  # [K][S][N][D]
    prev_logw: np.ndarray          # [K][S][N]
    p_prev: np.ndarray             # [K][S][N][D] velocities drawn by the move


class SMC2Run:
    """Device state of one SMC^2 run: two populations, the move's velocities, the counter."""

    def __init__(self, w, precision=smc2.MIXED, resampler=smc2.SYSTEMATIC, ess_frac=0.5,
                 ckpt_interval=0, tile=0, persistent=0, random_walk=0, gamma=None, device=0,
                 seed=None, store_noise=0):
        self.w = w
        self.dev = torch.device("cuda", device)
        self.model = smc2.Model.from_workload(w)
        self.opts = smc2.pf_opts(precision=precision, resampler=resampler, ess_frac=ess_frac,
                                 ckpt_interval=ckpt_interval, want_grad=1, tile=tile,
                                 persistent=persistent, store_noise=store_noise)
        self.gamma = float(w.gamma if gamma is None else gamma)
        self.random_walk = int(random_walk)
        self.seed = int(w.seed if seed is None else seed)
        S, N, D = w.S, w.N, w.D
        self.ctx = smc2.Context(self.model, self.opts, S, N, w.M, w.T_len, w.T_max, device=device)
        f64 = dict(dtype=torch.float64, device=self.dev)

        def pop():
            return dict(theta=torch.zeros((S, N, D), **f64), logpost=torch.zeros((S, N), **f64),
                        grad_logpost=torch.zeros((S, N, D), **f64),
                        loglik=torch.zeros((S, N), **f64), logw=torch.zeros((S, N), **f64))
        self.cur, self.prev = pop(), pop()
        self.p_prev = torch.zeros((S, N, D), **f64)
        self.y = torch.tensor(w.y, **f64).contiguous()
        self.iteration = torch.ones(1, dtype=torch.int32, device=self.dev)
        self.anc = torch.zeros((S, N), dtype=torch.int32, device=self.dev)
        self.ess = torch.zeros(S, **f64)
        self.estimate = torch.zeros((S, 2, D), **f64)
        self.recycle = torch.zeros((S, 1 + 4 * D), **f64)
        self.resampled = torch.zeros(S, dtype=torch.int32, device=self.dev)
        self._cur_c = smc2.population(**self.cur)
        self._prev_c = smc2.population(**self.prev)
        self.graph = None
        self.k = 0

    # -- the three calls of one iteration ------------------------------------------------------
    def _pf(self, stream=None):
        self.ctx.pf(self.cur["theta"], self.y, self.seed, self.iteration, self.cur["loglik"],
                    self.cur["grad_logpost"], stream=stream)

    def _reweight(self, first, stream=None):
        w = self.w
        smc2.smc2_reweight_resample(self.ctx.h, self.model, w.S, w.N, self.gamma,
                                    self.random_walk, self._cur_c,
                                    None if first else self._prev_c,
                                    None if first else self.p_prev, int(first), self.seed,
                                    self.iteration, 1, self.anc, self.ess, self.resampled,
                                    self.estimate, self.recycle, stream=stream)

    def _move(self, stream=None):
        w = self.w
        smc2.smc2_langevin_move(self.ctx.h, self.model, w.S, w.N, self.gamma, self.random_walk,
                                self.prev["theta"], self.prev["grad_logpost"], self.seed,
                                self.iteration, self.cur["theta"], self.p_prev, stream=stream)

    def _carry(self):
        for key in self.cur:
            self.prev[key].copy_(self.cur[key])

    def first_iteration(self):
        """k = 1: theta ~ prior, filter, weights = likelihood, normalise, ESS, resample."""
        w = self.w
        self.iteration.fill_(1)
        self.recycle.zero_()
        smc2.smc2_prior_init(self.ctx.h, self.model, w.S, w.N, self.seed, self.cur["theta"])
        self._pf()
        self._reweight(first=True)
        self._carry()
        self.k = 1

    def next_iteration(self):
        """k >= 2, eager: move, filter, reweight/resample, carry the population forward."""
        self._move()
        self._pf()
        self._reweight(first=False)
        self._carry()
        self.k += 1

    def capture(self, warmup=True):
        """Capture one k >= 2 iteration into a HIP graph (call after first_iteration)."""
        s = torch.cuda.Stream(device=self.dev)
        s.wait_stream(torch.cuda.current_stream())
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=s):
            self._move(stream=s)
            self._pf(stream=s)
            self._reweight(first=False, stream=s)
            for key in self.cur:
                self.prev[key].copy_(self.cur[key])
        torch.cuda.current_stream().wait_stream(s)

    def replay(self):
        self.graph.replay()
        self.k += 1

    def snapshot(self):
        c = self.cur
        return dict(theta=c["theta"].cpu().numpy(), loglik=c["loglik"].cpu().numpy(),
                    logw=c["logw"].cpu().numpy(), ess=self.ess.cpu().numpy(),
                    resampled=self.resampled.cpu().numpy(), anc=self.anc.cpu().numpy(),
                    estimate=self.estimate.cpu().numpy())

    def recycled_estimate(self):
        """Recycled E[theta], E[theta^2] over the iterations so far (Sec. III-C), [S][2][D], as
        the reweighting kernel left them in the recycle rows."""
        D = self.w.D
        return self.recycle[:, 1 + 2 * D:].cpu().numpy().reshape(-1, 2, D)

    def close(self):
        self.graph = None
        self.ctx.close()


def run_smc2(w, K=None, record=True, use_graph=False, **kw):
    """Run K iterations; with record=True also returns the pre-resampling records per k."""
    K = int(w.K if K is None else K)
    run = SMC2Run(w, **kw)
    recs = []

    for k in range(1, K + 1):
        if record:
            recs.append(_iteration_recorded(run, k))
        elif k == 1:
            run.first_iteration()
        elif use_graph:
            if run.graph is None:
                run.capture()
            run.replay()
        else:
            run.next_iteration()
    out = None
    if record:
        out = Records(**{f: np.stack([r[f] for r in recs]) for f in Records.__dataclass_fields__})
    return run, out


def _iteration_recorded(run, k):
    """One eager iteration; returns the proposed theta with its filter outputs (before the
    outer resampling permutes them), the weights, ESS and ancestors after it, and the inputs
    the reweighting step read (previous population and the move's velocities)."""
    w = run.w
    prev = {key: v.cpu().numpy() for key, v in run.prev.items()}
    if k == 1:
        run.iteration.fill_(1)
        smc2.smc2_prior_init(run.ctx.h, run.model, w.S, w.N, run.seed, run.cur["theta"])
    else:
        run._move()
    run._pf()
    theta = run.cur["theta"].cpu().numpy()
    loglik = run.cur["loglik"].cpu().numpy()
    grad = run.cur["grad_logpost"].cpu().numpy()
    p_prev = run.p_prev.cpu().numpy()
    run._reweight(first=(k == 1))
    snap = run.snapshot()
    run._carry()
    run.k = k
    return dict(theta=theta, loglik=loglik, grad=grad, logw=snap["logw"], ess=snap["ess"],
                resampled=snap["resampled"], anc=snap["anc"], estimate=snap["estimate"],
                prev_theta=prev["theta"],
                prev_logpost=prev["logpost"], prev_grad_logpost=prev["grad_logpost"],
                prev_logw=prev["logw"], p_prev=p_prev)


def pilot_gamma(w, candidates=(0.01, 0.02, 0.04, 0.085, 0.175), K=10, random_walk=0, **kw):
    """Step-size pilot as the paper chose its step sizes (Sec. IV-A: several runs over a range
    of step sizes, the best kept): a K-iteration run per candidate, scored by the mean ESS over
    the iterations (the data-generating parameters are unknown in use).  Returns
    (best gamma, {gamma: mean ESS / N})."""
    scores = {}
    for g in candidates:
        run, rec = run_smc2(w, K=K, random_walk=random_walk, gamma=g, **kw)
        run.close()
        scores[float(g)] = float(np.mean(rec.ess)) / w.N
    best = max(scores, key=scores.get)
    return best, scores


def mse_per_iteration(rec, theta_true, s=0):
    """Squared error of each iteration's realised E[theta] against reference parameters,
    averaged over the D components ([K])."""
    return np.mean((rec.estimate[:, s, 0, :] - np.asarray(theta_true)) ** 2, axis=1)
