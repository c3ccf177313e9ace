"""Pins of the oracle's CRN particle filter and its gradient.

Each test ties the oracle to something other than itself: the Kalman filter's exact likelihood
(itself pinned to scipy's joint Gaussian density), brute force on tiny inputs, the paper's
resampling index formula (App. B), invariants of normalised weights and ESS (Sec. II), and, for
the gradient, an independent differentiation mechanism (complex step) and finite differences
with the random numbers held fixed (Sec. II-A).
"""
import numpy as np
import pytest
from scipy import stats

from paper_2407_17296_amd import synth


def _model(oracle, w):
    return oracle.Model(w.kind, w.d, w.D, w.prior_mu, w.prior_sd)


def _y(w, s=0):
    return w.y[s, :w.T_len[s]]


# ---------------------------------------------------------------- Kalman pinned to scipy ----

def _lg_joint_cov(a, sx, sy, T):
    """Covariance of y_{1:T} of the 1-D LG model with x_0 ~ N(0,1), written from its moments."""
    var_x = np.zeros(T + 1)
    var_x[0] = 1.0
    for t in range(1, T + 1):
        var_x[t] = a * a * var_x[t - 1] + sx * sx
    C = np.zeros((T, T))
    for s in range(1, T + 1):
        for t in range(1, T + 1):
            lo, hi = min(s, t), max(s, t)
            C[s - 1, t - 1] = a ** (hi - lo) * var_x[lo]
    return C + sy * sy * np.eye(T)


@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_kalman_matches_joint_gaussian(oracle, T):
    rng = np.random.default_rng(T)
    m = oracle.Model(oracle.LG1D, 1, 3)
    for _ in range(5):
        th = np.array([rng.uniform(-1.2, 1.2), rng.normal(0, 0.5), rng.normal(0, 0.5)])
        y = rng.normal(size=T)
        C = _lg_joint_cov(th[0], np.exp(th[1]), np.exp(th[2]), T)
        want = stats.multivariate_normal(np.zeros(T), C).logpdf(y)
        ll, _ = oracle.kalman(m, th, y)
        assert ll == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_kalman_diag_is_sum_of_scalar_filters(oracle):
    rng = np.random.default_rng(3)
    d, T = 3, 4
    m = oracle.Model(oracle.LG_DIAG, d, d + 2)
    th = np.concatenate([rng.uniform(0.5, 0.95, d), [0.1, -0.4]])
    y = rng.normal(size=(T, d))
    want = sum(stats.multivariate_normal(np.zeros(T), _lg_joint_cov(th[q], np.exp(th[d]),
                                                                    np.exp(th[d + 1]), T)).logpdf(y[:, q])
               for q in range(d))
    ll, _ = oracle.kalman(m, th, y)
    assert ll == pytest.approx(want, rel=1e-12)


def test_kalman_score_matches_fd_of_joint_gaussian(oracle):
    rng = np.random.default_rng(4)
    T = 4
    m = oracle.Model(oracle.LG1D, 1, 3)
    th = np.array([0.7, 0.2, -0.3])
    y = rng.normal(size=T)

    def lj(t):
        return stats.multivariate_normal(np.zeros(T), _lg_joint_cov(t[0], np.exp(t[1]), np.exp(t[2]), T)).logpdf(y)

    h = 1e-6
    fd = np.array([(lj(th + h * e) - lj(th - h * e)) / (2 * h) for e in np.eye(3)])
    _, g = oracle.kalman(m, th, y)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7)


# --------------------------------------------------------- likelihood: brute force, Kalman ----

def test_T1_is_log_mean_of_likelihoods(oracle):
    """T = 1: no resampling happens (never at t = T), so l = log (1/M) sum_j g(y_1 | x_1^j)."""
    M, seed, k, fid = 257, 42, 3, 9
    m = oracle.Model(oracle.LG1D, 1, 3)
    th = np.array([0.6, -0.2, 0.3])
    y = np.array([[0.4]])
    x1 = []
    for j in range(M):
        x0 = oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.INIT_NORMAL), 0, j)
        e1 = oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.STEP_NORMAL), 1, j)
        x1.append(th[0] * x0 + np.exp(th[1]) * e1)
    g = stats.norm(np.array(x1), np.exp(th[2])).logpdf(0.4)
    want = np.log(np.mean(np.exp(g)))
    r = oracle.pf(m, th, y, M, seed, k, fid)
    assert r["loglik"] == pytest.approx(want, rel=1e-13)


def test_M1_is_single_path_likelihood(oracle):
    """M = 1 never resamples (ESS = 1 is not below M/2): l = sum_t log g(y_t | x_t) on one path."""
    w = synth.make(3, T=30)
    m = _model(oracle, w)
    th = np.array([0.3, -0.1])
    seed, k, fid = 5, 1, 0
    x = oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.INIT_NORMAL), 0, 0)
    ll = 0.0
    for t in range(1, 31):
        e = oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.STEP_NORMAL), t, 0)
        x = x / 2 + 25 * x / (1 + x * x) + 8 * np.cos(1.2 * t) + np.exp(th[0]) * e
        ll += stats.norm(x * x / 20, np.exp(th[1])).logpdf(w.y[0, t - 1, 0])
    r = oracle.pf(m, th, _y(w), 1, seed, k, fid, want_trace=True)
    assert r["flags"].sum() == 0
    assert r["loglik"] == pytest.approx(ll, rel=1e-12)


def test_M1_stochastic_volatility_single_path(oracle):
    """The SV model on one path: x_0 from the stationary N(mu, s^2 / (1 - phi^2)), x_t = mu +
    phi (x_{t-1} - mu) + s e_t, y_t ~ N(0, exp(x_t)) (y = exp(x/2) w), with theta = (mu,
    atanh phi, log s); the filter's estimate with M = 1 is that path's log-likelihood."""
    w = synth.make(4, S=1, T=60)
    m = _model(oracle, w)
    th = np.array([-0.8, np.arctanh(0.9), np.log(0.3)])
    mu, phi, sd = th[0], np.tanh(th[1]), np.exp(th[2])
    seed, k, fid = 11, 2, 5
    x = mu + sd / np.sqrt(1 - phi * phi) * oracle.lib().orc_filter_normal(
        seed, fid, oracle.c3(k, oracle.INIT_NORMAL), 0, 0)
    ll = 0.0
    T = int(w.T_len[0])
    for t in range(1, T + 1):
        e = oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.STEP_NORMAL), t, 0)
        x = mu + phi * (x - mu) + sd * e
        ll += stats.norm(0.0, np.exp(x / 2)).logpdf(w.y[0, t - 1, 0])
    r = oracle.pf(m, th, _y(w), 1, seed, k, fid, want_trace=True)
    assert r["flags"].sum() == 0
    assert r["loglik"] == pytest.approx(ll, rel=1e-12)


def test_T1_stochastic_volatility_is_log_mean_of_likelihoods(oracle):
    """T = 1 for the SV model: l = log (1/M) sum_j N(y_1; 0, exp(x_1^j)) over the M particles
    drawn from the stationary law and moved one step."""
    w = synth.make(4, S=1, T=1)
    m = _model(oracle, w)
    th = np.array([0.4, np.arctanh(0.7), np.log(0.5)])
    mu, phi, sd = th[0], np.tanh(th[1]), np.exp(th[2])
    M, seed, k, fid = 300, 8, 4, 2
    lg = []
    for j in range(M):
        x0 = mu + sd / np.sqrt(1 - phi * phi) * oracle.lib().orc_filter_normal(
            seed, fid, oracle.c3(k, oracle.INIT_NORMAL), 0, j)
        x1 = mu + phi * (x0 - mu) + sd * oracle.lib().orc_filter_normal(
            seed, fid, oracle.c3(k, oracle.STEP_NORMAL), 1, j)
        lg.append(stats.norm(0.0, np.exp(x1 / 2)).logpdf(w.y[0, 0, 0]))
    want = np.log(np.mean(np.exp(np.array(lg))))
    r = oracle.pf(m, th, _y(w), M, seed, k, fid)
    assert r["loglik"] == pytest.approx(want, rel=1e-12)


def test_M1_diagonal_16_dimensional_single_path(oracle):
    """The 16-dimensional diagonal LG model on one path: x_0 ~ N(0, I), x_t[q] = A_qq x_{t-1}[q]
    + sx e_t[q], y_t[q] ~ N(x_t[q], sy^2), component q of slot j drawn as element 16 j + q of the
    step's noise; with M = 1 the estimate is that path's log-likelihood."""
    w = synth.make(2, T=15)
    m = _model(oracle, w)
    rng = np.random.default_rng(3)
    th = np.concatenate([rng.uniform(0.5, 0.95, 16), [np.log(0.8), np.log(0.6)]])
    seed, k, fid = 13, 2, 1
    nrm = lambda c, t, g: oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, c), t, g)
    x = np.array([nrm(oracle.INIT_NORMAL, 0, q) for q in range(16)])
    ll = 0.0
    for t in range(1, 16):
        e = np.array([nrm(oracle.STEP_NORMAL, t, q) for q in range(16)])
        x = th[:16] * x + np.exp(th[16]) * e
        ll += stats.norm(x, np.exp(th[17])).logpdf(w.y[0, t - 1]).sum()
    r = oracle.pf(m, th, _y(w), 1, seed, k, fid, want_trace=True)
    assert r["flags"].sum() == 0
    assert r["loglik"] == pytest.approx(ll, rel=1e-12)


def test_diagonal_16_dimensional_estimate_is_unbiased(oracle):
    """E[p_hat] = p for the 16-dimensional model against its Kalman likelihood, and the estimate
    sits at the Kalman value.  The parameters (sx = 0.5, sy = 3) keep the bootstrap weights
    spread over many particles: at the workload's own (sx = 1, sy = 0.5) the log-weights of 16
    components differ by tens of nats, and exp(l_hat - l) is too skewed for a 60-seed mean."""
    w = synth.make(2, T=5)
    m = _model(oracle, w)
    th = np.concatenate([w.theta_true[:16], [np.log(0.5), np.log(3.0)]])
    lkf, _ = oracle.kalman(m, th, _y(w))
    ll = np.array([oracle.pf(m, th, _y(w), 1024, 500 + s, 1, 0, want_grad=False)["loglik"]
                   for s in range(60)])
    r = np.exp(ll - lkf)
    se = r.std(ddof=1) / np.sqrt(len(r))
    assert abs(r.mean() - 1.0) < 4 * se + 1e-3
    assert abs(ll.mean() - lkf) < 0.05  # measured: 0.006 (sd of l_hat 0.08)


def test_unbiased_likelihood_estimate(oracle):
    """E[p_hat] = p (eq. likelihood_pf_ is unbiased): the seed-mean of exp(l_hat - l_KF) -> 1."""
    w = synth.make(0, T=20)
    m = _model(oracle, w)
    th = w.theta_true
    lkf, _ = oracle.kalman(m, th, _y(w))
    r = np.array([np.exp(oracle.pf(m, th, _y(w), 512, 1000 + s, 1, 0, want_grad=False)["loglik"] - lkf)
                  for s in range(80)])
    se = r.std(ddof=1) / np.sqrt(len(r))
    assert abs(r.mean() - 1.0) < 4 * se + 1e-3


def test_loglik_converges_to_kalman(oracle):
    w = synth.make(0)
    m = _model(oracle, w)
    th = w.theta_true
    lkf, _ = oracle.kalman(m, th, _y(w))
    err = {}
    for M in (64, 4096):
        err[M] = np.mean([abs(oracle.pf(m, th, _y(w), M, 7 + s, 1, 0, want_grad=False)["loglik"] - lkf)
                          for s in range(8)])
    # the bootstrap filter's error here is about 12 / sqrt(M) (T = 50, sy = 0.5)
    assert err[4096] < 0.4
    assert err[4096] < err[64] / 4  # about M^-1/2: a factor 8 from M = 64 to 4096


# ----------------------------------------------------------------- gradient pins ----

CASES = [(0, None), (3, 40), (4, 60), (2, 20)]


@pytest.mark.parametrize("index,T", CASES)
@pytest.mark.parametrize("resampler", [0, 1])
def test_tangent_equals_complex_step(oracle, index, T, resampler):
    """Forward tangent (App. A) == complex-step derivative of the same filter, with every
    decision taken on real parts; the ancestry must be identical for the comparison to hold."""
    w = synth.make(index, T=T)
    m = _model(oracle, w)
    rng = np.random.default_rng(index)
    M = 64 if w.d == 1 else 16
    th = w.theta_true + 0.1 * rng.standard_normal(w.D)
    r = oracle.pf(m, th, _y(w), M, w.seed, 2, 5, resampler=resampler, want_trace=True)
    assert r["flags"].sum() > 0  # resampling is exercised
    for p in range(w.D):
        ll, dl, anc = oracle.pf_complex_step(m, th, _y(w), M, w.seed, 2, 5, p, resampler=resampler)
        assert np.array_equal(anc, r["ancestors"])
        assert ll == pytest.approx(r["loglik"], rel=1e-14)
        assert dl == pytest.approx(r["grad"][p], rel=1e-11, abs=1e-11 * (1 + abs(r["loglik"])))


@pytest.mark.parametrize("index,T", [(0, None), (3, 30), (4, 40)])
def test_tangent_matches_central_differences_with_fixed_ancestry(oracle, index, T):
    """Central differences with the random numbers fixed (CRN), used only where the ancestry at
    theta +- h is identical to that at theta (resampling is piecewise constant in theta)."""
    w = synth.make(index, T=T)
    m = _model(oracle, w)
    th = w.theta_true.copy()
    M = 32
    r = oracle.pf(m, th, _y(w), M, w.seed, 1, 3, want_trace=True)
    h = 1e-7
    checked = 0
    for p in range(w.D):
        e = np.zeros(w.D)
        e[p] = h
        rp = oracle.pf(m, th + e, _y(w), M, w.seed, 1, 3, want_grad=False, want_trace=True)
        rm = oracle.pf(m, th - e, _y(w), M, w.seed, 1, 3, want_grad=False, want_trace=True)
        if not (np.array_equal(rp["ancestors"], r["ancestors"]) and
                np.array_equal(rm["ancestors"], r["ancestors"])):
            continue
        fd = (rp["loglik"] - rm["loglik"]) / (2 * h)
        assert fd == pytest.approx(r["grad"][p], rel=2e-5, abs=2e-5)
        checked += 1
    assert checked >= 1


def test_score_converges_to_kalman_score_without_resampling(oracle):
    """With resampling switched off the CRN-PF score is the gradient of an importance-sampling
    estimate whose limit is the exact score."""
    w = synth.make(0, T=3)
    m = _model(oracle, w)
    th = w.theta_true
    _, gkf = oracle.kalman(m, th, _y(w))
    g = np.mean([oracle.pf(m, th, _y(w), 32768, 11 + s, 1, 0, ess_frac=0.0)["grad"]
                 for s in range(2)], axis=0)
    assert np.allclose(g, gkf, atol=0.05 * (1 + np.abs(gkf)))


def test_resampling_reports_the_known_bias(oracle):
    """With resampling on, the CRN-PF score drops the derivative of the resampling index
    (App. B: d kappa/d theta = 0 almost surely), which biases it (the paper says so in Sec. I).
    Reported, not asserted away: the gap to the Kalman score stays finite and does not vanish
    for the scale parameter as M grows."""
    w = synth.make(0)
    m = _model(oracle, w)
    th = w.theta_true
    _, gkf = oracle.kalman(m, th, _y(w))
    g = oracle.pf(m, th, _y(w), 8192, 3, 1, 0)["grad"]
    assert np.all(np.isfinite(g))
    assert abs(g[1] - gkf[1]) > 1.0  # the bias on d/d log sx is large and visible


# ----------------------------------------------------------- resampling rule and invariants ----

def test_resampling_index_equals_paper_counting_formula(oracle):
    """kappa_i = sum_j [nu_i > c_j] (App. B) with c the normalised cumulative weights; the
    sampled particle is kappa_i (1-based).  Weights are dyadic so every comparison is exact."""
    rng = np.random.default_rng(8)
    for M in (1, 2, 7, 64, 300):
        w = rng.integers(0, 9, size=M).astype(float)
        if w.sum() == 0:
            w[0] = 1
        w = w / 8.0
        nu = (rng.integers(0, 2**20, size=M) + 1) / 2.0**20
        c = np.cumsum(w) / w.sum()
        kappa = np.array([np.sum(n > c[:-1]) + 1 if M > 1 else 1 for n in nu])
        # ties and the M-1 cap: lower bound over P_m >= nu * P_{M-1}
        a = oracle.resample_lower_bound(w, nu)
        kap2 = np.array([min(np.sum(n > c), M - 1) + 1 for n in nu])
        assert np.array_equal(a + 1, kap2)
        assert np.array_equal(kappa, kap2)
        assert np.all(w[a] > 0)  # never selects a zero-weight particle


def test_systematic_offspring_counts_and_order(oracle):
    rng = np.random.default_rng(9)
    for M in (16, 512):
        w = rng.exponential(size=M) ** 3
        nu = 0.37
        a = oracle.resample_lower_bound(w, (np.arange(M) + nu) / M)
        assert np.all(np.diff(a) >= 0)
        counts = np.bincount(a, minlength=M)
        assert counts.sum() == M
        MW = M * w / w.sum()
        assert np.all((counts == np.floor(MW)) | (counts == np.ceil(MW)))


def test_multinomial_offspring_counts_are_multinomial(oracle):
    rng = np.random.default_rng(10)
    M = 8
    w = np.array([1, 2, 3, 4, 0.5, 0.25, 5, 0.25])
    total = np.zeros(M)
    reps = 4000
    for _ in range(reps):
        nu = 1.0 - rng.random(M)  # (0, 1]
        total += np.bincount(oracle.resample_lower_bound(w, nu), minlength=M)
    expected = reps * M * w / w.sum()
    chi2 = np.sum((total - expected) ** 2 / expected)
    assert stats.chi2(M - 1).sf(chi2) > 1e-4


def test_resampling_policy_flags(oracle):
    w = synth.make(0)
    m = _model(oracle, w)
    th = w.theta_true
    T = w.T_len[0]
    always = oracle.pf(m, th, _y(w), 64, 1, 1, 0, ess_frac=2.0, want_trace=True)
    never = oracle.pf(m, th, _y(w), 64, 1, 1, 0, ess_frac=0.0, want_trace=True)
    adaptive = oracle.pf(m, th, _y(w), 64, 1, 1, 0, ess_frac=0.5, want_trace=True)
    assert always["flags"][:-1].all() and always["flags"][-1] == 0  # never at t = T
    assert never["flags"].sum() == 0 and (never["ancestors"] == -1).all()
    assert 0 < adaptive["flags"].sum() < T - 1
    for t in np.nonzero(always["flags"])[0]:
        assert np.all(np.diff(always["ancestors"][t]) >= 0)


def test_nonfinite_inputs_give_minus_inf(oracle):
    w = synth.make(0)
    m = _model(oracle, w)
    r = oracle.pf(m, np.array([np.nan, 0.0, 0.0]), _y(w), 16, 1, 1, 0)
    assert r["loglik"] == -np.inf and np.all(r["grad"] == 0)
    # an observation noise so small that no particle can explain the data
    r = oracle.pf(m, np.array([0.8, 0.0, -400.0]), _y(w), 16, 1, 1, 0)
    assert r["loglik"] == -np.inf and np.all(r["grad"] == 0)


def test_empty_series(oracle):
    m = oracle.Model(oracle.LG1D, 1, 3)
    r = oracle.pf(m, np.zeros(3), np.zeros((0, 1)), 8, 1, 1, 0)
    assert r["loglik"] == 0.0 and np.all(r["grad"] == 0.0)


def test_steps_sum_to_loglik(oracle):
    w = synth.make(4, S=1, T=80)
    m = _model(oracle, w)
    r = oracle.pf(m, w.theta_true, _y(w), 128, 2, 1, 0, want_trace=True)
    assert np.sum(r["s"]) == pytest.approx(r["loglik"], rel=1e-13)
