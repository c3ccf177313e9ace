"""Pins of the oracle's SMC^2 outer step (paper Sec. III).

The Langevin proposal SMC1 and its L-kernel are pinned against the Metropolis-adjusted Langevin
ratio written with scipy's Gaussian density and against the reversibility of the one-step
leapfrog map; the whole sampler is pinned on a problem with no data, whose posterior is the
prior (a closed form), and on invariants of its weights.
"""
import numpy as np
import pytest
from scipy import stats

from paper_2407_17296_amd import synth


def test_lkernel_ratio_is_the_langevin_proposal_ratio(oracle):
    """With the velocity form (C12), L(theta_{k-1}|theta_k)/q(theta_k|theta_{k-1}) equals
    N(theta_{k-1}; theta_k + F(theta_k), G) / N(theta_k; theta_{k-1} + F(theta_{k-1}), G)."""
    rng = np.random.default_rng(0)
    for D in (1, 3, 18):
        for gamma in (0.01, 0.085, 0.5):
            th0 = rng.normal(size=D)
            g0 = rng.normal(size=D) * 3
            xi = rng.normal(size=D)
            th1, p0 = oracle.langevin_move(gamma, th0, g0, xi)
            g1 = rng.normal(size=D) * 3
            G = gamma * gamma
            fwd = stats.norm(th0 + 0.5 * G * g0, gamma).logpdf(th1).sum()
            bwd = stats.norm(th1 + 0.5 * G * g1, gamma).logpdf(th0).sum()
            got = oracle.lkernel_log_ratio(gamma, g0, g1, p0)
            assert got == pytest.approx(bwd - fwd, rel=1e-9, abs=1e-9)


def test_langevin_move_mean_and_spread(oracle):
    """SMC1: theta_k ~ N(theta_{k-1} + (gamma^2/2) grad log pi, gamma^2 I) (Sec. III-D)."""
    rng = np.random.default_rng(1)
    D, gamma, n = 2, 0.3, 20000
    th0, g0 = np.array([0.5, -1.0]), np.array([2.0, -4.0])
    out = np.array([oracle.langevin_move(gamma, th0, g0, rng.normal(size=D))[0] for _ in range(n)])
    mean = th0 + 0.5 * gamma**2 * g0
    assert np.all(np.abs(out.mean(0) - mean) < 5 * gamma / np.sqrt(n))
    assert np.all(np.abs(out.std(0) - gamma) < 5 * gamma / np.sqrt(2 * n))


def test_leapfrog_reversibility(oracle):
    """The one-step map from (theta_k, -p_k) returns to (theta_{k-1}, -p_{k-1}) (Sec. III-E)."""
    rng = np.random.default_rng(2)
    D, gamma = 4, 0.2
    A = rng.normal(size=(D, D))
    A = A @ A.T + D * np.eye(D)

    def grad(t):
        return -A @ t

    th0, xi = rng.normal(size=D), rng.normal(size=D)
    th1, p0 = oracle.langevin_move(gamma, th0, grad(th0), xi)
    pk = p0 + 0.5 * gamma**2 * (grad(th0) + grad(th1))
    back, p_back = oracle.langevin_move(gamma, th1, grad(th1), -pk / gamma)
    assert np.allclose(back, th0, atol=1e-12)
    assert np.allclose(p_back + 0.5 * gamma**2 * (grad(th1) + grad(back)), -p0, atol=1e-12)


def test_log_prior_is_gaussian(oracle):
    m = oracle.Model(oracle.LG1D, 1, 3, prior_mu=[0.1, -0.2, 0.3], prior_sd=[1.0, 2.0, 0.5])
    th = np.array([0.4, 0.7, -0.1])
    v, g = oracle.log_prior(m, th)
    assert v == pytest.approx(stats.norm([0.1, -0.2, 0.3], [1.0, 2.0, 0.5]).logpdf(th).sum(), rel=1e-14)
    assert np.allclose(g, -(th - [0.1, -0.2, 0.3]) / np.array([1.0, 2.0, 0.5]) ** 2)


@pytest.mark.slow
@pytest.mark.parametrize("proposal", [1, 0])
def test_no_data_posterior_is_the_prior(oracle, proposal):
    """T = 0: pi = prior N(0, I); the filter returns l = 0 and grad = 0, so SMC^2 with the
    Langevin proposal and its L-kernel (proposal 1), or with the random walk and its symmetric
    kernel (proposal 0, SMC0), must keep the prior's moments."""
    m = oracle.Model(oracle.LG1D, 1, 3)
    N, K, gamma = 4096, 6, 0.7
    rec = oracle.smc2_run(m, np.zeros((0, 1)), N, 4, K, gamma, seed=123, proposal=proposal)
    assert np.all(rec["loglik"] == 0.0)
    for k in range(K):
        lw = rec["logw"][k]
        W = np.exp(lw - lw.max())
        W /= W.sum()
        th = rec["theta"][k]
        mean = W @ th
        var = W @ (th - mean) ** 2
        ess = 1.0 / np.sum(W**2)
        assert rec["ess"][k] == pytest.approx(ess, rel=1e-10)
        assert np.all(np.abs(mean) < 6 / np.sqrt(ess))
        assert np.all(np.abs(var - 1.0) < 6 * np.sqrt(2 / ess))


def test_smc2_records_and_invariants(oracle):
    w = synth.make(0)
    m = oracle.Model(w.kind, w.d, w.D, w.prior_mu, w.prior_sd)
    rec = oracle.smc2_run(m, w.y[0], w.N, w.M, w.K, w.gamma, w.seed)
    rec2 = oracle.smc2_run(m, w.y[0], w.N, w.M, w.K, w.gamma, w.seed)
    for key in rec:
        assert np.array_equal(rec[key], rec2[key])  # deterministic given the seed
    assert np.all((rec["ess"] >= 1 - 1e-9) & (rec["ess"] <= w.N + 1e-9))
    # k = 1: weights are the likelihoods (q_1 = prior)
    assert np.array_equal(rec["logw"][0], rec["loglik"][0])
    # resampled iterations carry ancestors in range, others the identity
    for k in range(w.K):
        if rec["resampled"][k]:
            assert rec["ess"][k] < w.N / 2
            assert np.all(np.diff(rec["anc"][k]) >= 0)
        else:
            assert np.array_equal(rec["anc"][k], np.arange(w.N))
    # the first iteration's theta are prior draws from the PRIOR_NORMAL stream
    z = np.array([[oracle.lib().orc_normal(w.seed, 0xFFFFFFFF, i, oracle.c3(1, oracle.PRIOR_NORMAL), p)
                   for p in range(w.D)] for i in range(w.N)])
    assert np.array_equal(rec["theta"][0], z)
    # the estimate of the PF at each recorded theta is the PF of that theta
    r = oracle.pf(m, rec["theta"][3][5], w.y[0], w.M, w.seed, 4, 5)
    assert r["loglik"] == rec["loglik"][3][5]
    assert np.array_equal(r["grad"], rec["grad"][3][5])


def test_smc2_reaches_the_posterior_mode(oracle):
    """On the 1-D LG workload the sampler's weighted mean reaches the region of the exact
    posterior's mode (log posterior from the Kalman filter plus the N(0, I) prior), a qualitative
    check of the whole outer loop.  With T = 50 the posterior mode, not the data-generating
    parameter, is the target."""
    from scipy.optimize import minimize
    w = synth.make(0)
    m = oracle.Model(w.kind, w.d, w.D, w.prior_mu, w.prior_sd)

    def logpost(t):
        return oracle.kalman(m, t, w.y[0])[0] - 0.5 * np.sum(np.asarray(t) ** 2)

    mode = minimize(lambda t: -logpost(t), w.theta_true, method="Nelder-Mead").x
    rec = oracle.smc2_run(m, w.y[0], 128, 128, 15, 0.085, w.seed)
    lw = rec["logw"][-1]
    W = np.exp(lw - lw.max())
    W /= W.sum()
    est = W @ rec["theta"][-1]
    assert logpost(est) > logpost(mode) - 1.5
    assert logpost(est) > logpost(np.zeros(w.D)) + 2.0  # better than the prior mean


# ---- realised estimates and recycling (eqs. realised_estimates, recycling_I,
#      opt_recycling_constant) ------------------------------------------------------------------

def test_realised_estimate_special_cases(oracle):
    """Equal weights give the sample mean and mean square with l = N; a single finite weight
    gives that sample with l = 1; a constant added to every log-weight changes nothing; no
    finite weight gives NaN moments and l = 0."""
    rng = np.random.default_rng(3)
    th = rng.standard_normal((40, 3))
    m, s2, l = oracle.realised_estimate(np.zeros(40), th)
    assert np.allclose(m, th.mean(0), rtol=1e-13) and np.allclose(s2, (th ** 2).mean(0), rtol=1e-13)
    assert l == pytest.approx(40.0, rel=1e-13)
    lw = np.full(40, -np.inf)
    lw[7] = -3.0
    m, s2, l = oracle.realised_estimate(lw, th)
    assert np.array_equal(m, th[7]) and np.allclose(s2, th[7] ** 2) and l == 1.0
    lw = rng.standard_normal(40) * 2
    a = oracle.realised_estimate(lw, th)
    b = oracle.realised_estimate(lw + 123.4, th)
    assert np.allclose(a[0], b[0], rtol=1e-12) and np.allclose(a[1], b[1], rtol=1e-12)
    assert a[2] == pytest.approx(b[2], rel=1e-12)
    w = np.exp(lw - lw.max())
    assert a[2] == pytest.approx(w.sum() ** 2 / (w * w).sum(), rel=1e-13)
    m, s2, l = oracle.realised_estimate(np.full(40, -np.inf), th)
    assert np.all(np.isnan(m)) and l == 0.0


def test_realised_estimate_recovers_an_importance_sampling_target(oracle):
    """Draws from N(0, 1) weighted by N(theta; 1.5, 0.7^2) / N(theta; 0, 1) estimate the mean and
    second moment of N(1.5, 0.7^2): 1.5 and 1.5^2 + 0.49 (a sign or normalisation error in the
    weighting shows up here)."""
    rng = np.random.default_rng(4)
    th = rng.standard_normal((200000, 1))
    lw = stats.norm.logpdf(th[:, 0], 1.5, 0.7) - stats.norm.logpdf(th[:, 0])
    m, s2, l = oracle.realised_estimate(lw, th)
    assert abs(m[0] - 1.5) < 5.0 / np.sqrt(l)
    assert abs(s2[0] - (1.5 ** 2 + 0.49)) < 20.0 / np.sqrt(l)
    assert 0.1 * len(th) < l < len(th)


def test_recycling_constants(oracle):
    """c_k = l_k / sum l: equal l averages the estimates, one nonzero l selects its iteration,
    K = 1 is the identity, and the result is the l-weighted mean."""
    est = np.array([[1.0, -2.0], [3.0, 0.5], [-1.0, 4.0]])
    assert np.allclose(oracle.recycle([2.0, 2.0, 2.0], est), est.mean(0), rtol=1e-14)
    assert np.allclose(oracle.recycle([0.0, 5.0, 0.0], est), est[1], rtol=1e-14)
    assert np.allclose(oracle.recycle([7.0], est[:1]), est[0], rtol=1e-14)
    l = np.array([1.0, 3.0, 6.0])
    assert np.allclose(oracle.recycle(l, est), (l[:, None] * est).sum(0) / l.sum(), rtol=1e-14)


def test_random_walk_move_is_the_smc0_proposal(oracle):
    """SMC0 proposes N(theta, gamma^2 I) (Sec. III-D): over 4096 moves with the move stream's
    normals, (theta_new - theta) / gamma is standard normal (KS), independent of theta, and the
    velocity equals the step."""
    rng = np.random.default_rng(4)
    gamma, N, D = 0.175, 4096, 3
    c3 = oracle.c3(5, oracle.MOVE_NORMAL)
    steps, thetas = [], []
    for i in range(N):
        th = rng.standard_normal(D) * 2.0
        xi = [oracle.lib().orc_normal(99, 0xFFFFFFFF, i, c3, p) for p in range(D)]
        tn, pp = oracle.random_walk_move(gamma, th, xi)
        assert np.array_equal(pp, tn - th) or np.allclose(pp, tn - th, rtol=1e-15, atol=1e-15)
        steps.append((tn - th) / gamma)
        thetas.append(th)
    z, th = np.array(steps), np.array(thetas)
    assert stats.kstest(z.ravel(), "norm").pvalue > 1e-4
    for p in range(D):
        assert abs(np.corrcoef(z[:, p], th[:, p])[0, 1]) < 5 / np.sqrt(N)
