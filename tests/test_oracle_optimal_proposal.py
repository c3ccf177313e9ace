"""Pins of the oracle's particle filter with the "optimal" proposal of the 1-D LG model
(Sec. IV-A): q(x_t | x_{t-1}, y_t) = N(rho^2 (y_t / sy^2 + a x_{t-1} / sx^2), rho^2) with
1/rho^2 = 1/sx^2 + 1/sy^2, and incremental weight p(y_t | x_{t-1}) = N(y_t; a x_{t-1},
sx^2 + sy^2) (the predictive density; the paper's printed weight is garbled).

Each test ties it to something other than the filter itself: brute force written out from the
two densities above, the Kalman filter's exact likelihood and score, and complex-step and
finite-difference derivatives of the same estimate with the random numbers held fixed.
"""
import numpy as np
import pytest
from scipy import stats

from paper_2407_17296_amd import synth


def _opt(oracle):
    return oracle.Model(oracle.LG1D_OPT, 1, 3)


def _boot(oracle):
    return oracle.Model(oracle.LG1D, 1, 3)


def _proposal(th, xprev, y, e):
    a, vx, vy = th[0], np.exp(2 * th[1]), np.exp(2 * th[2])
    rho2 = 1.0 / (1.0 / vx + 1.0 / vy)
    return rho2 * (y / vy + a * xprev / vx) + np.sqrt(rho2) * e


def _pred_logpdf(th, xprev, y):
    a, vx, vy = th[0], np.exp(2 * th[1]), np.exp(2 * th[2])
    return stats.norm(a * xprev, np.sqrt(vx + vy)).logpdf(y)


def test_T1_is_log_mean_of_predictive_densities(oracle):
    """T = 1: l = log (1/M) sum_j N(y_1; a x_0^j, sx^2 + sy^2) with x_0^j ~ N(0, 1)."""
    M, seed, k, fid = 129, 11, 2, 4
    th = np.array([0.7, -0.3, 0.2])
    x0 = np.array([oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.INIT_NORMAL), 0, j)
                   for j in range(M)])
    want = np.log(np.mean(np.exp(_pred_logpdf(th, x0, -0.6))))
    r = oracle.pf(_opt(oracle), th, np.array([[-0.6]]), M, seed, k, fid)
    assert r["loglik"] == pytest.approx(want, rel=1e-13)


def test_M1_is_single_path_predictive_likelihood(oracle):
    """M = 1: the path moves by the proposal and l = sum_t log N(y_t; a x_{t-1}, sx^2 + sy^2)."""
    w = synth.make(0, T=25)
    th = np.array([0.5, 0.1, -0.4])
    seed, k, fid = 3, 1, 0
    x = oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.INIT_NORMAL), 0, 0)
    ll = 0.0
    for t in range(1, 26):
        y = w.y[0, t - 1, 0]
        ll += _pred_logpdf(th, x, y)
        e = oracle.lib().orc_filter_normal(seed, fid, oracle.c3(k, oracle.STEP_NORMAL), t, 0)
        x = _proposal(th, x, y, e)
    r = oracle.pf(_opt(oracle), th, w.y[0, :25], 1, seed, k, fid, want_trace=True)
    assert r["flags"].sum() == 0
    assert r["loglik"] == pytest.approx(ll, rel=1e-12)


def test_unbiased_and_lower_variance_than_bootstrap(oracle):
    """E[p_hat] = p for the optimal proposal too, and its estimate varies less than the
    bootstrap filter's at the same M (the reason the paper uses it)."""
    w = synth.make(0, T=20)
    th = w.theta_true
    y = w.y[0, :20]
    lkf, _ = oracle.kalman(_opt(oracle), th, y)
    lkf_b, _ = oracle.kalman(_boot(oracle), th, y)
    assert lkf == lkf_b
    lo = np.array([oracle.pf(_opt(oracle), th, y, 64, 500 + s, 1, 0, want_grad=False)["loglik"]
                   for s in range(80)])
    lb = np.array([oracle.pf(_boot(oracle), th, y, 64, 500 + s, 1, 0, want_grad=False)["loglik"]
                   for s in range(80)])
    r = np.exp(lo - lkf)
    assert abs(r.mean() - 1.0) < 4 * r.std(ddof=1) / np.sqrt(len(r)) + 1e-3
    assert lo.std() < 0.5 * lb.std()


@pytest.mark.parametrize("resampler", [0, 1])
def test_tangent_equals_complex_step(oracle, resampler):
    w = synth.make(1, T=60)
    th = w.theta_true + np.array([0.03, -0.05, 0.04])
    m = _opt(oracle)
    r = oracle.pf(m, th, w.y[0, :60], 64, w.seed, 2, 5, resampler=resampler, ess_frac=0.9,
                  want_trace=True)
    assert r["flags"].sum() > 0
    for p in range(3):
        ll, dl, anc = oracle.pf_complex_step(m, th, w.y[0, :60], 64, w.seed, 2, 5, p,
                                             resampler=resampler, ess_frac=0.9)
        assert np.array_equal(anc, r["ancestors"])
        assert ll == pytest.approx(r["loglik"], rel=1e-14)
        assert dl == pytest.approx(r["grad"][p], rel=1e-11, abs=1e-11 * (1 + abs(r["loglik"])))


def test_tangent_matches_central_differences_with_fixed_ancestry(oracle):
    w = synth.make(0)
    th = w.theta_true.copy()
    m = _opt(oracle)
    r = oracle.pf(m, th, w.y[0], 32, w.seed, 1, 3, ess_frac=0.9, want_trace=True)
    h, checked = 1e-7, 0
    for p in range(3):
        e = np.zeros(3)
        e[p] = h
        rp = oracle.pf(m, th + e, w.y[0], 32, w.seed, 1, 3, ess_frac=0.9, want_grad=False,
                       want_trace=True)
        rm = oracle.pf(m, th - e, w.y[0], 32, w.seed, 1, 3, ess_frac=0.9, want_grad=False,
                       want_trace=True)
        if not (np.array_equal(rp["ancestors"], r["ancestors"]) and
                np.array_equal(rm["ancestors"], r["ancestors"])):
            continue
        fd = (rp["loglik"] - rm["loglik"]) / (2 * h)
        assert fd == pytest.approx(r["grad"][p], rel=2e-5, abs=2e-5)
        checked += 1
    assert checked >= 1


def test_score_converges_to_kalman_score_without_resampling(oracle):
    w = synth.make(0, T=3)
    th = w.theta_true
    _, gkf = oracle.kalman(_opt(oracle), th, w.y[0, :3])
    g = np.mean([oracle.pf(_opt(oracle), th, w.y[0, :3], 32768, 21 + s, 1, 0, ess_frac=0.0)["grad"]
                 for s in range(2)], axis=0)
    assert np.allclose(g, gkf, atol=0.03 * (1 + np.abs(gkf)))
