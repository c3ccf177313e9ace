"""Pins of the oracle's SIR model (Sec. IV-B) and of the uniform priors it is sampled under.

The model's infection term, recovery term, noise, initial state and observation are tied to facts
that do not come from the oracle's own formulas:
  - with no infection (beta = 0) the infected count is a Gaussian AR(1) chain observed in Gaussian
    noise, so y_{1:T} is jointly Gaussian and scipy's density is the exact likelihood;
  - with no noise, the whole population infected at the start and no infection possible, the
    infected count decays geometrically: a closed form;
  - with no noise, no recovery and beta = 1, the susceptible fraction squares every day,
    S_t / N = (S_0 / N)^(2^t): a closed form that fixes the infection term's form, its sign in
    both compartments and its scaling by the population;
  - scaling the population, the initial infections, the noise and the observation sd by c scales
    the whole process by c (the infection term is homogeneous of degree one), so the
    log-likelihood of c * y shifts by exactly -T log c;
  - the gradient against the complex-step derivative and central differences of the same filter
    with the random numbers held fixed.
"""
import numpy as np
import pytest
from scipy import stats

from paper_2407_17296_amd import synth

NPOP, I0, VAR, SY = synth.SIR_CONSTANTS


def _sir(oracle, constants=None):
    return oracle.Model(oracle.SIR, 2, 2, np.zeros(2), np.ones(2),
                        prior_kind=[oracle.PRIOR_KIND_UNIFORM] * 2, constants=constants)


def _loglik(oracle, m, theta, y, M=1, seed=5, k=1, fid=0, want_grad=True):
    return oracle.pf(m, theta, np.asarray(y, dtype=float).reshape(-1, 1), M, seed, k, fid,
                     want_grad=want_grad)


def _ar1_joint(a, q, i0, sy, T):
    """Mean and covariance of y_{1:T} when I_t = a I_{t-1} + sqrt(q) v, I_0 = i0 fixed,
    y_t = I_t + sy w: written from the chain's moments."""
    mean = i0 * a ** np.arange(1, T + 1)
    var = np.array([q * sum(a ** (2 * k) for k in range(t)) for t in range(1, T + 1)])
    C = np.empty((T, T))
    for s in range(T):
        for t in range(T):
            lo, hi = min(s, t), max(s, t)
            C[s, t] = a ** (hi - lo) * var[lo]
    return mean, C + sy * sy * np.eye(T)


def test_no_infection_is_a_gaussian_chain(oracle):
    """beta = 0: I_t = (1 - gamma) I_{t-1} + s_e (e_g - e_b), variance 2 s_e^2 per step; the
    filter's estimate at many particles sits at scipy's exact joint-Gaussian log-density."""
    T, gam, i0 = 20, 0.3, 100.0  # many initial infections, so that the decay shows in y
    a, q = 1.0 - gam, 2.0 * VAR
    mean, C = _ar1_joint(a, q, i0, SY, T)
    y = np.random.default_rng(1).multivariate_normal(mean, C)
    exact = stats.multivariate_normal(mean, C).logpdf(y)
    m = _sir(oracle, constants=[NPOP, i0, VAR, SY])
    est = [_loglik(oracle, m, [0.0, gam], y, M=4096, seed=s, want_grad=False)["loglik"]
           for s in range(4)]
    assert abs(np.mean(est) - exact) < 0.02, (np.mean(est), exact)
    # a different recovery rate is measurably worse: the chain's coefficient is 1 - gamma
    mean2, C2 = _ar1_joint(1.0 - 0.6, q, i0, SY, T)
    assert stats.multivariate_normal(mean2, C2).logpdf(y) < exact - 1.0


def test_no_infection_gradient_in_gamma_matches_the_exact_one(oracle):
    """d/d gamma of the exact log-likelihood (central differences of scipy's density) against the
    filter's gradient at many particles; the infection rate's gradient is that of a model in
    which beta multiplies I S / N_pop, finite at beta = 0."""
    T, gam, h, i0 = 20, 0.3, 1e-5, 100.0
    mean, C = _ar1_joint(1.0 - gam, 2.0 * VAR, i0, SY, T)
    y = np.random.default_rng(2).multivariate_normal(mean, C)

    def exact(g):
        mu, Cg = _ar1_joint(1.0 - g, 2.0 * VAR, i0, SY, T)
        return stats.multivariate_normal(mu, Cg).logpdf(y)

    want = (exact(gam + h) - exact(gam - h)) / (2 * h)
    m = _sir(oracle, constants=[NPOP, i0, VAR, SY])
    got = np.mean([_loglik(oracle, m, [0.0, gam], y, M=4096, seed=s)["grad"][1]
                   for s in range(4)])
    assert got == pytest.approx(want, rel=0.05, abs=0.5)


@pytest.mark.parametrize("gam", [0.1, 0.45])
def test_whole_population_infected_decays_geometrically(oracle, gam):
    """No noise, S_0 = 0: no infection can happen and I_t = N (1 - gamma)^t exactly; with y at
    that path every residual is zero and the log-likelihood is T log N(0; 0, s_y^2)."""
    T, npop = 12, 500.0
    m = _sir(oracle, constants=[npop, npop, 0.0, 2.0])
    y = npop * (1.0 - gam) ** np.arange(1, T + 1)
    for beta in (0.0, 0.7):  # beta cannot matter: S stays 0
        out = _loglik(oracle, m, [beta, gam], y, M=8)
        assert out["loglik"] == pytest.approx(T * stats.norm(0, 2.0).logpdf(0.0), rel=1e-12)
        assert out["grad"][0] == 0.0
        assert abs(out["grad"][1]) < 1e-9


@pytest.mark.parametrize("s0_frac", [0.99, 0.7, 0.3])
def test_infection_term_closed_form(oracle, s0_frac):
    """No noise, no recovery, beta = 1: the susceptible fraction u = S/N obeys u_t = u_{t-1}^2
    (the infection term beta I S / N moves I S / N from S to I and S + I stays N), so
    I_t = N (1 - u_0^(2^t)).  Observed exactly, the log-likelihood is T log N(0; 0, s_y^2), and
    moving y off the path by r lowers it by r^2 / (2 s_y^2) per step."""
    T, npop = 6, 800.0
    i0 = npop * (1.0 - s0_frac)
    m = _sir(oracle, constants=[npop, i0, 0.0, 3.0])
    y = npop * (1.0 - s0_frac ** (2.0 ** np.arange(1, T + 1)))
    base = T * stats.norm(0, 3.0).logpdf(0.0)
    assert _loglik(oracle, m, [1.0, 0.0], y, M=4)["loglik"] == pytest.approx(base, rel=1e-11)
    r = np.linspace(-2.0, 2.0, T)
    got = _loglik(oracle, m, [1.0, 0.0], y + r, M=4)["loglik"]
    assert got == pytest.approx(base - np.sum(r * r) / (2 * 9.0), rel=1e-11)


@pytest.mark.parametrize("c", [0.5, 3.0])
def test_population_scaling(oracle, c):
    """Scaling N_pop, I_0, s_e and s_y by c scales every particle path by c under the same random
    numbers (the infection term is homogeneous of degree one), so the filter takes the same
    decisions and log p(c y) = log p(y) - T log c; the gradient is unchanged."""
    w = synth.make(5)
    y = w.y[0, :, 0]
    T = len(y)
    m1 = _sir(oracle)
    mc = _sir(oracle, constants=[c * NPOP, c * I0, c * c * VAR, c * SY])
    for th in ([0.6, 0.3], [0.45, 0.2]):
        a = oracle.pf(m1, th, y.reshape(-1, 1), 64, 9, 2, 3, want_trace=True)
        b = oracle.pf(mc, th, (c * y).reshape(-1, 1), 64, 9, 2, 3, want_trace=True)
        assert np.array_equal(a["ancestors"], b["ancestors"])
        assert b["loglik"] == pytest.approx(a["loglik"] - T * np.log(c), rel=1e-11, abs=1e-9)
        np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-8, atol=1e-8)


def test_default_constants_are_the_papers(oracle):
    """constants = NULL means (N_pop, I_0, s_e^2, s_y) = (763, 1, 0.5, 5)."""
    w = synth.make(5)
    y = w.y[0, :, 0].reshape(-1, 1)
    a = oracle.pf(_sir(oracle), [0.5, 0.25], y, 32, 3, 1, 0)
    b = oracle.pf(_sir(oracle, constants=[763.0, 1.0, 0.5, 5.0]), [0.5, 0.25], y, 32, 3, 1, 0)
    assert a["loglik"] == b["loglik"] and np.array_equal(a["grad"], b["grad"])


@pytest.mark.parametrize("p", [0, 1])
def test_gradient_matches_complex_step(oracle, p):
    """The forward-mode tangent (full 2 x 2 state Jacobian) against the complex-step derivative of
    the same filter, which shares none of the tangent code."""
    w = synth.make(5)
    y = w.y[0, :, 0].reshape(-1, 1)
    m = _sir(oracle)
    for th in ([0.6, 0.3], [0.35, 0.55]):
        g = oracle.pf(m, th, y, 64, 11, 1, 2)["grad"]
        _, dl, _ = oracle.pf_complex_step(m, th, y, 64, 11, 1, 2, p)
        assert g[p] == pytest.approx(dl, rel=1e-9, abs=1e-9)


def test_gradient_matches_central_differences(oracle):
    w = synth.make(5)
    y = w.y[0, :, 0].reshape(-1, 1)
    m = _sir(oracle)
    th, h = np.array([0.55, 0.32]), 1e-7
    out = oracle.pf(m, th, y, 128, 4, 3, 1, want_trace=True)
    for p in range(2):
        e = np.zeros(2)
        e[p] = h
        hi = oracle.pf(m, th + e, y, 128, 4, 3, 1, want_trace=True)
        lo = oracle.pf(m, th - e, y, 128, 4, 3, 1, want_trace=True)
        # the random numbers are common and the ancestors unchanged, so the estimate is smooth
        assert np.array_equal(hi["ancestors"], out["ancestors"])
        assert np.array_equal(lo["ancestors"], out["ancestors"])
        fd = (hi["loglik"] - lo["loglik"]) / (2 * h)
        assert out["grad"][p] == pytest.approx(fd, rel=1e-6)


def test_one_particle_brute_force(oracle):
    """M = 1 never resamples (ESS = 1 = M), so the estimate is the observation density summed
    along the one path its noise drives; the path is rebuilt here from the stream's normals."""
    w = synth.make(5)
    y = w.y[0, :10, 0]
    th = (0.6, 0.3)
    seed, k, fid = 21, 4, 7
    c3 = oracle.c3(k, oracle.STEP_NORMAL)
    S, I = NPOP - I0, I0
    se = np.sqrt(VAR)
    want = 0.0
    for t in range(1, len(y) + 1):
        eb, eg = (oracle.lib().orc_filter_normal(seed, fid, c3, t, g) for g in (0, 1))
        inf = th[0] * I * S / NPOP
        S, I = S - inf + se * eb, I + inf - th[1] * I - se * eb + se * eg
        want += stats.norm(I, SY).logpdf(y[t - 1])
    got = _loglik(oracle, _sir(oracle), th, y, M=1, seed=seed, k=k, fid=fid)["loglik"]
    assert got == pytest.approx(want, rel=1e-12)


# ------------------------------------------------------------------ uniform priors ----------

def test_uniform_log_prior(oracle):
    m = oracle.Model(oracle.SIR, 2, 2, [0.0, 0.2], [1.0, 0.7],
                     prior_kind=[oracle.PRIOR_KIND_UNIFORM] * 2)
    lp, g = oracle.log_prior(m, [0.4, 0.5])
    assert lp == pytest.approx(-np.log(1.0) - np.log(0.5), rel=1e-15)
    assert np.array_equal(g, [0.0, 0.0])
    for th in ([-0.01, 0.5], [0.4, 0.71], [1.2, 0.1]):
        assert oracle.log_prior(m, th)[0] == -np.inf
    # a mixed prior: the normal parameter keeps its Gaussian term and gradient
    mm = oracle.Model(oracle.SIR, 2, 2, [0.0, 1.0], [1.0, 2.0],
                      prior_kind=[oracle.PRIOR_KIND_UNIFORM, oracle.PRIOR_KIND_NORMAL])
    lp, g = oracle.log_prior(mm, [0.5, 2.0])
    assert lp == pytest.approx(stats.norm(1.0, 2.0).logpdf(2.0), rel=1e-14)
    assert g[0] == 0.0 and g[1] == pytest.approx(-0.25, rel=1e-14)


def test_first_iteration_draws_are_uniform(oracle):
    """theta_1 ~ prior: under U(0, 1) priors the first iteration's samples pass a KS test and lie
    inside the support."""
    w = synth.make(5, N=2048)
    m = oracle.Model(oracle.SIR, 2, 2, w.prior_mu, w.prior_sd, w.prior_kind, w.constants)
    rec = oracle.smc2_run(m, w.y[0, :5], N=2048, M=2, K=1, gamma=0.006, seed=w.seed)
    th = rec["theta"][0]
    assert th.min() > 0.0 and th.max() <= 1.0
    for p in range(2):
        assert stats.kstest(th[:, p], "uniform").pvalue > 1e-3


def test_samples_leaving_the_support_get_zero_weight(oracle):
    """A Langevin step that lands outside U(0, 1) has posterior zero, so its weight is zero from
    then on (eq. l_weights), and the population's estimate stays inside the support."""
    w = synth.make(5, N=64)
    m = oracle.Model(oracle.SIR, 2, 2, w.prior_mu, w.prior_sd, w.prior_kind, w.constants)
    rec = oracle.smc2_run(m, w.y[0], N=64, M=64, K=4, gamma=0.3, seed=w.seed)
    th, lw = rec["theta"], rec["logw"]
    outside = (th < 0.0) | (th > 1.0)
    bad = outside.any(axis=2)
    assert bad[1:].any()  # the large step does leave the support
    assert np.all(lw[bad] == -np.inf)
    assert np.all(np.isfinite(lw[~bad]) | (lw[~bad] == -np.inf))


def test_overflowed_particles_take_no_part_in_the_gradient(oracle):
    """With a vague observation (s_y = 200) nothing is resampled, and particles whose infected
    count went negative grow without bound until their state overflows; their weight is then
    exactly zero.  The gradient (such particles taking no part, C32) is finite and equals central
    differences of the estimate with the random numbers held fixed."""
    w = synth.make(5)
    m = _sir(oracle, constants=[NPOP, I0, VAR, 200.0])
    y = w.y[0, :, 0].reshape(-1, 1)
    th, h = np.array([0.6809537166263908, 0.23789620003663003]), 1e-7
    out = oracle.pf(m, th, y, 64, w.seed, 1, 7, want_trace=True)
    assert out["flags"].sum() == 0 and np.all(np.isfinite(out["grad"]))
    for p in range(2):
        e = np.zeros(2)
        e[p] = h
        fd = (oracle.pf(m, th + e, y, 64, w.seed, 1, 7)["loglik"] -
              oracle.pf(m, th - e, y, 64, w.seed, 1, 7)["loglik"]) / (2 * h)
        assert out["grad"][p] == pytest.approx(fd, rel=1e-6)
