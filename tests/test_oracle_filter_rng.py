"""Pins of the oracle's per-filter random numbers: the noise of every particle and step and the
resampling uniforms, and where the filter draws them.

The paper draws the propagation noise in advance (eq. reparam_epsilon), fixes it per filter
(common random numbers, Sec. II-A), and draws the resampling uniforms on (0, 1] independently
per particle and step (App. B).  The counter contract realises that: element g = j d + q of
step t is normal g mod 4 of the Philox block (g / 4, t, filter, stream) (Box-Muller pair
(g mod 4) / 2, cosine branch for even g); multinomial offspring i takes word i mod 4 of block
(i / 4, t), systematic resampling word 0 of block (0xFFFFFFFF, t).  These tests pin that map to
rocRAND's independent Philox engine, check the distribution and the independence across slots,
pair partners, blocks and steps, and check by brute force on a two-step filter that the filter
resamples with exactly those uniforms.  The last test plants plausible mistakes in a copy of the
oracle and shows that each fails at least one pin.
"""
import os
import tempfile

import numpy as np
import pytest
from scipy import stats

from test_oracle_rng import _rocrand_ref

SEED = 0x243F6A8885A308D3
FID = 77


def _c3(oracle, k, stream):
    return oracle.c3(k, stream)


def _normal_table(oracle, L, t_steps, slots, k=3, stream=None):
    """z[t][g] for steps t_steps and elements g in [0, slots)."""
    c3 = _c3(oracle, k, oracle.STEP_NORMAL if stream is None else stream)
    f = L.orc_filter_normal
    return np.array([[f(SEED, FID, c3, t, g) for g in range(slots)] for t in t_steps])


def _uniform_table(oracle, L, t_steps, slots, k=3):
    """Multinomial uniforms u[t][i] for offspring i in [0, slots)."""
    c3 = _c3(oracle, k, oracle.RESAMPLE_UNIFORM)
    f = L.orc_filter_uniform
    return np.array([[f(SEED, FID, c3, t, i >> 2, i & 3) for i in range(slots)]
                     for t in t_steps])


def pin_noise_word_mapping(oracle, L):
    """Element g of step t is Box-Muller pair (g mod 4) / 2 of block (g / 4, t): its words from
    rocRAND's engine, cosine branch for even g, sine for odd."""
    for stream, k in ((oracle.STEP_NORMAL, 3), (oracle.INIT_NORMAL, 1)):
        c3 = _c3(oracle, k, stream)
        for t in (0, 1, 7, 250):
            rows = [[b, t, FID, c3, SEED & 0xFFFFFFFF, SEED >> 32] for b in range(8)]
            words = _rocrand_ref(rows)
            for g in range(32):
                w = words[g // 4]
                pr = (g % 4) // 2
                u1 = (float(w[2 * pr]) + 1.0) * 2.0**-32
                u2 = float(w[2 * pr + 1]) * 2.0**-32
                r = np.sqrt(-2.0 * np.log(u1))
                want = r * (np.sin(2 * np.pi * u2) if g % 2 else np.cos(2 * np.pi * u2))
                got = L.orc_filter_normal(SEED, FID, c3, t, g)
                assert got == pytest.approx(want, rel=1e-13, abs=1e-13), (stream, t, g)


def pin_uniform_word_mapping(oracle, L):
    """Uniform (c0, word) of step t is (w + 1) 2^-32 of word `word` of block (c0, t)."""
    c3 = _c3(oracle, 4, oracle.RESAMPLE_UNIFORM)
    for t in (1, 2, 99):
        c0s = list(range(6)) + [0xFFFFFFFF]
        rows = [[c0, t, FID, c3, SEED & 0xFFFFFFFF, SEED >> 32] for c0 in c0s]
        words = _rocrand_ref(rows)
        for c0, w in zip(c0s, words):
            for word in range(4):
                want = (float(w[word]) + 1.0) * 2.0**-32
                assert L.orc_filter_uniform(SEED, FID, c3, t, c0, word) == want, (t, c0, word)


def _corr_ok(a, b, what):
    n = a.size
    r = np.corrcoef(a.ravel(), b.ravel())[0, 1]
    assert abs(r) < 5.0 / np.sqrt(n), (what, r, n)


def pin_noise_distribution_and_independence(oracle, L):
    """Over 40 steps x 4096 elements: N(0, 1) by a KS test; no correlation between elements
    1, 2, 3 and 4 apart (inside a block, across the two pairs of a block, across blocks), between
    the two values of each Box-Muller pair in value and in square, and between consecutive steps
    of one element."""
    z = _normal_table(oracle, L, range(1, 41), 4096)
    assert stats.kstest(z.ravel(), "norm").pvalue > 1e-4
    assert abs(z.mean()) < 5 / np.sqrt(z.size) and abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    for lag in (1, 2, 3, 4):
        _corr_ok(z[:, :-lag], z[:, lag:], "elements %d apart" % lag)
    # the two values of a pair (even g and g + 1), in value and in square (one radius each)
    _corr_ok(z[:, 0::2], z[:, 1::2], "pair partners")
    _corr_ok(z[:, 0::2] ** 2, z[:, 1::2] ** 2, "pair partners squared")
    # the two pairs of one block
    _corr_ok(z[:, 0::4] ** 2, z[:, 2::4] ** 2, "pairs of one block squared")
    _corr_ok(z[:-1], z[1:], "consecutive steps")
    # the initial draw is its own stream
    z0 = _normal_table(oracle, L, [0], 4096, k=3, stream=oracle.INIT_NORMAL)
    assert stats.kstest(z0.ravel(), "norm").pvalue > 1e-4
    _corr_ok(z0, z[:1], "initial draw against step 1")


def pin_uniform_distribution_and_independence(oracle, L):
    """Multinomial uniforms over 40 steps x 4096 offspring are U(0, 1] (KS) and uncorrelated
    across offspring 1..4 apart and across steps; the systematic offsets of 20,000 steps are
    U(0, 1]."""
    u = _uniform_table(oracle, L, range(1, 41), 4096)
    assert u.min() > 0.0 and u.max() <= 1.0
    assert stats.kstest(u.ravel(), "uniform").pvalue > 1e-4
    for lag in (1, 2, 3, 4):
        _corr_ok(u[:, :-lag], u[:, lag:], "offspring %d apart" % lag)
    _corr_ok(u[:-1], u[1:], "consecutive steps")
    c3 = _c3(oracle, 3, oracle.RESAMPLE_UNIFORM)
    nu = np.array([L.orc_filter_uniform(SEED, FID, c3, t, 0xFFFFFFFF, 0)
                   for t in range(1, 20001)])
    assert nu.min() > 0.0 and nu.max() <= 1.0
    assert stats.kstest(nu, "uniform").pvalue > 1e-4
    _corr_ok(nu[:-1], nu[1:], "systematic offsets of consecutive steps")


def pin_filter_resamples_with_the_stream(oracle, L):
    """A two-step 1-D LG filter that resamples after step 1 (ess_frac 2): its ancestors equal
    the lower-bound rule applied to the weights g(y_1 | x_1^j), written out from the model with
    the stream's noise, at the stream's resampling positions (multinomial: uniform i of the
    offspring's word; systematic: (i + nu) / M)."""
    a_, lsx, lsy = 0.8, np.log(0.9), np.log(0.6)
    theta = np.array([a_, lsx, lsy])
    y = np.array([[0.4], [-0.3]])
    m = oracle.Model(oracle.LG1D, 1, 3)
    k = 5
    c3i, c3s, c3r = (_c3(oracle, k, s) for s in (oracle.INIT_NORMAL, oracle.STEP_NORMAL,
                                                  oracle.RESAMPLE_UNIFORM))
    for M in (8, 37, 64):
        x0 = np.array([L.orc_filter_normal(SEED, FID, c3i, 0, j) for j in range(M)])
        e1 = np.array([L.orc_filter_normal(SEED, FID, c3s, 1, j) for j in range(M)])
        x1 = a_ * x0 + np.exp(lsx) * e1
        lam = stats.norm.logpdf(y[0, 0], loc=x1, scale=np.exp(lsy))
        w = np.exp(lam - lam.max())
        u_mult = np.array([L.orc_filter_uniform(SEED, FID, c3r, 1, i >> 2, i & 3)
                           for i in range(M)])
        nu = L.orc_filter_uniform(SEED, FID, c3r, 1, 0xFFFFFFFF, 0)
        u_sys = (np.arange(M) + nu) / M
        for resampler, u in ((oracle.MULTINOMIAL, u_mult), (oracle.SYSTEMATIC, u_sys)):
            r = oracle.pf(m, theta, y, M, SEED, k, FID, resampler=resampler, ess_frac=2.0,
                          want_trace=True, L=L)
            assert r["flags"][0] == 1
            want = oracle.resample_lower_bound(w, u)
            assert np.array_equal(r["ancestors"][0], want), (M, resampler)


PINS = [pin_noise_word_mapping, pin_uniform_word_mapping,
        pin_noise_distribution_and_independence, pin_uniform_distribution_and_independence,
        pin_filter_resamples_with_the_stream]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_filter_random_numbers(oracle, pin):
    pin(oracle, oracle.lib())


# Plausible mistakes in the per-filter random numbers, each planted in a copy of the oracle.
MUTANTS = {
    "pair index g & 1": [("uint32_t pr = (g & 3u) >> 1;", "uint32_t pr = g & 1u;")],
    "block index g / 2": [("block_words(seed, g >> 2, t, fid, c3, w);",
                           "block_words(seed, g >> 1, t, fid, c3, w);")],
    "sine and cosine swapped": [("return (g & 1u) ? r * std::sin(ang) : r * std::cos(ang);",
                                 "return (g & 1u) ? r * std::cos(ang) : r * std::sin(ang);")],
    "uniform word swapped": [("return ((double)w[word & 3u] + 1.0) * 0x1p-32;",
                              "return ((double)w[(word ^ 1u) & 3u] + 1.0) * 0x1p-32;")],
    "multinomial word fixed": [("(uint32_t)t, (uint32_t)i >> 2, (uint32_t)i & 3u);",
                                "(uint32_t)t, (uint32_t)i >> 2, 0u);")],
    "systematic word 1": [("(uint32_t)t, 0xFFFFFFFFu, 0u);", "(uint32_t)t, 0xFFFFFFFFu, 1u);")],
    "uniform step index off by one": [("block_words(seed, c0, t, fid, c3, w);\n  return",
                                       "block_words(seed, c0, t + 1, fid, c3, w);\n  return")],
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_fail_a_pin(oracle, name):
    with tempfile.TemporaryDirectory() as d:
        L = oracle.build_variant(os.path.join(d, "liboracle_mutant.so"), MUTANTS[name])
        failed = []
        for pin in PINS:
            try:
                pin(oracle, L)
            except AssertionError:
                failed.append(pin.__name__)
        assert failed, "planted mistake %r passed every pin" % name
        print("  %s: caught by %s" % (name, ", ".join(failed)))
