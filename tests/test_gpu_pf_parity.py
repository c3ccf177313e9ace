"""GPU parity of the fused CRN-PF forward+adjoint kernel against the FP64 oracle, through the C ABI.

Bars: plain FP64 form -- ancestors bit-exact, log-likelihood relative error <= 1e-12, gradient
relative error (2-norm over theta) <= 1e-9; mixed form -- abs(d loglik) <= 1e-4 * T, gradient
relative error <= 1e-3, ancestor-mismatch rate reported.
"""
import numpy as np
import pytest

from gpu_util import gpu_pf, oracle_pf, rel_err, say, spread_theta
from paper_2407_17296_amd import smc2, synth

pytestmark = pytest.mark.gpu

LL_TOL, G_TOL = 1e-12, 1e-9


def _check_fp64(oracle, w, theta, ll, g, traces, k=1, resampler=0, ess_frac=0.5, items=None):
    items = items or [(s, i) for s in range(w.S) for i in range(w.N)]
    worst_l = worst_g = 0.0
    for (s, i) in items:
        r = oracle_pf(oracle, w, theta, s, i, k=k, resampler=resampler, ess_frac=ess_frac,
                      want_trace=(s, i) in traces)
        if r["loglik"] == -np.inf:
            assert ll[s, i] == -np.inf and np.all(g[s, i] == 0), (s, i)
            continue
        el = abs(ll[s, i] - r["loglik"]) / max(abs(r["loglik"]), 1e-300)
        eg = rel_err(g[s, i], r["grad"])
        worst_l, worst_g = max(worst_l, el), max(worst_g, eg)
        assert el <= LL_TOL, (s, i, ll[s, i], r["loglik"])
        assert eg <= G_TOL, (s, i, g[s, i], r["grad"])
        if (s, i) in traces:
            fl, anc = traces[(s, i)]
            assert np.array_equal(fl, r["flags"]), (s, i)
            assert np.array_equal(anc, r["ancestors"]), (s, i)
    say("  worst rel err loglik %.2e grad %.2e over %d items" % (worst_l, worst_g, len(items)))


@pytest.mark.parametrize("resampler", [smc2.SYSTEMATIC, smc2.MULTINOMIAL])
def test_fp64_small_lg1d_all_items(oracle, resampler):
    w = synth.make(0)
    theta = synth.prior_draws(w)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, resampler=resampler, k=2, trace_items=items)
    _check_fp64(oracle, w, theta, ll, g, tr, k=2, resampler=resampler)


def test_fp64_growth_ragged_particles_and_segments(oracle):
    """M = 100 (a 128-particle tile with a ragged tail), T = 37, checkpoints every 5 steps."""
    w = synth.make(3, N=6, M=100, T=37)
    theta = spread_theta(w, 0.3, seed=1)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, ckpt=5, k=4, trace_items=items)
    _check_fp64(oracle, w, theta, ll, g, tr, k=4)


@pytest.mark.parametrize("persistent", [0, 1])
def test_fp64_sv_uneven_series(oracle, persistent):
    """Three series of lengths 13, 0 and 29 (an empty series included), longest first."""
    w = synth.make(4, S=3, N=4, M=256, T=40)
    w.T_len = np.array([13, 0, 29], dtype=np.int32)
    w.y = np.ascontiguousarray(w.y[:, :29])
    theta = spread_theta(w, 0.3, seed=2)
    items = [(s, i) for s in range(w.S) for i in range(w.N)]
    tr_items = items if not persistent else []
    ll, g, tr = gpu_pf(w, theta, k=3, persistent=persistent, trace_items=tr_items)
    assert np.all(ll[1] == 0.0) and np.all(g[1] == 0.0)  # T = 0: loglik 0, gradient 0
    _check_fp64(oracle, w, theta, ll, g, tr, k=3)


def test_fp64_lg_diag16(oracle):
    w = synth.make(2, N=3, M=64, T=12)
    theta = spread_theta(w, 0.05, seed=3)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, ckpt=4, k=2, trace_items=items)
    _check_fp64(oracle, w, theta, ll, g, tr, k=2)


def test_fp64_edge_cases(oracle):
    """M = 1 (never resamples), a NaN parameter and parameters no particle can explain."""
    w = synth.make(0, N=4, M=1)
    theta = spread_theta(w, 0.2, seed=4)
    theta[0, 1, 0] = np.nan
    theta[0, 2, 2] = -400.0  # observation noise so small that every weight underflows
    ll, g, tr = gpu_pf(w, theta, k=1, trace_items=[(0, 0)])
    assert ll[0, 1] == -np.inf and np.all(g[0, 1] == 0)
    assert ll[0, 2] == -np.inf and np.all(g[0, 2] == 0)
    _check_fp64(oracle, w, theta, ll, g, tr, items=[(0, 0), (0, 3)])


def test_fp64_always_and_never_resample(oracle):
    w = synth.make(0, N=4)
    theta = spread_theta(w, 0.3, seed=5)
    for frac in (0.0, 2.0):
        items = [(0, i) for i in range(w.N)]
        ll, g, tr = gpu_pf(w, theta, ess_frac=frac, k=1, trace_items=items)
        _check_fp64(oracle, w, theta, ll, g, tr, ess_frac=frac)


@pytest.mark.parametrize("tile", [7, 8])
def test_fp64_full_size_lg1d_sampled(oracle, tile):
    """The 1-D LG workload at full size (N = 1024, M = 1024, T = 250) in the benchmark's launch
    shape family; the oracle checks a sample of items one by one."""
    w = synth.make(1)
    theta = spread_theta(w, 0.3, seed=6)
    sample = [(0, i) for i in (0, 1, 257, 511, 768, 1023)]
    ll, g, tr = gpu_pf(w, theta, tile=tile, k=5, trace_items=sample)
    assert np.all(np.isfinite(ll))
    _check_fp64(oracle, w, theta, ll, g, tr, k=5, items=sample)


def test_fp64_tiles_agree():
    """Launch shapes of equal capacity give the same answer up to summation order."""
    w = synth.make(1, N=64)
    theta = spread_theta(w, 0.3, seed=7)
    ll7, g7, _ = gpu_pf(w, theta, tile=7, k=2)
    ll8, g8, _ = gpu_pf(w, theta, tile=8, k=2)
    assert np.allclose(ll7, ll8, rtol=1e-13, atol=0)
    assert np.allclose(g7, g8, rtol=1e-10, atol=1e-10)


def test_fp64_persistent_equals_grid():
    w = synth.make(3, N=300, M=512, T=60)
    theta = spread_theta(w, 0.3, seed=8)
    a = gpu_pf(w, theta, k=2, persistent=0)
    b = gpu_pf(w, theta, k=2, persistent=1)
    assert np.array_equal(a[0], b[0])
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------- mixed precision ----

def _check_mixed(oracle, w, theta, ll, g, traces, k, items, label):
    T = int(w.T_len.max())
    worst_dl = worst_g = 0.0
    mism = tot = 0
    fails = []
    for (s, i) in items:
        r = oracle_pf(oracle, w, theta, s, i, k=k, want_trace=(s, i) in traces)
        dl = abs(ll[s, i] - r["loglik"])
        eg = rel_err(g[s, i], r["grad"])
        worst_dl, worst_g = max(worst_dl, dl), max(worst_g, eg)
        if dl > 1e-4 * w.T_len[s] or eg > 1e-3:
            fails.append((s, i, dl, eg, r["loglik"]))
        if (s, i) in traces:
            fl, anc = traces[(s, i)]
            both = (fl == 1) & (r["flags"] == 1)
            mism += int(np.sum(anc[both] != r["ancestors"][both]))
            tot += int(np.sum(both)) * w.M
    say("  %s: worst |dl| %.2e (gate %.2e) grad rel %.2e; ancestor mismatch %d / %d = %.2e; "
        "gate failures %d / %d" % (label, worst_dl, 1e-4 * T, worst_g, mism, tot,
                                    mism / max(tot, 1), len(fails), len(items)))
    for f in fails:
        say("    fail s=%d i=%d |dl|=%.3e grad_rel=%.3e |loglik|=%.1f" % f)
    return fails


@pytest.mark.parametrize("index,kw", [(0, {}), (3, dict(N=64)), (1, dict(N=16)),
                                      (4, dict(S=2, N=8, T=300)), (2, dict(N=4, M=256, T=40))])
def test_mixed_within_tolerance(oracle, index, kw):
    w = synth.make(index, **kw)
    theta = spread_theta(w, 0.1 if w.d > 1 else 0.3, seed=10 + index)
    items = [(s, i) for s in range(w.S) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, precision=smc2.MIXED, k=2, trace_items=items[:8])
    fails = _check_mixed(oracle, w, theta, ll, g, tr, 2, items, w.name)
    assert not fails
