"""GPU parity of the fused CRN-PF forward+adjoint kernel against the FP64 oracle, through the C ABI.

Bars: plain FP64 form -- ancestors bit-exact, log-likelihood relative error <= 1e-12, gradient
relative error (2-norm over theta) <= 1e-9; mixed form -- abs(d loglik) <= 1e-4 * T, gradient
relative error <= 1e-3, ancestor-mismatch rate reported.
"""
import numpy as np
import pytest

from gpu_util import (gpu_pf, oracle_batch, oracle_pf, oracle_sensitivity, paired_mean_zero,
                      rel_err, say, spread_theta)
from paper_2407_17296_amd import smc2, synth

pytestmark = pytest.mark.gpu

LL_TOL, G_TOL = 1e-12, 1e-9
EPS64, EPS32 = 2.0**-52, 2.0**-24


def _check_fp64(oracle, w, theta, ll, g, traces, k=1, resampler=0, ess_frac=0.5, items=None,
                min_gated=0.5):
    """Gate every item at which the oracle is stable at FP64 resolution (its ancestry and
    value do not move under a one-ulp perturbation of theta); report the others."""
    items = items or [(s, i) for s in range(w.S) for i in range(w.N)]
    worst_l = worst_g = 0.0
    gated, ill = 0, []
    for (s, i) in items:
        r, dl, dg, same = oracle_sensitivity(oracle, w, theta, s, i, k, EPS64, resampler, ess_frac)
        if r["loglik"] == -np.inf:
            assert ll[s, i] == -np.inf and np.all(g[s, i] == 0), (s, i)
            gated += 1
            continue
        el = abs(ll[s, i] - r["loglik"]) / max(abs(r["loglik"]), 1e-300)
        eg = rel_err(g[s, i], r["grad"])
        if not (same and dl <= 1e-13 * max(1.0, abs(r["loglik"])) and dg <= 1e-10):
            ill.append((s, i, el, eg, dl, dg))
            continue
        gated += 1
        worst_l, worst_g = max(worst_l, el), max(worst_g, eg)
        assert el <= LL_TOL, (s, i, ll[s, i], r["loglik"])
        assert eg <= G_TOL, (s, i, g[s, i], r["grad"])
        if (s, i) in traces:
            fl, anc = traces[(s, i)]
            assert np.array_equal(fl, r["flags"]), (s, i)
            assert np.array_equal(anc, r["ancestors"]), (s, i)
    say("  FP64: %d/%d items gated, worst rel err loglik %.2e grad %.2e; %d ill-conditioned at "
        "FP64 resolution (reported)" % (gated, len(items), worst_l, worst_g, len(ill)))
    for (s, i, el, eg, dl, dg) in ill:
        say("    ill s=%d i=%d theta=%s rel err loglik %.1e grad %.1e; oracle moves %.1e / %.1e "
            "under one ulp" % (s, i, np.array2string(theta[s, i], precision=2), el, eg, dl, dg))
    assert gated >= min_gated * len(items)


@pytest.mark.parametrize("store_noise", [1, 0])
@pytest.mark.parametrize("resampler", [smc2.SYSTEMATIC, smc2.MULTINOMIAL])
def test_fp64_small_lg1d_all_items(oracle, resampler, store_noise):
    w = synth.make(0)
    theta = synth.prior_draws(w)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, resampler=resampler, k=2, trace_items=items,
                       store_noise=store_noise)
    _check_fp64(oracle, w, theta, ll, g, tr, k=2, resampler=resampler)


@pytest.mark.parametrize("ckpt", [5, 1])
def test_fp64_growth_ragged_particles_and_segments(oracle, ckpt):
    """M = 100 (a 128-particle tile with a ragged tail), T = 37, checkpoints every 5 steps
    (a ragged last segment) or at every step (the adjoint recomputes nothing)."""
    w = synth.make(3, N=6, M=100, T=37)
    theta = spread_theta(w, 0.3, seed=1)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, ckpt=ckpt, k=4, trace_items=items)
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


@pytest.mark.parametrize("M,store_noise,tile", [(256, 1, 0), (256, 0, 0), (2048, 1, 14),
                                                (2048, 0, 14)])
def test_fp64_lg_diag16_every_step_checkpoints(oracle, M, store_noise, tile):
    """The 16-dimensional state with a checkpoint every step (the reverse sweep that streams
    blocks of four components), noise stored or regenerated, at 256 particles and at the largest
    filter, 2048 particles, on the FP64 shape that holds it (eight waves x four particles per
    lane), every item with its ancestry."""
    w = synth.make(2, N=3, M=M, T=12)
    theta = spread_theta(w, 0.05, seed=60 + M + store_noise)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, tile=tile, ckpt=1, k=2, store_noise=store_noise,
                       trace_items=items)
    _check_fp64(oracle, w, theta, ll, g, tr, k=2)


def test_fp64_lg_diag16_sixteen_waves_is_not_built():
    """Sixteen waves x two particles per lane (tile 17) is built for the mixed form of the
    16-dimensional state only: an FP64 reservation on it is refused as unsupported."""
    w = synth.make(2, N=3, M=2048, T=12)
    model = smc2.Model.from_workload(w)
    with pytest.raises(smc2.SMC2Error) as e:
        smc2.Context(model, smc2.pf_opts(precision=smc2.FP64, tile=17, ckpt_interval=1), w.S,
                     w.N, w.M, w.T_len, w.T_max)
    assert e.value.status == smc2.SMC2_E_UNSUPPORTED
    ctx = smc2.Context(model, smc2.pf_opts(precision=smc2.MIXED, tile=17, ckpt_interval=1),
                       w.S, w.N, w.M, w.T_len, w.T_max)
    ctx.close()


@pytest.mark.parametrize("index,kw,tile,ckpt,store_noise", [
    (3, dict(N=4, M=512, T=100), 5, 1, 1),      # growth: one wave x 8 per lane, every step
    (4, dict(S=2, N=3, M=256), 3, 32, 0),       # SV: full series, a checkpoint every 32 steps
    (5, dict(N=4), 4, 1, 1),                    # SIR: four waves x 1 per lane
])
def test_fp64_other_workloads_in_their_benchmarked_configuration(oracle, index, kw, tile, ckpt,
                                                                  store_noise):
    """The launch shape, checkpoint interval and noise mode the autotuner picks for the growth,
    SV and SIR workloads, at their full series lengths, every item with its ancestry."""
    w = synth.make(index, **kw)
    theta = spread_theta(w, 0.05, seed=70 + index)
    items = [(s, i) for s in range(w.S) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, tile=tile, ckpt=ckpt, k=2, store_noise=store_noise,
                       trace_items=items)
    _check_fp64(oracle, w, theta, ll, g, tr, k=2, items=items)


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


@pytest.mark.parametrize("tile", [8, 9, 10, 11])
def test_fp64_full_size_lg1d_sampled(oracle, tile):
    """The 1-D LG workload at full size (N = 1024, M = 1024, T = 250) in the benchmark's launch
    shape family; the oracle checks a sample of items one by one."""
    w = synth.make(1)
    theta = spread_theta(w, 0.3, seed=6)
    sample = [(0, i) for i in (0, 1, 257, 511, 768, 1023)]
    ll, g, tr = gpu_pf(w, theta, tile=tile, k=5, trace_items=sample)
    assert np.all(np.isfinite(ll))
    _check_fp64(oracle, w, theta, ll, g, tr, k=5, items=sample)


def test_fp64_tiles_agree(oracle):
    """Launch shapes of equal capacity give the same answer up to summation order, wherever the
    filter is stable at FP64 resolution (its ancestry does not move under a one-ulp change)."""
    w = synth.make(1, N=48)
    theta = spread_theta(w, 0.1, seed=7)
    stable = [i for i in range(w.N)
              if oracle_sensitivity(oracle, w, theta, 0, i, 2, EPS64)[3]]
    say("  %d / %d items stable at FP64 resolution" % (len(stable), w.N))
    assert len(stable) >= w.N // 2
    ref_l, ref_g, _ = gpu_pf(w, theta, tile=8, k=2)
    for tile in (9, 10, 11):
        ll, g, _ = gpu_pf(w, theta, tile=tile, k=2)
        dl = np.max(np.abs(ll[0, stable] - ref_l[0, stable]) / np.abs(ref_l[0, stable]))
        dg = max(rel_err(g[0, i], ref_g[0, i]) for i in stable)
        say("  tile %d vs tile 8: max rel loglik %.1e, grad %.1e" % (tile, dl, dg))
        # each tile is held to 1e-12 / 1e-9 against the oracle, so two tiles to twice that
        assert dl <= 2e-12 and dg <= 2e-9, tile


@pytest.mark.parametrize("ckpt", [0, 1])
def test_fp64_persistent_equals_grid(ckpt):
    w = synth.make(3, N=300, M=512, T=60)
    theta = spread_theta(w, 0.3, seed=8)
    a = gpu_pf(w, theta, k=2, persistent=0, ckpt=ckpt)
    b = gpu_pf(w, theta, k=2, persistent=1, ckpt=ckpt)
    assert np.array_equal(a[0], b[0])
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("ckpt", [0, 1])
def test_fp64_persistent_many_items_per_workgroup(ckpt):
    """16384 filters of 64 particles over T = 150 steps: far more items than the persistent grid
    holds, so each workgroup runs several filters in turn, each past the 64-step blocks of its
    resampling words; estimates bit-identical to one workgroup per item."""
    w = synth.make(1, N=16384, M=64, T=150)
    theta = spread_theta(w, 0.05, seed=9)
    a = gpu_pf(w, theta, k=2, persistent=0, ckpt=ckpt)
    b = gpu_pf(w, theta, k=2, persistent=1, ckpt=ckpt)
    assert np.array_equal(a[0], b[0])
    assert np.allclose(a[1], b[1], rtol=1e-12, atol=1e-12)


def test_fp64_checkpoint_intervals_agree(oracle):
    """Every checkpoint interval (every step, a few steps, the square root of T) yields the
    same estimate and the same gradient up to the scatter's summation order."""
    w = synth.make(4, S=3, N=4, M=256, T=40)
    w.T_len = np.array([40, 17, 33], dtype=np.int32)
    theta = spread_theta(w, 0.3, seed=10)
    ref = gpu_pf(w, theta, k=2, ckpt=0)
    for ckpt in (1, 3, 8):
        ll, g, _ = gpu_pf(w, theta, k=2, ckpt=ckpt)
        assert np.array_equal(ll, ref[0]), ckpt
        worst = max(rel_err(g[s, i], ref[1][s, i]) for s in range(w.S) for i in range(w.N))
        say("  ckpt %d vs sqrt(T): max relative gradient difference %.1e" % (ckpt, worst))
        assert worst <= 1e-12, ckpt


@pytest.mark.parametrize("precision", [smc2.FP64, smc2.MIXED])
@pytest.mark.parametrize("index,kw,ckpt,spread", [
    (3, dict(N=6, M=100, T=37), 5, 0.3),
    (3, dict(N=6, M=100, T=37), 1, 0.3),
    (4, dict(S=3, N=4, M=256, T=40), 0, 0.3),
    (2, dict(N=3, M=64, T=12), 4, 0.05),
])
def test_stored_and_regenerated_noise_agree(index, kw, ckpt, spread, precision):
    """The adjoint reads back the forward's stored noise or regenerates it from the counter
    stream: the same numbers either way.  The forward sweep is the same code, so the estimates
    agree bit for bit; the gradients agree up to the order in which the adjoint's scatter-add
    to shared parents lands (workgroup atomics), i.e. to rounding."""
    w = synth.make(index, **kw)
    theta = spread_theta(w, spread, seed=9)
    a = gpu_pf(w, theta, precision=precision, ckpt=ckpt, k=2, store_noise=1)
    b = gpu_pf(w, theta, precision=precision, ckpt=ckpt, k=2, store_noise=0)
    assert np.array_equal(a[0], b[0])
    tol = 1e-12 if precision == smc2.FP64 else 1e-5
    worst = max(rel_err(a[1][s, i], b[1][s, i]) for s in range(w.S) for i in range(w.N))
    say("  stored vs regenerated noise: max relative gradient difference %.1e" % worst)
    assert worst <= tol


# ------------------------------------------------------------------- mixed precision ----

def _mixed_report(oracle, w, theta, ll, g, traces, k, items, label):
    """|d loglik| and gradient errors of the mixed form against the FP64 oracle per item, with
    the index of the first step whose ancestors differ (after it the two particle systems
    evolve apart: one different parent shifts the cumulative weights above it)."""
    rows = []
    mism = tot = 0
    for (s, i) in items:
        r = oracle_pf(oracle, w, theta, s, i, k=k, want_trace=(s, i) in traces)
        dl = abs(ll[s, i] - r["loglik"])
        eg = rel_err(g[s, i], r["grad"])
        first = -1
        if (s, i) in traces:
            fl, anc = traces[(s, i)]
            both = (fl == 1) & (r["flags"] == 1)
            mism += int(np.sum(anc[both] != r["ancestors"][both]))
            tot += int(np.sum(both)) * w.M
            bad = np.nonzero(np.any(anc != r["ancestors"], axis=1) | (fl != r["flags"]))[0]
            first = int(bad[0]) + 1 if len(bad) else 0
        ok = dl <= 1e-4 * int(w.T_len[s]) and eg <= 1e-3
        rows.append((s, i, ok, dl, eg, r["loglik"], first))
    n_ok = sum(r[2] for r in rows)
    say("  %s mixed: %d/%d items within |dl| <= 1e-4 T and grad rel <= 1e-3; ancestor mismatch "
        "%d / %d = %.2e; median |dl| %.2e, median grad rel %.2e" % (
            label, n_ok, len(rows), mism, tot, mism / max(tot, 1),
            np.median([r[3] for r in rows]), np.median([r[4] for r in rows])))
    for (s, i, ok, dl, eg, l, first) in rows:
        if not ok:
            say("    outside s=%d i=%d |dl|=%.3e grad_rel=%.3e loglik=%.1f first differing "
                "ancestry step %s" % (s, i, dl, eg, l, first if first else "none traced"))
    return n_ok, rows


# Workloads whose filters are insensitive at FP32 resolution at these sizes (few or no ancestor
# flips per filter): the mixed form must meet the bars on at least 90% of the items.
@pytest.mark.parametrize("index,kw,spread", [(0, {}, 0.3), (3, dict(N=32, M=64, T=30), 0.3),
                                             (4, dict(S=2, N=8, T=300), 0.3),
                                             (2, dict(N=4, M=256, T=40), 0.1),
                                             (1, dict(N=32, M=64, T=50), 0.1)])
def test_mixed_within_tolerance(oracle, index, kw, spread):
    w = synth.make(index, **kw)
    theta = spread_theta(w, spread, seed=10 + index)
    items = [(s, i) for s in range(w.S) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, precision=smc2.MIXED, k=2, trace_items=items)
    n_ok, _ = _mixed_report(oracle, w, theta, ll, g, tr, 2, items, w.name)
    assert n_ok >= 0.9 * len(items)


@pytest.mark.parametrize("index", [1, 3, 4])
def test_mixed_and_oracle_estimate_the_same_likelihood(oracle, index):
    """The mixed form and the oracle are the same estimator: N independent filters (distinct
    random streams) at one theta, each paired with the oracle's filter on its own stream; the
    paired differences of loglik and of the gradient have mean zero within 4 standard errors.
    (Filter by filter, up to the first resampling step that differs, the mixed form is held to
    the oracle in test_gpu_mixed_vs_oracle.)"""
    w = synth.make(index, N=512, S=1)
    theta = np.broadcast_to(w.theta_true, (1, w.N, w.D)).copy()
    l32, g32, _ = gpu_pf(w, theta, precision=smc2.MIXED, k=7)
    items = [(0, i) for i in range(w.N)]
    lo, go = oracle_batch(oracle, w, theta, items, 7)
    d = l32[0] - lo
    dg = g32[0] - go
    m, se = paired_mean_zero(d, "loglik")
    mg, seg = paired_mean_zero(dg, "grad")
    say("  %s: loglik mean oracle %.4f mixed %.4f (sd %.3f); paired diff %.2e +- %.2e; grad "
        "diff %s +- %s" % (w.name, lo.mean(), l32.mean(), lo.std(), m, se,
                           np.array2string(mg, precision=3), np.array2string(seg, precision=3)))


def test_lg1d_estimates_sit_at_the_kalman_value():
    """Both forms' loglik means lie within the lognormal bias (var/2) plus 4 SE of the exact
    Kalman log-likelihood on the full-size 1-D LG workload."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                    "oracle"))
    import pyoracle
    w = synth.make(1, N=512)
    theta = np.broadcast_to(w.theta_true, (1, w.N, w.D)).copy()
    m = pyoracle.Model(w.kind, w.d, w.D)
    lkf, _ = pyoracle.kalman(m, w.theta_true, w.y[0])
    for prec in (smc2.FP64, smc2.MIXED):
        l, _, _ = gpu_pf(w, theta, precision=prec, k=9)
        sd = l.std()
        say("  precision %d: mean loglik %.4f, Kalman %.4f, sd %.3f" % (prec, l.mean(), lkf, sd))
        assert abs(l.mean() - lkf) < 0.5 * sd * sd + 4 * sd / np.sqrt(w.N) + 0.05


# ----------------------------------------------- the optimal proposal of Sec. IV-A ----

def _opt(w):
    """The same data, filtered with the LG model's optimal proposal."""
    w.kind = smc2.LG1D_OPT
    w.name = w.name + "_opt"
    return w


@pytest.mark.parametrize("resampler", [smc2.SYSTEMATIC, smc2.MULTINOMIAL])
def test_fp64_optimal_proposal_small(oracle, resampler):
    w = _opt(synth.make(0))
    theta = synth.prior_draws(w)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, resampler=resampler, k=2, ess_frac=0.9, trace_items=items)
    _check_fp64(oracle, w, theta, ll, g, tr, k=2, resampler=resampler, ess_frac=0.9)


@pytest.mark.parametrize("ckpt", [0, 1])
def test_fp64_optimal_proposal_full_size_sampled(oracle, ckpt):
    w = _opt(synth.make(1))
    theta = spread_theta(w, 0.3, seed=12)
    sample = [(0, i) for i in (0, 3, 300, 700, 1023)]
    ll, g, tr = gpu_pf(w, theta, tile=10, ckpt=ckpt, k=3, ess_frac=0.9, trace_items=sample)
    assert np.all(np.isfinite(ll))
    _check_fp64(oracle, w, theta, ll, g, tr, k=3, ess_frac=0.9, items=sample)


def test_mixed_optimal_proposal_within_tolerance(oracle):
    w = _opt(synth.make(1, N=32, M=64, T=50))
    theta = spread_theta(w, 0.1, seed=13)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, precision=smc2.MIXED, k=2, trace_items=items)
    n_ok, _ = _mixed_report(oracle, w, theta, ll, g, tr, 2, items, w.name)
    assert n_ok >= 0.9 * len(items)


def test_optimal_proposal_estimates_sit_at_the_kalman_value(oracle):
    """512 independent filters at one theta on the full-size data: both proposals' mean
    likelihood estimate sits at the Kalman value (lognormal bias aside), and the optimal
    proposal's spread is far smaller than the bootstrap filter's."""
    w = synth.make(1, N=512)
    th = np.tile(w.theta_true, (1, w.N, 1))
    m = oracle.Model(smc2.LG1D, 1, 3)
    lkf, _ = oracle.kalman(m, w.theta_true, w.y[0])
    out = {}
    for kind in (smc2.LG1D, smc2.LG1D_OPT):
        w.kind = kind
        ll, _, _ = gpu_pf(w, th, precision=smc2.MIXED, k=2, want_grad=0)
        out[kind] = (ll[0].mean() - lkf, ll[0].std())
        say("  kind %d: mean loglik - Kalman %.3f, sd %.3f" % (kind, *out[kind]))
    assert abs(out[smc2.LG1D_OPT][0]) < 3 * out[smc2.LG1D_OPT][1] + 0.5 * out[smc2.LG1D_OPT][1] ** 2
    assert out[smc2.LG1D_OPT][1] < 0.5 * out[smc2.LG1D][1]


@pytest.mark.parametrize("precision", [smc2.FP64, smc2.MIXED])
def test_launches_are_reproducible(precision):
    """Two launches on the same inputs give the same estimates bit for bit (the forward sweep
    has a fixed order throughout); the gradients agree to rounding, the order in which the
    adjoint's workgroup atomics add offspring into shared parents being the only difference."""
    w = synth.make(1, N=64)
    theta = spread_theta(w, 0.2, seed=14)
    a = gpu_pf(w, theta, precision=precision, k=2, tile=10)
    b = gpu_pf(w, theta, precision=precision, k=2, tile=10)
    assert np.array_equal(a[0], b[0])
    tol = 1e-12 if precision == smc2.FP64 else 1e-5
    worst = max(rel_err(a[1][s, i], b[1][s, i]) for s in range(w.S) for i in range(w.N))
    say("  relaunch: max relative gradient difference %.1e" % worst)
    assert worst <= tol


def test_mixed_form_has_no_loglik_bias_over_many_streams(oracle):
    """The mixed form against the oracle on 5120 filters of the full-size 1-D LG workload at the
    data-generating theta (five iterations' random streams, each filter paired with the
    oracle's on the same stream): the mean paired difference of the log-likelihood estimate is
    zero within 4 standard errors, and the standard error is small enough that a bias of 1e-4 T
    (0.025 nats) would show."""
    w = synth.make(1, N=1024, S=1)
    theta = np.broadcast_to(w.theta_true, (1, w.N, w.D)).copy()
    items = [(0, i) for i in range(w.N)]
    ds = []
    for k in (7, 8, 9, 10, 11):
        l32, _, _ = gpu_pf(w, theta, precision=smc2.MIXED, k=k, want_grad=0)
        lo, _ = oracle_batch(oracle, w, theta, items, k, want_grad=False)
        ds.append(l32[0] - lo)
    d = np.concatenate(ds)
    se = d.std(ddof=1) / np.sqrt(len(d))
    say("  mixed - oracle loglik over %d filters: %.4f +- %.4f" % (len(d), d.mean(), se))
    assert se < 0.025 / 2
    assert abs(d.mean()) <= 4 * se


@pytest.mark.parametrize("precision", [smc2.FP64, smc2.MIXED])
def test_wide_state_persistent_equals_grid(precision):
    """The 16-dimensional state in the persistent grid (workgroups pulling several items in turn,
    the per-wave parameter-adjoint rows in LDS reused) against one workgroup per item."""
    w = synth.make(2, N=40, M=256, T=30)
    theta = spread_theta(w, 0.05, seed=52)
    a = gpu_pf(w, theta, precision=precision, k=2, persistent=0, ckpt=1)
    b = gpu_pf(w, theta, precision=precision, k=2, persistent=1, ckpt=1)
    assert np.array_equal(a[0], b[0])
    tol = 1e-12 if precision == smc2.FP64 else 1e-5
    worst = max(rel_err(a[1][0, i], b[1][0, i]) for i in range(w.N))
    say("  d = 16 persistent vs grid: max relative gradient difference %.1e" % worst)
    assert worst <= tol


@pytest.mark.parametrize("tile,store_noise", [(9, 1), (9, 0), (10, 1)])
def test_full_size_in_the_benchmarked_configuration(oracle, tile, store_noise):
    """The launch configurations the benchmark's tuner picks on the full-size 1-D LG workload
    (a checkpoint at every step, noise stored or regenerated): the FP64 form against the oracle
    on sampled items, and the mixed form against the oracle statistically (each filter paired
    with the oracle's on the same stream)."""
    w = synth.make(1)
    theta = spread_theta(w, 0.3, seed=53)
    sample = [(0, i) for i in (3, 400, 1000)]
    ll, g, tr = gpu_pf(w, theta, tile=tile, ckpt=1, store_noise=store_noise, k=6,
                       trace_items=sample)
    _check_fp64(oracle, w, theta, ll, g, tr, k=6, items=sample, min_gated=0.3)
    wt = synth.make(1, N=1024)
    at = np.broadcast_to(wt.theta_true, (1, wt.N, wt.D)).copy()
    l32, g32, _ = gpu_pf(wt, at, precision=smc2.MIXED, tile=tile, ckpt=1,
                         store_noise=store_noise, k=12)
    lo, go = oracle_batch(oracle, wt, at, [(0, i) for i in range(wt.N)], 12)
    m, se = paired_mean_zero(l32[0] - lo, "loglik")
    paired_mean_zero(g32[0] - go, "grad")
    say("  tile %d store_noise %d: mixed - oracle loglik %.3f +- %.3f" % (tile, store_noise, m, se))


@pytest.mark.parametrize("index,M,T", [(0, 4096, 30), (0, 4000, 30), (3, 4096, 20),
                                       (2, 2048, 10), (5, 2048, 20)])
def test_fp64_largest_particle_counts(oracle, index, M, T):
    """The largest filters the library builds (4096 particles for scalar states, 2048 for the
    two- and 16-component ones), full and ragged, every item with its ancestry."""
    w = synth.make(index, N=3, M=M, T=T)
    theta = spread_theta(w, 0.05, seed=54 + M)
    items = [(0, i) for i in range(w.N)]
    ll, g, tr = gpu_pf(w, theta, k=2, trace_items=items)
    _check_fp64(oracle, w, theta, ll, g, tr, k=2)
