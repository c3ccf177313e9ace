"""GPU parity of the SMC^2 outer step (Langevin move, filter, L-kernel reweighting, ESS and
resampling) against the oracle's full run, and of a captured HIP graph against eager calls."""
import numpy as np
import pytest

from gpu_util import say
from paper_2407_17296_amd import driver, smc2, synth

pytestmark = pytest.mark.gpu


def _oracle_run(oracle, w, K, s=0):
    m = oracle.Model(w.kind, w.d, w.D, w.prior_mu, w.prior_sd)
    return oracle.smc2_run(m, w.y[s, :w.T_len[s]], w.N, w.M, K, w.gamma, w.seed, series=s)


@pytest.mark.parametrize("index,kw,K", [(0, {}, 10), (3, dict(N=64, M=128, T=40), 6)])
def test_fp64_smc2_trajectory_matches_oracle(oracle, index, kw, K):
    w = synth.make(index, **kw)
    say("  smc2 %s N=%d M=%d K=%d" % (w.name, w.N, w.M, K))
    run, rec = driver.run_smc2(w, K=K, precision=smc2.FP64)
    run.close()
    o = _oracle_run(oracle, w, K)
    for k in range(K):
        assert np.allclose(rec.theta[k, 0], o["theta"][k], rtol=0, atol=1e-10), k
        assert np.allclose(rec.loglik[k, 0], o["loglik"][k], rtol=1e-11, atol=1e-11), k
        assert np.allclose(rec.grad[k, 0], o["grad"][k], rtol=1e-8, atol=1e-8), k
        assert rec.ess[k, 0] == pytest.approx(o["ess"][k], rel=1e-10), k
        assert rec.resampled[k, 0] == o["resampled"][k], k
        assert np.array_equal(rec.anc[k, 0], o["anc"][k]), k
        lw = o["logw"][k]
        if o["resampled"][k]:
            mx = lw.max()
            want = mx + np.log(np.sum(np.exp(lw - mx))) - np.log(w.N)
            assert np.allclose(rec.logw[k, 0], want, rtol=1e-11, atol=1e-10), k
        else:
            assert np.allclose(rec.logw[k, 0], lw, rtol=1e-11, atol=1e-10), k
    say("  %d iterations match; resampled at %s" % (K, list(np.nonzero(o["resampled"])[0] + 1)))


def test_multi_series_outer_step_is_per_series(oracle):
    w = synth.make(4, S=3, N=16, M=64, T=30)
    K = 4
    run, rec = driver.run_smc2(w, K=K, precision=smc2.FP64)
    run.close()
    for s in range(w.S):
        o = _oracle_run(oracle, w, K, s=s)
        for k in range(K):
            assert np.allclose(rec.theta[k, s], o["theta"][k], atol=1e-10), (s, k)
            assert np.array_equal(rec.anc[k, s], o["anc"][k]), (s, k)


def test_graph_replay_equals_eager():
    """One captured iteration replayed K-1 times equals K-1 eager iterations, replay by replay,
    with eager work and synchronisation between the replays."""
    import torch
    w = synth.make(0, N=32)
    K = 6
    eager = driver.SMC2Run(w, precision=smc2.FP64)
    graph = driver.SMC2Run(w, precision=smc2.FP64)
    eager.first_iteration()
    graph.first_iteration()
    graph.capture()
    # capture does not execute: the population is still the k = 1 result
    for k in range(2, K + 1):
        eager.next_iteration()
        graph.replay()
        torch.cuda.synchronize()
        a, b = eager.snapshot(), graph.snapshot()
        for key in a:
            assert np.allclose(a[key], b[key], rtol=1e-12, atol=1e-12), (k, key)
        assert int(graph.iteration.item()) == k + 1
    eager.close()
    graph.close()


def test_all_zero_weights_set_the_device_status():
    import torch
    w = synth.make(0, N=8)
    run = driver.SMC2Run(w, precision=smc2.FP64)
    run.first_iteration()
    torch.cuda.synchronize()
    assert smc2.smc2_ctx_device_status(run.ctx.h) == smc2.SMC2_OK
    # every sample gets an observation noise no particle can match: all weights zero
    run.cur["theta"][..., 2] = -400.0
    run._pf()
    run._reweight(first=True)
    assert smc2.smc2_ctx_device_status(run.ctx.h) == smc2.SMC2_E_NONFINITE
    assert np.all(run.ess.cpu().numpy() == 0.0)
    run.close()
