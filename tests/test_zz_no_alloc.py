"""The no-allocation reweighting entry point against the context one, through the C ABI: two
calls in a row on the same GPU (the second smaller, so it reuses the shared scratch array the
first left filled), each compared output by output with smc2_reweight_resample on the same
inputs; the size limit and the status word."""
import numpy as np
import pytest

from gpu_util import say
from paper_2407_17296_amd import smc2

pytestmark = pytest.mark.gpu


def _population(S, N, D, rng, dev):
    import torch
    f64 = dict(dtype=torch.float64, device=dev)

    def t(a):
        return torch.tensor(np.ascontiguousarray(a), **f64)
    # log-likelihoods spread over several nats so that the weights are uneven and the call
    # resamples (its gather goes through the scratch)
    cur = dict(theta=t(rng.standard_normal((S, N, D))), logpost=t(np.zeros((S, N))),
               grad_logpost=t(rng.standard_normal((S, N, D))),
               loglik=t(-50.0 + 3.0 * rng.standard_normal((S, N))), logw=t(np.zeros((S, N))))
    prev = dict(theta=t(rng.standard_normal((S, N, D))),
                logpost=t(-50.0 + rng.standard_normal((S, N))),
                grad_logpost=t(rng.standard_normal((S, N, D))),
                loglik=t(-50.0 + rng.standard_normal((S, N))),
                logw=t(-np.log(N) + 0.1 * rng.standard_normal((S, N))))
    p_prev = t(0.05 * rng.standard_normal((S, N, D)))
    return cur, prev, p_prev


def _outputs(S, N, D, dev):
    import torch
    return dict(anc=torch.full((S, N), -7, dtype=torch.int32, device=dev),
                ess=torch.full((S,), np.nan, dtype=torch.float64, device=dev),
                res=torch.full((S,), -7, dtype=torch.int32, device=dev),
                est=torch.full((S, 2, D), np.nan, dtype=torch.float64, device=dev),
                rec=torch.zeros((S, 1 + 4 * D), dtype=torch.float64, device=dev),
                it=torch.tensor([3], dtype=torch.int32, device=dev))


def _call(model, S, N, gamma, rw, cur, prev, p_prev, out, seed, noalloc, ctx=None, status=None):
    c = smc2.population(**cur)
    p = smc2.population(**prev)
    args = (S, N, gamma, rw, c, p, p_prev, 0, seed, out["it"], 1, out["anc"], out["ess"],
            out["res"], out["est"], out["rec"])
    if noalloc:
        smc2.smc2_reweight_resample_noalloc(model, *args, status=status)
    else:
        smc2.smc2_reweight_resample(ctx.h, model, *args)


@pytest.mark.parametrize("rw", [0, 1])
def test_noalloc_equals_context_call_twice(rw):
    import torch
    dev = torch.device("cuda:0")
    model = smc2.Model(smc2.LG1D, 1, 3)
    D = 3
    for call, (S, N) in enumerate(((3, 1500), (2, 700))):
        rng = np.random.default_rng(100 + call)
        say("  call %d: S=%d N=%d random_walk=%d" % (call + 1, S, N, rw))
        cur_a, prev, p_prev = _population(S, N, D, rng, dev)
        cur_b = {k: v.clone() for k, v in cur_a.items()}
        out_a, out_b = _outputs(S, N, D, dev), _outputs(S, N, D, dev)
        ctx = smc2.Context(model, smc2.pf_opts(), S, N, 64, np.full(S, 4, np.int32), 4)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        _call(model, S, N, 0.1, rw, cur_a, prev, p_prev, out_a, 17 + call, False, ctx=ctx)
        _call(model, S, N, 0.1, rw, cur_b, prev, p_prev, out_b, 17 + call, True, status=status)
        torch.cuda.synchronize()
        ctx.close()
        assert int(status.item()) == 0
        assert out_a["res"].cpu().numpy().sum() >= 1  # the scratch's gather was exercised
        for k in cur_a:
            a, b = cur_a[k].cpu().numpy(), cur_b[k].cpu().numpy()
            assert np.array_equal(a, b, equal_nan=True), (call, k)
        for k in out_a:
            a, b = out_a[k].cpu().numpy(), out_b[k].cpu().numpy()
            assert np.array_equal(a, b, equal_nan=True), (call, k)
        say("    resampled %s, ESS %s: equal to the context call" % (
            out_b["res"].cpu().numpy(), np.array2string(out_b["ess"].cpu().numpy(), precision=1)))


def test_noalloc_refuses_sizes_beyond_its_scratch_and_sets_the_status():
    import torch
    dev = torch.device("cuda:0")
    model = smc2.Model(smc2.LG1D, 1, 3)
    D = 3
    # 64 series of 4096 samples need 64 * 4096 * 8 doubles, twice the fixed scratch
    S, N = 64, 4096
    rng = np.random.default_rng(7)
    cur, prev, p_prev = _population(S, N, D, rng, dev)
    out = _outputs(S, N, D, dev)
    with pytest.raises(smc2.SMC2Error, match="scratch") as e:
        _call(model, S, N, 0.1, 0, cur, prev, p_prev, out, 5, True)
    assert e.value.status == smc2.SMC2_E_INVALID_ARG
    # every weight zero in one series: the caller's status word is set
    S, N = 2, 64
    cur, prev, p_prev = _population(S, N, D, rng, dev)
    cur["loglik"][1] = -np.inf
    out = _outputs(S, N, D, dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    _call(model, S, N, 0.1, 0, cur, prev, p_prev, out, 5, True, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == smc2.SMC2_E_NONFINITE
    assert out["ess"].cpu().numpy()[1] == 0.0
