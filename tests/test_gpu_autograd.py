"""The filter as a torch.autograd.Function: its forward value and the gradient that backward
propagates are the fused kernel's log-likelihood and adjoint gradient, checked against the FP64
oracle."""
import numpy as np
import pytest

from gpu_util import oracle_pf, rel_err, spread_theta
from paper_2407_17296_amd import smc2, synth

pytestmark = pytest.mark.gpu


def test_pf_loglik_autograd_matches_oracle(oracle):
    import torch
    dev = torch.device("cuda:0")
    w = synth.make(0, N=6)
    theta_np = spread_theta(w, 0.2, seed=51)
    model = smc2.Model.from_workload(w)
    ctx = smc2.Context(model, smc2.pf_opts(precision=smc2.FP64), w.S, w.N, w.M, w.T_len, w.T_max)
    theta = torch.tensor(theta_np, dtype=torch.float64, device=dev, requires_grad=True)
    y = torch.tensor(w.y, dtype=torch.float64, device=dev)
    it = torch.tensor([2], dtype=torch.int32, device=dev)
    ll = smc2.PFLogLik.apply(theta, y, ctx, w.seed, it)
    coef = torch.linspace(0.5, 2.0, w.N, dtype=torch.float64, device=dev).reshape(1, -1)
    (coef * ll).sum().backward()
    torch.cuda.synchronize()
    got_l = ll.detach().cpu().numpy()
    got_g = theta.grad.cpu().numpy()
    c = coef.cpu().numpy()
    ctx.close()
    for i in range(w.N):
        r = oracle_pf(oracle, w, theta_np, 0, i, k=2)
        assert got_l[0, i] == pytest.approx(r["loglik"], rel=1e-12)
        assert rel_err(got_g[0, i], c[0, i] * r["grad"]) <= 1e-9


def test_pf_loglik_autograd_refuses_a_context_without_gradients():
    """A context reserved with want_grad = 0 has no gradient to hand to backward: the autograd
    function refuses it instead of returning an unwritten buffer as the gradient."""
    import torch
    dev = torch.device("cuda:0")
    w = synth.make(0, N=4)
    model = smc2.Model.from_workload(w)
    ctx = smc2.Context(model, smc2.pf_opts(precision=smc2.FP64, want_grad=0), w.S, w.N, w.M,
                       w.T_len, w.T_max)
    theta = torch.zeros((w.S, w.N, w.D), dtype=torch.float64, device=dev, requires_grad=True)
    y = torch.tensor(w.y, dtype=torch.float64, device=dev)
    it = torch.tensor([2], dtype=torch.int32, device=dev)
    with pytest.raises(ValueError, match="want_grad"):
        smc2.PFLogLik.apply(theta, y, ctx, w.seed, it)
    ctx.close()
