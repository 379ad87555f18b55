"""GPU checks of the torch.autograd.Function wrappers: their gradients are
the library's hand-written adjoints (the same numbers as calling the _bwd
entry points directly) and agree with the FP64 oracle's autograd."""
import pytest
import torch

import synthetic_inputs as si
from oracle import cnn, ic, learned, projection, timestep
from tests.gpu_common import L, announce, cpu64, dev, need_gpu, oracle_prm, rel_l2

pytestmark = pytest.mark.gpu

KW = dict(nu=0.01, dt=0.04, forcing_amp=1.0, forcing_k=4.0, drag=0.1)


def _weights(b, n, seed):
    g = torch.Generator().manual_seed(seed)
    return (torch.randn(b, n, n, generator=g, dtype=torch.float64).float(),
            torch.randn(b, n, n, generator=g, dtype=torch.float64).float())


def test_fv_step_function_is_the_adjoint():
    L_ = need_gpu()
    from paper_2507_01975_amd import autograd as A
    announce("autograd fv_step")
    n, b = 32, 2
    s = L_.Solver(n, n, b)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=11)
    u = dev(u0, torch.float32).requires_grad_(True)
    v = dev(v0, torch.float32).requires_grad_(True)
    coef = dev(torch.tensor(si.random_field(12, (b, 64, n, n), scale=0.1)),
               torch.float32).requires_grad_(True)
    wu, wv = _weights(b, n, 13)
    prm = L_.params(**KW)
    uo, vo = A.fv_step(s, prm, u, v, coef)
    ((wu.cuda() * uo).sum() + (wv.cuda() * vo).sum()).backward()
    # the same numbers as the entry point
    gc = torch.zeros_like(coef)
    gu, gv = s.fv_step_bwd(prm, u.detach(), v.detach(), wu.cuda(), wv.cuda(), coef=coef.detach(),
                           gcoef=gc)
    assert torch.equal(u.grad, gu) and torch.equal(v.grad, gv) and torch.equal(coef.grad, gc)
    # and the oracle's autograd
    ua = cpu64(u).requires_grad_(True)
    va = cpu64(v).requires_grad_(True)
    ra = cpu64(coef).requires_grad_(True)
    x, y = timestep.fv_step(ua, va, oracle_prm(n, n, **KW), coef=learned.constrain(ra))
    ((wu.double() * x).sum() + (wv.double() * y).sum()).backward()
    assert rel_l2(u.grad, ua.grad) < 1e-4 and rel_l2(v.grad, va.grad) < 1e-4
    assert rel_l2(coef.grad, ra.grad) < 1e-4


def test_project_function_is_self_adjoint():
    L_ = need_gpu()
    from paper_2507_01975_amd import autograd as A
    announce("autograd project")
    n, b = 64, 3
    s = L_.Solver(n, n, b)
    u0 = torch.tensor(si.smooth_field(21, b, n, n)).float()
    v0 = torch.tensor(si.smooth_field(22, b, n, n)).float()
    u = u0.cuda().requires_grad_(True)
    v = v0.cuda().requires_grad_(True)
    wu, wv = _weights(b, n, 23)
    uo, vo = A.project(s, u, v)
    ((wu.cuda() * uo).sum() + (wv.cuda() * vo).sum()).backward()
    pu, pv, _ = projection.project(wu.double(), wv.double(), oracle_prm(n, n))
    assert rel_l2(u.grad, pu) < 1e-5 and rel_l2(v.grad, pv) < 1e-5
    # the forward left its inputs untouched
    assert torch.equal(u.detach().cpu(), u0) and torch.equal(v.detach().cpu(), v0)


def _net(L_, seed, last_scale=0.05):
    ws, bs = si.cnn_weights(seed, cnn.LAYERS, last_scale=last_scale)
    return L_.NetParams([torch.tensor(w) for w in ws], [torch.tensor(b) for b in bs])


def test_learned_step_function_parameter_gradients():
    L_ = need_gpu()
    from paper_2507_01975_amd import autograd as A
    announce("autograd learned step")
    n, b = 32, 2
    s = L_.Solver(n, n, b)
    net = _net(L_, seed=31)
    params = list(net.master_w) + list(net.b)
    for p in params:
        p.requires_grad_(True)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=32)
    u = dev(u0, torch.float32).requires_grad_(True)
    v = dev(v0, torch.float32).requires_grad_(True)
    wu, wv = _weights(b, n, 33)
    prm = L_.params(k_c=1, **KW)
    uo, vo = A.learned_step(s, prm, net, u, v, 1)
    ((wu.cuda() * uo).sum() + (wv.cuda() * vo).sum()).backward()
    dW = L_.NetGradBuffers(net)
    gu, gv = s.learned_fv_step_bwd(prm, net, u.detach(), v.detach(), 1, wu.cuda(), wv.cuda(), dW)
    assert torch.equal(u.grad, gu) and torch.equal(v.grad, gv)
    for l in range(6):
        assert torch.equal(net.master_w[l].grad, dW.w[l]), l
        assert torch.equal(net.b[l].grad, dW.b[l]), l
    # against the bf16-emulating oracle's autograd
    wb = [w.double().cpu() for w in net.bf16_weights()]
    wr = [w.clone().requires_grad_(True) for w in wb]
    br = [cpu64(q).requires_grad_(True) for q in net.b]
    ua, va = cpu64(u).requires_grad_(True), cpu64(v).requires_grad_(True)
    x, y, _ = learned.learned_fv_step(ua, va, oracle_prm(n, n, k_c=1, **KW), wr, br, 1, bf16=True)
    ((wu.double() * x).sum() + (wv.double() * y).sum()).backward()
    assert rel_l2(u.grad, ua.grad) < 1e-3 and rel_l2(v.grad, va.grad) < 1e-3
    for l in range(6):
        gw = net.master_w[l].grad.permute(0, 3, 1, 2).contiguous()
        assert rel_l2(gw, wr[l].grad) < 3e-2, l


def test_rollout_function_matches_chained_steps():
    """The checkpointed rollout backward (4 steps, checkpoints every 2) gives
    the gradient of the chain of single learned steps, bit for bit (the
    recomputed segments run the same deterministic kernels on the same
    states)."""
    L_ = need_gpu()
    from paper_2507_01975_amd import autograd as A
    announce("autograd rollout")
    n, b, T = 32, 2, 4
    s = L_.Solver(n, n, b)
    prm = L_.params(k_c=1, fallback_enable=0, **KW)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=41)
    g = torch.Generator().manual_seed(42)
    wts = torch.randn(T, 2, b, n, n, generator=g, dtype=torch.float64).float().cuda()

    def run(use_rollout):
        net = _net(L_, seed=43)
        params = list(net.master_w) + list(net.b)
        for p in params:
            p.requires_grad_(True)
        u = dev(u0, torch.float32).requires_grad_(True)
        v = dev(v0, torch.float32).requires_grad_(True)
        if use_rollout:
            tu, tv = A.rollout(s, prm, net, u, v, T, first_index=1, checkpoint_every=2)
        else:
            xs, ys = [], []
            x, y = u, v
            for k in range(T):
                x, y = A.learned_step(s, prm, net, x, y, k + 1)
                xs.append(x)
                ys.append(y)
            tu, tv = torch.stack(xs), torch.stack(ys)
        ((wts[:, 0] * tu).sum() + (wts[:, 1] * tv).sum()).backward()
        return u.grad, v.grad, [p.grad for p in params], tu.detach()

    ru, rv, rp, rtu = run(True)
    cu, cv, cp, ctu = run(False)
    # the same kernels in the same order on the same values: bit for bit
    assert torch.equal(rtu, ctu)
    assert torch.equal(ru, cu) and torch.equal(rv, cv)
    for a, c in zip(rp, cp):
        assert torch.equal(a, c)


def test_learned_d_step_function_parameter_gradients():
    """The two-network step as an autograd Function returns the numbers of the
    step adjoint entry point bit for bit, for the state and both networks."""
    L_ = need_gpu()
    from paper_2507_01975_amd import autograd as A
    announce("autograd learned_d step")
    n, b = 32, 2
    s = L_.Solver(n, n, b)
    net = _net(L_, seed=41)
    dnet = _net(L_, seed=42)
    params = list(net.master_w) + list(net.b) + list(dnet.master_w) + list(dnet.b)
    for p in params:
        p.requires_grad_(True)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=43)
    u = dev(u0, torch.float32).requires_grad_(True)
    v = dev(v0, torch.float32).requires_grad_(True)
    wu, wv = _weights(b, n, 44)
    prm = L_.params(k_c=1, **KW)
    uo, vo = A.learned_d_step(s, prm, net, dnet, u, v, 1)
    ((wu.cuda() * uo).sum() + (wv.cuda() * vo).sum()).backward()
    dW, dWd = L_.NetGradBuffers(net), L_.NetGradBuffers(dnet)
    gu, gv = s.learned_d_fv_step_bwd(prm, net, dnet, u.detach(), v.detach(), 1, wu.cuda(),
                                     wv.cuda(), dW, dWd)
    assert torch.equal(u.grad, gu) and torch.equal(v.grad, gv)
    for l in range(6):
        assert torch.equal(net.master_w[l].grad, dW.w[l]), l
        assert torch.equal(dnet.master_w[l].grad, dWd.w[l]), l
        assert torch.equal(net.b[l].grad, dW.b[l]) and torch.equal(dnet.b[l].grad, dWd.b[l]), l
