"""GPU checks of the hand-written adjoint of the FV step: FP64 adjoint
against FP64 central finite differences of the device's own forward step
(16^2, 4 steps), FP32 adjoint against the oracle's autograd, the projection's
symmetry, and the coefficient gradient."""
import math

import pytest
import torch

import synthetic_inputs as si
from oracle import fv, ic, learned, timestep
from tests.gpu_common import L, announce, cpu64, dev, need_gpu, oracle_prm, rel_l2

pytestmark = pytest.mark.gpu

KW = dict(nu=0.01, dt=0.04, forcing_amp=1.0, forcing_k=4.0, drag=0.1)


def _setup(L_, n, b, dtype, seed=3, learned_coef=True):
    s = L_.Solver(n, n, b, dtype=dtype)
    u, v = ic.grf_peak(b, n, n, L, L, seed=seed)
    u, v = dev(u, dtype), dev(v, dtype)
    coef = None
    if learned_coef:
        coef = dev(torch.tensor(si.random_field(seed + 1, (b, 64, n, n), scale=0.1)), torch.float32)
    return s, u, v, coef


@pytest.mark.parametrize("learned_coef", [False, True])
def test_fp64_adjoint_vs_central_differences_4_steps(learned_coef):
    L_ = need_gpu()
    announce("adjoint fd", learned_coef)
    n, b, steps = 16, 2, 4
    s, u, v, coef = _setup(L_, n, b, torch.float64, learned_coef=learned_coef)
    prm = L_.params(**KW)
    g = torch.Generator().manual_seed(0)
    wu = dev(torch.randn(b, n, n, generator=g, dtype=torch.float64), torch.float64)
    wv = dev(torch.randn(b, n, n, generator=g, dtype=torch.float64), torch.float64)

    def loss(a, c):
        x, y = a
        x, y = s.fv_step(prm, x, y, nsteps=steps, coef=c)
        return ((wu * x).sum() + (wv * y).sum()).item()

    # reverse sweep through the 4 steps
    states = [(u, v)]
    for _ in range(steps):
        states.append(s.fv_step(prm, *states[-1], coef=coef))
    gu, gv = wu.clone(), wv.clone()
    gc = torch.zeros_like(coef) if coef is not None else None
    for k in reversed(range(steps)):
        gu, gv = s.fv_step_bwd(prm, *states[k], gu, gv, coef=coef, gcoef=gc)
    for trial in range(3):
        du = dev(torch.randn(b, n, n, generator=g, dtype=torch.float64), torch.float64)
        dv = dev(torch.randn(b, n, n, generator=g, dtype=torch.float64), torch.float64)
        dc = None
        if coef is not None:
            dc = torch.randn(coef.shape, generator=g, dtype=torch.float32).cuda() * 1e-4
        h = 1e-6
        # the coefficients are float32: the step actually taken is cp - coef
        cp = cm = coef
        if coef is not None:
            cp = coef + dc
            cm = coef - dc
        fd_u = (loss((u + h * du, v + h * dv), coef) - loss((u - h * du, v - h * dv), coef)) / (2 * h)
        ad_u = (gu * du).sum().item() + (gv * dv).sum().item()
        assert abs(fd_u - ad_u) <= 1e-6 * abs(ad_u) + 1e-9, (trial, fd_u, ad_u)
        if coef is not None:
            fd_c = (loss((u, v), cp) - loss((u, v), cm)) / 2.0
            # the steps taken are cp - coef and coef - cm (float32 rounding);
            # the central difference matches their mean to O(|dc|^2)
            ad_c = (gc.double() * (cp.double() - cm.double()) * 0.5).sum().item()
            assert abs(fd_c - ad_c) <= 1e-5 * abs(ad_c) + 1e-12, (trial, fd_c, ad_c)


def test_fp32_adjoint_vs_oracle_autograd():
    L_ = need_gpu()
    announce("adjoint fp32 vs autograd")
    n, b = 32, 2
    s, u, v, coef = _setup(L_, n, b, torch.float32, seed=5)
    prm = L_.params(**KW)
    g = torch.Generator().manual_seed(1)
    wu = torch.randn(b, n, n, generator=g, dtype=torch.float64).float()
    wv = torch.randn(b, n, n, generator=g, dtype=torch.float64).float()
    gc = torch.zeros_like(coef)
    gu, gv = s.fv_step_bwd(prm, u, v, wu.cuda(), wv.cuda(), coef=coef, gcoef=gc)
    # oracle
    ua = cpu64(u).requires_grad_(True)
    va = cpu64(v).requires_grad_(True)
    ra = cpu64(coef).requires_grad_(True)
    x, y = timestep.fv_step(ua, va, oracle_prm(n, n, **KW), coef=learned.constrain(ra))
    ((wu.double() * x).sum() + (wv.double() * y).sum()).backward()
    assert rel_l2(gu, ua.grad) < 1e-4 and rel_l2(gv, va.grad) < 1e-4
    assert rel_l2(gc, ra.grad) < 1e-4


def test_plain_adjoint_vs_oracle_autograd_nonsquare():
    L_ = need_gpu()
    announce("adjoint plain nonsquare")
    nx, ny, b = 32, 16, 3
    s = L_.Solver(nx, ny, b, dtype=torch.float64, ly=L / 2)
    u, v = ic.grf_peak(b, nx, ny, L, L / 2, seed=9)
    g = torch.Generator().manual_seed(2)
    wu = torch.randn(b, ny, nx, generator=g, dtype=torch.float64)
    wv = torch.randn(b, ny, nx, generator=g, dtype=torch.float64)
    gu, gv = s.fv_step_bwd(L_.params(**KW), dev(u, torch.float64), dev(v, torch.float64),
                           dev(wu, torch.float64), dev(wv, torch.float64))
    ua = u.clone().requires_grad_(True)
    va = v.clone().requires_grad_(True)
    x, y = timestep.fv_step(ua, va, oracle_prm(nx, ny, ly=L / 2, **KW))
    ((wu * x).sum() + (wv * y).sum()).backward()
    assert rel_l2(gu, ua.grad) < 1e-12 and rel_l2(gv, va.grad) < 1e-12


def test_projection_is_self_adjoint_on_device():
    L_ = need_gpu()
    announce("projection symmetric")
    n, b = 32, 2
    s = L_.Solver(n, n, b, dtype=torch.float64)
    g = torch.Generator().manual_seed(3)
    a = [dev(torch.randn(b, n, n, generator=g, dtype=torch.float64), torch.float64) for _ in range(4)]
    pa = [x.clone() for x in a[:2]]
    pb = [x.clone() for x in a[2:]]
    s.project(*pa)
    s.project_bwd(*pb)
    lhs = (pa[0] * a[2]).sum() + (pa[1] * a[3]).sum()
    rhs = (a[0] * pb[0]).sum() + (a[1] * pb[1]).sum()
    assert abs(lhs.item() - rhs.item()) < 1e-11 * abs(lhs.item())


def _net(L_, seed, last_scale=0.05):
    from oracle import cnn
    ws, bs = si.cnn_weights(seed, cnn.LAYERS, last_scale=last_scale)
    net = L_.NetParams([torch.tensor(w) for w in ws], [torch.tensor(b) for b in bs])
    wb = [w.double().cpu() for w in net.bf16_weights()]
    bb = [b.double().cpu() for b in net.b]
    return net, wb, bb


@pytest.mark.parametrize("nx,ny,b", [(16, 16, 2), (32, 16, 1), (64, 64, 2)])
def test_cnn_backward_vs_oracle_autograd(nx, ny, b):
    from oracle import cnn
    L_ = need_gpu()
    announce("cnn backward", nx, ny, b)
    net, wb, bb = _net(L_, seed=2, last_scale=1.0)
    u, v = ic.grf_peak(b, nx, ny, L, L, seed=4)
    u, v = u.float(), v.float()
    s = L_.Solver(nx, ny, b)
    g = torch.Generator().manual_seed(5)
    R = torch.randn(b, 66, ny, nx, generator=g, dtype=torch.float64)
    dW = L_.NetGradBuffers(net)
    gu, gv = s.cnn_backward(net, dev(u, torch.float32), dev(v, torch.float32),
                            dev(R, torch.float32), dW)
    x = torch.stack([u.double(), v.double()], dim=1).requires_grad_(True)
    wr = [w.clone().requires_grad_(True) for w in wb]
    br = [q.clone().requires_grad_(True) for q in bb]
    out = cnn.cnn_forward(x, wr, br, bf16=True)
    (R * out).sum().backward()
    for l in range(6):
        gw = dW.w[l].permute(0, 3, 1, 2).contiguous()   # [Cout][3][3][Cin] -> [Cout][Cin][3][3]
        assert rel_l2(gw, wr[l].grad) < 2e-2, l
        assert rel_l2(dW.b[l], br[l].grad) < 2e-2, l
    assert rel_l2(gu, x.grad[:, 0]) < 2e-2 and rel_l2(gv, x.grad[:, 1]) < 2e-2


def test_learned_step_backward_vs_oracle_autograd():
    from oracle import cnn
    L_ = need_gpu()
    announce("learned step backward")
    n, b = 32, 2
    net, wb, bb = _net(L_, seed=3, last_scale=0.05)
    u, v = ic.grf_peak(b, n, n, L, L, seed=6)
    u, v = u.float(), v.float()
    s = L_.Solver(n, n, b)
    prm = L_.params(k_c=1, **KW)
    g = torch.Generator().manual_seed(6)
    wu = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    wv = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    dW = L_.NetGradBuffers(net)
    gu, gv = s.learned_fv_step_bwd(prm, net, dev(u, torch.float32), dev(v, torch.float32), 1,
                                   dev(wu, torch.float32), dev(wv, torch.float32), dW)
    ua = u.double().requires_grad_(True)
    va = v.double().requires_grad_(True)
    wr = [w.clone().requires_grad_(True) for w in wb]
    br = [q.clone().requires_grad_(True) for q in bb]
    x, y, _ = learned.learned_fv_step(ua, va, oracle_prm(n, n, k_c=1, **KW), wr, br, 1, bf16=True)
    ((wu * x).sum() + (wv * y).sum()).backward()
    assert rel_l2(gu, ua.grad) < 1e-3 and rel_l2(gv, va.grad) < 1e-3
    for l in range(6):
        gw = dW.w[l].permute(0, 3, 1, 2).contiguous()
        assert rel_l2(gw, wr[l].grad) < 3e-2, l
        assert rel_l2(dW.b[l], br[l].grad) < 3e-2, l
