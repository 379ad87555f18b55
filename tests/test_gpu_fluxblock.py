"""GPU parity of the flux block (Sec. 3.4, Eqs. 5-8) through the C ABI
against the FP64 oracle: the FV step with uniform 5x4 kernels and face
fields, its adjoint (state, kernel and field gradients), the two FNOs and
the model step.

Tolerances: the FV step and its adjoint keep the plain step's bars (rel-L2
1e-5 per FP32 step, 1e-12 in FP64; adjoint 1e-4 in FP32).  The FNO runs in
FP32 through L layers of two 2D FFTs (O(log2 N) rounding steps each) and a
C-term complex sum per mode: about L (2 log2 N + C) 2^-24 ~ 6 (24 + 16)
6e-8 ~ 1.4e-5 relative; the bar is 1e-4."""
import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle import fluxblock, fno, fv, ic, timestep
from tests.gpu_common import assert_fields_close, L, announce, cpu64, dev, need_gpu, oracle_prm, rel_l2

pytestmark = pytest.mark.gpu

KW = dict(nu=0.01, dt=0.02, forcing_amp=1.0, forcing_k=4.0, drag=0.1)


def _stencils(seed, scale=0.05):
    w = np.stack([si.stencil_weights(seed, scale), si.stencil_weights(seed + 1, scale)])
    return torch.tensor(w, dtype=torch.float32)                     # [2, 4, 20]


def _fields(seed, b, n, m, scale=0.05):
    return torch.tensor(si.random_field(seed, (b, 8, m, n), scale=scale), dtype=torch.float32)


def _record(w32, f32):
    w = w32.double()
    f = f32.double() if f32 is not None else None
    return {"wi": w[0], "wd": w[1], "fi": f[:, :4] if f is not None else None,
            "fd": f[:, 4:] if f is not None else None}


@pytest.mark.parametrize("nx,ny,b,dtype,tol", [
    (64, 64, 2, torch.float32, 1e-5), (128, 32, 3, torch.float32, 1e-5),
    (32, 32, 2, torch.float64, 1e-12)])
def test_fluxblock_fv_step_matches_oracle(nx, ny, b, dtype, tol):
    L_ = need_gpu()
    announce("fluxblock fv step", nx, ny, b, dtype)
    s = L_.Solver(nx, ny, b, dtype=dtype)
    u0, v0 = ic.grf_peak(b, nx, ny, L, L, seed=5)
    u = dev(u0, dtype)
    v = dev(v0, dtype)
    w = _stencils(7)
    f = _fields(9, b, nx, ny)
    prm = L_.params(**KW)
    uo, vo = s.fluxblock_fv_step(prm, w.cuda(), f.cuda(), u, v, nsteps=2)
    ref = timestep.fv_step(cpu64(u), cpu64(v), oracle_prm(nx, ny, **KW), nsteps=2,
                           flux=_record(w, f))
    assert rel_l2(uo, ref[0]) < tol and rel_l2(vo, ref[1]) < tol


def test_empty_flux_block_is_the_plain_step():
    """Zero kernels and fields leave the physics operator: the plain step's
    result up to the different association of the viscous product (the flux
    block forms nu * (D + learned), the plain path nu * D_sum / (24 h))."""
    L_ = need_gpu()
    announce("fluxblock zero")
    n, b = 64, 2
    s = L_.Solver(n, n, b)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=6)
    u, v = dev(u0, torch.float32), dev(v0, torch.float32)
    prm = L_.params(**KW)
    w = torch.zeros(2, 4, 20, device="cuda")
    f = torch.zeros(b, 8, n, n, device="cuda")
    a = s.fluxblock_fv_step(prm, w, f, u, v)
    p = s.fv_step(prm, u, v)
    assert rel_l2(a[0], p[0]) < 1e-6 and rel_l2(a[1], p[1]) < 1e-6


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_fluxblock_fv_step_bwd_matches_oracle_autograd(dtype, tol):
    L_ = need_gpu()
    announce("fluxblock fv step bwd", dtype)
    n, b = 32, 2
    s = L_.Solver(n, n, b, dtype=dtype)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=15)
    u, v = dev(u0, dtype), dev(v0, dtype)
    w = _stencils(17)
    f = _fields(19, b, n, n)
    g = torch.Generator().manual_seed(3)
    gu_out = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    gv_out = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    prm = L_.params(**KW)
    gw = torch.zeros(2, 4, 20, device="cuda")
    gf = torch.zeros(b, 8, n, n, device="cuda")
    gu, gv = s.fluxblock_fv_step_bwd(prm, w.cuda(), f.cuda(), u, v, dev(gu_out, dtype),
                                     dev(gv_out, dtype), gstencil=gw, gfields=gf)
    ua, va = cpu64(u).requires_grad_(True), cpu64(v).requires_grad_(True)
    wr = w.double().requires_grad_(True)
    fr = f.double().requires_grad_(True)
    rec = {"wi": wr[0], "wd": wr[1], "fi": fr[:, :4], "fd": fr[:, 4:]}
    x, y = timestep.fv_step(ua, va, oracle_prm(n, n, **KW), flux=rec)
    ((gu_out * x).sum() + (gv_out * y).sum()).backward()
    assert rel_l2(gu, ua.grad) < tol and rel_l2(gv, va.grad) < tol
    # the kernel and field gradients are stored in float32 whatever the grid
    # dtype: one rounding, 2^-24 relative
    gtol = max(tol, 2e-7)
    assert rel_l2(gw, wr.grad) < gtol
    assert rel_l2(gf, fr.grad) < gtol


def _fno_pair(seed, cfg, out_scale=0.05):
    layers, modes, width = si.FLUXBLOCK_FNO[cfg]
    a_i = si.fno_weights(seed, width, layers, modes, out_scale=out_scale)
    a_d = si.fno_weights(seed + 1, width, layers, modes, out_scale=out_scale)
    return a_i, a_d


@pytest.mark.parametrize("cfg,n,b,ny", [("forced", 64, 4, 64), ("decaying", 128, 2, 128),
                                         ("forced", 128, 2, 128), ("decaying", 64, 3, 32)])
def test_fno_forward_matches_oracle(cfg, n, b, ny):
    """Both FNOs at the paper's hyper-parameters (forced: 6 layers, 32 modes,
    width 16; decaying: 4 layers, 16 modes, width 8) on 64^2, 128^2 (16
    values per thread in the transforms) and a non-square 64 x 32 grid; the
    last layer is given O(1) weights so the fields are not small."""
    L_ = need_gpu()
    announce("fno forward", cfg, n, ny, b)
    s = L_.Solver(n, ny, b)
    a_i, a_d = _fno_pair(21, cfg, out_scale=1.0)
    net = L_.FluxNetParams(_stencils(23), L_.FnoParams.from_arrays(a_i),
                           L_.FnoParams.from_arrays(a_d))
    u0, v0 = ic.grf_peak(b, n, ny, L, L, seed=25)
    u, v = dev(u0, torch.float32), dev(v0, torch.float32)
    got = s.fno_forward(net, u, v)
    x = torch.stack([cpu64(u), cpu64(v)], dim=1)
    ref_i = fno.fno_forward(x, fno.from_arrays(a_i))
    ref_d = fno.fno_forward(x, fno.from_arrays(a_d))
    assert rel_l2(got[:, :4], ref_i) < 1e-4
    assert rel_l2(got[:, 4:], ref_d) < 1e-4


def test_fno_forward_one_operator_and_none():
    """An absent operator gives zero fields; a present one is unaffected."""
    L_ = need_gpu()
    announce("fno forward absent")
    n, b = 64, 2
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(31, "decaying", out_scale=1.0)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=33)
    u, v = dev(u0, torch.float32), dev(v0, torch.float32)
    only_d = L_.FluxNetParams(_stencils(1), None, L_.FnoParams.from_arrays(a_d))
    got = s.fno_forward(only_d, u, v)
    assert torch.count_nonzero(got[:, :4]).item() == 0
    x = torch.stack([cpu64(u), cpu64(v)], dim=1)
    assert rel_l2(got[:, 4:], fno.fno_forward(x, fno.from_arrays(a_d))) < 1e-4
    none = L_.FluxNetParams(_stencils(1))
    assert torch.count_nonzero(s.fno_forward(none, u, v)).item() == 0


@pytest.mark.parametrize("cfg,n,b", [("forced", 64, 4), ("decaying", 128, 2)])
def test_fluxblock_step_matches_oracle(cfg, n, b):
    L_ = need_gpu()
    announce("fluxblock step", cfg, n, b)
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(41, cfg)
    w = _stencils(43)
    net = L_.FluxNetParams(w, L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=45)
    u, v = dev(u0, torch.float32), dev(v0, torch.float32)
    kw = KW if cfg == "forced" else dict(nu=1e-3, dt=0.0035)
    prm = L_.params(**kw)
    uo, vo, f = s.fluxblock_step(prm, net, u, v, want_fields=True)
    params = {"wi": w[0].double(), "wd": w[1].double(), "fno_i": fno.from_arrays(a_i),
              "fno_d": fno.from_arrays(a_d)}
    ru, rv = fluxblock.fluxblock_step(cpu64(u), cpu64(v), oracle_prm(n, n, **kw), params)
    assert rel_l2(uo, ru) < 1e-5 and rel_l2(vo, rv) < 1e-5
    # the step used the fields it returned
    a = s.fluxblock_fv_step(prm, net.stencil_w, f, u, v)
    assert torch.equal(a[0], uo) and torch.equal(a[1], vo)


def _fno_grads_ref(x, a, gF):
    """Oracle autograd of sum(gF * FNO(x)) in every parameter and in x."""
    p = fno.from_arrays(a)
    leaves = [p["P_w"], p["P_b"], p["Q_w"], p["Q_b"]]
    for lay in p["layers"]:
        leaves += [lay["R"], lay["W"], lay["b"]]
    for t in leaves:
        t.requires_grad_(True)
    xr = x.clone().requires_grad_(True)
    (gF * fno.fno_forward(xr, p)).sum().backward()
    return p, xr.grad


def _check_fno_grads(gb, p, tol):
    assert rel_l2(gb.lift_w, p["P_w"].grad) < tol
    assert rel_l2(gb.lift_b, p["P_b"].grad) < tol
    assert rel_l2(gb.proj_w, p["Q_w"].grad) < tol
    # the output bias of the derivative operator has an exactly zero gradient
    # inside the step (a uniform offset of every face derivative cancels in
    # the flux differences): compare on the scale of the projection weights
    scale = max(p["Q_b"].grad.norm().item(), p["Q_w"].grad.norm().item())
    assert (gb.proj_b.double().cpu() - p["Q_b"].grad).norm().item() < tol * scale
    spec = gb.spec_complex()
    for l, lay in enumerate(p["layers"]):
        assert rel_l2(gb.point_w[l], lay["W"].grad) < tol, l
        # (the last layer's bias feeds the projection linearly: the same
        # exact zero for the derivative operator)
        sc = max(lay["b"].grad.norm().item(), lay["W"].grad.norm().item())
        assert (gb.point_b[l].double().cpu() - lay["b"].grad).norm().item() < tol * sc, l
        r = spec[l].cpu()
        ref = lay["R"].grad
        err = ((r.to(torch.complex128) - ref).abs().norm() / ref.abs().norm()).item()
        assert err < tol, (l, err)


@pytest.mark.parametrize("cfg,n,b", [("forced", 64, 2), ("decaying", 128, 2)])
def test_fno_backward_matches_oracle_autograd(cfg, n, b):
    """Every FNO parameter gradient (the complex spectral weights in torch's
    d/dRe + i d/dIm convention) and the input gradient, both operators."""
    L_ = need_gpu()
    announce("fno backward", cfg, n, b)
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(51, cfg, out_scale=1.0)
    net = L_.FluxNetParams(_stencils(53), L_.FnoParams.from_arrays(a_i),
                           L_.FnoParams.from_arrays(a_d))
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=55)
    u, v = dev(u0, torch.float32), dev(v0, torch.float32)
    gF = torch.tensor(si.random_field(57, (b, 8, n, n)), dtype=torch.float32)
    gb = L_.FluxNetGradBuffers(net)
    gu, gv = s.fno_backward(net, u, v, gF.cuda(), gb)
    x = torch.stack([cpu64(u), cpu64(v)], dim=1)
    p_i, gx_i = _fno_grads_ref(x, a_i, gF[:, :4].double())
    p_d, gx_d = _fno_grads_ref(x, a_d, gF[:, 4:].double())
    _check_fno_grads(gb.fno[0], p_i, 1e-4)
    _check_fno_grads(gb.fno[1], p_d, 1e-4)
    gx = gx_i + gx_d
    assert rel_l2(gu, gx[:, 0]) < 1e-4 and rel_l2(gv, gx[:, 1]) < 1e-4
    # deterministic: a second call accumulates exactly the same numbers
    before = [t.clone() for f in gb.fno for t in f.tensors()]
    gu2, gv2 = s.fno_backward(net, u, v, gF.cuda(), gb)
    assert torch.equal(gu, gu2) and torch.equal(gv, gv2)
    for t0, t1 in zip(before, [t for f in gb.fno for t in f.tensors()]):
        assert torch.equal(2 * t0, t1)


def test_fluxblock_step_bwd_matches_oracle_autograd():
    """The gradient of the whole flux-block step: state, uniform kernels and
    both FNOs (forced configuration at 64^2)."""
    L_ = need_gpu()
    announce("fluxblock step bwd")
    n, b = 64, 2
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(61, "forced", out_scale=0.2)
    w = _stencils(63)
    net = L_.FluxNetParams(w, L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=65)
    u, v = dev(u0, torch.float32), dev(v0, torch.float32)
    g = torch.Generator().manual_seed(67)
    gu_out = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    gv_out = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    prm = L_.params(**KW)
    gb = L_.FluxNetGradBuffers(net)
    gu, gv = s.fluxblock_step_bwd(prm, net, u, v, dev(gu_out, torch.float32),
                                  dev(gv_out, torch.float32), gb)
    p_i, p_d = fno.from_arrays(a_i), fno.from_arrays(a_d)
    leaves = []
    for p in (p_i, p_d):
        leaves += [p["P_w"], p["P_b"], p["Q_w"], p["Q_b"]]
        for lay in p["layers"]:
            leaves += [lay["R"], lay["W"], lay["b"]]
    wr = w.double().requires_grad_(True)
    for t in leaves:
        t.requires_grad_(True)
    ua, va = cpu64(u).requires_grad_(True), cpu64(v).requires_grad_(True)
    params = {"wi": wr[0], "wd": wr[1], "fno_i": p_i, "fno_d": p_d}
    x, y = fluxblock.fluxblock_step(ua, va, oracle_prm(n, n, **KW), params)
    ((gu_out * x).sum() + (gv_out * y).sum()).backward()
    assert rel_l2(gu, ua.grad) < 1e-4 and rel_l2(gv, va.grad) < 1e-4
    assert rel_l2(gb.stencil_w, wr.grad) < 1e-4
    _check_fno_grads(gb.fno[0], p_i, 1e-4)
    _check_fno_grads(gb.fno[1], p_d, 1e-4)


def test_fluxblock_autograd_function_is_the_adjoint():
    L_ = need_gpu()
    from paper_2507_01975_amd import autograd as A
    announce("fluxblock autograd")
    n, b = 64, 2
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(71, "decaying", out_scale=0.2)
    net = L_.FluxNetParams(_stencils(73), L_.FnoParams.from_arrays(a_i),
                           L_.FnoParams.from_arrays(a_d))
    params = A._fluxblock_params(net)
    for p in params:
        p.requires_grad_(True)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=75)
    u = dev(u0, torch.float32).requires_grad_(True)
    v = dev(v0, torch.float32).requires_grad_(True)
    prm = L_.params(**KW)
    wu, wv = (torch.randn(b, n, n, generator=torch.Generator().manual_seed(77)).cuda()
              for _ in range(2))
    uo, vo = A.fluxblock_step(s, prm, net, u, v)
    ((wu * uo).sum() + (wv * vo).sum()).backward()
    gb = L_.FluxNetGradBuffers(net)
    gu, gv = s.fluxblock_step_bwd(prm, net, u.detach(), v.detach(), wu, wv, gb)
    assert torch.equal(u.grad, gu) and torch.equal(v.grad, gv)
    ref = [gb.stencil_w] + [t for f in gb.fno for t in f.tensors()]
    for p, r in zip(params, ref):
        assert torch.equal(p.grad, r)


def test_train_fluxblock_reduces_the_loss():
    """Teacher-student: labels from the same model with perturbed uniform
    kernels; a few Adam iterations of the unrolled loss bring the student's
    kernels toward the teacher's (the gradient itself is pinned above)."""
    L_ = need_gpu()
    from paper_2507_01975_amd import train as T
    announce("fluxblock training")
    n, b, steps = 64, 4, 10
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(81, "decaying", out_scale=0.1)
    w = _stencils(83, scale=0.01)
    teacher = L_.FluxNetParams(w + torch.tensor(si.random_field(85, (2, 4, 20), scale=0.02),
                                                dtype=torch.float32),
                               L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    student = L_.FluxNetParams(w, L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    prm = L_.params(nu=1e-3, dt=0.02)
    u, v = s.init_state(L_.IC_GRF_PEAK, seed=87)
    lu, lv = [u], [v]
    for _ in range(steps):
        u, v = s.fluxblock_step(prm, teacher, u, v)
        lu.append(u)
        lv.append(v)
    labels = (torch.stack(lu), torch.stack(lv))
    hist = T.train_fluxblock(s, student, labels, prm, iters=12, unroll=4, lr=3e-3, log_every=1)
    assert hist[-1][1] < 0.5 * hist[0][1], hist


def _tc_arrays(seed, kc, out_scale=0.1):
    # the paper's temporal-correction FNO: 4 layers, 32 modes, width 8
    return si.fno_weights(seed, 8, 4, 32, n_in=2 * kc, n_out=2, out_scale=out_scale)


def test_complete_model_rollout_matches_oracle():
    """Flux block + temporal correction every k_c = 2 steps (Eq. 2), forced
    configuration at 64^2: every state of a 4-step rollout."""
    L_ = need_gpu()
    announce("complete model rollout")
    n, b, kc, T = 64, 2, 2, 4
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(91, "forced")
    w = _stencils(93)
    a_tc = _tc_arrays(95, kc)
    net = L_.FluxNetParams(w, L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    tc = L_.FnoParams.from_arrays(a_tc)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=97)
    prm = L_.params(k_c=kc, **KW)
    hu, hv = [dev(u0, torch.float32)], [dev(v0, torch.float32)]
    for k in range(1, T + 1):
        pu = hu[-kc:] if len(hu) >= kc else [hu[0]] * (kc - len(hu)) + hu
        pv = hv[-kc:] if len(hv) >= kc else [hv[0]] * (kc - len(hv)) + hv
        u, v = s.fluxblock_tc_step(prm, net, tc, pu, pv, k)
        hu.append(u)
        hv.append(v)
    params = {"wi": w[0].double(), "wd": w[1].double(), "fno_i": fno.from_arrays(a_i),
              "fno_d": fno.from_arrays(a_d), "tc": fno.from_arrays(a_tc)}
    ru, rv = fluxblock.model_rollout(cpu64(hu[0]), cpu64(hv[0]), oracle_prm(n, n, k_c=kc, **KW),
                                     params, T)
    for k in range(T):
        assert rel_l2(hu[k + 1], ru[k]) < 1e-5 and rel_l2(hv[k + 1], rv[k]) < 1e-5, k


def test_complete_model_step_bwd_matches_oracle_autograd():
    """The adjoint of a corrected step (k = k_c = 2): gradients of both
    history states, the flux block and the correction's FNO."""
    L_ = need_gpu()
    announce("complete model step bwd")
    n, b, kc = 64, 2, 2
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(101, "decaying", out_scale=0.2)
    w = _stencils(103)
    a_tc = _tc_arrays(105, kc, out_scale=0.5)
    net = L_.FluxNetParams(w, L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    tc = L_.FnoParams.from_arrays(a_tc)
    u0, v0 = ic.grf_peak(b, n, n, L, L, seed=107)
    prm = L_.params(k_c=kc, **KW)
    hu = [dev(u0, torch.float32)]
    hv = [dev(v0, torch.float32)]
    u1, v1 = s.fluxblock_step(prm, net, hu[0], hv[0])
    hu.append(u1)
    hv.append(v1)
    g = torch.Generator().manual_seed(109)
    gu_out = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    gv_out = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    gb = L_.FluxNetGradBuffers(net)
    gtc = L_.FnoGradBuffers(tc)
    ghu = [torch.zeros_like(x) for x in hu]
    ghv = [torch.zeros_like(x) for x in hv]
    s.fluxblock_tc_step_bwd(prm, net, tc, hu, hv, kc, dev(gu_out, torch.float32),
                            dev(gv_out, torch.float32), ghu, ghv, gb, gtc)
    p_i, p_d, p_tc = fno.from_arrays(a_i), fno.from_arrays(a_d), fno.from_arrays(a_tc)
    leaves = []
    for p in (p_i, p_d, p_tc):
        leaves += [p["P_w"], p["P_b"], p["Q_w"], p["Q_b"]]
        for lay in p["layers"]:
            leaves += [lay["R"], lay["W"], lay["b"]]
    for t in leaves:
        t.requires_grad_(True)
    wr = w.double().requires_grad_(True)
    xs = [cpu64(t).requires_grad_(True) for t in hu + hv]
    params = {"wi": wr[0], "wd": wr[1], "fno_i": p_i, "fno_d": p_d, "tc": p_tc}
    x, y = fluxblock.model_step(xs[:2], xs[2:], oracle_prm(n, n, k_c=kc, **KW), params, kc)
    ((gu_out * x).sum() + (gv_out * y).sum()).backward()
    for j in range(2):
        assert rel_l2(ghu[j], xs[j].grad) < 1e-4, j
        assert rel_l2(ghv[j], xs[2 + j].grad) < 1e-4, j
    assert rel_l2(gb.stencil_w, wr.grad) < 1e-4
    _check_fno_grads(gb.fno[0], p_i, 1e-4)
    _check_fno_grads(gb.fno[1], p_d, 1e-4)
    _check_fno_grads(gtc, p_tc, 1e-4)


def test_train_complete_model_reduces_the_loss():
    """Teacher-student with the temporal correction: the student's
    correction starts at zero output and learns the teacher's."""
    L_ = need_gpu()
    from paper_2507_01975_amd import train as T
    announce("complete model training")
    n, b, kc, steps = 64, 4, 2, 10
    s = L_.Solver(n, n, b)
    a_i, a_d = _fno_pair(111, "decaying", out_scale=0.1)
    w = _stencils(113, scale=0.01)
    net = L_.FluxNetParams(w, L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    teacher_tc = L_.FnoParams.from_arrays(_tc_arrays(115, kc, out_scale=0.3))
    student_tc = L_.FnoParams.from_arrays(_tc_arrays(115, kc, out_scale=0.0))
    prm = L_.params(nu=1e-3, dt=0.02, k_c=kc)
    u, v = s.init_state(L_.IC_GRF_PEAK, seed=117)
    lu, lv = [u], [v]
    for k in range(1, steps + 1):
        hu = [lu[max(0, k - kc + j)] for j in range(kc)]
        hv = [lv[max(0, k - kc + j)] for j in range(kc)]
        u, v = s.fluxblock_tc_step(prm, net, teacher_tc, hu, hv, k)
        lu.append(u)
        lv.append(v)
    labels = (torch.stack(lu), torch.stack(lv))
    hist = T.train_fluxblock(s, net, labels, prm, iters=12, unroll=4, lr=3e-3, log_every=1,
                             tc=student_tc)
    assert hist[-1][1] < 0.5 * hist[0][1], hist


def test_kolmogorov64_full_size_fluxblock_step_and_correction():
    """The flux-block step at the benchmark's configuration (64^2, batch 64,
    the forced-flow FNOs of 6 layers, 32 modes, width 16, the bench's
    weights) in the launch configuration it times, every trajectory against
    the oracle in L2 and element by element; then one step of the complete
    model with the temporal correction (k_c = 4), also on every trajectory."""
    L_ = need_gpu()
    announce("kolmogorov64 flux-block step")
    w = si.WORKLOADS["kolmogorov64"]
    n, B = w["nx"], w["batch"]
    layers, modes, width = si.FLUXBLOCK_FNO["forced"]
    ws = np.stack([si.stencil_weights(0, 0.01), si.stencil_weights(1, 0.01)])
    a_i = si.fno_weights(2, width, layers, modes)
    a_d = si.fno_weights(3, width, layers, modes)
    net = L_.FluxNetParams(ws, L_.FnoParams.from_arrays(a_i), L_.FnoParams.from_arrays(a_d))
    s = L_.Solver(n, n, B)
    gu, gv = s.init_state(L_.IC_GRF_PEAK, seed=200)
    kw = dict(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"], forcing_k=w["forcing_k"],
              drag=w["drag"])
    uo, vo = s.fluxblock_step(L_.params(**kw), net, gu, gv)
    params = {"wi": torch.tensor(ws[0]), "wd": torch.tensor(ws[1]),
              "fno_i": fno.from_arrays(a_i), "fno_d": fno.from_arrays(a_d)}
    ru, rv = fluxblock.fluxblock_step(cpu64(gu), cpu64(gv), oracle_prm(n, n, **kw), params)
    for b in range(B):
        assert_fields_close(uo[b], ru[b], what=("u", b))
        assert_fields_close(vo[b], rv[b], what=("v", b))
    kc = 4
    a_tc = si.fno_weights(9, 8, 4, 32, n_in=2 * kc, n_out=2)
    tc = L_.FnoParams.from_arrays(a_tc)
    hu = [gu, uo, gu, uo]
    hv = [gv, vo, gv, vo]
    cu, cv = s.fluxblock_tc_step(L_.params(k_c=kc, **kw), net, tc, hu, hv, kc)
    params["tc"] = fno.from_arrays(a_tc)
    ru, rv = fluxblock.model_step([cpu64(x) for x in hu], [cpu64(x) for x in hv],
                                  oracle_prm(n, n, k_c=kc, **kw), params, kc)
    for b in range(B):
        assert_fields_close(cu[b], ru[b], what=("u", b))
        assert_fields_close(cv[b], rv[b], what=("v", b))
