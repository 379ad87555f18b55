"""GPU parity of the per-cell learned derivative stencils (Sec. 3.4, the
m = d operator in per-cell form) against the FP64 oracle through the C ABI:
the FV step with given raw derivative values (several tile shapes, RK4 and
SSP-RK3), its adjoint, the learned step with the derivative network beside
the coefficient network, its adjoint, the rollout and training."""
import pytest
import torch

import synthetic_inputs as si
from oracle import cnn, ic, learned, timestep
from oracle.projection import project
from tests.gpu_common import assert_fields_close, L, announce, cpu64, dev, need_gpu, oracle_prm, rel_l2

pytestmark = pytest.mark.gpu

KW = dict(nu=1e-2, dt=0.02, forcing_amp=1.0, forcing_k=4.0, drag=0.1)


def _fields(nx, ny, b, seed):
    u, v = ic.grf_peak(b, nx, ny, L, L, seed=seed)
    u, v = u.float().double(), v.float().double()
    coef = torch.tensor(si.random_field(seed + 1, (b, 64, ny, nx), scale=0.1)).float()
    dcoef = torch.tensor(si.random_field(seed + 2, (b, 64, ny, nx), scale=0.1)).float()
    return u, v, coef, dcoef


@pytest.mark.parametrize("nx,ny,b,rk,nsteps", [(32, 32, 2, 0, 1), (64, 16, 3, 0, 2),
                                               (128, 64, 1, 0, 1), (8, 8, 2, 0, 1),
                                               (32, 16, 2, 1, 1)])
def test_fv_step_d_matches_oracle(nx, ny, b, rk, nsteps):
    L_ = need_gpu()
    announce("fv_step_d", nx, ny, b, rk, nsteps)
    u, v, coef, dcoef = _fields(nx, ny, b, seed=11)
    s = L_.Solver(nx, ny, b)
    prm = L_.params(rk=rk, **KW)
    uo, vo = s.fv_step_d(prm, dev(u, torch.float32), dev(v, torch.float32), coef.cuda(),
                         dcoef.cuda(), nsteps=nsteps)
    oprm = oracle_prm(nx, ny, rk=rk, **KW)
    eu, ev = timestep.fv_step(u, v, oprm, learned.constrain(coef.double()), nsteps=nsteps,
                              dcoef=learned.constrain_deriv(dcoef.double()))
    e = (rel_l2(uo, eu), rel_l2(vo, ev))
    print("rel-L2", e)
    assert e[0] < 1e-5 and e[1] < 1e-5


def test_zero_derivative_values_give_the_coefficient_step():
    L_ = need_gpu()
    announce("fv_step_d zero")
    nx = ny = 64
    b = 2
    u, v, coef, _ = _fields(nx, ny, b, seed=12)
    s = L_.Solver(nx, ny, b)
    prm = L_.params(**KW)
    z = torch.zeros(b, 64, ny, nx, device="cuda")
    ud, vd = s.fv_step_d(prm, dev(u, torch.float32), dev(v, torch.float32), coef.cuda(), z)
    uc, vc = s.fv_step(prm, dev(u, torch.float32), dev(v, torch.float32), coef=coef.cuda())
    # the same step; the face derivative is summed in another order
    assert rel_l2(ud, uc) < 1e-6 and rel_l2(vd, vc) < 1e-6


@pytest.mark.parametrize("nx,ny,b", [(32, 32, 2), (32, 16, 1)])
def test_fv_step_d_adjoint_vs_oracle_autograd(nx, ny, b):
    L_ = need_gpu()
    announce("fv_step_d_bwd", nx, ny, b)
    u, v, coef, dcoef = _fields(nx, ny, b, seed=13)
    s = L_.Solver(nx, ny, b)
    prm = L_.params(**KW)
    g = torch.Generator().manual_seed(3)
    wu = torch.randn(b, ny, nx, generator=g, dtype=torch.float64).float()
    wv = torch.randn(b, ny, nx, generator=g, dtype=torch.float64).float()
    gc = torch.zeros(b, 64, ny, nx, device="cuda")
    gd = torch.zeros_like(gc)
    gu, gv = s.fv_step_d_bwd(prm, dev(u, torch.float32), dev(v, torch.float32), wu.cuda(),
                             wv.cuda(), coef.cuda(), dcoef.cuda(), gcoef=gc, gdcoef=gd)
    ua = u.clone().requires_grad_(True)
    va = v.clone().requires_grad_(True)
    ra = coef.double().requires_grad_(True)
    da = dcoef.double().requires_grad_(True)
    x, y = timestep.fv_step(ua, va, oracle_prm(nx, ny, **KW), learned.constrain(ra),
                            dcoef=learned.constrain_deriv(da))
    ((wu.double() * x).sum() + (wv.double() * y).sum()).backward()
    e = (rel_l2(gu, ua.grad), rel_l2(gv, va.grad), rel_l2(gc, ra.grad), rel_l2(gd, da.grad))
    print("rel-L2 gu gv gcoef gdcoef", e)
    assert max(e) < 1e-4


def _net(L_, seed, last_scale=0.05):
    ws, bs = si.cnn_weights(seed, cnn.LAYERS, last_scale=last_scale)
    net = L_.NetParams([torch.tensor(w) for w in ws], [torch.tensor(b) for b in bs])
    wb = [w.double().cpu() for w in net.bf16_weights()]
    bb = [b.double().cpu() for b in net.b]
    return net, wb, bb


@pytest.mark.parametrize("n,ny,b", [(32, 32, 3), (64, 64, 2), (64, 32, 3), (8, 8, 1)])
def test_learned_d_step_matches_oracle(n, ny, b):
    """Square, non-square and an 8 x 8 grid (sides not multiples of 16: the
    network's untiled path, float outputs)."""
    L_ = need_gpu()
    announce("learned_d_step", n, ny, b)
    net, wb, bb = _net(L_, seed=21)
    dnet, dwb, dbb = _net(L_, seed=22)
    u, v = ic.grf_peak(b, n, ny, L, L, seed=23)
    u, v = u.float().double(), v.float().double()
    s = L_.Solver(n, ny, b)
    prm = L_.params(k_c=1, **KW)
    uo, vo, no, dno = s.learned_d_fv_step(prm, net, dnet, dev(u, torch.float32),
                                          dev(v, torch.float32), 1, want_net_out=True)
    # the bf16-plane form (no outputs asked for) gives the same step bit for bit
    up, vp = s.learned_d_fv_step(prm, net, dnet, dev(u, torch.float32), dev(v, torch.float32), 1)
    assert torch.equal(up, uo) and torch.equal(vp, vo)
    # the FV step with the device's network outputs
    out, dout = cpu64(no), cpu64(dno)
    oprm = oracle_prm(n, ny, k_c=1, **KW)
    eu, ev = timestep.fv_step(u, v, oprm, learned.constrain(out[:, :64]),
                              dcoef=learned.constrain_deriv(dout[:, :64]))
    eu, ev, _ = project(eu + out[:, 64], ev + out[:, 65], oprm)
    assert rel_l2(uo, eu) < 1e-5 and rel_l2(vo, ev) < 1e-5
    # the whole step against the bf16-emulating oracle
    lu, lv, lo = learned.learned_fv_step(u, v, oprm, wb, bb, 1, bf16=True, dnet=(dwb, dbb))
    x = torch.stack([u, v], dim=1)
    dref = cnn.cnn_forward(x, dwb, dbb, bf16=True)
    e = (rel_l2(no, lo), rel_l2(dno[:, :64], dref[:, :64]), rel_l2(uo, lu), rel_l2(vo, lv))
    print("rel-L2 net dnet u v", e)
    assert e[0] < 5e-3 and e[1] < 5e-3 and e[2] < 1e-4 and e[3] < 1e-4


def test_zero_derivative_network_gives_the_learned_step():
    L_ = need_gpu()
    announce("learned_d zero dnet")
    n, b = 32, 2
    net, _, _ = _net(L_, seed=24)
    ws, bs = si.cnn_weights(25, cnn.LAYERS, last_scale=0.05)
    ws[-1] = ws[-1] * 0
    bs[-1] = bs[-1] * 0
    dnet = L_.NetParams([torch.tensor(w) for w in ws], [torch.tensor(q) for q in bs])
    u, v = ic.grf_peak(b, n, n, L, L, seed=26)
    s = L_.Solver(n, n, b)
    prm = L_.params(k_c=2, **KW)
    for k in (1, 2):
        ud, vd = s.learned_d_fv_step(prm, net, dnet, dev(u, torch.float32),
                                     dev(v, torch.float32), k)
        ul, vl = s.learned_fv_step(prm, net, dev(u, torch.float32), dev(v, torch.float32), k)
        assert rel_l2(ud, ul) < 1e-6 and rel_l2(vd, vl) < 1e-6, k


def test_learned_d_step_backward_vs_oracle_autograd():
    L_ = need_gpu()
    announce("learned_d_step backward")
    n, b = 32, 2
    net, wb, bb = _net(L_, seed=31)
    dnet, dwb, dbb = _net(L_, seed=32)
    u, v = ic.grf_peak(b, n, n, L, L, seed=33)
    u, v = u.float(), v.float()
    s = L_.Solver(n, n, b)
    prm = L_.params(k_c=1, **KW)
    g = torch.Generator().manual_seed(34)
    wu = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    wv = torch.randn(b, n, n, generator=g, dtype=torch.float64)
    dW = L_.NetGradBuffers(net)
    dWd = L_.NetGradBuffers(dnet)
    gu, gv = s.learned_d_fv_step_bwd(prm, net, dnet, dev(u, torch.float32),
                                     dev(v, torch.float32), 1, dev(wu, torch.float32),
                                     dev(wv, torch.float32), dW, dWd)
    ua = u.double().requires_grad_(True)
    va = v.double().requires_grad_(True)
    wr = [w.clone().requires_grad_(True) for w in wb]
    br = [q.clone().requires_grad_(True) for q in bb]
    dwr = [w.clone().requires_grad_(True) for w in dwb]
    dbr = [q.clone().requires_grad_(True) for q in dbb]
    x, y, _ = learned.learned_fv_step(ua, va, oracle_prm(n, n, k_c=1, **KW), wr, br, 1,
                                      bf16=True, dnet=(dwr, dbr))
    ((wu * x).sum() + (wv * y).sum()).backward()
    assert rel_l2(gu, ua.grad) < 1e-3 and rel_l2(gv, va.grad) < 1e-3
    for grads, ref_w, ref_b in ((dW, wr, br), (dWd, dwr, dbr)):
        for l in range(6):
            gw = grads.w[l].permute(0, 3, 1, 2).contiguous()
            if l == 5:
                # output channels 64, 65 of the derivative network are unused
                assert rel_l2(gw[:64], ref_w[l].grad[:64]) < 3e-2
                assert rel_l2(grads.b[l][:64], ref_b[l].grad[:64]) < 3e-2
                if grads is dWd:
                    assert float(gw[64:].abs().max()) == 0.0
                    assert float(grads.b[l][64:].abs().max()) == 0.0
            else:
                assert rel_l2(gw, ref_w[l].grad) < 3e-2, l
                assert rel_l2(grads.b[l], ref_b[l].grad) < 3e-2, l


def test_rollout_d_equals_step_sequence():
    L_ = need_gpu()
    announce("rollout_d")
    n, b = 32, 2
    net, _, _ = _net(L_, seed=41)
    dnet, _, _ = _net(L_, seed=42)
    u, v = ic.grf_peak(b, n, n, L, L, seed=43)
    u, v = dev(u, torch.float32), dev(v, torch.float32)
    s = L_.Solver(n, n, b)
    prm = L_.params(k_c=2, **KW)
    tu, tv = s.rollout_d(prm, net, dnet, u, v, 4, save_every=2)
    cu, cv = u.clone(), v.clone()
    for k in range(1, 5):
        cu, cv = s.learned_d_fv_step(prm, net, dnet, cu, cv, k)
        if k % 2 == 0:
            assert torch.equal(tu[k // 2 - 1], cu) and torch.equal(tv[k // 2 - 1], cv), k


def test_rollout_d_bwd_equals_step_adjoints():
    """The checkpointed unrolled backward equals the per-step adjoints chained
    by hand (the same kernels in the same order), bit for bit."""
    L_ = need_gpu()
    announce("rollout_d_bwd")
    n, b, T = 32, 2, 3
    net, _, _ = _net(L_, seed=51)
    dnet, _, _ = _net(L_, seed=52)
    u, v = ic.grf_peak(b, n, n, L, L, seed=53)
    u, v = dev(u, torch.float32), dev(v, torch.float32)
    s = L_.Solver(n, n, b)
    prm = L_.params(k_c=1, **KW)
    g = torch.Generator().manual_seed(54)
    gtu = torch.randn(T, b, n, n, generator=g).cuda()
    gtv = torch.randn(T, b, n, n, generator=g).cuda()
    dW, dWd = L_.NetGradBuffers(net), L_.NetGradBuffers(dnet)
    gu0, gv0 = s.rollout_d_bwd(prm, net, dnet, u, v, T, dW, dWd, checkpoint_every=2,
                               g_traj=(gtu, gtv), want_input_grad=True)
    states = [(u, v)]
    for k in range(1, T + 1):
        states.append(s.learned_d_fv_step(prm, net, dnet, *states[-1], k))
    eW, eWd = L_.NetGradBuffers(net), L_.NetGradBuffers(dnet)
    gu, gv = torch.zeros_like(u), torch.zeros_like(v)
    for k in range(T, 0, -1):
        gu, gv = gu + gtu[k - 1], gv + gtv[k - 1]
        gu, gv = s.learned_d_fv_step_bwd(prm, net, dnet, *states[k - 1], k, gu.contiguous(),
                                         gv.contiguous(), eW, eWd)
    assert torch.equal(gu0, gu) and torch.equal(gv0, gv)
    for l in range(6):
        assert torch.equal(dW.w[l], eW.w[l]) and torch.equal(dWd.w[l], eWd.w[l]), l
        assert torch.equal(dW.b[l], eW.b[l]) and torch.equal(dWd.b[l], eWd.b[l]), l


def test_training_with_derivative_network_lowers_loss():
    L_ = need_gpu()
    from paper_2507_01975_amd import train as T
    announce("training with the derivative network 256->32")
    fine_n, n = 256, 32
    r = fine_n // n
    dtf = 2.19e-4 * 2048 / fine_n
    phys = dict(nu=1e-3, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    lab = T.generate_labels(fine_n, n, 4, 300, 120, dtf, phys, warmup_steps=1500)
    s = L_.Solver(n, n, 4)
    net = T.init_network(seed=1)
    dnet = T.init_network(seed=2)
    prm = L_.params(dt=r * dtf, k_c=1, fallback_enable=0, **phys)
    hist = T.train(s, net, lab, prm, iters=150, unroll=8, lr=1e-4, log_every=25, dnet=dnet,
                   progress=lambda m: print(m, flush=True))
    first = hist[0][1]
    last = hist[-1][1]
    assert last < 0.8 * first, hist


def test_kolmogorov64_full_size_learned_d_step():
    """The two-network step at the benchmark's inference configuration (64^2,
    batch 64, the forced-flow parameters and time step) in the launch
    configuration the benchmark times (bf16 planes); every trajectory
    against the oracle given the device's network outputs, and the
    derivative network's output of trajectory 63 against the bf16-emulating
    oracle network."""
    L_ = need_gpu()
    announce("kolmogorov64 learned_d step")
    w = si.WORKLOADS["kolmogorov64"]
    n, B = w["nx"], w["batch"]
    net, _, _ = _net(L_, seed=0, last_scale=1e-3)
    dnet, dwb, dbb = _net(L_, seed=1, last_scale=1e-3)
    s = L_.Solver(n, n, B)
    gu, gv = s.init_state(L_.IC_GRF_PEAK, seed=200)
    kw = dict(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"], forcing_k=w["forcing_k"],
              drag=w["drag"])
    prm = L_.params(k_c=1, **kw)
    uo, vo, no, dno = s.learned_d_fv_step(prm, net, dnet, gu, gv, 1, want_net_out=True)
    pu, pv = s.learned_d_fv_step(prm, net, dnet, gu, gv, 1)
    assert torch.equal(pu, uo) and torch.equal(pv, vo)
    oprm = oracle_prm(n, n, k_c=1, **kw)
    out, dout = cpu64(no), cpu64(dno)
    eu, ev = timestep.fv_step(cpu64(gu), cpu64(gv), oprm, learned.constrain(out[:, :64]),
                              dcoef=learned.constrain_deriv(dout[:, :64]))
    eu, ev, _ = project(eu + out[:, 64], ev + out[:, 65], oprm)
    for b in range(B):
        assert_fields_close(uo[b], eu[b], what=("u", b))
        assert_fields_close(vo[b], ev[b], what=("v", b))
    x = torch.stack([cpu64(gu[B - 1:B]), cpu64(gv[B - 1:B])], dim=1)
    ref = cnn.cnn_forward(x, dwb, dbb, bf16=True)
    assert rel_l2(dno[B - 1:B, :64], ref[:, :64]) < 5e-3
    d = s.diagnostics(uo, vo).cpu()
    assert (d[:, 5] == 1).all()
