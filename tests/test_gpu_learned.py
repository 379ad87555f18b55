"""GPU parity of the learned path: the BF16 MFMA coefficient network, the
learned step (coefficients + temporal correction), the rollout and its
guard, against the FP64 oracle through the C ABI."""
import math

import pytest
import torch

import synthetic_inputs as si
from oracle import cnn, fv, ic, learned, timestep
from tests.gpu_common import assert_fields_close, L, announce, cpu64, dev, need_gpu, oracle_prm, rel_l2

pytestmark = pytest.mark.gpu

KW = dict(nu=1e-3, dt=0.05, forcing_amp=1.0, forcing_k=4.0, drag=0.1)


def _net(L_, seed=0, last_scale=1e-3):
    ws, bs = si.cnn_weights(seed, cnn.LAYERS, last_scale=last_scale)
    net = L_.NetParams([torch.tensor(w) for w in ws], [torch.tensor(b) for b in bs])
    wb = [w.double().cpu() for w in net.bf16_weights()]
    bb = [b.double().cpu() for b in net.b]
    return net, wb, bb


@pytest.mark.parametrize("nx,ny,b", [(8, 8, 1), (16, 16, 3), (32, 16, 2), (64, 64, 4)])
def test_cnn_forward(nx, ny, b):
    L_ = need_gpu()
    announce("cnn_forward", nx, ny, b)
    net, wb, bb = _net(L_, seed=1, last_scale=1.0)
    u, v = ic.grf_peak(b, nx, ny, L, L, seed=3)
    u, v = u.float(), v.float()
    s = L_.Solver(nx, ny, b)
    out = s.cnn_forward(net, dev(u, torch.float32), dev(v, torch.float32))
    x = torch.stack([u.double(), v.double()], dim=1)
    ref64 = cnn.cnn_forward(x, wb, bb)
    refbf = cnn.cnn_forward(x, wb, bb, bf16=True)
    assert rel_l2(out, ref64) < 2e-2
    # layer by layer from the device's own bf16 inputs: each layer matches the
    # oracle's layer to FP32 accumulation and bf16 rounding of its output
    prev = cnn.round_bf16(x)
    errs = []
    for li in range(6):
        z = cnn.conv3x3_circular(prev, wb[li], bb[li])
        if li < 5:
            ref = cnn.round_bf16(cnn.gelu(z))
            got = cpu64(s.cnn_activation(li))
            # each value within one bf16 ulp (a rounding flip), flips rare
            scale = torch.maximum(got.abs(), ref.abs())
            ulp = 2.0 ** -7 * scale + 1e-6 * ref.pow(2).mean().sqrt()
            assert ((got - ref).abs() <= 1.01 * ulp).all(), li
            flips = ((got - ref).abs() > 1e-6 * ref.pow(2).mean().sqrt()).double().mean().item()
            errs.append((rel_l2(got, ref), flips))
            assert rel_l2(got, ref) < 1e-4 and flips < 1e-2, (li, errs)
            prev = got
        else:
            # the 64 stencil-coefficient outputs are stored at bf16 (within
            # one bf16 ulp of the oracle's rounding), the 2 correction
            # channels at FP32
            got = cpu64(out)
            ref = cnn.round_bf16(z[:, :64])
            scale = torch.maximum(got[:, :64].abs(), ref.abs())
            ulp = 2.0 ** -7 * scale + 1e-6 * ref.pow(2).mean().sqrt()
            assert ((got[:, :64] - ref).abs() <= 1.01 * ulp).all()
            errs.append((rel_l2(out[:, :64], ref), rel_l2(out[:, 64:], z[:, 64:])))
            assert rel_l2(out[:, :64], ref) < 1e-4 and rel_l2(out[:, 64:], z[:, 64:]) < 1e-5, errs
    print("per-layer rel-L2 and rounding-flip fraction:", errs)
    # end to end, rounding flips compound through the layers
    assert rel_l2(out, refbf) < 5e-3


def test_learned_step_matches_oracle_given_network_output():
    L_ = need_gpu()
    announce("learned_step")
    nx = ny = 32
    b = 3
    net, wb, bb = _net(L_, seed=2, last_scale=0.05)
    u, v = ic.grf_peak(b, nx, ny, L, L, seed=5)
    u, v = u.float().double(), v.float().double()
    s = L_.Solver(nx, ny, b)
    prm = L_.params(k_c=1, **KW)
    uo, vo, no = s.learned_fv_step(prm, net, dev(u, torch.float32), dev(v, torch.float32), 1,
                                   want_net_out=True)
    out = cpu64(no)
    # the FV step with the device's coefficients and correction
    oprm = oracle_prm(nx, ny, k_c=1, **KW)
    eu, ev = timestep.fv_step(u, v, oprm, learned.constrain(out[:, :64]))
    from oracle.projection import project
    eu, ev, _ = project(eu + out[:, 64], ev + out[:, 65], oprm)
    assert rel_l2(uo, eu) < 1e-5 and rel_l2(vo, ev) < 1e-5
    # and the whole learned step against the bf16-emulating oracle
    lu, lv, lo = learned.learned_fv_step(u, v, oprm, wb, bb, 1, bf16=True)
    assert rel_l2(no, lo) < 5e-3
    assert rel_l2(uo, lu) < 1e-4


@pytest.mark.parametrize("n,b", [(32, 3), (64, 4)])
def test_packed_coefficients_equal_float_output_path(n, b):
    """Without a requested network output the 64 stencil values stay in bf16
    per cell inside the handle; the step equals, bit for bit, the step that
    reads them as bf16-rounded floats from the network output; so does the
    two-network step with learned derivative stencils."""
    L_ = need_gpu()
    announce("packed coefficients", n, b)
    net, _, _ = _net(L_, seed=2, last_scale=0.05)
    dnet, _, _ = _net(L_, seed=5, last_scale=0.05)
    s = L_.Solver(n, n, b)
    u, v = s.init_state(L_.IC_GRF_PEAK, seed=11)
    prm = L_.params(k_c=1, **KW)
    pu, pv = s.learned_fv_step(prm, net, u, v, 1)
    fu, fv, _ = s.learned_fv_step(prm, net, u, v, 1, want_net_out=True)
    assert torch.equal(pu, fu) and torch.equal(pv, fv)
    pu, pv = s.learned_d_fv_step(prm, net, dnet, u, v, 1)
    fu, fv, _, _ = s.learned_d_fv_step(prm, net, dnet, u, v, 1, want_net_out=True)
    assert torch.equal(pu, fu) and torch.equal(pv, fv)


@pytest.mark.parametrize("nx,ny,b", [(32, 16, 3), (64, 64, 4), (128, 64, 2)])
def test_fused_first_layer_equals_layer_by_layer_forward(nx, ny, b):
    """The learned step evaluates the network with layer 1 computed inside
    layer 2's tiles (grids whose sides are multiples of 16); its network
    output equals, bit for bit, the layer-by-layer forward of cnn_forward,
    and so does the derivative network's."""
    L_ = need_gpu()
    announce("fused first layer", nx, ny, b)
    net, _, _ = _net(L_, seed=4, last_scale=1.0)
    dnet, _, _ = _net(L_, seed=6, last_scale=1.0)
    s = L_.Solver(nx, ny, b)
    u, v = s.init_state(L_.IC_GRF_PEAK, seed=13)
    ref = s.cnn_forward(net, u, v).clone()
    dref = s.cnn_forward(dnet, u, v).clone()
    prm = L_.params(k_c=1, **KW)
    _, _, got = s.learned_fv_step(prm, net, u, v, 1, want_net_out=True)
    assert torch.equal(got, ref)
    _, _, got, dgot = s.learned_d_fv_step(prm, net, dnet, u, v, 1, want_net_out=True)
    assert torch.equal(got, ref) and torch.equal(dgot, dref)


def test_zero_head_reproduces_plain_fv_and_kc():
    L_ = need_gpu()
    announce("zero head")
    n, b = 32, 2
    ws, bs = si.cnn_weights(0, cnn.LAYERS)
    ws[-1][:] = 0
    bs[-1][:] = 0
    bs[-1][64] = 0.1   # constant TC in u
    net = L_.NetParams([torch.tensor(w) for w in ws], [torch.tensor(x) for x in bs])
    s = L_.Solver(n, n, b)
    u, v = s.init_state(L_.IC_GRF_PEAK, seed=4)
    pu, pv = s.fv_step(L_.params(**KW), u, v)
    prm = L_.params(k_c=2, **KW)
    lu, lv = s.learned_fv_step(prm, net, u, v, 1)       # 1 % 2 != 0: no correction
    assert (lu - pu).abs().max().item() < 1e-6 and (lv - pv).abs().max().item() < 1e-6
    lu, lv = s.learned_fv_step(prm, net, u, v, 2)       # correction added
    du = (lu.double() - pu.double()).mean(dim=(-2, -1))
    assert torch.allclose(du.cpu(), torch.full((b,), 0.1, dtype=torch.float64), atol=1e-6)


def test_rollout_equals_step_sequence():
    L_ = need_gpu()
    announce("rollout")
    n, b = 32, 2
    net, _, _ = _net(L_, seed=3)
    s = L_.Solver(n, n, b)
    u0, v0 = s.init_state(L_.IC_GRF_PEAK, seed=6)
    prm = L_.params(k_c=2, fallback_enable=0, **KW)
    tu, tv = s.rollout(prm, u0, v0, nsteps=6, save_every=2, net=net)
    u, v = u0.clone(), v0.clone()
    for k in range(6):
        u, v = s.learned_fv_step(prm, net, u, v, k + 1)
        if (k + 1) % 2 == 0:
            assert torch.equal(tu[(k + 1) // 2 - 1], u) and torch.equal(tv[(k + 1) // 2 - 1], v)
    # plain rollout
    tu, tv = s.rollout(L_.params(**KW), u0, v0, nsteps=3, save_every=3)
    pu, pv = s.fv_step(L_.params(**KW), u0, v0, nsteps=3)
    assert torch.equal(tu[0], pu) and torch.equal(tv[0], pv)


@pytest.mark.parametrize("guard", [False, True])
def test_rollout_matches_oracle(guard):
    """ldsv_rollout of the coefficient network (Eq. 2 with k_c = 2: the
    correction on even steps only) against the oracle: (1) each step from
    the device's previous state with the device's network output, through
    the oracle's FV step and correction schedule, to the FP32 step
    tolerance; (2) the snapshots every 2 steps against the oracle's own
    learned rollout (BF16-emulating network) over 6 steps.  With the guard
    on (a bound it never reaches) the result is the same bit for bit."""
    L_ = need_gpu()
    announce("rollout vs oracle, guard", guard)
    n, b, T, kc = 32, 3, 6, 2
    net, wb, bb = _net(L_, seed=3, last_scale=0.05)
    u, v = ic.grf_peak(b, n, n, L, L, seed=9)
    u, v = u.float().double(), v.float().double()
    s = L_.Solver(n, n, b)
    gprm = dict(k_c=kc, fallback_enable=1 if guard else 0,
                guard_threshold=1e3 if guard else 0.0, **KW)
    prm = L_.params(**gprm)
    flags = torch.zeros(b, dtype=torch.int32, device="cuda")
    u0, v0 = dev(u, torch.float32), dev(v, torch.float32)
    tu, tv = s.rollout(prm, u0, v0, nsteps=T, save_every=1, net=net,
                       fallback_flags=flags if guard else None)
    oprm = oracle_prm(n, n, k_c=kc, **KW)
    from oracle.projection import project
    prev_u, prev_v = u0, v0
    for k in range(1, T + 1):
        out = cpu64(s.cnn_forward(net, prev_u.contiguous(), prev_v.contiguous()))
        eu, ev = timestep.fv_step(cpu64(prev_u), cpu64(prev_v), oprm,
                                  learned.constrain(out[:, :64]))
        if k % kc == 0:
            eu, ev, _ = project(eu + out[:, 64], ev + out[:, 65], oprm)
        for bb_ in range(b):
            assert rel_l2(tu[k - 1, bb_], eu[bb_]) < 1e-5, (k, bb_)
            assert rel_l2(tv[k - 1, bb_], ev[bb_]) < 1e-5, (k, bb_)
        prev_u, prev_v = tu[k - 1], tv[k - 1]
    su, sv = s.rollout(prm, u0, v0, nsteps=T, save_every=2, net=net)
    assert torch.equal(su, tu[1::2]) and torch.equal(sv, tv[1::2])
    ou, ov = learned.learned_rollout(u, v, oprm, wb, bb, T, first_index=1, bf16=True)
    fu, fv_ = learned.learned_rollout(u, v, oprm, wb, bb, T, first_index=1, bf16=False)
    errs = [max(rel_l2(su[t], ou[2 * t + 1]), rel_l2(sv[t], ov[2 * t + 1])) for t in range(T // 2)]
    e64 = [max(rel_l2(su[t], fu[2 * t + 1]), rel_l2(sv[t], fv_[2 * t + 1])) for t in range(T // 2)]
    spread = [max(rel_l2(ou[2 * t + 1], fu[2 * t + 1]), rel_l2(ov[2 * t + 1], fv_[2 * t + 1]))
              for t in range(T // 2)]
    print("rollout rel-L2 at steps 2, 4, 6: vs the bf16-emulating oracle", errs,
          "vs the FP64 oracle", e64, "bf16 oracle vs FP64 oracle", spread)
    # A rounding flip (one bf16 ulp) of a hidden activation moves the next
    # layer's inputs by enough to flip others: the flips cascade through the
    # five hidden layers, so the device's network output differs from the
    # bf16-emulating oracle's by about as much as bf16 storage itself moves
    # the output away from FP64 (a few 1e-3, bounded in test_cnn_forward).
    # The rollout therefore differs from either oracle by about the oracle's
    # own bf16-vs-FP64 spread: at most twice that spread, and within the
    # BF16-network tolerance (2e-2) of the FP64 oracle.
    for t in range(T // 2):
        assert errs[t] < 2.0 * spread[t] + 1e-5, (errs, spread)
        assert e64[t] < 2.0 * spread[t] + 1e-5 and e64[t] < 2e-2, (e64, spread)
    if guard:
        torch.cuda.synchronize()
        assert flags.tolist() == [0] * b
        p0 = L_.params(k_c=kc, fallback_enable=0, **KW)
        nu_, nv_ = s.rollout(p0, u0, v0, nsteps=T, save_every=2, net=net)
        assert torch.equal(nu_, su) and torch.equal(nv_, sv)


def test_guard_fallback_matches_oracle_plain_step():
    """A trajectory over the guard bound is recomputed with the plain FV step:
    its state after the rollout equals the oracle's plain steps from the
    same start, the others the oracle's learned steps given the device's
    network output."""
    L_ = need_gpu()
    announce("guard vs oracle")
    n, b = 32, 3
    kw = dict(KW, dt=0.005)
    net, _, _ = _net(L_, seed=4)
    s = L_.Solver(n, n, b)
    u0, v0 = s.init_state(L_.IC_GRF_PEAK, seed=7)
    u0[2] *= 8.0
    v0[2] *= 8.0
    bound = 4.0 * float((u0[:2].abs() + v0[:2].abs()).max())
    prm = L_.params(k_c=1, guard_threshold=bound, fallback_enable=1, **kw)
    flags = torch.zeros(b, dtype=torch.int32, device="cuda")
    tu, tv = s.rollout(prm, u0, v0, nsteps=2, save_every=1, net=net, fallback_flags=flags)
    torch.cuda.synchronize()
    assert flags.tolist() == [0, 0, 2]
    oprm = oracle_prm(n, n, k_c=1, **kw)
    pu, pv = timestep.fv_step(cpu64(u0[2:]), cpu64(v0[2:]), oprm, nsteps=2)
    assert rel_l2(tu[1, 2], pu[0]) < 1e-5 and rel_l2(tv[1, 2], pv[0]) < 1e-5
    from oracle.projection import project
    cu, cv = u0[:2].contiguous(), v0[:2].contiguous()
    s2 = L_.Solver(n, n, 2)
    for k in range(2):
        out = cpu64(s2.cnn_forward(net, cu, cv))
        eu, ev = timestep.fv_step(cpu64(cu), cpu64(cv), oprm, learned.constrain(out[:, :64]))
        eu, ev, _ = project(eu + out[:, 64], ev + out[:, 65], oprm)
        assert rel_l2(tu[k, :2], eu) < 1e-5 and rel_l2(tv[k, :2], ev) < 1e-5, k
        cu, cv = tu[k, :2].contiguous(), tv[k, :2].contiguous()


def test_guard_falls_back_to_plain_fv_for_the_failing_trajectory_only():
    L_ = need_gpu()
    announce("guard")
    n, b = 32, 3
    kw = dict(KW, dt=0.005)
    net, _, _ = _net(L_, seed=4)
    s = L_.Solver(n, n, b)
    u0, v0 = s.init_state(L_.IC_GRF_PEAK, seed=7)
    u0[2] *= 8.0
    v0[2] *= 8.0
    flags = torch.zeros(b, dtype=torch.int32, device="cuda")
    bound = 4.0 * float((u0[:2].abs() + v0[:2].abs()).max())
    prm = L_.params(k_c=1, guard_threshold=bound, fallback_enable=1, **kw)
    tu, tv = s.rollout(prm, u0, v0, nsteps=2, save_every=1, net=net, fallback_flags=flags)
    torch.cuda.synchronize()
    assert flags.tolist() == [0, 0, 2]
    assert torch.isfinite(tu).all() and torch.isfinite(tv).all()
    # untouched trajectories follow the learned steps; the failing one the plain steps
    u, v = u0.clone(), v0.clone()
    pu, pv = u0.clone(), v0.clone()
    for k in range(2):
        u, v = s.learned_fv_step(prm, net, u, v, k + 1)
        pu, pv = s.fv_step(L_.params(**kw), pu, pv)
    assert torch.equal(tu[1, :2], u[:2])
    # the redo (detection and the plain step of the pair in one kernel on
    # grids up to 64^2) evaluates the plain step's expressions in its own
    # kernel: equal to the plain step up to FP32 rounding
    assert_fields_close(tu[1, 2], pu[2], rel=1e-6, elem=1e-6, what="redone u")
    assert_fields_close(tv[1, 2], pv[2], rel=1e-6, elem=1e-6, what="redone v")
    # with the fallback disabled the call reports the failure
    prm = L_.params(k_c=1, guard_threshold=bound, fallback_enable=0, **kw)
    with pytest.raises(L_.LdsvError) as e:
        s.rollout(prm, u0, v0, nsteps=1, save_every=1, net=net)
    assert e.value.code == L_.ENONFINITE


@pytest.mark.parametrize("n,b,bad", [(32, 4, 1), (128, 4, 2)])
def test_guard_fallback_beside_a_good_partner(n, b, bad):
    """The plain-FV redo of one trajectory of a packed pair: its good
    partner keeps its learned result bit for bit, the redone one follows the
    oracle's plain steps; at 32^2 the one-launch guard (the redo of the pair
    in LDS, whose projection transforms the two trajectories at once), at
    128^2 the detection kernel and the plain step masked to the flagged
    trajectory."""
    L_ = need_gpu()
    announce("guard beside a good partner", n, b, bad)
    kw = dict(KW, dt=0.005 * 32 / n)
    net, _, _ = _net(L_, seed=4)
    s = L_.Solver(n, n, b)
    u0, v0 = s.init_state(L_.IC_GRF_PEAK, seed=7)
    u0[bad] *= 8.0
    v0[bad] *= 8.0
    good = [i for i in range(b) if i != bad]
    bound = 4.0 * float((u0[good].abs() + v0[good].abs()).max())
    prm = L_.params(k_c=1, guard_threshold=bound, fallback_enable=1, **kw)
    flags = torch.zeros(b, dtype=torch.int32, device="cuda")
    tu, tv = s.rollout(prm, u0, v0, nsteps=2, save_every=1, net=net, fallback_flags=flags)
    torch.cuda.synchronize()
    assert flags.tolist() == [2 if i == bad else 0 for i in range(b)]
    # each step of the good trajectories is the learned step of the rollout's
    # previous state (which holds the redone trajectory), bit for bit
    prev_u, prev_v = u0, v0
    for k in range(2):
        lu, lv = s.learned_fv_step(prm, net, prev_u.contiguous(), prev_v.contiguous(), k + 1)
        assert torch.equal(tu[k, good], lu[good]) and torch.equal(tv[k, good], lv[good]), k
        prev_u, prev_v = tu[k], tv[k]
    oprm = oracle_prm(n, n, k_c=1, **kw)
    pu, pv = timestep.fv_step(cpu64(u0[bad:bad + 1]), cpu64(v0[bad:bad + 1]), oprm, nsteps=2)
    assert_fields_close(tu[1, bad], pu[0], what="redone trajectory u")
    assert_fields_close(tv[1, bad], pv[0], what="redone trajectory v")


@pytest.mark.parametrize("n", [32, 128])
def test_guarded_rollout_replays_as_a_captured_graph(n):
    """With the fallback enabled the guarded rollout reads nothing back, so
    it can be captured in a HIP graph: replays (with a trajectory that trips
    the guard at every step, so the redo runs inside the graph) match the
    eager call bit for bit, flags included; at 32^2 the one-kernel redo, at
    128^2 the masked plain step."""
    L_ = need_gpu()
    announce("guarded rollout graph capture", n)
    b = 3
    kw = dict(KW, dt=0.005 * 32 / n)
    net, _, _ = _net(L_, seed=4)
    s = L_.Solver(n, n, b)
    u0, v0 = s.init_state(L_.IC_GRF_PEAK, seed=7)
    u0[1] *= 8.0
    v0[1] *= 8.0
    bound = 4.0 * float((u0[0::2].abs() + v0[0::2].abs()).max())
    prm = L_.params(k_c=2, guard_threshold=bound, fallback_enable=1, **kw)
    flags = torch.zeros(b, dtype=torch.int32, device="cuda")
    ru, rv = s.rollout(prm, u0, v0, nsteps=4, save_every=2, net=net, fallback_flags=flags)
    torch.cuda.synchronize()
    rflags = flags.clone()
    assert rflags.tolist() == [0, 4, 0]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gu, gv = s.rollout(prm, u0, v0, nsteps=4, save_every=2, net=net, fallback_flags=flags)
    torch.cuda.synchronize()
    for _ in range(3):
        flags.zero_()
        s.fv_step(L_.params(**kw), u0, v0)   # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(gu, ru) and torch.equal(gv, rv) and torch.equal(flags, rflags)


def test_nan_network_falls_back_everywhere():
    L_ = need_gpu()
    announce("nan guard")
    n, b = 16, 2
    ws, bs = si.cnn_weights(5, cnn.LAYERS)
    bs[-1][3] = float("nan")
    net = L_.NetParams([torch.tensor(w) for w in ws], [torch.tensor(x) for x in bs])
    s = L_.Solver(n, n, b)
    u0, v0 = s.init_state(L_.IC_GRF_PEAK, seed=8)
    flags = torch.zeros(b, dtype=torch.int32, device="cuda")
    prm = L_.params(k_c=1, fallback_enable=1, **KW)
    tu, tv = s.rollout(prm, u0, v0, nsteps=3, save_every=3, net=net, fallback_flags=flags)
    pu, pv = s.fv_step(L_.params(**KW), u0, v0, nsteps=3)
    torch.cuda.synchronize()
    assert flags.tolist() == [3, 3]
    assert_fields_close(tu[0], pu, rel=1e-6, elem=1e-6, what="all redone u")
    assert_fields_close(tv[0], pv, rel=1e-6, elem=1e-6, what="all redone v")


def test_bf16_conversion_rounds_to_nearest_even():
    """The hardware float -> bf16 conversion used for weights and activations
    against round-to-nearest-even (torch's CPU conversion): random values,
    exact ties with even and odd kept bit, subnormals, signed zeros, the
    overflow boundary and infinities; NaN only as NaN."""
    L_ = need_gpu()
    announce("bf16 rounding")
    g = torch.Generator().manual_seed(7)
    rnd = torch.randint(0, 2**31 - 1, (1 << 16,), generator=g, dtype=torch.int64)
    hi = (rnd & 0x7FFF7FFF) | ((rnd & 1) << 31)           # random sign, exponent, mantissa
    ties = (hi & ~0xFFFF) | 0x8000                          # exactly half-way
    near = (hi & ~0xFFFF) | 0x7FFF                          # just below half-way
    above = (hi & ~0xFFFF) | 0x8001                         # just above
    special = torch.tensor([0x00000000, 0x80000000, 0x00000001, 0x00008000, 0x00018000,
                            0x007FFFFF, 0x7F7F7FFF, 0x7F7F8000, 0x7F7FFFFF, 0x7F800000,
                            0xFF800000, 0x3F808000, 0x3F818000, 0xBF808000], dtype=torch.int64)
    bits = torch.cat([hi, ties, near, above, special]).to(torch.int64)
    bits = torch.where(bits >= 2**31, bits - 2**32, bits).to(torch.int32)
    x = bits.view(torch.float32)
    finite = ~torch.isnan(x)
    x = x[finite].contiguous()
    xd = x.cuda()
    out = torch.empty(x.numel(), dtype=torch.int16, device="cuda")
    L_._check(L_._lib.ldsv_to_bf16(L_._ptr(xd), L_._ptr(out), x.numel(), L_._stream()))
    torch.cuda.synchronize()
    ref = x.to(torch.bfloat16).view(torch.int16)
    assert torch.equal(out.cpu(), ref)
    nan = torch.tensor([float("nan")], dtype=torch.float32).cuda()
    o1 = torch.empty(1, dtype=torch.int16, device="cuda")
    L_._check(L_._lib.ldsv_to_bf16(L_._ptr(nan), L_._ptr(o1), 1, L_._stream()))
    assert torch.isnan(o1.cpu().view(torch.bfloat16).float()).all()


def test_kolmogorov64_full_size_learned_step():
    """The learned step at the benchmark's inference configuration (64^2,
    batch 64, the forced-flow parameters and time step), in the launch
    configuration the benchmark times; every trajectory is checked against
    the oracle given the device's network output, and the network
    output of trajectory 63 against the bf16-emulating oracle network."""
    L_ = need_gpu()
    announce("kolmogorov64 learned step")
    w = si.WORKLOADS["kolmogorov64"]
    n, B = w["nx"], w["batch"]
    net, wb, bb = _net(L_, seed=0)
    s = L_.Solver(n, n, B)
    gu, gv = s.init_state(L_.IC_GRF_PEAK, seed=200)
    kw = dict(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"], forcing_k=w["forcing_k"],
              drag=w["drag"])
    uo, vo, no = s.learned_fv_step(L_.params(k_c=1, **kw), net, gu, gv, 1, want_net_out=True)
    # without a request for the network output the step reads bf16
    # coefficient planes instead of the float output: the same values, the
    # same result bit for bit
    pu, pv = s.learned_fv_step(L_.params(k_c=1, **kw), net, gu, gv, 1)
    assert torch.equal(pu, uo) and torch.equal(pv, vo)
    oprm = oracle_prm(n, n, k_c=1, **kw)
    from oracle.projection import project
    # every trajectory, in L2 and element by element
    out = cpu64(no)
    eu, ev = timestep.fv_step(cpu64(gu), cpu64(gv), oprm, learned.constrain(out[:, :64]))
    eu, ev, _ = project(eu + out[:, 64], ev + out[:, 65], oprm)
    for b in range(B):
        assert_fields_close(uo[b], eu[b], what=("u", b))
        assert_fields_close(vo[b], ev[b], what=("v", b))
    x = torch.stack([cpu64(gu[B - 1:B]), cpu64(gv[B - 1:B])], dim=1)
    ref = cnn.cnn_forward(x, wb, bb, bf16=True)
    assert rel_l2(no[B - 1:B], ref) < 5e-3
    d = s.diagnostics(uo, vo).cpu()
    assert (d[:, 5] == 1).all()


def test_rollout_bwd_replays_as_a_captured_graph():
    """The unrolled backward records no memset nodes, so it can be captured
    in a HIP graph: three rounds of replays over two windows (new inputs
    copied into the captured buffers, eager work and synchronisations
    between replays) match the eager calls bit for bit."""
    L_ = need_gpu()
    announce("rollout_bwd graph capture")
    n, b, unroll = 32, 2, 6
    net, _, _ = _net(L_, seed=7, last_scale=0.05)
    s = L_.Solver(n, n, b)
    prm = L_.params(k_c=2, fallback_enable=0, **KW)
    u, v = ic.grf_peak(b, n, n, L, L, seed=8)
    u, v = dev(u, torch.float32), dev(v, torch.float32)
    tu, tv = s.rollout(prm, u, v, unroll + 3)
    lu, lv = torch.cat([u[None], tu]), torch.cat([v[None], tv])
    dW = L_.NetGradBuffers(net)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    u0s, v0s = lu[0].clone(), lv[0].clone()
    yus, yvs = lu[1:1 + unroll].clone(), lv[1:1 + unroll].clone()

    def load(t0):
        u0s.copy_(lu[t0])
        v0s.copy_(lv[t0])
        yus.copy_(lu[t0 + 1:t0 + 1 + unroll])
        yvs.copy_(lv[t0 + 1:t0 + 1 + unroll])

    def call():
        dW.zero_()
        loss.zero_()
        s.rollout_bwd(prm, net, u0s, v0s, unroll, dW, checkpoint_every=4, first_index=1,
                      labels=(yus, yvs), loss_scale=1.0 / unroll, loss=loss)

    refs = []
    for t0 in (0, 3):
        load(t0)
        call()
        torch.cuda.synchronize()
        refs.append(([x.clone() for x in dW.w + dW.b], loss.clone()))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    torch.cuda.synchronize()
    for _ in range(3):
        for k, t0 in enumerate((0, 3)):
            load(t0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(loss, refs[k][1]), (t0, loss, refs[k][1])
            for x, r in zip(dW.w + dW.b, refs[k][0]):
                assert torch.equal(x, r)
