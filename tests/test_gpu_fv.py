"""GPU parity of the plain FV path (residual, projection, RK steps, initial
conditions, diagnostics) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle import fv, ic, learned, metrics, projection, timestep
from tests.gpu_common import assert_fields_close, L, announce, cpu64, dev, need_gpu, oracle_prm, rel_l2

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 1), (16, 16, 3), (32, 16, 2), (64, 64, 2), (128, 32, 1)]


def _fields(seed, b, ny, nx, dtype):
    u = torch.tensor(si.smooth_field(seed, b, ny, nx))
    v = torch.tensor(si.smooth_field(seed + 1, b, ny, nx))
    # round to the device precision so both sides see identical inputs
    return u.to(dtype).double(), v.to(dtype).double()


@pytest.mark.parametrize("nx,ny,b", SHAPES)
@pytest.mark.parametrize("mask", [fv.ALL_PHYSICS, fv.ADVECTION, fv.VISCOSITY])
def test_rhs_mac_f32(nx, ny, b, mask):
    L_ = need_gpu()
    announce("rhs_mac_f32", nx, ny, b, mask)
    u, v = _fields(1, b, ny, nx, torch.float32)
    kw = dict(nu=0.01, forcing_amp=1.0, forcing_k=4.0, drag=0.1, mask=mask)
    s = L_.Solver(nx, ny, b)
    ru, rv = s.rhs(L_.params(**kw), dev(u, torch.float32), dev(v, torch.float32))
    torch.cuda.synchronize()
    eu, ev = fv.ns_rhs(u, v, oracle_prm(nx, ny, **kw))
    assert rel_l2(ru, eu) < 1e-5 and rel_l2(rv, ev) < 1e-5


@pytest.mark.parametrize("nx,ny,b", SHAPES)
def test_rhs_mac_f64(nx, ny, b):
    L_ = need_gpu()
    announce("rhs_mac_f64", nx, ny, b)
    u, v = _fields(2, b, ny, nx, torch.float64)
    kw = dict(nu=0.02, forcing_amp=0.5, forcing_k=2.0, drag=0.3)
    s = L_.Solver(nx, ny, b, dtype=torch.float64)
    ru, rv = s.rhs(L_.params(**kw), dev(u, torch.float64), dev(v, torch.float64))
    eu, ev = fv.ns_rhs(u, v, oracle_prm(nx, ny, **kw))
    assert rel_l2(ru, eu) < 1e-13 and rel_l2(rv, ev) < 1e-13


@pytest.mark.parametrize("nx,ny,b", [(16, 16, 2), (32, 16, 1), (64, 64, 3)])
def test_rhs_learned_coefficients(nx, ny, b):
    L_ = need_gpu()
    announce("rhs_learned", nx, ny, b)
    u, v = _fields(3, b, ny, nx, torch.float32)
    raw = torch.tensor(si.random_field(5, (b, 64, ny, nx), scale=0.2)).float()
    kw = dict(nu=0.01, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    s = L_.Solver(nx, ny, b)
    ru, rv = s.rhs(L_.params(**kw), dev(u, torch.float32), dev(v, torch.float32),
                   coef=dev(raw, torch.float32))
    eu, ev = fv.ns_rhs(u, v, oracle_prm(nx, ny, **kw), learned.constrain(raw.double()))
    assert rel_l2(ru, eu) < 1e-5 and rel_l2(rv, ev) < 1e-5
    # conservation holds for any coefficients: sum of the flux part is zero
    s2 = L_.Solver(nx, ny, b)
    ru, rv = s2.rhs(L_.params(nu=0.01, mask=L_.ADVECTION | L_.VISCOSITY), dev(u, torch.float32),
                    dev(v, torch.float32), coef=dev(raw, torch.float32))
    assert ru.double().sum(dim=(-2, -1)).abs().max().item() < 1e-3 * ru.abs().max().item()


@pytest.mark.parametrize("nx,ny,b", [(8, 8, 1), (16, 16, 3), (64, 32, 2)])
def test_rhs_burgers_f64(nx, ny, b):
    L_ = need_gpu()
    announce("rhs_burgers", nx, ny, b)
    u, v = _fields(4, b, ny, nx, torch.float64)
    s = L_.Solver(nx, ny, b, dtype=torch.float64, layout=L_.COLLOCATED)
    ru, rv = s.rhs(L_.params(nu=0.01, rk=L_.SSPRK3), dev(u, torch.float64), dev(v, torch.float64))
    eu, ev = fv.burgers_rhs(u, v, oracle_prm(nx, ny, nu=0.01))
    assert rel_l2(ru, eu) < 1e-13 and rel_l2(rv, ev) < 1e-13


# grids up to 4096 cells take the single-workgroup LDS projection, and so do
# grids up to 16384 cells (and 128 KB of complex pair field) when there are
# at least 256 trajectory pairs; the rest take the three-pass version:
# (64, 64), (128, 128, 3), (128, 128, 512) and (256, 64) cover every side
@pytest.mark.parametrize("nx,ny,b", SHAPES + [(32, 32, 3), (64, 64, 5), (128, 128, 3),
                                              (128, 128, 512), (256, 64, 2), (512, 512, 2),
                                              (256, 1024, 1)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_projection(nx, ny, b, dtype):
    L_ = need_gpu()
    announce("project", nx, ny, b, dtype)
    u, v = _fields(6, b, ny, nx, dtype)
    s = L_.Solver(nx, ny, b, dtype=dtype)
    gu, gv = dev(u, dtype), dev(v, dtype)
    p = s.project(gu, gv, want_p=True)
    prm = oracle_prm(nx, ny)
    eu, ev, ep = projection.project(u, v, prm)
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    assert rel_l2(gu, eu) < tol and rel_l2(gv, ev) < tol
    assert rel_l2(p, ep) < tol
    # discretely divergence-free up to transform roundoff: an error of
    # eps*sqrt(log2 N)*|p| spread over all wavenumbers, amplified by the
    # largest eigenvalue of D G
    eps = 6e-8 if dtype == torch.float32 else 1.2e-16
    lam_max = 4 / (L / nx) ** 2 + 4 / (L / ny) ** 2
    d_out = projection.divergence(cpu64(gu), cpu64(gv), prm)
    bound = 4 * eps * math.sqrt(math.log2(nx * ny)) * lam_max * ep.pow(2).mean().sqrt()
    assert d_out.pow(2).mean().sqrt() < bound
    d_in = projection.divergence(u, v, prm)
    assert d_out.norm() < 1e-3 * d_in.norm()


@pytest.mark.parametrize("nx,ny,b", [(16, 16, 3), (64, 64, 2), (128, 64, 1)])
def test_rk4_step_f32(nx, ny, b):
    L_ = need_gpu()
    announce("rk4_f32", nx, ny, b)
    u, v = ic.grf_peak(b, nx, ny, L, L * ny / nx, seed=7)
    u, v = u.float().double(), v.float().double()
    kw = dict(nu=1e-3, dt=0.5 * (L / nx), forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    s = L_.Solver(nx, ny, b, ly=L * ny / nx)
    uo, vo = s.fv_step(L_.params(**kw), dev(u, torch.float32), dev(v, torch.float32))
    eu, ev = timestep.fv_step(u, v, oracle_prm(nx, ny, ly=L * ny / nx, **kw))
    assert rel_l2(uo, eu) < 1e-5 and rel_l2(vo, ev) < 1e-5


@pytest.mark.parametrize("nx,ny,b", [(8, 8, 1), (16, 16, 3), (32, 16, 2)])
def test_rk4_steps_f64(nx, ny, b):
    L_ = need_gpu()
    announce("rk4_f64", nx, ny, b)
    u, v = ic.grf_peak(b, nx, ny, L, L, seed=8)
    kw = dict(nu=1e-2, dt=0.05, forcing_amp=1.0, forcing_k=2.0, drag=0.1)
    s = L_.Solver(nx, ny, b, dtype=torch.float64)
    gu, gv = dev(u, torch.float64), dev(v, torch.float64)
    uo, vo = s.fv_step(L_.params(**kw), gu, gv, nsteps=5, out=(gu, gv))   # in place
    eu, ev = timestep.fv_step(u, v, oracle_prm(nx, ny, **kw), nsteps=5)
    assert rel_l2(uo, eu) < 1e-12 and rel_l2(vo, ev) < 1e-12


def test_learned_coefficient_step_f32():
    L_ = need_gpu()
    announce("fv_step_coef")
    nx = ny = 32
    b = 2
    u, v = ic.grf_peak(b, nx, ny, L, L, seed=9)
    u, v = u.float().double(), v.float().double()
    raw = torch.tensor(si.random_field(11, (b, 64, ny, nx), scale=0.05)).float()
    kw = dict(nu=1e-3, dt=0.05, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    s = L_.Solver(nx, ny, b)
    uo, vo = s.fv_step(L_.params(**kw), dev(u, torch.float32), dev(v, torch.float32),
                       coef=dev(raw, torch.float32))
    eu, ev = timestep.fv_step(u, v, oracle_prm(nx, ny, **kw), coef=learned.constrain(raw.double()))
    assert rel_l2(uo, eu) < 1e-5 and rel_l2(vo, ev) < 1e-5


def test_burgers_config_200_steps_f64():
    """The Burgers workload (64^2, FP64, SSP-RK3, CFL 0.5, 200 steps): initial
    condition, CFL time step and the whole trajectory against the oracle."""
    L_ = need_gpu()
    announce("burgers64 200 steps")
    w = si.WORKLOADS["burgers64"]
    n = w["nx"]
    s = L_.Solver(n, n, 1, dtype=torch.float64, layout=L_.COLLOCATED)
    gu, gv = s.init_state(L_.IC_FOURIER_MODES, seed=0)
    eu, ev = ic.fourier_modes(1, n, n, L, L, seed=0)
    assert rel_l2(gu, eu) < 1e-13 and rel_l2(gv, ev) < 1e-13
    dt = s.cfl_dt(gu, gv, w["cfl"])
    prm = oracle_prm(n, n, nu=w["nu"], rk=timestep.SSPRK3, layout=timestep.COLLOCATED)
    dt_ref = timestep.cfl_dt(eu, ev, prm, w["cfl"])
    assert dt == pytest.approx(dt_ref, rel=1e-14)
    prm["dt"] = dt_ref
    uo, vo = s.fv_step(L_.params(nu=w["nu"], dt=dt, rk=L_.SSPRK3), gu, gv, nsteps=w["steps"])
    ou, ov = timestep.fv_step(eu, ev, prm, nsteps=w["steps"])
    assert rel_l2(uo, ou) < 1e-10 and rel_l2(vo, ov) < 1e-10


@pytest.mark.parametrize("kind,nx,ny,b", [("grf", 32, 32, 3), ("grf", 64, 16, 2),
                                          ("tgv", 16, 16, 2), ("shear", 64, 64, 2)])
def test_initial_conditions_f64(kind, nx, ny, b):
    L_ = need_gpu()
    announce("init", kind, nx, ny, b)
    s = L_.Solver(nx, ny, b, dtype=torch.float64)
    if kind == "grf":
        gu, gv = s.init_state(L_.IC_GRF_PEAK, seed=12)
        eu, ev = ic.grf_peak(b, nx, ny, L, L, seed=12)
    elif kind == "tgv":
        gu, gv = s.init_state(L_.IC_TGV, seed=0, k=2.0, amp=0.7)
        eu, ev = ic.taylor_green(b, nx, ny, L, L, amp=0.7, k=2)
    else:
        gu, gv = s.init_state(L_.IC_SHEAR_LAYER, seed=3)
        eu, ev = ic.shear_layer(b, nx, ny, L, L, seed=3)
    assert rel_l2(gu, eu) < 1e-12 and rel_l2(gv, ev) < 1e-12


def test_decaying512_full_size_step():
    """One RK4 step of the decaying-flow workload at its full size (512^2,
    batch 16, FP32) in the launch configuration the benchmark times;
    trajectories 0 and 15 are checked against the oracle."""
    L_ = need_gpu()
    announce("decaying512 step")
    w = si.WORKLOADS["decaying512"]
    n, B = w["nx"], w["batch"]
    s = L_.Solver(n, n, B)
    gu, gv = s.init_state(L_.IC_GRF_PEAK, seed=0)
    kw = dict(nu=w["nu"], dt=w["dt"])
    uo, vo = s.fv_step(L_.params(**kw), gu, gv)
    # every trajectory against the oracle, in L2 and element by element
    eu, ev = timestep.fv_step(cpu64(gu), cpu64(gv), oracle_prm(n, n, **kw))
    for b in range(B):
        assert_fields_close(uo[b], eu[b], what=("u", b))
        assert_fields_close(vo[b], ev[b], what=("v", b))
    # the state stays discretely divergence-free (relative to its vorticity)
    # and finite
    d = s.diagnostics(uo, vo).cpu()
    w = s.vorticity(uo, vo).double()
    w_norm = w.pow(2).sum(dim=(-2, -1)).sqrt().cpu()
    assert (d[:, 4] < 1e-4 * w_norm).all() and (d[:, 5] == 1).all()


def test_determinism_bitwise():
    L_ = need_gpu()
    announce("determinism")
    s = L_.Solver(64, 64, 4)
    gu, gv = s.init_state(L_.IC_GRF_PEAK, seed=1)
    prm = L_.params(nu=1e-3, dt=0.02, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    a = s.fv_step(prm, gu, gv, nsteps=3)
    b = s.fv_step(prm, gu, gv, nsteps=3)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_diagnostics_vorticity_pcc_downsample():
    L_ = need_gpu()
    announce("diagnostics")
    n, b = 32, 3
    u, v = ic.grf_peak(b, n, n, L, L, seed=4)
    u, v = (u + 0.3).float().double(), (v - 0.2).float().double()
    s = L_.Solver(n, n, b)
    gu, gv = dev(u, torch.float32), dev(v, torch.float32)
    d = s.diagnostics(gu, gv).cpu()
    assert torch.allclose(d[:, 0], (u.abs() + v.abs()).amax(dim=(-2, -1)), rtol=1e-6)
    assert torch.allclose(d[:, 1], 0.5 * (u * u + v * v).mean(dim=(-2, -1)), rtol=1e-6)
    assert torch.allclose(d[:, 2], u.mean(dim=(-2, -1)), atol=1e-7)
    w = s.vorticity(gu, gv)
    ew = metrics.vorticity(u, v, L / n, L / n)
    assert rel_l2(w, ew) < 1e-6
    p = s.pcc(w, gu).cpu()
    assert torch.allclose(p, metrics.pcc(ew, u), atol=1e-6)
    # fine 128^2 -> coarse 32^2
    uf, vf = ic.grf_peak(b, 4 * n, 4 * n, L, L, seed=5)
    uf, vf = uf.float().double(), vf.float().double()
    uc, vc = s.downsample(4, dev(uf, torch.float32), dev(vf, torch.float32))
    euc, evc = metrics.downsample_mac(uf, vf, 4)
    assert rel_l2(uc, euc) < 1e-6 and rel_l2(vc, evc) < 1e-6


def test_error_paths():
    L_ = need_gpu()
    s = L_.Solver(16, 16, 1)
    u = s.new_state()
    with pytest.raises(L_.LdsvError) as e:
        s.fv_step(L_.params(nu=1e-3, dt=0.01), u, u, nsteps=0)
    assert e.value.code == L_.EINVAL
    c = L_.Solver(16, 16, 1, layout=L_.COLLOCATED)
    with pytest.raises(L_.LdsvError):
        c.project(c.new_state(), c.new_state())


@pytest.mark.parametrize("nx,ny", [(2048, 16), (16, 2048)])
def test_projection_extreme_aspect_fp32(nx, ny):
    """The longest rows and columns the FP32 MAC grid allows (2048): the row
    passes switch to 512-thread blocks with one row each, the column pass to
    4-column blocks."""
    L_ = need_gpu()
    announce("project extreme", nx, ny)
    u, v = _fields(9, 1, ny, nx, torch.float32)
    s = L_.Solver(nx, ny, 1)
    gu, gv = dev(u, torch.float32), dev(v, torch.float32)
    p = s.project(gu, gv, want_p=True)
    prm = oracle_prm(nx, ny)
    eu, ev, ep = projection.project(u, v, prm)
    # FP32 transform roundoff in p, about eps sqrt(log2 N) rms(p) spread over
    # all wavenumbers, reaches u through G, which amplifies the highest ones
    # by up to 2 / min(dx, dy): at this aspect ratio that bound exceeds the
    # 1e-5 of the step tests
    eps = 6e-8
    hmin = min(L / nx, L / ny)
    rms = lambda t: t.pow(2).mean().sqrt().item()
    bound = 2 * eps * math.sqrt(math.log2(nx * ny)) * (2 / hmin) * rms(ep) / min(rms(u), rms(v))
    tol = max(1e-5, bound)
    print("extreme-aspect projection tolerance %.3g" % tol)
    assert rel_l2(gu, eu) < tol and rel_l2(gv, ev) < tol
    assert rel_l2(p, ep) < 1e-5


def test_streaming_full_size_step():
    """One plain RK4 step at the streaming shape of the benchmark (1024^2,
    batch 128, FP32; 537 MB per field) in the launch configuration it times;
    trajectories 0 and 127 against the oracle."""
    L_ = need_gpu()
    announce("streaming 1024^2 x 128 step")
    n, B = 1024, 128
    s = L_.Solver(n, n, B)
    gu, gv = s.init_state(L_.IC_GRF_PEAK, seed=0)
    kw = dict(nu=2e-4, dt=0.1 * 2 * math.pi / n)
    uo, vo = s.fv_step(L_.params(**kw), gu, gv)
    # eight trajectories spread over the batch (every 18th), in L2 and
    # element by element
    for b in list(range(0, B, 18)) + [B - 1]:
        u0, v0 = cpu64(gu[b:b + 1]), cpu64(gv[b:b + 1])
        eu, ev = timestep.fv_step(u0, v0, oracle_prm(n, n, **kw))
        assert_fields_close(uo[b], eu[0], what=("u", b))
        assert_fields_close(vo[b], ev[0], what=("v", b))
    s.close()


def test_decaying512_2000_step_rollout_matches_oracle_golden():
    """The full 2000-step run of the decaying workload (512^2, batch 16, FP32,
    the benchmark's launch shape) against the FP64 oracle's rollout of
    trajectory 0 from the same float32 initial state (tests/golden/
    decaying512_rollout.json, written by make_decaying512_rollout.py with
    the oracle only): energy and enstrophy every 100 steps, the final state
    on every 16th row and column, and its Fourier coefficients |k| <= 4,
    each within 1e-3.  Decaying turbulence at this Reynolds number amplifies
    the FP32 roundoff of each step (1e-7 relative) over the 1.75 simulated
    seconds, well below 1e-3."""
    import json
    import os
    L_ = need_gpu()
    announce("decaying512 2000-step rollout vs golden")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "decaying512_rollout.json")))
    w = si.WORKLOADS["decaying512"]
    n, B = w["nx"], w["batch"]
    assert gold["n"] == n and gold["dt"] == w["dt"] and gold["nu"] == w["nu"]
    s = L_.Solver(n, n, B)
    u0, v0 = s.init_state(L_.IC_GRF_PEAK, seed=0)
    every = gold["series"]["step"][1]
    tu, tv = s.rollout(L_.params(nu=w["nu"], dt=w["dt"]), u0, v0, gold["steps"], save_every=every)
    h = L / n
    en, ens = [], []
    for st in [(u0, v0)] + [(tu[t], tv[t]) for t in range(tu.shape[0])]:
        en.append(s.diagnostics(st[0].contiguous(), st[1].contiguous())[0, 1].item())
        wv = s.vorticity(st[0].contiguous(), st[1].contiguous())[0].double()
        ens.append(0.5 * wv.pow(2).mean().item())
    e_en = max(abs(a - b) / abs(b) for a, b in zip(en, gold["series"]["energy"]))
    e_ens = max(abs(a - b) / abs(b) for a, b in zip(ens, gold["series"]["enstrophy"]))
    k = gold["final"]["stride"]
    fu, fv_ = tu[-1, 0, ::k, ::k], tv[-1, 0, ::k, ::k]
    gu_, gv_ = torch.tensor(gold["final"]["u"]), torch.tensor(gold["final"]["v"])
    e_state = max(rel_l2(fu, gu_), rel_l2(fv_, gv_))
    km = gold["modes"]["kmax"]
    ks = list(range(-km, km + 1))
    e_modes = 0.0
    for q, nm in ((tu[-1, 0], "u"), (tv[-1, 0], "v")):
        f = torch.fft.fft2(q.double().cpu()) / (n * n)
        got = torch.stack([torch.stack([f[ky % n, kx % n] for kx in ks]) for ky in ks])
        ref = torch.complex(torch.tensor(gold["modes"][nm + "_re"], dtype=torch.float64),
                            torch.tensor(gold["modes"][nm + "_im"], dtype=torch.float64))
        e_modes = max(e_modes, ((got - ref).abs().pow(2).sum().sqrt() / ref.abs().pow(2).sum().sqrt()).item())
    print("2000-step rollout vs FP64 oracle: energy %.2e, enstrophy %.2e, sampled state %.2e, "
          "low modes %.2e" % (e_en, e_ens, e_state, e_modes))
    assert e_en < 1e-3 and e_ens < 1e-3 and e_state < 1e-3 and e_modes < 1e-3
    s.close()
