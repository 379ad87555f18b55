"""GPU parity of the shear-flow system with a passive scalar (velocity and
scalar stepped together) against the FP64 oracle, on the paper's
non-square domain [0, 8] x [0, 4]."""
import pytest
import torch

from oracle import ic, scalar
from tests.gpu_common import assert_fields_close, announce, cpu64, dev, need_gpu, oracle_prm, rel_l2

pytestmark = pytest.mark.gpu

LX, LY = 8.0, 4.0
KW = dict(nu=1e-3, dt=0.01)


# tiles: 64 x 16 (128 x 64, 64 x 32), 32 x 8 (32 x 8), 8 x 8 (16 x 16)
@pytest.mark.parametrize("nx,ny,b,dtype,tol", [
    (128, 64, 3, torch.float32, 1e-5), (64, 32, 2, torch.float32, 1e-5),
    (64, 32, 2, torch.float64, 1e-12), (32, 8, 2, torch.float64, 1e-12),
    (16, 16, 1, torch.float64, 1e-12)])
def test_scalar_step_matches_oracle(nx, ny, b, dtype, tol):
    L_ = need_gpu()
    announce("scalar step", nx, ny, b, dtype)
    s = L_.Solver(nx, ny, b, lx=LX, ly=LY, dtype=dtype)
    u0, v0 = ic.shear_layer(b, nx, ny, LX, LY, seed=3, delta=0.1)
    s0 = ic.shear_scalar(b, nx, ny, LX, LY, delta=0.1)
    u, v, c = dev(u0, dtype), dev(v0, dtype), dev(s0, dtype)
    prm = L_.params(**KW)
    uo, vo, so = s.fv_step_scalar(prm, 2e-3, u, v, c, nsteps=3)
    ru, rv, rs = scalar.fv_step_scalar(cpu64(u), cpu64(v), cpu64(c),
                                       oracle_prm(nx, ny, lx=LX, ly=LY, diffusivity=2e-3, **KW),
                                       nsteps=3)
    assert rel_l2(uo, ru) < tol and rel_l2(vo, rv) < tol and rel_l2(so, rs) < tol
    # the velocity is the plain step's, and the total of s is conserved
    pu, pv = s.fv_step(prm, u, v, nsteps=3)
    assert torch.equal(pu, uo) and torch.equal(pv, vo)
    tot0 = cpu64(c).sum(dim=(-2, -1))
    tot = cpu64(so).sum(dim=(-2, -1))
    rt = 1e-6 if dtype == torch.float32 else 1e-13
    assert ((tot - tot0).abs() / tot0.abs()).max().item() < rt


def test_scalar_init_and_in_place():
    L_ = need_gpu()
    announce("scalar init, in place")
    nx, ny, b = 128, 64, 2
    s = L_.Solver(nx, ny, b, lx=LX, ly=LY, dtype=torch.float64)
    c = s.init_scalar(delta=0.1)
    assert torch.allclose(c.cpu(), ic.shear_scalar(b, nx, ny, LX, LY, delta=0.1), atol=1e-15)
    u, v = s.init_state(L_.IC_SHEAR_LAYER, seed=5, delta=0.1)
    prm = L_.params(**KW)
    ref = s.fv_step_scalar(prm, 1e-3, u, v, c, nsteps=2)
    s.fv_step_scalar(prm, 1e-3, u, v, c, nsteps=2, out=(u, v, c))
    assert torch.equal(u, ref[0]) and torch.equal(v, ref[1]) and torch.equal(c, ref[2])


def test_shear_scalar_full_size_step():
    """One step of velocity and passive scalar at the benchmark's fine
    resolution (2048 x 1024 on [0, 8] x [0, 4], batch 8, FP32) in the launch
    configuration it times; trajectories 0, 3 and 7 against the oracle, in
    L2 and element by element."""
    import synthetic_inputs as si
    L_ = need_gpu()
    announce("shear_scalar full-size step")
    w = si.WORKLOADS["shear_scalar"]
    nx, ny, B = w["nx"], w["ny"], w["batch"]
    s = L_.Solver(nx, ny, B, lx=w["lx"], ly=w["ly"])
    u, v = s.init_state(L_.IC_SHEAR_LAYER, seed=1000, delta=w["delta"])
    c = s.init_scalar(delta=w["delta"])
    prm = L_.params(nu=w["nu"], dt=w["dt"])
    uo, vo, co = s.fv_step_scalar(prm, w["diffusivity"], u, v, c)
    oprm = oracle_prm(nx, ny, lx=w["lx"], ly=w["ly"], nu=w["nu"], dt=w["dt"],
                      diffusivity=w["diffusivity"])
    for b in (0, 3, B - 1):
        ru, rv, rc = scalar.fv_step_scalar(cpu64(u[b:b + 1]), cpu64(v[b:b + 1]),
                                           cpu64(c[b:b + 1]), oprm)
        assert_fields_close(uo[b], ru[0], what=("u", b))
        assert_fields_close(vo[b], rv[0], what=("v", b))
        assert_fields_close(co[b], rc[0], what=("s", b))
