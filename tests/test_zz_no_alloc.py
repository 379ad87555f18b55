"""ldsv_fv_step_noalloc (the handle-less FV step whose workspace is the
library's fixed device scratch array) against ldsv_fv_step through the C
ABI: two calls in a row, the second on a smaller grid, then an FP64
collocated call, each equal to the handle path; a grid beyond the scratch
array is refused before any work is enqueued."""
import pytest
import torch

import synthetic_inputs as si
from oracle import ic, timestep
from tests.gpu_common import L, announce, assert_fields_close, dev, need_gpu, oracle_prm

pytestmark = pytest.mark.gpu


def test_noalloc_step_matches_handle_step():
    L_ = need_gpu()
    # call 1: 128^2 x 8 FP32, two steps (the three-pass projection)
    nx = ny = 128
    b = 8
    announce("fv_step_noalloc", nx, ny, b)
    u, v = ic.grf_peak(b, nx, ny, L, L, seed=21)
    u, v = u.float().double(), v.float().double()
    kw = dict(nu=1e-3, dt=0.5 * (L / nx), forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    prm = L_.params(**kw)
    gu, gv = dev(u, torch.float32), dev(v, torch.float32)
    nu_, nv_ = L_.fv_step_noalloc(prm, gu, gv, nsteps=2)
    s = L_.Solver(nx, ny, b)
    hu, hv = s.fv_step(prm, gu, gv, nsteps=2)
    torch.cuda.synchronize()
    assert_fields_close(nu_, hu, rel=1e-6, elem=1e-6, what="noalloc vs handle, call 1 u")
    assert_fields_close(nv_, hv, rel=1e-6, elem=1e-6, what="noalloc vs handle, call 1 v")
    eu, ev = timestep.fv_step(u, v, oracle_prm(nx, ny, **kw), nsteps=2)
    assert_fields_close(nu_, eu, what="noalloc vs oracle u")
    assert_fields_close(nv_, ev, what="noalloc vs oracle v")
    del s

    # call 2, smaller: 64 x 32 on [0, 2pi) x [0, pi), 3 trajectories, raw
    # learned coefficients, in place (the one-workgroup LDS projection)
    nx, ny, b = 64, 32, 3
    announce("fv_step_noalloc", nx, ny, b, "coef, in place")
    u, v = ic.grf_peak(b, nx, ny, L, L / 2, seed=22)
    coef = torch.tensor(si.random_field(23, (b, 64, ny, nx), scale=0.1)).float().cuda()
    kw2 = dict(nu=1e-3, dt=0.02, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    prm2 = L_.params(**kw2)
    s2 = L_.Solver(nx, ny, b, ly=L / 2)
    hu, hv = s2.fv_step(prm2, dev(u, torch.float32), dev(v, torch.float32), coef=coef, nsteps=3)
    gu, gv = dev(u, torch.float32), dev(v, torch.float32)
    ru, rv = L_.fv_step_noalloc(prm2, gu, gv, nsteps=3, coef=coef, out=(gu, gv), ly=L / 2)
    torch.cuda.synchronize()
    assert ru.data_ptr() == gu.data_ptr()
    assert_fields_close(gu, hu, rel=1e-6, elem=1e-6, what="noalloc vs handle, call 2 u")
    assert_fields_close(gv, hv, rel=1e-6, elem=1e-6, what="noalloc vs handle, call 2 v")
    del s2

    # call 3: FP64 collocated Burgers 32^2, SSP-RK3
    n = 32
    announce("fv_step_noalloc", n, n, 1, "f64 collocated")
    u, v = ic.fourier_modes(1, n, n, L, L, seed=24)
    kw3 = dict(nu=0.01, dt=0.01)
    prm3 = L_.params(rk=L_.SSPRK3, **kw3)
    s3 = L_.Solver(n, n, 1, dtype=torch.float64, layout=L_.COLLOCATED)
    hu, hv = s3.fv_step(prm3, dev(u, torch.float64), dev(v, torch.float64), nsteps=4)
    nu_, nv_ = L_.fv_step_noalloc(prm3, dev(u, torch.float64), dev(v, torch.float64), nsteps=4,
                                  layout=L_.COLLOCATED)
    torch.cuda.synchronize()
    assert_fields_close(nu_, hu, rel=1e-13, elem=1e-13, what="noalloc vs handle, f64 u")
    assert_fields_close(nv_, hv, rel=1e-13, elem=1e-13, what="noalloc vs handle, f64 v")


def test_noalloc_rejects_grid_beyond_scratch():
    L_ = need_gpu()
    announce("fv_step_noalloc rejection")
    # 256^2 x 32 FP32 needs ~56 MiB of workspace: refused on the host
    u = torch.zeros(32, 256, 256, device="cuda")
    v = torch.zeros_like(u)
    with pytest.raises(L_.LdsvError) as e:
        L_.fv_step_noalloc(L_.params(nu=1e-3, dt=1e-3), u, v)
    assert e.value.code == L_.ESHAPE and "scratch" in str(e.value)
