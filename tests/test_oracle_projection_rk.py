"""Pins for the oracle's projection, Poisson solve and time integrators."""
import math

import numpy as np
import pytest
import torch

from oracle import fv, ic, projection, timestep

L = 2 * math.pi


def _dense_operators(nx, ny, dx, dy):
    """D (N x 2N) and G (2N x N) built entry by entry from the MAC stencil
    positions: u[j,i] is the west face of cell (i,j), v[j,i] the south face."""
    n = nx * ny
    D = np.zeros((n, 2 * n))
    G = np.zeros((2 * n, n))
    idx = lambda j, i: (j % ny) * nx + (i % nx)
    for j in range(ny):
        for i in range(nx):
            c = idx(j, i)
            # outflow through east face (u of cell i+1) minus west face (u of cell i)
            D[c, idx(j, i + 1)] += 1 / dx
            D[c, idx(j, i)] -= 1 / dx
            D[c, n + idx(j + 1, i)] += 1 / dy
            D[c, n + idx(j, i)] -= 1 / dy
            # pressure gradient at the west face of cell (i,j): p(i,j) - p(i-1,j)
            G[idx(j, i), idx(j, i)] += 1 / dx
            G[idx(j, i), idx(j, i - 1)] -= 1 / dx
            G[n + idx(j, i), idx(j, i)] += 1 / dy
            G[n + idx(j, i), idx(j - 1, i)] -= 1 / dy
    return D, G


@pytest.mark.parametrize("shape", [(8, 8), (8, 6)])
def test_poisson_matches_dense_least_squares(shape):
    nx, ny = shape
    dx, dy = L / nx, L / ny
    D, G = _dense_operators(nx, ny, dx, dy)
    assert np.allclose(G, -D.T)
    g = np.random.default_rng(0)
    u = g.standard_normal((ny, nx))
    v = g.standard_normal((ny, nx))
    prm = {"dx": dx, "dy": dy}
    d = projection.divergence(torch.tensor(u), torch.tensor(v), prm).numpy()
    assert np.allclose(d.ravel(), D @ np.concatenate([u.ravel(), v.ravel()]), atol=1e-13)
    A = D @ G
    p_ls = np.linalg.lstsq(A, d.ravel(), rcond=None)[0]
    p_ls -= p_ls.mean()
    p = projection.poisson_solve(torch.tensor(d), prm).numpy().ravel()
    assert abs(p.mean()) < 1e-13
    assert np.linalg.norm(A @ p - d.ravel()) / np.linalg.norm(d) < 1e-12
    assert np.allclose(p, p_ls, atol=1e-12)


def test_projection_invariants():
    g = torch.Generator().manual_seed(1)
    n = 16
    prm = {"dx": L / n, "dy": L / 12}
    a = torch.randn(2, 2, 12, n, generator=g, dtype=torch.float64)
    b = torch.randn(2, 2, 12, n, generator=g, dtype=torch.float64)
    pa = projection.project(a[0], a[1], prm)[:2]
    pb = projection.project(b[0], b[1], prm)[:2]
    # divergence-free
    assert projection.divergence(*pa, prm).abs().max() < 1e-12
    # idempotent
    ppa = projection.project(*pa, prm)[:2]
    assert max((x - y).abs().max() for x, y in zip(ppa, pa)) < 1e-13
    # symmetric: <Pa, b> = <a, Pb>
    lhs = sum((x * y).sum() for x, y in zip(pa, (b[0], b[1])))
    rhs = sum((x * y).sum() for x, y in zip((a[0], a[1]), pb))
    assert abs(lhs - rhs) < 1e-11
    # mean preserved
    assert torch.allclose(pa[0].mean(dim=(-2, -1)), a[0].mean(dim=(-2, -1)), atol=1e-14)
    assert torch.allclose(pa[1].mean(dim=(-2, -1)), a[1].mean(dim=(-2, -1)), atol=1e-14)
    # a gradient field is removed entirely
    phi = torch.randn(12, n, generator=g, dtype=torch.float64)
    gx, gy = projection.gradient(phi, prm)
    r = projection.project(gx, gy, prm)[:2]
    assert max(x.abs().max() for x in r) < 1e-12


def test_rk4_viscous_tgv_amplification_closed_form():
    # advection off: u_n = G(z)^n u_0 with z = nu dt (mu_x + mu_y) and
    # G(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 (the RK4 stability polynomial)
    n = 16
    h = L / n
    nu, dt, steps = 0.2, 0.05, 7
    u, v = ic.taylor_green(1, n, n, L, L, k=2)
    prm = fv.grid_params(n, n, nu=nu, dt=dt, mask=fv.VISCOSITY)
    un, vn = timestep.fv_step(u, v, prm, nsteps=steps)
    th = 2 * h
    mu = -math.sin(th / 2) * (27 * math.sin(th / 2) - math.sin(1.5 * th)) / (6 * h * h)
    z = nu * dt * 2 * mu
    G = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    assert torch.allclose(un, G ** steps * u, rtol=1e-12, atol=1e-14)
    assert torch.allclose(vn, G ** steps * v, rtol=1e-12, atol=1e-14)


def test_ssprk3_linear_decay_closed_form():
    # SSP-RK3 on R = -d u (drag only): u_n = (1 - z + z^2/2 - z^3/6)^n u_0, z = d dt
    n = 8
    prm = fv.grid_params(n, n, dt=0.1, drag=0.7, mask=fv.FORCING, rk=timestep.SSPRK3)
    u = torch.randn(1, n, n, dtype=torch.float64)
    v = torch.randn(1, n, n, dtype=torch.float64)
    un, vn = timestep.fv_step(u, v, prm, nsteps=5)
    z = 0.07
    G = 1 - z + z * z / 2 - z ** 3 / 6
    # projection is applied (MAC layout): compare the projected initial field
    pu, pv, _ = projection.project(u, v, prm)
    assert torch.allclose(un, G ** 5 * pu, atol=1e-13)
    assert torch.allclose(vn, G ** 5 * pv, atol=1e-13)


def test_tgv_decay_second_order_to_exact_solution():
    # TGV is an exact NS solution decaying as exp(-2 nu k^2 t); the
    # nonlinear term is a gradient, removed by the projection
    nu, T = 0.05, 0.5
    errs = []
    for n in (16, 32, 64):
        u, v = ic.taylor_green(1, n, n, L, L)
        dt = 0.25 * L / 64
        steps = int(round(T / dt))
        prm = fv.grid_params(n, n, nu=nu, dt=T / steps)
        un, vn = timestep.fv_step(u, v, prm, nsteps=steps)
        ex = math.exp(-2 * nu * T)
        errs.append(max((un - ex * u).abs().max().item(), (vn - ex * v).abs().max().item()))
    o1 = math.log2(errs[0] / errs[1])
    o2 = math.log2(errs[1] / errs[2])
    assert 1.7 < o1 < 2.5 and 1.7 < o2 < 2.5, errs


def _order(step_fn, u, v, prm, T, dts):
    ref_dt = dts[-1] / 8
    n = int(round(T / ref_dt))
    ru, rv = step_fn(u, v, dict(prm, dt=T / n), n)
    errs = []
    for dt in dts:
        m = int(round(T / dt))
        a, b = step_fn(u, v, dict(prm, dt=T / m), m)
        errs.append(max((a - ru).abs().max().item(), (b - rv).abs().max().item()))
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)], errs


def test_rk4_with_projection_fourth_order_in_time():
    n = 16
    u, v = ic.grf_peak(1, n, n, L, L, seed=3, kpeak=2.0)
    prm = fv.grid_params(n, n, nu=0.02, forcing_amp=0.5, forcing_k=2.0, drag=0.1)
    step = lambda a, b, p, m: timestep.fv_step(a, b, p, nsteps=m)
    orders, errs = _order(step, u, v, prm, 0.4, [0.1, 0.05, 0.025])
    assert all(3.6 < o < 4.5 for o in orders), (orders, errs)


def test_ssprk3_third_order_in_time_burgers():
    n = 16
    u, v = ic.fourier_modes(1, n, n, L, L, seed=2)
    prm = fv.grid_params(n, n, nu=0.05, rk=timestep.SSPRK3, layout=timestep.COLLOCATED)
    step = lambda a, b, p, m: timestep.fv_step(a, b, p, nsteps=m)
    orders, errs = _order(step, u, v, prm, 0.2, [0.04, 0.02, 0.01])
    assert all(2.7 < o < 3.4 for o in orders), (orders, errs)


def test_burgers_1d_cole_hopf_convergence():
    # u = 2 nu k b e^{-nu k^2 t} sin(kx) / (a + b e^{-nu k^2 t} cos(kx)) solves
    # u_t + u u_x = nu u_xx (Cole-Hopf with phi = a + b e^{-nu k^2 t} cos kx)
    nu, a, b, T = 0.1, 1.2, 1.0, 0.5
    exact = lambda x, t: (2 * nu * b * math.exp(-nu * t) * torch.sin(x)
                          / (a + b * math.exp(-nu * t) * torch.cos(x)))
    errs = []
    for n in (64, 128, 256):
        x = (torch.arange(n, dtype=torch.float64) + 0.5) * L / n
        u = exact(x, 0.0).view(1, 1, n).expand(1, 4, n).clone()
        v = torch.zeros_like(u)
        dt = 0.002
        prm = fv.grid_params(n, 4, lx=L, ly=L * 4 / n, nu=nu, dt=dt, rk=timestep.SSPRK3,
                             layout=timestep.COLLOCATED)
        un, vn = timestep.fv_step(u, v, prm, nsteps=int(round(T / dt)))
        assert vn.abs().max() == 0
        errs.append((un[0, 0] - exact(x, T)).abs().max().item())
    o1 = math.log2(errs[0] / errs[1])
    o2 = math.log2(errs[1] / errs[2])
    assert 1.8 < o1 < 2.4 and 1.9 < o2 < 2.4, errs


def test_mean_momentum_decays_by_drag_polynomial():
    # sin(4y) has zero mean and flux differences telescope, so the mean of u
    # evolves only through the drag: <u>_n = <u>_0 G(-d dt)^n (RK4 polynomial)
    from oracle.learned import constrain
    n = 16
    u, v = ic.grf_peak(2, n, n, L, L, seed=4)
    u = u + 0.7
    v = v - 0.4
    g = torch.Generator().manual_seed(2)
    coef = constrain(0.1 * torch.randn(2, 64, n, n, generator=g, dtype=torch.float64))
    dt, d = 0.05, 0.1
    prm = fv.grid_params(n, n, nu=1e-3, dt=dt, forcing_amp=1.0, forcing_k=4.0, drag=d)
    un, vn = timestep.fv_step(u, v, prm, coef=coef, nsteps=6)
    z = -d * dt
    G = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    assert torch.allclose(un.mean(dim=(-2, -1)), u.mean(dim=(-2, -1)) * G ** 6, atol=1e-13)
    assert torch.allclose(vn.mean(dim=(-2, -1)), v.mean(dim=(-2, -1)) * G ** 6, atol=1e-13)
    # decaying flow (no drag): mean conserved exactly
    prm = fv.grid_params(n, n, nu=1e-3, dt=dt)
    un, vn = timestep.fv_step(u, v, prm, coef=coef, nsteps=6)
    assert torch.allclose(un.mean(dim=(-2, -1)), u.mean(dim=(-2, -1)), atol=1e-13)
    assert projection.divergence(un, vn, prm).abs().max() < 1e-11
