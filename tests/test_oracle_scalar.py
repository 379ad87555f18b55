"""Pins for the oracle's passive scalar (the shear-flow system): exact
conservation, invariance of a constant, and the closed-form amplification
of a Fourier mode under pure diffusion and under uniform advection (the
kernel symbols through the RK4 stability polynomial)."""
import math

import numpy as np
import torch

from oracle import fv, ic, scalar

LX, LY = 8.0, 4.0   # the shear-flow domain [0, 8] x [0, 4]


def _prm(nx, ny, **kw):
    return fv.grid_params(nx, ny, lx=LX, ly=LY, **kw)


def _rk4_poly(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_scalar_total_is_conserved():
    nx, ny = 64, 32
    u, v = ic.shear_layer(2, nx, ny, LX, LY, seed=3, delta=0.1)
    s = ic.shear_scalar(2, nx, ny, LX, LY, delta=0.1) + 0.1 * torch.rand(2, ny, nx,
                                                                        dtype=torch.float64)
    prm = _prm(nx, ny, nu=1e-3, diffusivity=1e-3, dt=0.01)
    r = scalar.scalar_rhs(u, v, s, prm)
    assert r.sum(dim=(-2, -1)).abs().max().item() < 1e-12 * r.abs().max().item() * nx * ny
    _, _, s5 = scalar.fv_step_scalar(u, v, s, prm, nsteps=5)
    assert torch.allclose(s5.sum(dim=(-2, -1)), s.sum(dim=(-2, -1)), rtol=1e-13)


def test_constant_scalar_stays_constant():
    nx, ny = 32, 16
    u, v = ic.shear_layer(1, nx, ny, LX, LY, seed=4, delta=0.1)
    s = torch.full((1, ny, nx), 0.7, dtype=torch.float64)
    _, _, s2 = scalar.fv_step_scalar(u, v, s, _prm(nx, ny, nu=1e-3, diffusivity=2e-3, dt=0.01), 2)
    assert (s2 - 0.7).abs().max().item() < 1e-14


def test_pure_diffusion_of_a_mode_closed_form():
    """u = 0: s = cos(2 pi m x / Lx) is an eigenfunction with eigenvalue
    lam = -D (4/h^2) sin(th/2) (27 sin(th/2) - sin(3 th/2)) / 24 (the compact
    difference of the fourth-order face derivative), th = 2 pi m / nx, so n
    RK4 steps multiply it by G(dt lam)^n."""
    nx, ny, m, D, dt, n = 32, 16, 3, 0.05, 0.02, 4
    h = LX / nx
    th = 2 * math.pi * m / nx
    lam = -D * 4 / h ** 2 * math.sin(th / 2) * (27 * math.sin(th / 2) - math.sin(1.5 * th)) / 24
    x = (np.arange(nx) + 0.5) * h
    s0 = torch.tensor(np.cos(2 * math.pi * m * x / LX)).view(1, 1, -1).expand(1, ny, nx)
    zero = torch.zeros(1, ny, nx, dtype=torch.float64)
    prm = _prm(nx, ny, diffusivity=D, dt=dt, mask=fv.VISCOSITY)
    _, _, sn = scalar.fv_step_scalar(zero, zero, s0.contiguous(), prm, nsteps=n)
    assert torch.allclose(sn, _rk4_poly(dt * lam) ** n * s0, atol=1e-13)


def test_uniform_advection_of_a_mode_closed_form():
    """u = U, v = 0: the midpoint flux difference has symbol -i U sin(th)/h on
    exp(i th i), so s = Re(exp(i k x)) goes to Re(G(-i U dt sin(th)/h)^n
    exp(i k x)).  (A uniform u is divergence-free and a fixed point of the
    projection with no viscosity.)"""
    nx, ny, m, U, dt, n = 32, 8, 2, 0.8, 0.05, 3
    h = LX / nx
    th = 2 * math.pi * m / nx
    z = -1j * U * dt * math.sin(th) / h
    x = (np.arange(nx) + 0.5) * h
    s0 = torch.tensor(np.cos(2 * math.pi * m * x / LX)).view(1, 1, -1).expand(1, ny, nx)
    u = torch.full((1, ny, nx), U, dtype=torch.float64)
    v = torch.zeros(1, ny, nx, dtype=torch.float64)
    prm = _prm(nx, ny, dt=dt, mask=fv.ADVECTION)
    un, vn, sn = scalar.fv_step_scalar(u, v, s0.contiguous(), prm, nsteps=n)
    ref = (_rk4_poly(z) ** n * np.exp(1j * 2 * math.pi * m * x / LX)).real
    assert np.abs(sn[0].numpy() - ref[None, :]).max() < 1e-13
    assert torch.allclose(un, u, atol=1e-14)


def test_shear_scalar_profile():
    s = ic.shear_scalar(1, 8, 64, LX, LY, delta=0.1)
    col = s[0, :, 0]
    assert col.min().item() > -1e-12 and col.max().item() < 1 + 1e-12
    # a layer at y = L/4 and 3L/4: ~0 at y = 0, ~1 at y = L/2
    assert col[0].item() < 1e-3 and abs(col[31].item() - 1) < 1e-3
