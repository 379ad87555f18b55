"""Pins of the oracle's per-cell learned derivative stencils (Sec. 3.4, the
m = d operator in per-cell form): the constraint against a KKT solve, the
exactness on linear fields, written-out sums on a tiny grid, conservation,
the reduction to the fourth-order kernel, and the autograd gradient against
central differences."""
import math

import numpy as np
import pytest
import torch

from oracle import fv, learned, timestep
from oracle.cnn import LAYERS

D = torch.float64


def _prm(nx, ny, **kw):
    return fv.grid_params(nx, ny, nu=kw.pop("nu", 0.05), dt=kw.pop("dt", 1e-3), **kw)


def test_constraint_is_the_kkt_projection():
    """w = argmin |w - (w_P + r)|^2 subject to sum(w) = 0, sum(w x) = 1 and
    sum(w b) = 0, solved as a KKT system with numpy, equals constrain_deriv
    for every kind."""
    g = torch.Generator().manual_seed(0)
    raw = torch.randn(2, 64, 3, 2, generator=g, dtype=D)
    w = learned.constrain_deriv(raw).numpy()
    x = np.array([a - 0.5 for a, _ in fv.FOOTPRINT])
    y = np.array([float(b) for _, b in fv.FOOTPRINT])
    A = np.stack([np.ones(16), x, y])
    K = np.zeros((19, 19))
    K[:16, :16] = np.eye(16)
    K[:16, 16:] = A.T
    K[16:, :16] = A
    wp = fv.plain_deriv_coefficients().numpy()
    for b in range(2):
        for kind in range(4):
            for j in range(3):
                for i in range(2):
                    t = wp[16 * kind:16 * kind + 16] + raw[b, 16 * kind:16 * kind + 16, j, i].numpy()
                    sol = np.linalg.solve(K, np.concatenate([t, [0.0, 1.0, 0.0]]))
                    np.testing.assert_allclose(w[b, 16 * kind:16 * kind + 16, j, i], sol[:16],
                                               rtol=0, atol=1e-13)


def test_constraint_moments_and_null_directions():
    g = torch.Generator().manual_seed(1)
    raw = torch.randn(1, 64, 4, 4, generator=g, dtype=D)
    w = learned.constrain_deriv(raw).reshape(1, 4, 16, 4, 4)
    x = torch.tensor([a - 0.5 for a, _ in fv.FOOTPRINT], dtype=D).reshape(1, 1, 16, 1, 1)
    y = torch.tensor([float(b) for _, b in fv.FOOTPRINT], dtype=D).reshape(1, 1, 16, 1, 1)
    assert w.sum(2).abs().max() < 1e-13
    assert ((w * x).sum(2) - 1).abs().max() < 1e-13
    assert (w * y).sum(2).abs().max() < 1e-13
    # adding constants and multiples of x and b to the raw values changes nothing
    shift = (2.5 + 1.5 * x - 0.75 * y).expand(1, 4, 16, 4, 4).reshape(1, 64, 4, 4)
    assert (learned.constrain_deriv(raw + shift) - learned.constrain_deriv(raw)).abs().max() < 1e-13
    # r = 0 gives the fourth-order kernel [1, -27, 27, -1]/24 on the row b = 0
    w0 = learned.constrain_deriv(torch.zeros(1, 64, 1, 1, dtype=D))[0, :, 0, 0]
    for kind in range(4):
        ref = torch.zeros(16, dtype=D)
        ref[4:8] = torch.tensor([1.0, -27.0, 27.0, -1.0], dtype=D) / 24.0
        assert torch.equal(w0[16 * kind:16 * kind + 16], ref)


def test_face_derivative_exact_on_linear_fields():
    """Per-cell random weights differentiate a x + b y + c exactly at every
    face whose footprint does not wrap around the periodic box."""
    nx, ny = 16, 12
    dx, dy = 0.3, 0.7
    g = torch.Generator().manual_seed(2)
    w = learned.constrain_deriv(torch.randn(1, 64, ny, nx, generator=g, dtype=D))
    xs = torch.arange(nx, dtype=D) * dx
    ys = torch.arange(ny, dtype=D) * dy
    q = 1.7 * xs.view(1, -1) - 0.6 * ys.view(-1, 1) + 0.25
    q = q.unsqueeze(0)
    for kind in range(4):
        along_x = kind in (0, 2)
        d = fv._face_deriv(q, w, kind, along_x, dx if along_x else dy)[0]
        inner = d[2:ny - 3, 2:nx - 3]
        expect = 1.7 if along_x else -0.6
        assert (inner - expect).abs().max() < 1e-12, kind


def test_viscous_residual_against_written_out_sums():
    """The viscous part of ns_rhs with per-cell derivative weights against
    explicit loops over faces on a 6 x 5 grid (periodic indices)."""
    nx, ny = 6, 5
    prm = _prm(nx, ny, nu=0.3, mask=fv.VISCOSITY)
    dx, dy, nu = prm["dx"], prm["dy"], prm["nu"]
    g = torch.Generator().manual_seed(3)
    u = torch.randn(1, ny, nx, generator=g, dtype=D)
    v = torch.randn(1, ny, nx, generator=g, dtype=D)
    w = learned.constrain_deriv(torch.randn(1, 64, ny, nx, generator=g, dtype=D))
    ru, rv = fv.ns_rhs(u, v, prm, dcoef=w)

    def dface(q, kind, i, j):
        """Derivative of kind K at the face owned by cell (i, j)."""
        s_sum = 0.0
        for s, (a, b) in enumerate(fv.FOOTPRINT):
            if kind in (0, 2):
                val = q[0, (j + b) % ny, (i + a) % nx]
            else:
                val = q[0, (j + a) % ny, (i + b) % nx]
            s_sum += float(w[0, 16 * kind + s, j, i]) * float(val)
        return s_sum / (dx if kind in (0, 2) else dy)

    for j in range(ny):
        for i in range(nx):
            eu = nu * ((dface(u, 0, i, j) - dface(u, 0, i - 1 if i else nx - 1, j)) / dx +
                       (dface(u, 1, i, j) - dface(u, 1, i, j - 1 if j else ny - 1)) / dy)
            ev = nu * ((dface(v, 2, i, j) - dface(v, 2, i - 1 if i else nx - 1, j)) / dx +
                       (dface(v, 3, i, j) - dface(v, 3, i, j - 1 if j else ny - 1)) / dy)
            assert abs(float(ru[0, j, i]) - eu) < 1e-12
            assert abs(float(rv[0, j, i]) - ev) < 1e-12


def test_zero_raw_reduces_to_plain_residual_and_conserves():
    nx, ny = 16, 8
    prm = _prm(nx, ny, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    g = torch.Generator().manual_seed(4)
    u = torch.randn(2, ny, nx, generator=g, dtype=D)
    v = torch.randn(2, ny, nx, generator=g, dtype=D)
    w0 = learned.constrain_deriv(torch.zeros(2, 64, ny, nx, dtype=D))
    a = fv.ns_rhs(u, v, prm)
    b = fv.ns_rhs(u, v, prm, dcoef=w0)
    assert (a[0] - b[0]).abs().max() < 1e-13 and (a[1] - b[1]).abs().max() < 1e-13
    # the viscous fluxes telescope for arbitrary weights
    w = learned.constrain_deriv(torch.randn(2, 64, ny, nx, generator=g, dtype=D))
    pv = dict(prm, mask=fv.VISCOSITY)
    ru, rv = fv.ns_rhs(u, v, pv, dcoef=w)
    assert ru.sum(dim=(-1, -2)).abs().max() < 1e-11
    assert rv.sum(dim=(-1, -2)).abs().max() < 1e-11


def _net(seed, scale=0.05):
    g = torch.Generator().manual_seed(seed)
    ws, bs = [], []
    for ci, co in LAYERS:
        ws.append(torch.randn(co, ci, 3, 3, generator=g, dtype=D) * scale / math.sqrt(ci))
        bs.append(torch.randn(co, generator=g, dtype=D) * scale)
    return ws, bs


def test_zero_derivative_network_gives_the_learned_step():
    nx = ny = 16
    prm = _prm(nx, ny, k_c=1)
    g = torch.Generator().manual_seed(5)
    u = torch.randn(1, ny, nx, generator=g, dtype=D) * 0.3
    v = torch.randn(1, ny, nx, generator=g, dtype=D) * 0.3
    ws, bs = _net(6)
    dws, dbs = _net(7)
    dws[-1] = torch.zeros_like(dws[-1])
    dbs[-1] = torch.zeros_like(dbs[-1])
    a = learned.learned_fv_step(u, v, prm, ws, bs, 1)
    b = learned.learned_fv_step(u, v, prm, ws, bs, 1, dnet=(dws, dbs))
    assert (a[0] - b[0]).abs().max() < 1e-14 and (a[1] - b[1]).abs().max() < 1e-14
    # a non-zero derivative network changes the step
    c = learned.learned_fv_step(u, v, prm, ws, bs, 1, dnet=_net(7))
    assert (a[0] - c[0]).abs().max() > 1e-8


@pytest.mark.parametrize("seed", [8, 9])
def test_autograd_through_the_derivative_weights(seed):
    """d/d(raw) of a scalar loss of one FV step against central differences."""
    nx, ny = 8, 8
    prm = _prm(nx, ny, nu=0.2, dt=2e-2)
    g = torch.Generator().manual_seed(seed)
    u = torch.randn(1, ny, nx, generator=g, dtype=D)
    v = torch.randn(1, ny, nx, generator=g, dtype=D)
    lu = torch.randn(1, ny, nx, generator=g, dtype=D)
    raw = torch.randn(1, 64, ny, nx, generator=g, dtype=D) * 0.1
    direc = torch.randn(1, 64, ny, nx, generator=g, dtype=D)

    def loss(r):
        un, vn = timestep.fv_step(u, v, prm, dcoef=learned.constrain_deriv(r))
        return ((un - lu) ** 2).sum() + (vn ** 2).sum()

    r = raw.clone().requires_grad_(True)
    loss(r).backward()
    eps = 1e-6
    fd = (loss(raw + eps * direc) - loss(raw - eps * direc)) / (2 * eps)
    ad = (r.grad * direc).sum()
    assert abs(float(fd - ad)) < 1e-7 * max(1.0, abs(float(ad)))
