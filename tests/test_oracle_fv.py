"""Pins for the oracle's finite-volume stencils and residuals.

Each test checks the oracle against something fixed outside its own code:
trigonometric closed forms of the stencils, polynomial exactness, the
continuous PDE residual under grid refinement (consistency order), and
telescoping of the flux differences (discrete conservation).
"""
import math

import pytest
import torch

from oracle import fv
from oracle.learned import constrain

L = 2 * math.pi


def _mesh(nx, ny, xoff, yoff):
    dx, dy = L / nx, L / ny
    x = ((torch.arange(nx, dtype=torch.float64) + xoff) * dx).view(1, -1).expand(ny, nx)
    y = ((torch.arange(ny, dtype=torch.float64) + yoff) * dy).view(-1, 1).expand(ny, nx)
    return x, y


def test_stencil_symbols_closed_form():
    # q_m = sin(theta m): midpoint average = cos(theta/2) sin(theta (m+1/2));
    # S6 derivative = cos(theta (m+1/2)) (27 sin(theta/2) - sin(3 theta/2)) / (12 h)
    n = 32
    h = L / n
    for k in (1, 3, 7):
        th = k * h
        m = torch.arange(n, dtype=torch.float64)
        q = torch.sin(th * m).view(1, 1, n).expand(1, 4, n).clone()
        c = fv.plain_coefficients()
        face = fv.interp_x(q, c, 0)[0, 0]
        assert torch.allclose(face, math.cos(th / 2) * torch.sin(th * (m + 0.5)), atol=1e-14)
        d = fv.deriv4_x(q, h)[0, 0]
        sym = (27 * math.sin(th / 2) - math.sin(1.5 * th)) / (12 * h)
        assert torch.allclose(d, sym * torch.cos(th * (m + 0.5)), atol=1e-12)


def test_deriv4_exact_for_cubics_interp_exact_for_linear():
    n = 40
    h = 0.1
    x = torch.arange(n, dtype=torch.float64) * h
    q = (x ** 3 - 2 * x ** 2 + 0.5 * x).view(1, n).expand(3, n).clone()
    d = fv.deriv4_x(q, h)[0]
    xf = x + 0.5 * h
    exact = 3 * xf ** 2 - 4 * xf + 0.5
    assert torch.allclose(d[2:-3], exact[2:-3], rtol=1e-11, atol=1e-11)
    # and along y (transpose)
    dy = fv.deriv4_y(q.t().contiguous(), h)[:, 0]
    assert torch.allclose(dy[2:-3], exact[2:-3], rtol=1e-11, atol=1e-11)
    lin = (2 * x - 1).view(1, n).expand(5, n).clone()
    face = fv.interp_x(lin, fv.plain_coefficients(), 0)[2]
    assert torch.allclose(face[2:-3], (2 * xf - 1)[2:-3], atol=1e-13)


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_footprint_orientation_by_moments(kind):
    # A delta correction at footprint point s moves the face value of a linear
    # field by (a_s - 1/2) h along the face normal and by b_s h across it,
    # relative to the plain stencil (the footprint's centroid is the face).
    n = 24
    h = L / n
    along_x = kind in (0, 2)
    x, y = _mesh(n, n, 0.0, 0.0)
    for s, (a, b) in enumerate(fv.FOOTPRINT):
        raw = torch.zeros(1, 64, n, n, dtype=torch.float64)
        raw[:, 16 * kind + s] = 1.0
        c = constrain(raw)
        for field, is_x in ((x, True), (y, False)):
            q = field.unsqueeze(0).clone()
            f = fv.interp_x if along_x else fv.interp_y
            got = f(q, c, kind) - f(q, fv.plain_coefficients(), kind)
            if along_x:
                shift = (a - 0.5) * h if is_x else b * h
            else:
                shift = b * h if is_x else (a - 0.5) * h
            # away from the periodic seam
            assert torch.allclose(got[0, 4:-4, 4:-4], torch.full((n - 8, n - 8), shift,
                                  dtype=torch.float64), atol=1e-12), (s, is_x)


def _fields(x, y):
    u = torch.sin(x) * torch.cos(2 * y) + 0.3
    v = torch.cos(3 * x) * torch.sin(y) - 0.2
    return u, v


def _ns_exact(nx, ny, nu, amp, kf, drag):
    # continuous residual at the u points (i dx, (j+1/2) dy)
    x, y = _mesh(nx, ny, 0.0, 0.5)
    u, v = _fields(x, y)
    ux = torch.cos(x) * torch.cos(2 * y)
    uy = -2 * torch.sin(x) * torch.sin(2 * y)
    lap_u = -5 * torch.sin(x) * torch.cos(2 * y)
    vx = -3 * torch.sin(3 * x) * torch.sin(y)
    vy = torch.cos(3 * x) * torch.cos(y)
    ru = -(2 * u * ux) - (uy * v + u * vy) + nu * lap_u + amp * torch.sin(kf * y) - drag * u
    # continuous residual at the v points ((i+1/2) dx, j dy)
    x, y = _mesh(nx, ny, 0.5, 0.0)
    u, v = _fields(x, y)
    ux = torch.cos(x) * torch.cos(2 * y)
    uy = -2 * torch.sin(x) * torch.sin(2 * y)
    vx = -3 * torch.sin(3 * x) * torch.sin(y)
    vy = torch.cos(3 * x) * torch.cos(y)
    lap_v = -10 * torch.cos(3 * x) * torch.sin(y)
    rv = -(ux * v + u * vx) - 2 * v * vy + nu * lap_v - drag * v
    return ru, rv


def _ns_discrete(nx, ny, nu, amp, kf, drag):
    xu, yu = _mesh(nx, ny, 0.0, 0.5)
    xv, yv = _mesh(nx, ny, 0.5, 0.0)
    u = _fields(xu, yu)[0].unsqueeze(0)
    v = _fields(xv, yv)[1].unsqueeze(0)
    prm = fv.grid_params(nx, ny, nu=nu, forcing_amp=amp, forcing_k=kf, drag=drag)
    ru, rv = fv.ns_rhs(u, v, prm)
    return ru[0], rv[0]


@pytest.mark.parametrize("nonsquare", [False, True])
def test_ns_residual_second_order_consistency(nonsquare):
    nu, amp, kf, drag = 0.05, 1.0, 4.0, 0.1
    errs = []
    for n in (32, 64, 128):
        nx, ny = (n, n // 2) if nonsquare else (n, n)
        ru, rv = _ns_discrete(nx, ny, nu, amp, kf, drag)
        eu, ev = _ns_exact(nx, ny, nu, amp, kf, drag)
        errs.append(max((ru - eu).abs().max().item(), (rv - ev).abs().max().item()))
    o1 = math.log2(errs[0] / errs[1])
    o2 = math.log2(errs[1] / errs[2])
    assert errs[2] < 5e-2
    assert 1.8 < o1 < 2.3 and 1.8 < o2 < 2.3, errs


def test_viscous_operator_tgv_eigenvalue():
    # With advection and forcing off, R(TGV) = nu (mu_x + mu_y) TGV exactly,
    # mu(theta) = -sin(theta/2)(27 sin(theta/2) - sin(3 theta/2)) / (6 h^2).
    from oracle.ic import taylor_green
    n = 16
    h = L / n
    for k in (1, 2, 3):
        u, v = taylor_green(1, n, n, L, L, amp=1.0, k=k)
        prm = fv.grid_params(n, n, nu=0.3, mask=fv.VISCOSITY)
        ru, rv = fv.ns_rhs(u, v, prm)
        th = k * h
        mu = -math.sin(th / 2) * (27 * math.sin(th / 2) - math.sin(1.5 * th)) / (6 * h * h)
        assert torch.allclose(ru, 0.3 * 2 * mu * u, atol=1e-12)
        assert torch.allclose(rv, 0.3 * 2 * mu * v, atol=1e-12)


def test_flux_telescoping_conserves_momentum_any_coefficients():
    # the sum over cells of the advective and viscous residual vanishes for
    # any per-cell coefficients (each face value is owned by one cell)
    g = torch.Generator().manual_seed(0)
    n = 12
    u = torch.randn(2, n, n, generator=g, dtype=torch.float64)
    v = torch.randn(2, n, n, generator=g, dtype=torch.float64)
    raw = torch.randn(2, 64, n, n, generator=g, dtype=torch.float64)
    prm = fv.grid_params(n, n, nu=0.1, mask=fv.ADVECTION | fv.VISCOSITY)
    ru, rv = fv.ns_rhs(u, v, prm, constrain(raw))
    assert ru.sum(dim=(-2, -1)).abs().max() < 1e-10
    assert rv.sum(dim=(-2, -1)).abs().max() < 1e-10
    # but the residual itself is not trivially zero
    assert ru.abs().max() > 1.0


def _burgers_exact(n, nu):
    x, y = _mesh(n, n, 0.5, 0.5)
    u, v = _fields(x, y)
    ux = torch.cos(x) * torch.cos(2 * y)
    uy = -2 * torch.sin(x) * torch.sin(2 * y)
    vx = -3 * torch.sin(3 * x) * torch.sin(y)
    vy = torch.cos(3 * x) * torch.cos(y)
    ru = nu * (-5 * torch.sin(x) * torch.cos(2 * y)) - (u * ux + v * uy)
    rv = nu * (-10 * torch.cos(3 * x) * torch.sin(y)) - (u * vx + v * vy)
    return u, v, ru, rv


def test_burgers_residual_second_order_consistency():
    nu = 0.05
    errs = []
    for n in (32, 64, 128):
        u, v, eu, ev = _burgers_exact(n, nu)
        prm = fv.grid_params(n, n, nu=nu)
        ru, rv = fv.burgers_rhs(u.unsqueeze(0), v.unsqueeze(0), prm)
        errs.append(max((ru[0] - eu).abs().max().item(), (rv[0] - ev).abs().max().item()))
    o1 = math.log2(errs[0] / errs[1])
    o2 = math.log2(errs[1] / errs[2])
    assert 1.7 < o1 < 2.4 and 1.7 < o2 < 2.4, errs


def test_upwind_direction():
    # a > 0: value from the left (i-1, i); a < 0: from the right (i+1, i+2)
    q = torch.arange(8, dtype=torch.float64).view(1, 8) ** 2
    a = torch.ones_like(q)
    f = fv.upwind2_x(q, a)
    assert f[0, 3].item() == pytest.approx(-0.5 * 4 + 1.5 * 9)
    f = fv.upwind2_x(q, -a)
    assert f[0, 3].item() == pytest.approx(1.5 * 16 - 0.5 * 25)


def test_upwind_direction_y():
    # the mirror of the x test: b > 0 takes the value from below (j-1, j),
    # b < 0 from above (j+1, j+2)
    q = (torch.arange(8, dtype=torch.float64) ** 2).view(8, 1)
    b = torch.ones_like(q)
    f = fv.upwind2_y(q, b)
    assert f[3, 0].item() == pytest.approx(-0.5 * 4 + 1.5 * 9)
    f = fv.upwind2_y(q, -b)
    assert f[3, 0].item() == pytest.approx(1.5 * 16 - 0.5 * 25)
    # on a cubic profile the two biases differ: j^3 gives 36.5 from below and
    # 33.5 from above at the face between rows 3 and 4
    c = (torch.arange(8, dtype=torch.float64) ** 3).view(8, 1)
    assert fv.upwind2_y(c, b)[3, 0].item() == pytest.approx(-0.5 * 8 + 1.5 * 27)
    assert fv.upwind2_y(c, -b)[3, 0].item() == pytest.approx(1.5 * 64 - 0.5 * 125)


def _upwind_face(q_m2, q_m1, q_p1, q_p2, a):
    """Linear-upwind value at the face between m1 and p1 (written out)."""
    return (-q_m2 + 3.0 * q_m1) / 2.0 if a > 0 else (3.0 * q_p1 - q_p2) / 2.0


def test_burgers_residual_against_written_out_sums():
    # every cell of a 6 x 5 random field, both components, by explicit
    # index arithmetic: central advecting averages, linear-upwind advected
    # values chosen by the sign of the face velocity, flux form minus q div,
    # compact viscous differences (the collocated Burgers scheme)
    g = torch.Generator().manual_seed(11)
    ny, nx = 5, 6
    u = torch.randn(1, ny, nx, generator=g, dtype=torch.float64)
    v = torch.randn(1, ny, nx, generator=g, dtype=torch.float64)
    nu = 0.03
    prm = fv.grid_params(nx, ny, nu=nu)
    dx, dy = prm["dx"], prm["dy"]
    ru, rv = fv.burgers_rhs(u, v, prm)
    U, V = u[0].tolist(), v[0].tolist()
    for q, got in ((U, ru), (V, rv)):
        for j in range(ny):
            for i in range(nx):
                def Q(jj, ii):
                    return q[jj % ny][ii % nx]

                def A(jj, ii):   # east-face advecting velocity of cell (ii, jj)
                    return 0.5 * (U[jj % ny][ii % nx] + U[jj % ny][(ii + 1) % nx])

                def B(jj, ii):   # north-face advecting velocity
                    return 0.5 * (V[jj % ny][ii % nx] + V[(jj + 1) % ny][ii % nx])
                ae, aw = A(j, i), A(j, i - 1)
                bn, bs = B(j, i), B(j - 1, i)
                qe = _upwind_face(Q(j, i - 1), Q(j, i), Q(j, i + 1), Q(j, i + 2), ae)
                qw = _upwind_face(Q(j, i - 2), Q(j, i - 1), Q(j, i), Q(j, i + 1), aw)
                qn = _upwind_face(Q(j - 1, i), Q(j, i), Q(j + 1, i), Q(j + 2, i), bn)
                qs = _upwind_face(Q(j - 2, i), Q(j - 1, i), Q(j, i), Q(j + 1, i), bs)
                r = -((ae * qe - aw * qw) / dx + (bn * qn - bs * qs) / dy)
                r += Q(j, i) * ((ae - aw) / dx + (bn - bs) / dy)
                r += nu * ((Q(j, i + 1) - 2 * Q(j, i) + Q(j, i - 1)) / dx ** 2
                           + (Q(j + 1, i) - 2 * Q(j, i) + Q(j - 1, i)) / dy ** 2)
                assert got[0, j, i].item() == pytest.approx(r, rel=1e-12, abs=1e-12), (j, i)


def test_burgers_residual_commutes_with_transposition():
    # swapping the axes maps (u, v)(x, y) to (v, u)(y, x); the residual of the
    # swapped field is the swapped residual (a mirrored y bias breaks this)
    g = torch.Generator().manual_seed(12)
    n = 8
    u = torch.randn(2, n, n, generator=g, dtype=torch.float64)
    v = torch.randn(2, n, n, generator=g, dtype=torch.float64)
    prm = fv.grid_params(n, n, nu=0.02)
    ru, rv = fv.burgers_rhs(u, v, prm)
    su, sv = fv.burgers_rhs(v.transpose(-1, -2), u.transpose(-1, -2), prm)
    assert torch.allclose(su, rv.transpose(-1, -2), rtol=1e-13, atol=1e-13)
    assert torch.allclose(sv, ru.transpose(-1, -2), rtol=1e-13, atol=1e-13)
