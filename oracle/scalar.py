"""Passive scalar of the shear-flow system (oracle, float64): the NS velocity
on the MAC grid carries a scalar s (concentration or temperature) with
ds/dt - D lap s = -u . grad s (the shear-flow equations of the appendix on
the datasets).

TEST INFRASTRUCTURE ONLY (see the package header).

s lives at cell centres.  Finite-volume form over the cell (i, j), with the
MAC velocity already on its faces (u[j, i+1] on the east face, v[j+1, i] on
the north face):
  R_s = -[(u_e s~_e - u_w s~_w)/dx + (v_n s~_n - v_s s~_s)/dy]
        + D [((ds/dx)_e - (ds/dx)_w)/dx + ((ds/dy)_n - (ds/dy)_s)/dy]
with the physics kernels of the flux block (App. B.2, S6-S7 as read for the
velocity): s~ the midpoint average of the two cells a face separates and
ds/dn the fourth-order face derivative [1, -27, 27, -1]/(24 h).  For a
discretely divergence-free u the flux form equals -u . grad s up to the
discretisation, and the total amount of s is conserved exactly (the fluxes
telescope).

Time integration: the scalar rides the velocity's RK4 stages (App. B.5):
its stage residual uses the projected velocity stage state of the same
stage; the scalar itself is not projected.
"""
import torch

from . import fv
from .projection import project


def scalar_rhs(u, v, s, prm):
    dx, dy = prm["dx"], prm["dy"]
    D = prm.get("diffusivity", 0.0)
    mask = prm.get("mask", fv.ALL_PHYSICS)
    r = torch.zeros_like(s)
    if mask & fv.ADVECTION:
        fe = fv.sx(u, 1) * 0.5 * (s + fv.sx(s, 1))      # east face of cell i
        gn = fv.sy(v, 1) * 0.5 * (s + fv.sy(s, 1))      # north face of cell j
        r = r - (fe - fv.sx(fe, -1)) / dx - (gn - fv.sy(gn, -1)) / dy
    if mask & fv.VISCOSITY:
        sxd = fv.deriv4_x(s, dx)
        syd = fv.deriv4_y(s, dy)
        r = r + D * ((sxd - fv.sx(sxd, -1)) / dx + (syd - fv.sy(syd, -1)) / dy)
    return r


def rk4_step_scalar(u, v, s, prm):
    """One RK4 step of the velocity (projection per sub-step) and the scalar."""
    dt = prm["dt"]

    def proj(a, b):
        pu, pv, _ = project(a, b, prm)
        return pu, pv

    k1 = fv.ns_rhs(u, v, prm)
    q1 = scalar_rhs(u, v, s, prm)
    u1 = proj(u + 0.5 * dt * k1[0], v + 0.5 * dt * k1[1])
    s1 = s + 0.5 * dt * q1
    k2 = fv.ns_rhs(*u1, prm)
    q2 = scalar_rhs(*u1, s1, prm)
    u2 = proj(u + 0.5 * dt * k2[0], v + 0.5 * dt * k2[1])
    s2 = s + 0.5 * dt * q2
    k3 = fv.ns_rhs(*u2, prm)
    q3 = scalar_rhs(*u2, s2, prm)
    u3 = proj(u + dt * k3[0], v + dt * k3[1])
    s3 = s + dt * q3
    k4 = fv.ns_rhs(*u3, prm)
    q4 = scalar_rhs(*u3, s3, prm)
    un = u + dt / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0])
    vn = v + dt / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1])
    sn = s + dt / 6.0 * (q1 + 2.0 * q2 + 2.0 * q3 + q4)
    un, vn = proj(un, vn)
    return un, vn, sn


def fv_step_scalar(u, v, s, prm, nsteps=1):
    for _ in range(nsteps):
        u, v, s = rk4_step_scalar(u, v, s, prm)
    return u, v, s
