"""Time integration (oracle, float64).

RK4 (App. B.5, S15-S20; Sec. 3.2: the FV module runs a projection at the end
of every RK4 sub-step):
  k1 = R(u_n),  u1 = P(u_n + dt/2 k1)
  k2 = R(u1),   u2 = P(u_n + dt/2 k2)
  k3 = R(u2),   u3 = P(u_n + dt k3)
  k4 = R(u3),   u_{n+1} = P(u_n + dt/6 (k1 + 2 k2 + 2 k3 + k4))
The forcing is time independent, so the time argument of S17-S19 is unused.

SSP-RK3 (Shu and Osher, 1988) for the collocated Burgers configuration, which
has no pressure and so no projection:
  u1 = u + dt R(u);  u2 = 3/4 u + 1/4 (u1 + dt R(u1));
  u_{n+1} = 1/3 u + 2/3 (u2 + dt R(u2)).
"""
import torch

from . import fv
from .projection import project

RK4 = 0
SSPRK3 = 1
MAC = 0
COLLOCATED = 1


def rhs(u, v, prm, coef=None, flux=None, dcoef=None):
    if prm.get("layout", MAC) == COLLOCATED:
        return fv.burgers_rhs(u, v, prm)
    return fv.ns_rhs(u, v, prm, coef, flux, dcoef)


def _proj(u, v, prm):
    if prm.get("layout", MAC) == COLLOCATED:
        return u, v
    pu, pv, _ = project(u, v, prm)
    return pu, pv


def rk4_step(u, v, prm, coef=None, flux=None, dcoef=None):
    dt = prm["dt"]
    k1 = rhs(u, v, prm, coef, flux, dcoef)
    u1 = _proj(u + 0.5 * dt * k1[0], v + 0.5 * dt * k1[1], prm)
    k2 = rhs(*u1, prm, coef, flux, dcoef)
    u2 = _proj(u + 0.5 * dt * k2[0], v + 0.5 * dt * k2[1], prm)
    k3 = rhs(*u2, prm, coef, flux, dcoef)
    u3 = _proj(u + dt * k3[0], v + dt * k3[1], prm)
    k4 = rhs(*u3, prm, coef, flux, dcoef)
    un = u + dt / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0])
    vn = v + dt / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1])
    return _proj(un, vn, prm)


def ssprk3_step(u, v, prm, coef=None, flux=None, dcoef=None):
    dt = prm["dt"]
    r = rhs(u, v, prm, coef, flux, dcoef)
    u1, v1 = u + dt * r[0], v + dt * r[1]
    u1, v1 = _proj(u1, v1, prm)
    r = rhs(u1, v1, prm, coef, flux, dcoef)
    u2 = 0.75 * u + 0.25 * (u1 + dt * r[0])
    v2 = 0.75 * v + 0.25 * (v1 + dt * r[1])
    u2, v2 = _proj(u2, v2, prm)
    r = rhs(u2, v2, prm, coef, flux, dcoef)
    un = u / 3.0 + 2.0 / 3.0 * (u2 + dt * r[0])
    vn = v / 3.0 + 2.0 / 3.0 * (v2 + dt * r[1])
    return _proj(un, vn, prm)


def fv_step(u, v, prm, coef=None, nsteps=1, flux=None, dcoef=None):
    """The plain (or fixed-coefficient) FV module applied nsteps times; flux
    is an optional flux-block record and dcoef optional per-cell derivative
    weights (see fv), both held fixed over the steps."""
    step = ssprk3_step if prm.get("rk", RK4) == SSPRK3 else rk4_step
    for _ in range(nsteps):
        u, v = step(u, v, prm, coef, flux, dcoef)
    return u, v


def cfl_dt(u, v, prm, cfl):
    """dt = cfl * min(dx, dy) / max over cells of (|u| + |v|) (the Burgers
    configuration's CFL rule, evaluated once on the initial condition)."""
    h = min(prm["dx"], prm["dy"])
    speed = (u.abs() + v.abs()).max().item()
    return cfl * h / speed
