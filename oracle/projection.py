"""Pressure projection on the periodic MAC grid (oracle, float64).

Projection method (App. B.3, S8-S10): an intermediate velocity u* is made
divergence-free by solving a Poisson equation for the pressure and
subtracting its gradient.  Poisson solver (App. B.4, S11-S14): FFT, divide
by minus the squared wavenumber, zero mode left at zero, inverse FFT.

Discrete operators (App. B.1: mass conservation on the staggered cell):
  D(u, v)[j, i] = (u[j, i+1] - u[j, i]) / dx + (v[j+1, i] - v[j, i]) / dy
  G(p)          = ((p[j, i] - p[j, i-1]) / dx, (p[j, i] - p[j-1, i]) / dy)
so that G = -D^T.  The spectral division uses the eigenvalues of D G,
-lambda_h(k) = -[(2/dx)^2 sin^2(pi kx/Nx) + (2/dy)^2 sin^2(pi ky/Ny)]
(the modified wavenumbers of the compact pair; our reading of S12-S14, which
print the continuous wavenumbers: only this choice makes D u = 0 exactly
after the correction, which the paper states the step guarantees).  The
zero mode of p is zero (S12 excludes eta = 0; App. C.1 fixes the mean of p).

The time-step factor of S9/S10 cancels: u = u* - G p with D G p = D u*; the
returned p is that potential (the paper's pressure times dt).
"""
import math
import torch

from .fv import sx, sy


def divergence(u, v, prm):
    return (sx(u, 1) - u) / prm["dx"] + (sy(v, 1) - v) / prm["dy"]


def gradient(p, prm):
    return (p - sx(p, -1)) / prm["dx"], (p - sy(p, -1)) / prm["dy"]


def laplacian_eigenvalues(ny, nx, dx, dy, dtype=torch.float64):
    """lambda_h[ky, kx] >= 0 with D G e_k = -lambda_h e_k."""
    kx = torch.arange(nx, dtype=dtype)
    ky = torch.arange(ny, dtype=dtype)
    lx = (2.0 / dx) ** 2 * torch.sin(math.pi * kx / nx) ** 2
    ly = (2.0 / dy) ** 2 * torch.sin(math.pi * ky / ny) ** 2
    return ly.view(-1, 1) + lx.view(1, -1)


def poisson_solve(d, prm):
    """Solve D G p = d on the periodic grid by FFT (S11-S14), p-hat(0,0) = 0."""
    ny, nx = d.shape[-2], d.shape[-1]
    lam = laplacian_eigenvalues(ny, nx, prm["dx"], prm["dy"], d.dtype)
    inv = torch.zeros_like(lam)
    nz = lam > 0
    inv[nz] = -1.0 / lam[nz]
    dh = torch.fft.fft2(d)
    ph = dh * inv
    return torch.fft.ifft2(ph).real


def project(u, v, prm):
    """u <- u* - G p with D G p = D u*.  Returns (u, v, p)."""
    d = divergence(u, v, prm)
    p = poisson_solve(d, prm)
    gx, gy = gradient(p, prm)
    return u - gx, v - gy, p
