"""Seeded initial conditions (oracle, float64).

The paper draws random initial conditions from seeded Gaussian random fields
(App. C.1) and, for shear flow, tanh shear layers with a sinusoidal vertical
perturbation and random noise (S30-S31).  The exact spectra are not given;
the forms below are the ones this project fixes (see each function).  All
random numbers come from ``rng.NormalStream(seed, b)`` for trajectory b.

Modes are enumerated in one fixed order over the half plane:
for kx = 0..K, for ky = -K..K, keep (kx, ky) if kx > 0 or ky > 0, and
kx^2 + ky^2 <= K^2.  Physical wavevector: (2 pi kx / Lx, 2 pi ky / Ly).
"""
import math
import torch

from .rng import NormalStream

FOURIER_MODES = 0
GRF_PEAK = 1
TGV = 2
SHEAR_LAYER = 3


def half_plane_modes(kmax):
    modes = []
    for kx in range(0, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            if (kx > 0 or ky > 0) and kx * kx + ky * ky <= kmax * kmax:
                modes.append((kx, ky))
    return modes


def _wave(kx, ky, x, y, lx, ly):
    return 2.0 * math.pi * kx / lx * x + 2.0 * math.pi * ky / ly * y


def fourier_modes(batch, nx, ny, lx, ly, seed, kmax=4):
    """Collocated (u, v): for each component, sum over half-plane modes with
    0 < |k| <= 4 of (alpha cos(k.x) + beta sin(k.x)), alpha, beta ~ N(0, 1)
    (drawn alpha then beta, mode by mode, all of u before all of v), then one
    scale factor per trajectory so that max over cells of max(|u|, |v|) = 1."""
    x = ((torch.arange(nx, dtype=torch.float64) + 0.5) * lx / nx).view(1, -1)
    y = ((torch.arange(ny, dtype=torch.float64) + 0.5) * ly / ny).view(-1, 1)
    modes = half_plane_modes(kmax)
    us, vs = [], []
    for b in range(batch):
        g = NormalStream(seed, b)
        comps = []
        for _ in range(2):
            q = torch.zeros(ny, nx, dtype=torch.float64)
            for kx, ky in modes:
                al = g.normal()
                be = g.normal()
                ph = _wave(kx, ky, x, y, lx, ly)
                q = q + al * torch.cos(ph) + be * torch.sin(ph)
            comps.append(q)
        s = 1.0 / max(comps[0].abs().max().item(), comps[1].abs().max().item())
        us.append(comps[0] * s)
        vs.append(comps[1] * s)
    return torch.stack(us), torch.stack(vs)


def _streamfunction_corners(nx, ny, lx, ly, modes, amps, g):
    """psi at corners (i dx, j dy) = sum_k A_k (g1 cos(k.x) + g2 sin(k.x))."""
    x = (torch.arange(nx, dtype=torch.float64) * lx / nx).view(1, -1)
    y = (torch.arange(ny, dtype=torch.float64) * ly / ny).view(-1, 1)
    psi = torch.zeros(ny, nx, dtype=torch.float64)
    for (kx, ky), a in zip(modes, amps):
        g1 = g.normal()
        g2 = g.normal()
        ph = _wave(kx, ky, x, y, lx, ly)
        psi = psi + a * (g1 * torch.cos(ph) + g2 * torch.sin(ph))
    return psi


def _velocity_from_psi(psi, dx, dy):
    """u = d psi/dy at u-points, v = -d psi/dx at v-points; exactly
    divergence-free for the compact MAC divergence."""
    u = (torch.roll(psi, -1, dims=-2) - psi) / dy
    v = -(torch.roll(psi, -1, dims=-1) - psi) / dx
    return u, v


def grf_kmax(nx, ny):
    return max(1, min(16, min(nx, ny) // 2 - 1))


def grf_peak(batch, nx, ny, lx, ly, seed, kpeak=4.0):
    """MAC (u, v) from a Gaussian random streamfunction whose shell energy
    spectrum is E(k) ~ k^4 exp(-2 (k/kpeak)^2) (maximum at kpeak): mode
    amplitude A(k) = sqrt(E(k) / k^3) for integer modes 0 < |k| <= K with
    K = min(16, N/2 - 1).  Scaled to unit energy, 1/2 <u^2 + v^2> = 1, per
    trajectory (the decaying-flow configuration)."""
    dx, dy = lx / nx, ly / ny
    kmax = grf_kmax(nx, ny)
    modes = half_plane_modes(kmax)
    amps = []
    for kx, ky in modes:
        k = math.sqrt(kx * kx + ky * ky)
        amps.append(math.sqrt(k ** 4 * math.exp(-2.0 * (k / kpeak) ** 2) / k ** 3))
    us, vs = [], []
    for b in range(batch):
        g = NormalStream(seed, b)
        psi = _streamfunction_corners(nx, ny, lx, ly, modes, amps, g)
        u, v = _velocity_from_psi(psi, dx, dy)
        e = 0.5 * ((u * u).mean() + (v * v).mean())
        s = 1.0 / math.sqrt(e.item())
        us.append(u * s)
        vs.append(v * s)
    return torch.stack(us), torch.stack(vs)


def taylor_green(batch, nx, ny, lx, ly, amp=1.0, k=1):
    """u = A sin(k x) cos(k y), v = -A cos(k x) sin(k y) sampled at the MAC
    points (k in units of 2 pi / L).  On a square grid it is discretely
    divergence-free."""
    kx = 2.0 * math.pi * k / lx
    ky = 2.0 * math.pi * k / ly
    xu = (torch.arange(nx, dtype=torch.float64) * lx / nx).view(1, -1)
    yu = ((torch.arange(ny, dtype=torch.float64) + 0.5) * ly / ny).view(-1, 1)
    xv = ((torch.arange(nx, dtype=torch.float64) + 0.5) * lx / nx).view(1, -1)
    yv = (torch.arange(ny, dtype=torch.float64) * ly / ny).view(-1, 1)
    u = amp * torch.sin(kx * xu) * torch.cos(ky * yu)
    v = -amp * torch.cos(kx * xv) * torch.sin(ky * yv)
    return u.expand(batch, ny, nx).clone(), v.expand(batch, ny, nx).clone()


def shear_layer(batch, nx, ny, lx, ly, seed, delta=1.0 / 30.0, pert=0.05, noise_rms=1e-3,
                noise_kmax=8):
    """Doubly periodic shear layers: u = tanh((y - L/4)/delta) for y <= L/2 and
    -tanh((y - 3L/4)/delta) above, at u-points; v = pert sin(2 * 2 pi x / L) at
    v-points; plus a divergence-free noise field from a random streamfunction
    over modes 0 < |k| <= noise_kmax with unit N(0,1) amplitudes, scaled so
    that sqrt(1/2 <u_n^2 + v_n^2>) = noise_rms (the per-trajectory noise of
    S30-S31).  Every part is discretely divergence-free."""
    dx, dy = lx / nx, ly / ny
    yu = (torch.arange(ny, dtype=torch.float64) + 0.5) * dy
    prof = torch.where(yu <= 0.5 * ly, torch.tanh((yu - 0.25 * ly) / delta),
                       -torch.tanh((yu - 0.75 * ly) / delta))
    xv = (torch.arange(nx, dtype=torch.float64) + 0.5) * dx
    vper = pert * torch.sin(2.0 * 2.0 * math.pi * xv / lx)
    modes = half_plane_modes(noise_kmax)
    us, vs = [], []
    for b in range(batch):
        g = NormalStream(seed, b)
        psi = _streamfunction_corners(nx, ny, lx, ly, modes, [1.0] * len(modes), g)
        un, vn = _velocity_from_psi(psi, dx, dy)
        rms = math.sqrt(0.5 * ((un * un).mean() + (vn * vn).mean()).item())
        s = noise_rms / rms
        us.append(prof.view(-1, 1).expand(ny, nx) + s * un)
        vs.append(vper.view(1, -1).expand(ny, nx) + s * vn)
    return torch.stack(us), torch.stack(vs)


def shear_scalar(batch, nx, ny, lx, ly, delta=1.0 / 30.0):
    """The passive scalar aligned with the shear layers (our reading of the
    shear-flow IC): s = (1 + prof(y)) / 2 at cell centres, with prof the
    velocity's tanh profile (layers at L_y/4 and 3 L_y/4), so s runs from 0
    to 1 across each layer."""
    dy = ly / ny
    yc = (torch.arange(ny, dtype=torch.float64) + 0.5) * dy
    prof = torch.where(yc <= 0.5 * ly, torch.tanh((yc - 0.25 * ly) / delta),
                       -torch.tanh((yc - 0.75 * ly) / delta))
    return (0.5 * (1.0 + prof)).view(1, -1, 1).expand(batch, ny, nx).contiguous()


def init_state(kind, batch, nx, ny, lx, ly, seed, **kw):
    if kind == FOURIER_MODES:
        return fourier_modes(batch, nx, ny, lx, ly, seed)
    if kind == GRF_PEAK:
        return grf_peak(batch, nx, ny, lx, ly, seed, kw.get("kpeak", 4.0))
    if kind == TGV:
        return taylor_green(batch, nx, ny, lx, ly, kw.get("amp", 1.0), int(kw.get("k", 1)))
    if kind == SHEAR_LAYER:
        return shear_layer(batch, nx, ny, lx, ly, seed, kw.get("delta", 1.0 / 30.0),
                           kw.get("pert", 0.05), kw.get("noise_rms", 1e-3))
    raise ValueError(kind)
