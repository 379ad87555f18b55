"""Pins for the oracle's random numbers and initial conditions."""
import math
import os

import numpy as np
import pytest
import torch

from oracle import ic, projection
from oracle.rng import NormalStream, SplitMix64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        seed, vals = line.split(":")
        out[int(seed)] = [int(x) for x in vals.split()]
    return out


def test_splitmix64_published_outputs():
    for seed, vals in _golden().items():
        g = SplitMix64(seed)
        assert [g.next_u64() for _ in vals] == vals


def test_uniform_range_and_box_muller_moments():
    g = SplitMix64(7)
    u = np.array([g.uniform() for _ in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    s = NormalStream(3)
    z = np.array([s.normal() for _ in range(40000)])
    assert abs(z.mean()) < 0.02
    assert abs(z.var() - 1.0) < 0.03
    # fourth moment of a standard normal is 3
    assert abs((z ** 4).mean() - 3.0) < 0.15


def test_box_muller_pair_closed_form():
    # the first pair equals the transform of the first two uniforms
    s = NormalStream(11)
    g = SplitMix64(11)
    u1 = 1.0 - g.uniform()
    u2 = g.uniform()
    r = math.sqrt(-2 * math.log(u1))
    assert s.normal() == pytest.approx(r * math.cos(2 * math.pi * u2), abs=0, rel=1e-15)
    assert s.normal() == pytest.approx(r * math.sin(2 * math.pi * u2), abs=0, rel=1e-15)


def test_half_plane_mode_count():
    # 24 modes with 0 < |k| <= 4 in a half plane; no mode and its negative both
    modes = ic.half_plane_modes(4)
    assert len(modes) == 24
    s = set(modes)
    assert all((-a, -b) not in s for a, b in modes)
    assert (0, 0) not in s


def test_fourier_modes_ic_scaled_to_unit_max():
    L = 2 * math.pi
    u, v = ic.fourier_modes(2, 32, 32, L, L, seed=0)
    for b in range(2):
        m = max(u[b].abs().max().item(), v[b].abs().max().item())
        assert m == pytest.approx(1.0, rel=1e-14)
    # band limit: no energy above |k| = 4
    spec = torch.fft.fft2(u[0]).abs()
    k = torch.fft.fftfreq(32, 1.0 / 32)
    kk = torch.sqrt(k.view(-1, 1) ** 2 + k.view(1, -1) ** 2)
    assert spec[kk > 4.01].max() < 1e-10
    assert spec[0, 0] < 1e-10
    # trajectories differ
    assert (u[0] - u[1]).abs().max() > 0.1


def test_grf_divergence_free_unit_energy_peak():
    L = 2 * math.pi
    n = 64
    u, v = ic.grf_peak(3, n, n, L, L, seed=5)
    prm = {"dx": L / n, "dy": L / n}
    d = projection.divergence(u, v, prm)
    assert d.abs().max() < 1e-11
    e = 0.5 * ((u * u).mean(dim=(-2, -1)) + (v * v).mean(dim=(-2, -1)))
    assert torch.allclose(e, torch.ones(3, dtype=torch.float64), rtol=1e-13)
    # shell energy spectrum averaged over many seeds peaks at k = 4
    u, v = ic.grf_peak(24, n, n, L, L, seed=9)
    eu = torch.fft.fft2(u).abs() ** 2 + torch.fft.fft2(v).abs() ** 2
    eu = eu.mean(0)
    k = torch.fft.fftfreq(n, 1.0 / n)
    kk = torch.sqrt(k.view(-1, 1) ** 2 + k.view(1, -1) ** 2).round().long()
    shell = torch.zeros(n)
    shell.index_add_(0, kk.flatten(), eu.flatten().float())
    assert int(shell[1:20].argmax()) + 1 in (3, 4, 5)


def test_taylor_green_closed_form_and_divergence():
    L = 2 * math.pi
    n = 16
    u, v = ic.taylor_green(1, n, n, L, L)
    dx = L / n
    # u at (i dx, (j+1/2) dx)
    assert u[0, 3, 5].item() == pytest.approx(math.sin(5 * dx) * math.cos(3.5 * dx), rel=1e-14)
    assert v[0, 3, 5].item() == pytest.approx(-math.cos(5.5 * dx) * math.sin(3 * dx), rel=1e-14)
    d = projection.divergence(u, v, {"dx": dx, "dy": dx})
    assert d.abs().max() < 1e-13


def test_shear_layer_profile_and_noise():
    L = 2 * math.pi
    n = 64
    u, v = ic.shear_layer(2, n, n, L, L, seed=1, noise_rms=0.0)
    dy = L / n
    y = 10.5 * dy
    assert u[0, 10, 3].item() == pytest.approx(math.tanh((y - math.pi / 2) * 30), rel=1e-13)
    y = 50.5 * dy
    assert u[0, 50, 3].item() == pytest.approx(-math.tanh((y - 3 * math.pi / 2) * 30), rel=1e-13)
    x = 7.5 * dy
    assert v[0, 4, 7].item() == pytest.approx(0.05 * math.sin(2 * x), rel=1e-13)
    u, v = ic.shear_layer(2, n, n, L, L, seed=1, noise_rms=1e-3)
    d = projection.divergence(u, v, {"dx": dy, "dy": dy})
    assert d.abs().max() < 1e-10
    assert (u[0] - u[1]).abs().max() > 1e-5
