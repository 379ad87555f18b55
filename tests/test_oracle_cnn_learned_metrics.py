"""Pins for the oracle's network, learned step, metrics and gradients."""
import math

import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle import cnn, fv, ic, learned, metrics, projection, timestep

L = 2 * math.pi


def test_conv3x3_circular_brute_force():
    g = np.random.default_rng(0)
    b, ci, co, ny, nx = 2, 3, 4, 5, 4
    x = g.standard_normal((b, ci, ny, nx))
    w = g.standard_normal((co, ci, 3, 3))
    bias = g.standard_normal(co)
    ref = np.zeros((b, co, ny, nx))
    for n in range(b):
        for o in range(co):
            for j in range(ny):
                for i in range(nx):
                    acc = bias[o]
                    for c in range(ci):
                        for dj in (-1, 0, 1):
                            for di in (-1, 0, 1):
                                acc += w[o, c, dj + 1, di + 1] * x[n, c, (j + dj) % ny, (i + di) % nx]
                    ref[n, o, j, i] = acc
    got = cnn.conv3x3_circular(torch.tensor(x), torch.tensor(w), torch.tensor(bias)).numpy()
    assert np.allclose(got, ref, atol=1e-12)


def test_gelu_exact_erf_values():
    xs = [-3.0, -1.0, -0.25, 0.0, 0.5, 2.0, 6.0]
    got = cnn.gelu(torch.tensor(xs, dtype=torch.float64))
    for x, y in zip(xs, got.tolist()):
        assert y == pytest.approx(0.5 * x * (1 + math.erf(x / math.sqrt(2))), rel=1e-15, abs=1e-300)
    # GELU(x) - GELU(-x) = x
    t = torch.linspace(-4, 4, 33, dtype=torch.float64)
    assert torch.allclose(cnn.gelu(t) - cnn.gelu(-t), t, atol=1e-15)


def test_bf16_rounding_known_values():
    vals = torch.tensor([1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -8, -2.0 - 2 ** -7 - 2 ** -9],
                        dtype=torch.float64)
    out = cnn.round_bf16(vals).tolist()
    # bf16 keeps 8 significant bits: ulp(1) = 2^-7; ties go to even
    assert out == [1.0, 1.0 + 2 ** -7, 1.0, -2.0 - 2 ** -6]


def test_network_shape_and_parameter_count():
    assert cnn.param_count() == 187010
    ws, bs = si.cnn_weights(0, cnn.LAYERS)
    x = torch.randn(2, 2, 8, 8, dtype=torch.float64)
    out = cnn.cnn_forward(x, [torch.tensor(w) for w in ws], [torch.tensor(b) for b in bs])
    assert out.shape == (2, 66, 8, 8)


def test_network_translation_equivariance():
    # circular convolutions commute with periodic shifts
    ws, bs = si.cnn_weights(1, cnn.LAYERS, last_scale=1.0)
    ws = [torch.tensor(w) for w in ws]
    bs = [torch.tensor(b) for b in bs]
    x = torch.randn(1, 2, 8, 6, dtype=torch.float64)
    a = cnn.cnn_forward(torch.roll(x, (3, 2), (-2, -1)), ws, bs)
    b = torch.roll(cnn.cnn_forward(x, ws, bs), (3, 2), (-2, -1))
    assert torch.allclose(a, b, atol=1e-12)


def test_constraint_sums_to_one_and_zero_is_physics():
    raw = torch.randn(3, 64, 5, 4, dtype=torch.float64)
    c = learned.constrain(raw)
    s = c.reshape(3, 4, 16, 5, 4).sum(dim=2)
    assert torch.allclose(s, torch.ones_like(s), atol=1e-14)
    c0 = learned.constrain(torch.zeros(1, 64, 2, 2, dtype=torch.float64))
    assert torch.equal(c0[0, :, 0, 0], fv.plain_coefficients())


def _zero_last_layer(seed):
    ws, bs = si.cnn_weights(seed, cnn.LAYERS)
    ws = [torch.tensor(w) for w in ws]
    bs = [torch.tensor(b) for b in bs]
    ws[-1].zero_()
    bs[-1].zero_()
    return ws, bs


def test_learned_step_with_zero_head_is_plain_fv():
    n = 16
    u, v = ic.grf_peak(2, n, n, L, L, seed=1)
    prm = fv.grid_params(n, n, nu=1e-3, dt=0.02, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    ws, bs = _zero_last_layer(0)
    lu, lv, _ = learned.learned_fv_step(u, v, prm, ws, bs, step_index=1)
    pu, pv = timestep.fv_step(u, v, prm)
    assert torch.allclose(lu, pu, atol=1e-14) and torch.allclose(lv, pv, atol=1e-14)


def test_temporal_correction_every_kc_steps():
    # a constant TC of 0.1 in u raises mean(u) by 0.1 exactly at multiples of k_c
    n = 16
    u, v = ic.grf_peak(1, n, n, L, L, seed=2)
    prm = fv.grid_params(n, n, nu=1e-3, dt=0.02, k_c=2)
    ws, bs = _zero_last_layer(0)
    bs[-1][64] = 0.1
    m0 = u.mean().item()
    u1, v1, _ = learned.learned_fv_step(u, v, prm, ws, bs, step_index=1)
    assert u1.mean().item() == pytest.approx(m0, abs=1e-14)
    u2, v2, _ = learned.learned_fv_step(u1, v1, prm, ws, bs, step_index=2)
    assert u2.mean().item() == pytest.approx(m0 + 0.1, abs=1e-13)
    assert projection.divergence(u2, v2, prm).abs().max() < 1e-11


def test_pcc_vorticity_downsample():
    a = torch.randn(4, 8, 8, dtype=torch.float64)
    assert torch.allclose(metrics.pcc(a, a), torch.ones(4, dtype=torch.float64))
    assert torch.allclose(metrics.pcc(a, -a), -torch.ones(4, dtype=torch.float64))
    assert torch.allclose(metrics.pcc(a, 2 * a + 3), torch.ones(4, dtype=torch.float64))
    # vorticity of the TGV at corners: 2 sin(x) sin(y) (2 sin(h/2)/h)
    n = 16
    h = L / n
    u, v = ic.taylor_green(1, n, n, L, L)
    w = metrics.vorticity(u, v, h, h)[0]
    x = (torch.arange(n, dtype=torch.float64) * h).view(1, -1)
    y = (torch.arange(n, dtype=torch.float64) * h).view(-1, 1)
    assert torch.allclose(w, 2 * torch.sin(x) * torch.sin(y) * (2 * math.sin(h / 2) / h), atol=1e-13)
    # face averaging keeps a divergence-free field divergence-free and is exact
    # for fields linear along the face
    uf, vf = ic.grf_peak(1, 32, 32, L, L, seed=3)
    uc, vc = metrics.downsample_mac(uf, vf, 4)
    assert projection.divergence(uc, vc, {"dx": L / 8, "dy": L / 8}).abs().max() < 1e-11
    yu = ((torch.arange(32, dtype=torch.float64) + 0.5) * L / 32).view(-1, 1).expand(32, 32)
    uc, _ = metrics.downsample_mac(yu.unsqueeze(0), yu.unsqueeze(0), 4)
    yc = ((torch.arange(8, dtype=torch.float64) + 0.5) * L / 8).view(-1, 1).expand(8, 8)
    assert torch.allclose(uc[0], yc, atol=1e-14)
    # the coarse divergence is the block mean of the fine divergence
    g = torch.Generator().manual_seed(5)
    uf = torch.randn(1, 16, 16, generator=g, dtype=torch.float64)
    vf = torch.randn(1, 16, 16, generator=g, dtype=torch.float64)
    df = projection.divergence(uf, vf, {"dx": L / 16, "dy": L / 16})
    uc, vc = metrics.downsample_mac(uf, vf, 4)
    dc = projection.divergence(uc, vc, {"dx": L / 4, "dy": L / 4})
    assert torch.allclose(dc, metrics.downsample_collocated(df, 4), atol=1e-12)


def test_hct_and_first_drop():
    p = torch.tensor([0.99, 0.95, 0.91, 0.85, 0.92, 0.7])
    assert metrics.hct(p, 0.5, 0.8) == pytest.approx(2.5)
    assert metrics.first_drop_time(p, 0.5, 0.9) == pytest.approx(1.5)


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step is -lr * g / (|g| + eps)
    from oracle.optim import adam_step
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64)
    g = torch.tensor([0.3, -4.0, 1e-3], dtype=torch.float64)
    w1, m, v = adam_step(w, g, torch.zeros(3, dtype=torch.float64),
                         torch.zeros(3, dtype=torch.float64), 1, lr=0.01)
    assert torch.allclose(w1, w - 0.01 * g / (g.abs() + 1e-8), atol=1e-15)


def test_oracle_autograd_matches_central_differences():
    # the reference VJP of one RK4 step (learned coefficients + forcing), FP64
    n = 8
    g = torch.Generator().manual_seed(7)
    u, v = ic.grf_peak(1, n, n, L, L, seed=6)
    coef = learned.constrain(0.2 * torch.randn(1, 64, n, n, generator=g, dtype=torch.float64))
    prm = fv.grid_params(n, n, nu=0.01, dt=0.05, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    wu = torch.randn(1, n, n, generator=g, dtype=torch.float64)
    wv = torch.randn(1, n, n, generator=g, dtype=torch.float64)

    def loss(a, b, c):
        x, y = timestep.fv_step(a, b, prm, coef=c, nsteps=2)
        return (wu * x).sum() + (wv * y).sum()

    ua = u.clone().requires_grad_(True)
    va = v.clone().requires_grad_(True)
    ca = coef.clone().requires_grad_(True)
    loss(ua, va, ca).backward()
    for _ in range(3):
        du = torch.randn(1, n, n, generator=g, dtype=torch.float64)
        dv = torch.randn(1, n, n, generator=g, dtype=torch.float64)
        dc = torch.randn(1, 64, n, n, generator=g, dtype=torch.float64)
        h = 1e-6
        fd = (loss(u + h * du, v + h * dv, coef + h * dc)
              - loss(u - h * du, v - h * dv, coef - h * dc)) / (2 * h)
        ad = (ua.grad * du).sum() + (va.grad * dv).sum() + (ca.grad * dc).sum()
        assert abs(fd.item() - ad.item()) <= 1e-7 * abs(ad.item()) + 1e-9


def test_cfl_dt_against_the_rule():
    # dt = cfl * min(dx, dy) / max over cells and trajectories of |u| + |v|:
    # u = A cos(2 pi i / 16) peaks at i = 0, v = B sin(2 pi j / 8) at j = 2,
    # so the max is A + B on the second trajectory (scaled by 3)
    nx, ny = 16, 8
    prm = fv.grid_params(nx, ny, lx=2.0, ly=L)
    i = torch.arange(nx, dtype=torch.float64).view(1, -1)
    j = torch.arange(ny, dtype=torch.float64).view(-1, 1)
    a, b = 0.7, 0.4
    u = (a * torch.cos(2 * math.pi * i / nx)).expand(ny, nx)
    v = (b * torch.sin(2 * math.pi * j / ny)).expand(ny, nx)
    u = torch.stack([u, 3 * u])
    v = torch.stack([v, 3 * v])
    dt = timestep.cfl_dt(u, v, prm, 0.5)
    assert dt == pytest.approx(0.5 * min(2.0 / nx, L / ny) / (3 * (a + b)), rel=1e-14)
    # a single sign flip anywhere does not change |u| + |v|
    assert timestep.cfl_dt(-u, v, prm, 0.5) == pytest.approx(dt, rel=1e-15)


def test_mse_rmse_mae_against_written_out_sums():
    g = torch.Generator().manual_seed(21)
    pu, pv, lu, lv = (torch.randn(2, 3, 4, generator=g, dtype=torch.float64) for _ in range(4))
    n = pu.numel()
    su = sum((pu.flatten()[k].item() - lu.flatten()[k].item()) ** 2 for k in range(n))
    sv = sum((pv.flatten()[k].item() - lv.flatten()[k].item()) ** 2 for k in range(n))
    from oracle.optim import mse_loss
    assert mse_loss(pu, pv, lu, lv).item() == pytest.approx(0.5 * (su / n + sv / n), rel=1e-14)
    # its gradient is (pred - label) / n per component, the cotangent the
    # rollout backward feeds the adjoint
    a = pu.clone().requires_grad_(True)
    mse_loss(a, pv, lu, lv).backward()
    assert torch.allclose(a.grad, (pu - lu) / n, rtol=1e-14, atol=0)
    # RMSE and MAE (S32, S33): written-out sums, a constant error, and the
    # textbook inequality MAE <= RMSE
    d = [pu.flatten()[k].item() - lu.flatten()[k].item() for k in range(n)]
    assert metrics.rmse(pu, lu).item() == pytest.approx(math.sqrt(sum(x * x for x in d) / n),
                                                        rel=1e-14)
    assert metrics.mae(pu, lu).item() == pytest.approx(sum(abs(x) for x in d) / n, rel=1e-14)
    assert metrics.mae(pu, lu).item() <= metrics.rmse(pu, lu).item()
    c = torch.full_like(pu, -0.25)
    assert metrics.rmse(lu + c, lu).item() == pytest.approx(0.25, rel=1e-14)
    assert metrics.mae(lu + c, lu).item() == pytest.approx(0.25, rel=1e-14)
    e = torch.tensor([3.0, -4.0], dtype=torch.float64)
    z = torch.zeros(2, dtype=torch.float64)
    assert metrics.rmse(e, z).item() == pytest.approx(math.sqrt(12.5), rel=1e-15)
    assert metrics.mae(e, z).item() == pytest.approx(3.5, rel=1e-15)


def test_energy_and_enstrophy_of_the_taylor_green_vortex():
    # u = sin x cos y, v = -cos x sin y sampled on the MAC faces: the cell
    # means of sin^2 cos^2 are exactly 1/4 on any grid of 4+ cells, so the
    # energy is 1/4; the corner vorticity is 2 sin x sin y s with
    # s = 2 sin(h/2)/h, so the enstrophy is s^2 / 2
    for n in (8, 16):
        h = L / n
        u, v = ic.taylor_green(2, n, n, L, L)
        assert torch.allclose(metrics.energy(u, v), torch.full((2,), 0.25, dtype=torch.float64),
                              atol=1e-15)
        s = 2 * math.sin(h / 2) / h
        assert torch.allclose(metrics.enstrophy(u, v, h, h),
                              torch.full((2,), s * s / 2, dtype=torch.float64), atol=1e-14)
    # energy by Parseval on a random field
    g = torch.Generator().manual_seed(22)
    a = torch.randn(1, 8, 8, generator=g, dtype=torch.float64)
    b = torch.randn(1, 8, 8, generator=g, dtype=torch.float64)
    fa, fb = torch.fft.fft2(a), torch.fft.fft2(b)
    par = 0.5 * ((fa.abs() ** 2).sum() + (fb.abs() ** 2).sum()) / 64 ** 2
    assert metrics.energy(a, b).item() == pytest.approx(par.item(), rel=1e-13)


def test_adam_bias_correction_over_several_steps():
    # five steps with a constant gradient: m_t = g (1 - b1^t), v_t = g^2 (1 - b2^t),
    # so every bias-corrected step is -lr g / (|g| + eps), written out
    from oracle.optim import adam_step
    g = torch.tensor([0.5, -2.0, 1e-4], dtype=torch.float64)
    w = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64)
    m = torch.zeros(3, dtype=torch.float64)
    v = torch.zeros(3, dtype=torch.float64)
    lr, b1, b2 = 1e-3, 0.9, 0.999
    for t in range(1, 6):
        w, m, v = adam_step(w, g, m, v, t, lr=lr, b1=b1, b2=b2)
        assert torch.allclose(m, g * (1 - b1 ** t), rtol=1e-14, atol=0)
        assert torch.allclose(v, g * g * (1 - b2 ** t), rtol=1e-13, atol=0)
    assert torch.allclose(w, 1.0 - 5 * lr * g / (g.abs() + 1e-8), rtol=1e-12, atol=0)
