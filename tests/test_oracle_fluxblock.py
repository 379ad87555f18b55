"""Pins for the oracle's flux block (Sec. 3.4, Eqs. 5-8): the spectral
convolution against its written-out transform sums, the FNO's special cases
and symmetry, the uniform kernels against their Fourier symbols, and the
face-field terms against closed forms."""
import cmath
import math

import numpy as np
import pytest
import torch

import synthetic_inputs as si
from oracle import cnn, fluxblock, fno, fv, ic, timestep

L = 2 * math.pi


def _brute_spectral_conv(v, R):
    """The spectral convolution of the fno module header, summed term by term."""
    b, c, ny, nx = v.shape
    two_my, mx, _, co = R.shape
    my = two_my // 2
    rows = list(range(my)) + list(range(ny - my, ny))
    out = np.zeros((b, co, ny, nx))
    for n in range(b):
        V = {}
        for r, ky in enumerate(rows):
            for kx in range(mx):
                for i in range(c):
                    acc = 0j
                    for y in range(ny):
                        for x in range(nx):
                            acc += v[n, i, y, x] * cmath.exp(-2j * math.pi * (ky * y / ny + kx * x / nx))
                    V[(r, kx, i)] = acc
        for o in range(co):
            for y in range(ny):
                for x in range(nx):
                    acc = 0.0
                    for r, ky in enumerate(rows):
                        for kx in range(mx):
                            Y = sum(R[r, kx, i, o] * V[(r, kx, i)] for i in range(c))
                            w = 1.0 if kx == 0 or 2 * kx == nx else 2.0
                            acc += w * (Y * cmath.exp(2j * math.pi * (ky * y / ny + kx * x / nx))).real
                    out[n, o, y, x] = acc / (nx * ny)
    return out


@pytest.mark.parametrize("ny,nx,my,mx", [(8, 8, 2, 3), (6, 8, 3, 5), (8, 4, 1, 3)])
def test_spectral_conv_written_out_sums(ny, nx, my, mx):
    """Includes the full row band (2 my = ny) and the Nyquist column (mx = nx/2 + 1)."""
    g = np.random.default_rng(ny * 100 + nx)
    b, c, co = 1, 2, 3
    v = g.standard_normal((b, c, ny, nx))
    R = g.standard_normal((2 * my, mx, c, co)) + 1j * g.standard_normal((2 * my, mx, c, co))
    got = fno.spectral_conv(torch.tensor(v), torch.tensor(R)).numpy()
    ref = _brute_spectral_conv(v, R)
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_spectral_conv_identity_keeps_all_but_nyquist_column():
    """R = I on the band 2 My = Ny, Mx = Nx / 2 keeps every mode but the
    Nyquist column: out = v - (1/Nx) (sum_n v[y, n] (-1)^n) (-1)^x."""
    ny, nx, c = 8, 8, 2
    g = np.random.default_rng(3)
    v = g.standard_normal((2, c, ny, nx))
    R = np.zeros((ny, nx // 2, c, c), dtype=np.complex128)
    for i in range(c):
        R[:, :, i, i] = 1.0
    got = fno.spectral_conv(torch.tensor(v), torch.tensor(R)).numpy()
    sign = (-1.0) ** np.arange(nx)
    nyq = (v * sign).sum(axis=-1, keepdims=True) / nx * sign
    assert np.abs(got - (v - nyq)).max() < 1e-13


def _net(seed, width=4, layers=3, modes=2, n_out=4, out_scale=1.0):
    return fno.from_arrays(si.fno_weights(seed, width, layers, modes, n_out=n_out,
                                          out_scale=out_scale))


def test_fno_without_spectral_weights_is_a_pointwise_network():
    """R = 0: each pixel goes through lift, GELU layers and projection alone."""
    p = _net(5)
    for lay in p["layers"]:
        lay["R"] = torch.zeros_like(lay["R"])
    x = torch.tensor(si.random_field(6, (2, 2, 8, 8)))
    got = fno.fno_forward(x, p)
    P_w, P_b, Q_w, Q_b = (p[k].numpy() for k in ("P_w", "P_b", "Q_w", "Q_b"))
    xn = x.numpy()
    nl = len(p["layers"])
    for n in range(2):
        for y in range(8):
            for xx in range(8):
                h = [sum(P_w[o, i] * xn[n, i, y, xx] for i in range(2)) + P_b[o] for o in range(4)]
                for li, lay in enumerate(p["layers"]):
                    W, bb = lay["W"].numpy(), lay["b"].numpy()
                    z = [sum(W[o, i] * h[i] for i in range(4)) + bb[o] for o in range(4)]
                    h = [0.5 * t * (1 + math.erf(t / math.sqrt(2))) for t in z] if li < nl - 1 else z
                out = [sum(Q_w[k, o] * h[o] for o in range(4)) + Q_b[k] for k in range(4)]
                for k in range(4):
                    assert got[n, k, y, xx].item() == pytest.approx(out[k], abs=1e-13)


def test_fno_commutes_with_periodic_shifts():
    p = _net(7)
    x = torch.tensor(si.random_field(8, (1, 2, 8, 8)))
    a = fno.fno_forward(torch.roll(x, shifts=(3, 5), dims=(-2, -1)), p)
    b = torch.roll(fno.fno_forward(x, p), shifts=(3, 5), dims=(-2, -1))
    assert torch.allclose(a, b, atol=1e-13)


def test_fno_parameter_count_of_the_paper_networks():
    # forced flow: 6 layers, 32 modes, width 16; decaying: 4 layers, 16 modes, width 8
    assert fno.param_count(16, 6, 32) == 6 * (2 * 2 * 32 * 32 * 256 + 256 + 16) + 32 + 16 + 64 + 4
    a = si.fno_weights(0, 8, 4, 16)
    n = sum(np.asarray(z).size for k, z in a.items() if k != "layers")
    n += sum(np.asarray(z).size for l in a["layers"] for z in l.values())
    assert n == fno.param_count(8, 4, 16)


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_uniform_kernel_fourier_symbol(kind):
    """On q = Re(exp(i (tx i + ty j))) a uniform kernel returns
    Re(sigma exp(i (tx i + ty j))), sigma = sum_s w_s exp(i (t_n a_s + t_t b_s)),
    with t_n the phase step along the face normal (x for kinds 0, 2) and t_t
    across it."""
    n = 16
    w = torch.tensor(si.stencil_weights(11 + kind, scale=1.0)[kind])
    mx, my = 3, 5
    tx, ty = 2 * math.pi * mx / n, 2 * math.pi * my / n
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    q = torch.tensor(np.cos(tx * i + ty * j))
    along_x = kind in (0, 2)
    got = (fv.uniform_x(q, w) if along_x else fv.uniform_y(q, w)).numpy()
    tn, tt = (tx, ty) if along_x else (ty, tx)
    pts = [(s % 4 - 1, s // 4 - 1) for s in range(12)] + [(0, -2), (1, -2), (0, 2), (1, 2),
                                                          (-1, -2), (2, -2), (-1, 2), (2, 2)]
    sigma = sum(w[s].item() * cmath.exp(1j * (tn * a + tt * b)) for s, (a, b) in enumerate(pts))
    ref = (sigma * np.exp(1j * (tx * i + ty * j))).real
    assert np.abs(got - ref).max() < 1e-12


def _state(n=16, b=2, seed=3):
    u, v = ic.grf_peak(b, n, n, L, L, seed=seed)
    return u, v, fv.grid_params(n, n, nu=0.01, forcing_amp=1.0, forcing_k=4.0, drag=0.1)


def _record(n, b, seed, scale=0.05):
    g = np.random.default_rng(seed)
    return {"wi": torch.tensor(si.stencil_weights(seed, scale)),
            "wd": torch.tensor(si.stencil_weights(seed + 1, scale)),
            "fi": torch.tensor(g.standard_normal((b, 4, n, n)) * scale),
            "fd": torch.tensor(g.standard_normal((b, 4, n, n)) * scale)}


def test_empty_flux_block_is_the_physics_scheme():
    """O_L = O_F = 0 leaves the physics operator O_P (the plain FV residual)."""
    u, v, prm = _state()
    zero = {"wi": torch.zeros(4, 20, dtype=torch.float64),
            "wd": torch.zeros(4, 20, dtype=torch.float64),
            "fi": torch.zeros(2, 4, 16, 16, dtype=torch.float64),
            "fd": torch.zeros(2, 4, 16, 16, dtype=torch.float64)}
    a = fv.ns_rhs(u, v, prm, flux=zero)
    b = fv.ns_rhs(u, v, prm)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_flux_block_residual_is_conservative():
    """Each face value is single-valued whatever the flux block adds, so the
    advective and viscous fluxes telescope: sum over cells of R = 0 for the
    unforced equations."""
    u, v, prm = _state()
    prm = dict(prm, mask=fv.ADVECTION | fv.VISCOSITY)
    ru, rv = fv.ns_rhs(u, v, prm, flux=_record(16, 2, 21))
    scale = max(ru.abs().max().item(), rv.abs().max().item())
    assert ru.sum(dim=(-2, -1)).abs().max().item() < 1e-12 * scale * 256
    assert rv.sum(dim=(-2, -1)).abs().max().item() < 1e-12 * scale * 256


def test_interpolation_field_closed_form():
    """fi of kind 0 equal to a constant c adds c * ubar to every east face of
    the u volumes; with u = sin(x) at the u points, R_u changes by
    -c (sin((i+1) h) - sin((i-1) h)) / (2 h) = -c cos(i h) sin(h) / h.
    fi of kind 3 (north faces of the v volumes) with v = sin(y) at the v
    points changes R_v by -c cos(j h) sin(h) / h."""
    n, c = 16, 0.7
    h = L / n
    prm = dict(fv.grid_params(n, n), mask=fv.ADVECTION)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u = torch.tensor(np.sin(i * h))[None]
    v = torch.tensor(np.sin(j * h))[None]
    base = fv.ns_rhs(u, v, prm)
    for kind, comp, idx in ((0, 0, i), (3, 1, j)):
        fi = torch.zeros(1, 4, n, n, dtype=torch.float64)
        fi[:, kind] = c
        got = fv.ns_rhs(u, v, prm, flux={"fi": fi})
        ref = -c * np.cos(idx * h) * math.sin(h) / h
        assert np.abs((got[comp] - base[comp])[0].numpy() - ref).max() < 1e-12
        other = 1 - comp
        assert torch.allclose(got[other], base[other], atol=1e-14)


def test_derivative_field_closed_form():
    """fd of kind 1 (du/dy at the corners) equal to cos(j h) changes R_u by
    nu (cos(j h) - cos((j-1) h)) / h (the north-minus-south face difference)."""
    n, nu = 16, 0.3
    h = L / n
    prm = dict(fv.grid_params(n, n, nu=nu), mask=fv.VISCOSITY)
    u, v, _ = _state(n, 1, seed=4)
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    fd = torch.zeros(1, 4, n, n, dtype=torch.float64)
    fd[:, 1] = torch.tensor(np.cos(j * h))
    got = fv.ns_rhs(u, v, prm, flux={"fd": fd})
    base = fv.ns_rhs(u, v, prm)
    ref = nu * (np.cos(j * h) - np.cos((j - 1) * h)) / h
    assert np.abs((got[0] - base[0])[0].numpy() - ref).max() < 1e-12
    assert torch.allclose(got[1], base[1], atol=1e-14)


def test_uniform_derivative_kernel_scaling():
    """A uniform derivative kernel equal to the fourth-order weights (24 h
    times S6 divided by 24, i.e. [1, -27, 27, -1]/24 at b = 0) doubles the
    viscous term: the learned part is (1/h) sum_s w_s q_s."""
    u, v, prm = _state(16, 1, seed=5)
    prm = dict(prm, mask=fv.VISCOSITY)
    wd = torch.zeros(4, 20, dtype=torch.float64)
    for kind in range(4):
        wd[kind, 4:8] = torch.tensor([1.0, -27.0, 27.0, -1.0]) / 24.0
    got = fv.ns_rhs(u, v, prm, flux={"wd": wd})
    base = fv.ns_rhs(u, v, prm)
    assert torch.allclose(got[0], 2 * base[0], atol=1e-12)
    assert torch.allclose(got[1], 2 * base[1], atol=1e-12)


def test_flux_block_step_with_zero_operators_is_the_plain_step():
    u, v, prm = _state(16, 2, seed=6)
    prm = dict(prm, dt=0.02)
    p = {"wi": torch.zeros(4, 20, dtype=torch.float64),
         "wd": torch.zeros(4, 20, dtype=torch.float64),
         "fno_i": _net(9, out_scale=0.0), "fno_d": _net(10, out_scale=0.0)}
    a = fluxblock.fluxblock_step(u, v, prm, p)
    b = timestep.fv_step(u, v, prm)
    assert torch.allclose(a[0], b[0], atol=1e-14) and torch.allclose(a[1], b[1], atol=1e-14)


def test_flux_block_step_gradient_matches_finite_differences():
    """The oracle's autograd through the flux-block step (uniform kernels and
    one FNO weight) against central differences in FP64."""
    u, v, prm = _state(8, 1, seed=7)
    prm = dict(prm, dt=0.05)
    p = {"wi": torch.tensor(si.stencil_weights(31, 0.05)).requires_grad_(True),
         "wd": torch.tensor(si.stencil_weights(32, 0.05)).requires_grad_(True),
         "fno_i": _net(12, out_scale=0.1), "fno_d": _net(13, out_scale=0.1)}
    R = p["fno_i"]["layers"][1]["R"].requires_grad_(True)
    g = torch.Generator().manual_seed(1)
    wu = torch.randn(u.shape, generator=g, dtype=torch.float64)
    wv = torch.randn(v.shape, generator=g, dtype=torch.float64)

    def loss():
        a, b = fluxblock.fluxblock_step(u, v, prm, p)
        return (wu * a).sum() + (wv * b).sum()

    loss().backward()
    for t, idx in ((p["wi"], (0, 5)), (p["wi"], (3, 17)), (p["wd"], (1, 9)), (p["wd"], (2, 19))):
        with torch.no_grad():
            e = 1e-5
            t[idx] += e
            lp = loss().item()
            t[idx] -= 2 * e
            lm = loss().item()
            t[idx] += e
        fd = (lp - lm) / (2 * e)
        assert t.grad[idx].item() == pytest.approx(fd, rel=1e-6, abs=1e-10)
    k = (1, 1, 2, 3)
    for part, step in (("real", 1e-5), ("imag", 1e-5j)):
        with torch.no_grad():
            R[k] += step
            lp = loss().item()
            R[k] -= 2 * step
            lm = loss().item()
            R[k] += step
        # torch's gradient of a real loss in a complex weight is
        # d/d(Re R) + i d/d(Im R), the convention the library's adjoint keeps
        got = getattr(R.grad[k], part).item()
        assert got == pytest.approx((lp - lm) / 2e-5, rel=1e-6, abs=1e-10), part


def _tc_params(seed, kc, out_scale=0.05):
    p = {"wi": torch.tensor(si.stencil_weights(seed, 0.02)),
         "wd": torch.tensor(si.stencil_weights(seed + 1, 0.02)),
         "fno_i": _net(seed + 2, out_scale=0.05), "fno_d": _net(seed + 3, out_scale=0.05)}
    p["tc"] = fno.from_arrays(si.fno_weights(seed + 4, 4, 2, 2, n_in=2 * kc, n_out=2,
                                             out_scale=out_scale))
    return p


def test_temporal_correction_only_at_multiples_of_kc_and_projected():
    """Eq. 2: the correction enters at k = k_c, 2 k_c, ... only, and the
    corrected state is divergence-free."""
    from oracle import projection
    kc, n = 3, 16
    u0, v0, prm = _state(n, 2, seed=9)
    prm = dict(prm, dt=0.02, k_c=kc)
    p = _tc_params(40, kc)
    with_tc = fluxblock.model_rollout(u0, v0, prm, p, 6)
    no_tc = fluxblock.model_rollout(u0, v0, prm, dict(p, tc=None), 6)
    for k in range(1, 7):
        diff = (with_tc[0][k - 1] - no_tc[0][k - 1]).abs().max().item()
        if k < kc:
            assert diff == 0.0, k
        if k == kc:
            assert diff > 1e-6, k
    div = projection.divergence(with_tc[0][kc - 1], with_tc[1][kc - 1], prm)
    assert div.abs().max().item() < 1e-10


def test_temporal_correction_reads_the_history_oldest_first():
    """A correction whose lift reads only input plane 0 (and whose spectral
    and pointwise layers are switched off) depends on u_{k-k_c} alone: the
    planes are (u, v) per state, oldest first."""
    kc, n = 2, 16
    u0, v0, prm = _state(n, 1, seed=10)
    prm = dict(prm, dt=0.02, k_c=kc)
    p = _tc_params(50, kc, out_scale=1.0)
    tc = p["tc"]
    tc["P_w"] = torch.zeros_like(tc["P_w"])
    tc["P_w"][:, 0] = 1.0
    for lay in tc["layers"]:
        lay["R"] = torch.zeros_like(lay["R"])
    u1, v1 = fluxblock.fluxblock_step(u0, v0, prm, p)
    base = fno.fno_forward(fluxblock.tc_input([u0, u1], [v0, v1]), tc)
    # changing v_{k-2} or the later state leaves it; changing u_{k-2} does not
    same = fno.fno_forward(fluxblock.tc_input([u0, 2 * u1], [v0 + 1, 3 * v1]), tc)
    assert torch.allclose(base, same, atol=1e-14)
    other = fno.fno_forward(fluxblock.tc_input([u0 + 0.5, u1], [v0, v1]), tc)
    assert (other - base).abs().max().item() > 1e-6
    # and the same function of u_{k-2} as a per-pixel evaluation
    P_b, Q_w, Q_b = tc["P_b"], tc["Q_w"], tc["Q_b"]
    h = u0[:, None] + P_b.view(1, -1, 1, 1)
    nl = len(tc["layers"])
    for li, lay in enumerate(tc["layers"]):
        z = torch.einsum("oi,biyx->boyx", lay["W"], h) + lay["b"].view(1, -1, 1, 1)
        h = cnn.gelu(z) if li < nl - 1 else z
    ref = torch.einsum("ko,boyx->bkyx", Q_w, h) + Q_b.view(1, -1, 1, 1)
    assert torch.allclose(base, ref, atol=1e-13)


def test_temporal_correction_with_zero_output_is_the_flux_block_model():
    kc = 2
    u0, v0, prm = _state(16, 2, seed=11)
    prm = dict(prm, dt=0.02, k_c=kc)
    p = _tc_params(60, kc, out_scale=0.0)
    a = fluxblock.model_rollout(u0, v0, prm, p, 4)
    b = fluxblock.fluxblock_rollout(u0, v0, prm, p, 4)
    assert torch.allclose(a[0], b[0], atol=1e-14) and torch.allclose(a[1], b[1], atol=1e-14)
