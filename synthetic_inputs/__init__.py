"""Seeded synthetic inputs shared by the tests, the oracle checks and the
benchmark.  This module holds no arithmetic of the method: it only draws
random arrays (numpy PCG64 with a fixed seed) and builds the configuration
records of the workloads.

Workload records (sizes, physics parameters) follow the paper's flows
(App. C.1, Table S2) at the resolutions this project runs:

* burgers64   2D viscous Burgers, [0, 2pi)^2, 64^2 collocated, nu = 0.01,
              linear-upwind advection, SSP-RK3, dt from CFL 0.5, 200 steps, B = 1
* decaying512 decaying NS, [0, 2pi)^2, 512^2 MAC, nu = 1e-3, GRF peaked at k = 4
              with unit energy, RK4 with a projection per sub-step,
              dt = 2.19e-4 * 2048 / 512, 2000 steps, B = 16
* kolmogorov64 forced NS (sin 4y forcing, drag 0.1), nu = 1e-3, 64^2 learned,
              dt = 16 * 4.38e-4, inference B = 64; fine reference 1024^2
* decaying128_train  decaying NS, 128^2 learned, unroll 32, B = 8
* shear128    shear layers, nu = 2e-4, learned 128^2 vs plain 1024^2, B = 128
* shear_scalar  the shear-flow system with a passive scalar on [0, 8] x [0, 4]:
              fine 2048 x 1024 (coarse 128 x 64), Re = 1000 (nu = 1e-3),
              D = 1e-3, layer thickness w/5 = 0.1, dt = 0.1 dx, B = 8
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def rng(seed):
    return np.random.default_rng(seed)


def random_field(seed, shape, scale=1.0, dtype=np.float64):
    """White-noise field, N(0, scale^2)."""
    return (rng(seed).standard_normal(shape) * scale).astype(dtype)


def smooth_field(seed, batch, ny, nx, kmax=6, dtype=np.float64):
    """A random band-limited periodic field: sum of random Fourier modes with
    |kx|, |ky| <= kmax and N(0,1) complex amplitudes, normalised to unit rms.
    (Arbitrary test data; not the paper's initial conditions.)"""
    g = rng(seed)
    spec = np.zeros((batch, ny, nx), dtype=np.complex128)
    kx = min(kmax, nx // 2 - 1)
    ky = min(kmax, ny // 2 - 1)
    for j in range(-ky, ky + 1):
        for i in range(-kx, kx + 1):
            spec[:, j % ny, i % nx] = g.standard_normal(batch) + 1j * g.standard_normal(batch)
    f = np.fft.ifft2(spec).real
    f /= np.sqrt((f * f).mean(axis=(-2, -1), keepdims=True))
    return f.astype(dtype)


def cnn_weights(seed, layers, last_scale=1e-3, dtype=np.float64):
    """He-normal weights [Cout, Cin, 3, 3] and small biases for each layer; the
    last layer scaled by last_scale (small initial correction)."""
    g = rng(seed)
    ws, bs = [], []
    for li, (ci, co) in enumerate(layers):
        std = math.sqrt(2.0 / (ci * 9))
        w = g.standard_normal((co, ci, 3, 3)) * std
        b = g.standard_normal(co) * 0.01
        if li == len(layers) - 1:
            w = w * last_scale
            b = b * last_scale
        ws.append(w.astype(dtype))
        bs.append(b.astype(dtype))
    return ws, bs


WORKLOADS = {
    "burgers64": dict(layout="collocated", nx=64, ny=64, lx=TWO_PI, ly=TWO_PI, batch=1,
                      nu=0.01, rk="ssprk3", cfl=0.5, steps=200, ic="fourier_modes",
                      forcing_amp=0.0, forcing_k=0.0, drag=0.0, dtype="f64"),
    "decaying512": dict(layout="mac", nx=512, ny=512, lx=TWO_PI, ly=TWO_PI, batch=16,
                        nu=1e-3, rk="rk4", dt=2.19e-4 * 2048 / 512, steps=2000,
                        ic="grf_peak", forcing_amp=0.0, forcing_k=0.0, drag=0.0,
                        dtype="f32"),
    "kolmogorov64": dict(layout="mac", nx=64, ny=64, lx=TWO_PI, ly=TWO_PI, batch=64,
                         nu=1e-3, rk="rk4", dt=16 * 2.19e-4 * 2048 / 1024, steps=625,
                         ic="grf_peak", forcing_amp=1.0, forcing_k=4.0, drag=0.1,
                         dtype="f32", fine_n=1024, fine_batch=8),
    "decaying128_train": dict(layout="mac", nx=128, ny=128, lx=TWO_PI, ly=TWO_PI, batch=8,
                              nu=1e-3, rk="rk4", dt=4 * 2.19e-4 * 2048 / 512, unroll=32,
                              checkpoint_every=8, ic="grf_peak", forcing_amp=0.0,
                              forcing_k=0.0, drag=0.0, dtype="f32", fine_n=512),
    "shear_scalar": dict(layout="mac", nx=2048, ny=1024, lx=8.0, ly=4.0, batch=8, nu=1e-3,
                         diffusivity=1e-3, rk="rk4", dt=0.1 * (8.0 / 2048), steps=20,
                         ic="shear_layer", delta=0.1, forcing_amp=0.0, forcing_k=0.0, drag=0.0,
                         dtype="f32", coarse_nx=128, coarse_ny=64),
    "shear128": dict(layout="mac", nx=128, ny=128, lx=TWO_PI, ly=TWO_PI, batch=128,
                     nu=2e-4, rk="rk4", dt=8 * 0.1 * (TWO_PI / 1024), steps=4096,
                     ic="shear_layer", forcing_amp=0.0, forcing_k=0.0, drag=0.0,
                     dtype="f32", fine_n=1024),
}


def fno_weights(seed, width, layers, modes, n_in=2, n_out=4, out_scale=1e-2, dtype=np.float64):
    """Random FNO parameters as real arrays: lift P_w [width, n_in], P_b;
    per layer R_re, R_im [2 modes, modes, width, width] drawn with scale
    1 / width^2, pointwise W [width, width] (out, in) with scale 1 / sqrt(width)
    and b; projection Q_w [n_out, width] and Q_b scaled by out_scale (a small
    initial correction)."""
    g = rng(seed)
    a = {"P_w": g.standard_normal((width, n_in)) / math.sqrt(n_in),
         "P_b": g.standard_normal(width) * 0.01, "layers": []}
    for _ in range(layers):
        sc = 1.0 / (width * width)
        a["layers"].append({
            "R_re": g.standard_normal((2 * modes, modes, width, width)) * sc,
            "R_im": g.standard_normal((2 * modes, modes, width, width)) * sc,
            "W": g.standard_normal((width, width)) / math.sqrt(width),
            "b": g.standard_normal(width) * 0.01})
    a["Q_w"] = g.standard_normal((n_out, width)) / math.sqrt(width) * out_scale
    a["Q_b"] = g.standard_normal(n_out) * 0.01 * out_scale

    def cast(z):
        return {k: ([cast(l) for l in v] if isinstance(v, list) else v.astype(dtype))
                for k, v in z.items()}
    return cast(a)


def stencil_weights(seed, scale=1e-2, dtype=np.float64):
    """Random uniform 5x4 kernels [4 kinds, 20 points], N(0, scale^2)."""
    return (rng(seed).standard_normal((4, 20)) * scale).astype(dtype)


# flux-block networks of the paper's hyper-parameter table: (layers, modes, width)
FLUXBLOCK_FNO = {"forced": (6, 32, 16), "decaying": (4, 16, 8)}
