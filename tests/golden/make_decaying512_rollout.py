"""Writes decaying512_rollout.json: the FP64 oracle's 2000-step rollout of
one trajectory of the decaying 512^2 workload, the long-rollout pin of the
FP32 plain path.

    python tests/golden/make_decaying512_rollout.py [--threads N]

Calls only the oracle.  Workload: decaying 2D Navier-Stokes on the periodic
[0, 2 pi)^2 box, 512^2 MAC cells, nu = 1e-3, dt = 2.19e-4 * 2048 / 512, RK4
with a projection after every sub-step (Sec. 3.2; App. B.5 S15-S20); initial
condition: the Gaussian random streamfunction peaked at k = 4 with unit
energy, seed 0, trajectory 0 (App. C.1), rounded to float32 first because
the FP32 path starts from the float32 state.  Recorded: kinetic energy and
enstrophy every 100 steps, the final state on every 16th row and column,
and the final state's Fourier coefficients with |kx|, |ky| <= 4 (FFT
normalised by the cell count).  About 6 minutes on 8 cores.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

from oracle import fv, ic, metrics, timestep  # noqa: E402

N = 512
STEPS = 2000
EVERY = 100
STRIDE = 16
KMAX = 4
NU = 1e-3
DT = 2.19e-4 * 2048 / N


def low_modes(q):
    f = torch.fft.fft2(q) / (q.shape[-1] * q.shape[-2])
    ks = list(range(-KMAX, KMAX + 1))
    rows = [[f[ky % N, kx % N] for kx in ks] for ky in ks]
    return ([[float(z.real) for z in r] for r in rows], [[float(z.imag) for z in r] for r in rows])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    a = ap.parse_args()
    torch.set_num_threads(a.threads)
    L = 2 * math.pi
    u, v = ic.grf_peak(1, N, N, L, L, seed=0)
    u, v = u.float().double(), v.float().double()
    prm = fv.grid_params(N, N, nu=NU, dt=DT)
    h = L / N
    steps, en, ens = [0], [float(metrics.energy(u, v)[0])], [float(metrics.enstrophy(u, v, h, h)[0])]
    t0 = time.time()
    for k in range(1, STEPS + 1):
        u, v = timestep.fv_step(u, v, prm)
        if k % EVERY == 0:
            steps.append(k)
            en.append(float(metrics.energy(u, v)[0]))
            ens.append(float(metrics.enstrophy(u, v, h, h)[0]))
            print("step %d energy %.12e enstrophy %.12e (%.0f s)" % (k, en[-1], ens[-1],
                                                                    time.time() - t0), flush=True)
    ur, ui = low_modes(u[0])
    vr, vi = low_modes(v[0])
    out = {
        "what": "FP64 oracle rollout of the decaying 512^2 workload, trajectory 0 of seed 0, "
                "float32-rounded initial state; written by make_decaying512_rollout.py",
        "n": N, "nu": NU, "dt": DT, "steps": STEPS, "rk": "rk4, projection per sub-step",
        "series": {"step": steps, "energy": en, "enstrophy": ens},
        "final": {"stride": STRIDE,
                  "u": u[0, ::STRIDE, ::STRIDE].tolist(), "v": v[0, ::STRIDE, ::STRIDE].tolist()},
        "modes": {"kmax": KMAX, "u_re": ur, "u_im": ui, "v_re": vr, "v_im": vi},
    }
    with open(os.path.join(HERE, "decaying512_rollout.json"), "w") as f:
        json.dump(out, f)
        f.write("\n")
    print("wrote decaying512_rollout.json (%.0f s)" % (time.time() - t0))


if __name__ == "__main__":
    main()
