"""Data generation, training and evaluation drivers for the learned solver.

Everything numerical runs in libldsv.so through the ctypes binding; this
module only sequences the calls:

* ``generate_labels``  plain fine-grid FV trajectories down-sampled in space
  (MAC face averaging) and time (the coarse/fine step ratio), the coarse
  training labels of Sec. 4.1 (Table 1 / Table S2 recipe: fine simulation,
  warm-up, down-sampling);
* ``train``            Adam on the autoregressive rollout MSE (Eq. 13) with
  the hand-written adjoint (unrolled backward with checkpoints);
* ``evaluate``         vorticity correlation against the down-sampled fine
  reference per snapshot, the time until it first drops below a threshold,
  and the MSE at a fixed horizon (App. D.1 metrics).
"""
import math
import time

import torch

from . import ldsv


def physics(w):
    return dict(nu=w["nu"], forcing_amp=w.get("forcing_amp", 0.0),
                forcing_k=w.get("forcing_k", 0.0), drag=w.get("drag", 0.0))


def generate_labels(fine_n, coarse_n, batch, seed, nsteps, dt_fine, phys, warmup_steps=0,
                    ic=ldsv.IC_GRF_PEAK, lx=2 * math.pi, progress=None):
    """Coarse labels [nsteps + 1, B, n, n] (u and v): the fine plain-FV
    solution down-sampled every r fine steps, r = fine_n / coarse_n."""
    r = fine_n // coarse_n
    fine = ldsv.Solver(fine_n, fine_n, batch, lx=lx, ly=lx)
    coarse = ldsv.Solver(coarse_n, coarse_n, batch, lx=lx, ly=lx)
    u, v = fine.init_state(ic, seed)
    prm = ldsv.params(dt=dt_fine, **phys)
    if warmup_steps:
        chunk = 500
        done = 0
        while done < warmup_steps:
            k = min(chunk, warmup_steps - done)
            fine.fv_step(prm, u, v, nsteps=k, out=(u, v))
            done += k
            if progress:
                torch.cuda.synchronize()
                progress("warm-up %d/%d fine steps" % (done, warmup_steps))
    lu = torch.empty(nsteps + 1, batch, coarse_n, coarse_n, device="cuda")
    lv = torch.empty_like(lu)
    uc, vc = coarse.downsample(r, u, v)
    lu[0], lv[0] = uc, vc
    for t in range(nsteps):
        fine.fv_step(prm, u, v, nsteps=r, out=(u, v))
        uc, vc = coarse.downsample(r, u, v)
        lu[t + 1], lv[t + 1] = uc, vc
        if progress and (t + 1) % 200 == 0:
            torch.cuda.synchronize()
            progress("labels %d/%d coarse steps" % (t + 1, nsteps))
    torch.cuda.synchronize()
    fine.close()
    coarse.close()
    return lu, lv


class Adam:
    """Adam state over the network's FP32 master weights and biases; the
    update itself is the library's Adam kernel."""

    def __init__(self, net, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
        self.net = net
        self.params = net.master_w + net.b
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, grads):
        self.t += 1
        g = grads.w + grads.b
        for p, gp, m, v in zip(self.params, g, self.m, self.v):
            ldsv.adam_step(p, gp, m, v, self.t, self.lr, self.b1, self.b2, self.eps)
        self.net.refresh()


def train(solver, net, labels, prm, iters, unroll=32, checkpoint_every=8, lr=1e-4, seed=0,
          batch_from=None, progress=None, log_every=10):
    """Adam on the unrolled rollout MSE.  labels: (lu, lv) [T+1, B, n, n] with
    the solver's batch B.  Each iteration starts from labels[t0] at a random
    t0 and unrolls `unroll` learned steps.  Returns the loss history."""
    lu, lv = labels
    T = lu.shape[0] - 1
    g = torch.Generator().manual_seed(seed)
    opt = Adam(net, lr=lr)
    dW = ldsv.NetGradBuffers(net)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    t_start = time.perf_counter()
    for it in range(iters):
        t0 = int(torch.randint(0, T - unroll + 1, (1,), generator=g))
        dW.zero_()
        loss.zero_()
        solver.rollout_bwd(prm, net, lu[t0].contiguous(), lv[t0].contiguous(), unroll, dW,
                           checkpoint_every=checkpoint_every, first_index=1,
                           labels=(lu[t0 + 1:t0 + 1 + unroll].contiguous(),
                                   lv[t0 + 1:t0 + 1 + unroll].contiguous()),
                           loss_scale=1.0 / unroll, loss=loss)
        opt.step(dW)
        if (it + 1) % log_every == 0 or it == 0:
            l = loss.item()
            hist.append((it + 1, l))
            if progress:
                progress("iter %d loss %.6e (%.1f s)" % (it + 1, l, time.perf_counter() - t_start))
    return hist


def vorticity_pcc_series(solver, traj, labels):
    """PCC of corner vorticity per snapshot and trajectory: [T, B]."""
    tu, tv = traj
    lu, lv = labels
    out = []
    for t in range(tu.shape[0]):
        w = solver.vorticity(tu[t].contiguous(), tv[t].contiguous())
        wl = solver.vorticity(lu[t].contiguous(), lv[t].contiguous())
        out.append(solver.pcc(w, wl))
    return torch.stack(out)


def first_drop(pcc, dt, threshold=0.9):
    """Per trajectory: simulated time until the correlation first falls below
    threshold (snapshot t is at time (t+1) dt); the horizon if never."""
    T = pcc.shape[0]
    below = pcc < threshold
    res = []
    for b in range(pcc.shape[1]):
        idx = torch.nonzero(below[:, b])
        res.append(dt * (int(idx[0]) if idx.numel() else T))
    return res


def evaluate(solver, prm, labels, nsteps, net=None):
    """Rollout from labels[0] (plain FV if net is None) and compare with
    labels[1..nsteps]: returns dict with pcc [T, B], T_0.9 per trajectory,
    MSE per snapshot and wall time."""
    lu, lv = labels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = prm
    if net is not None:
        p = ldsv.params(nu=prm.nu, dt=prm.dt, forcing_amp=prm.forcing_amp,
                        forcing_k=prm.forcing_k, drag=prm.drag, rk=prm.rk,
                        mask=prm.physics_mask, k_c=prm.k_c, fallback_enable=1)
    flags = torch.zeros(solver.batch, dtype=torch.int32, device="cuda")
    tu, tv = solver.rollout(p, lu[0].contiguous(), lv[0].contiguous(), nsteps, 1, net=net,
                            fallback_flags=flags if net is not None else None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ref = (lu[1:nsteps + 1], lv[1:nsteps + 1])
    pcc = vorticity_pcc_series(solver, (tu, tv), ref)
    mse = (((tu - ref[0]) ** 2).mean(dim=(-2, -1)) + ((tv - ref[1]) ** 2).mean(dim=(-2, -1))) * 0.5
    return {"pcc": pcc, "t09": first_drop(pcc.cpu(), prm.dt), "mse": mse, "wall_s": wall,
            "fallbacks": flags.tolist() if net is not None else None}
