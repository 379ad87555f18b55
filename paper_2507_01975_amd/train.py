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
                    ic=ldsv.IC_GRF_PEAK, lx=2 * math.pi, progress=None, ic_resolutions=None):
    """Coarse labels [nsteps + 1, B, n, n] (u and v): the fine plain-FV
    solution down-sampled every r fine steps, r = fine_n / coarse_n.  With
    ic_resolutions (a sequence, possibly empty), returns ((u, v), ics) with
    ics = {N: (u, v)}: the state after the warm-up down-sampled to N x N (the
    common initial condition of a resolution sweep)."""
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
    ics = {}
    for N in ic_resolutions or ():
        if N == fine_n:
            ics[N] = (u.clone(), v.clone())
        else:
            sN = ldsv.Solver(N, N, batch, lx=lx, ly=lx)
            ics[N] = sN.downsample(fine_n // N, u, v)
            sN.close()
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
    if ic_resolutions is not None:
        return (lu, lv), ics
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
          batch_from=None, progress=None, log_every=10, windows=1, dnet=None):
    """Adam on the unrolled rollout MSE.  labels: (lu, lv) [T+1, B, n, n].
    Each iteration draws `windows` random start times t0 and unrolls `unroll`
    learned steps from labels[t0] for every trajectory of every window at
    once; the solver's batch is windows * B.  dnet: optional
    derivative-stencil network trained beside net.  Returns the loss
    history."""
    lu, lv = labels
    T = lu.shape[0] - 1
    assert solver.batch == windows * lu.shape[1], "solver batch must be windows * label batch"
    g = torch.Generator().manual_seed(seed)
    opt = Adam(net, lr=lr)
    dW = ldsv.NetGradBuffers(net)
    dopt = Adam(dnet, lr=lr) if dnet is not None else None
    dWd = ldsv.NetGradBuffers(dnet) if dnet is not None else None
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    t_start = time.perf_counter()
    for it in range(iters):
        t0s = [int(x) for x in torch.randint(0, T - unroll + 1, (windows,), generator=g)]
        u0 = torch.cat([lu[t] for t in t0s]).contiguous()
        v0 = torch.cat([lv[t] for t in t0s]).contiguous()
        yu = torch.cat([lu[t + 1:t + 1 + unroll] for t in t0s], dim=1).contiguous()
        yv = torch.cat([lv[t + 1:t + 1 + unroll] for t in t0s], dim=1).contiguous()
        dW.zero_()
        loss.zero_()
        if dnet is None:
            solver.rollout_bwd(prm, net, u0, v0, unroll, dW, checkpoint_every=checkpoint_every,
                               first_index=1, labels=(yu, yv), loss_scale=1.0 / unroll,
                               loss=loss)
        else:
            dWd.zero_()
            solver.rollout_d_bwd(prm, net, dnet, u0, v0, unroll, dW, dWd,
                                 checkpoint_every=checkpoint_every, first_index=1,
                                 labels=(yu, yv), loss_scale=1.0 / unroll, loss=loss)
            dopt.step(dWd)
        opt.step(dW)
        if (it + 1) % log_every == 0 or it == 0:
            l = loss.item()
            hist.append((it + 1, l))
            if progress:
                progress("iter %d loss %.6e (%.1f s)" % (it + 1, l, time.perf_counter() - t_start))
    return hist


def fluxblock_param_tensors(net):
    """The flux block's trainable tensors: the uniform kernels, then each
    present FNO's lift, spectral, pointwise and projection tensors."""
    out = [net.stencil_w]
    for f in net.fno:
        if f is not None:
            out += [f.lift_w, f.lift_b, f.spec_w, f.point_w, f.point_b, f.proj_w, f.proj_b]
    return out


def fluxblock_grad_tensors(grads):
    out = [grads.stencil_w]
    for f in grads.fno:
        if f is not None:
            out += f.tensors()
    return out


def _history(states, k, kc):
    """The k_c states u_{k-k_c} .. u_{k-1} (padded with u_0 before the first
    correction, where only the last one is read)."""
    idx = [max(0, k - kc + j) for j in range(kc)]
    return [states[i][0] for i in idx], [states[i][1] for i in idx]


def train_fluxblock(solver, net, labels, prm, iters, unroll=8, lr=1e-4, seed=0, progress=None,
                    log_every=10, tc=None):
    """Adam on the unrolled rollout MSE of the flux-block model (the paper's
    own learnable flux block, Sec. 3.4, trained on the Eq. 13 loss), with the
    temporal correction block when tc (an FnoParams with 2 prm.k_c inputs and
    2 outputs) is given: Eq. 2 with the window start as time 0.
    labels: (lu, lv) [T+1, B, n, n].  Each iteration unrolls `unroll` steps
    from a random labels[t0], keeping the states, then runs the step adjoint
    backwards through them with the loss gradient of every state added on
    the way (a corrected step also sends gradient to the earlier states of
    its history).  Returns the loss history."""
    lu, lv = labels
    T = lu.shape[0] - 1
    kc = prm.k_c
    g = torch.Generator().manual_seed(seed)
    params = fluxblock_param_tensors(net)
    grads = ldsv.FluxNetGradBuffers(net)
    gts = fluxblock_grad_tensors(grads)
    gtc = None
    if tc is not None:
        gtc = ldsv.FnoGradBuffers(tc)
        params += [tc.lift_w, tc.lift_b, tc.spec_w, tc.point_w, tc.point_b, tc.proj_w, tc.proj_b]
        gts += gtc.tensors()
    m = [torch.zeros_like(p) for p in params]
    v2 = [torch.zeros_like(p) for p in params]
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    t_start = time.perf_counter()
    for it in range(iters):
        t0 = int(torch.randint(0, T - unroll + 1, (1,), generator=g))
        states = [(lu[t0].contiguous(), lv[t0].contiguous())]
        for k in range(1, unroll + 1):
            if tc is None:
                states.append(solver.fluxblock_step(prm, net, *states[-1]))
            else:
                states.append(solver.fluxblock_tc_step(prm, net, tc, *_history(states, k, kc), k))
        grads.zero_()
        if gtc is not None:
            for t in gtc.tensors():
                t.zero_()
        loss.zero_()
        # cotangents of every state; complete for state k once steps > k are done
        gs = [(torch.zeros_like(states[0][0]), torch.zeros_like(states[0][1]))
              for _ in range(unroll + 1)]
        for k in range(unroll, 0, -1):
            mu, mv = solver.mse_grad(states[k][0], states[k][1], lu[t0 + k], lv[t0 + k],
                                     scale=1.0 / unroll, loss=loss)
            mu += gs[k][0]
            mv += gs[k][1]
            if tc is None:
                gu, gv = solver.fluxblock_step_bwd(prm, net, states[k - 1][0], states[k - 1][1],
                                                   mu, mv, grads)
                gs[k - 1][0].add_(gu)
                gs[k - 1][1].add_(gv)
            else:
                idx = [max(0, k - kc + j) for j in range(kc)]
                hu, hv = _history(states, k, kc)
                ghu, ghv = [], []
                for j, i in enumerate(idx):
                    # padded entries (before the first correction) are not read
                    if j < kc - 1 and k % kc != 0:
                        ghu.append(torch.zeros_like(mu))
                        ghv.append(torch.zeros_like(mv))
                    else:
                        ghu.append(gs[i][0])
                        ghv.append(gs[i][1])
                solver.fluxblock_tc_step_bwd(prm, net, tc, hu, hv, k, mu, mv, ghu, ghv, grads,
                                             gtc)
        for p, gp, mm, vv in zip(params, gts, m, v2):
            ldsv.adam_step(p, gp, mm, vv, it + 1, lr)
        if (it + 1) % log_every == 0 or it == 0:
            l = loss.item()  # summed over the unrolled states, as train() reports it
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
    below = ~(pcc >= threshold)  # a non-finite correlation counts as a drop
    res = []
    for b in range(pcc.shape[1]):
        idx = torch.nonzero(below[:, b])
        res.append(dt * (int(idx[0]) if idx.numel() else T))
    return res


def evaluate(solver, prm, labels, nsteps, net=None, dnet=None):
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
    if dnet is not None:
        tu, tv = solver.rollout_d(p, net, dnet, lu[0].contiguous(), lv[0].contiguous(), nsteps,
                                  1, fallback_flags=flags)
    else:
        tu, tv = solver.rollout(p, lu[0].contiguous(), lv[0].contiguous(), nsteps, 1, net=net,
                                fallback_flags=flags if net is not None else None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ref = (lu[1:nsteps + 1], lv[1:nsteps + 1])
    pcc = vorticity_pcc_series(solver, (tu, tv), ref)
    mse = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    for t in range(nsteps):
        solver.mse_grad(tu[t], tv[t], ref[0][t].contiguous(), ref[1][t].contiguous(),
                        loss=mse[t:t + 1], want_grad=False)
    return {"pcc": pcc, "t09": first_drop(pcc.cpu(), prm.dt), "mse": mse, "wall_s": wall,
            "fallbacks": flags.tolist() if net is not None else None}


def plain_sweep_pcc(N, n, ic, labels, dt_coarse, phys, horizon, lx=2 * math.pi, chunk=256):
    """Plain FV at N x N from ic (already at N), advanced N/n steps of dt
    dt_coarse * n / N per coarse step, down-sampled to n and compared with
    labels[1..horizon] by vorticity PCC: returns (pcc [T, B], wall seconds of
    the rollouts).  The rollout runs in chunks of `chunk` coarse steps, so
    only a chunk of fine snapshots is held at a time."""
    u, v = (t.contiguous() for t in ic)
    B = u.shape[0]
    rN = N // n
    sN = ldsv.Solver(N, N, B, lx=lx, ly=lx)
    sn = ldsv.Solver(n, n, B, lx=lx, ly=lx)
    prm = ldsv.params(dt=dt_coarse / rN, **phys)
    lu, lv = labels
    pccs = []
    wall = 0.0
    for c0 in range(0, horizon, chunk):
        k = min(chunk, horizon - c0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tu, tv = sN.rollout(prm, u, v, k * rN, save_every=rN)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        u, v = tu[-1].clone(), tv[-1].clone()
        cu = torch.empty(k, B, n, n, device="cuda")
        cv = torch.empty_like(cu)
        for t in range(k):
            if rN == 1:
                cu[t], cv[t] = tu[t], tv[t]
            else:
                cu[t], cv[t] = sn.downsample(rN, tu[t].contiguous(), tv[t].contiguous())
        del tu, tv
        pccs.append(vorticity_pcc_series(sn, (cu, cv), (lu[c0 + 1:c0 + k + 1],
                                                       lv[c0 + 1:c0 + k + 1])))
    sN.close()
    sn.close()
    return torch.cat(pccs), wall


def t09_summary(t09, horizon_s):
    """Mean, spread and censoring of per-trajectory T_0.9 values (a
    trajectory that never drops below 0.9 within the horizon is censored at
    the horizon)."""
    t = torch.tensor(t09, dtype=torch.float64)
    return {"mean": float(t.mean()), "min": float(t.min()), "max": float(t.max()),
            "std": float(t.std()) if t.numel() > 1 else 0.0,
            "censored": int((t >= horizon_s - 1e-12).sum()), "per_trajectory": list(t09)}


def throughput(N, B, prm, steps, net=None, warmup=3, lx=2 * math.pi, dnet=None,
               ic=ldsv.IC_GRF_PEAK):
    """(cell-steps/s, sim-time/s per trajectory, ms/step) of the plain or
    learned step (with the derivative-stencil network when dnet is given) at
    N x N, batch B, on device-resident state."""
    s = ldsv.Solver(N, N, B, lx=lx, ly=lx)
    u, v = s.init_state(ic, seed=7)
    if net is not None:
        # the learned solver as it runs: the rollout with the guard and the
        # plain-FV fallback on the device, one snapshot at the end
        prm = ldsv.params(nu=prm.nu, dt=prm.dt, forcing_amp=prm.forcing_amp,
                          forcing_k=prm.forcing_k, drag=prm.drag, rk=prm.rk,
                          mask=prm.physics_mask, k_c=prm.k_c, fallback_enable=1)
        flags = torch.zeros(B, dtype=torch.int32, device="cuda")

        def run(k):
            if dnet is None:
                s.rollout(prm, u, v, k, save_every=k, net=net, fallback_flags=flags)
            else:
                s.rollout_d(prm, net, dnet, u, v, k, k, fallback_flags=flags)
    else:
        def run(k):
            s.fv_step(prm, u, v, nsteps=k, out=(u, v))

    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.close()
    return N * N * B * steps / t, prm.dt * steps / t, 1e3 * t / steps


def corr_metric(fine_n=1024, n=64, sweep=(64, 128, 256, 512), train_batch=8, test_batch=16,
                train_fine_steps=10000, warmup_fine=4000, horizon=1200, iters=1500, unroll=16,
                windows=4, lr=1e-4, speed_batch=64, speed_steps=40, progress=None,
                seeds=(100, 200), fluxblock_iters=600, fluxblock_kc=4, deriv_iters=750):
    """The forced-flow measurement: train the 64^2 learned solver on labels
    down-sampled from fine plain FV, then on held-out seeds find T_0.9 (time
    until the vorticity PCC against the down-sampled fine reference first
    drops below 0.9) for the learned solver and for plain FV at each sweep
    resolution, and the throughput of the learned step and of the coarsest
    plain resolution that reaches the learned T_0.9.  With fluxblock_iters
    the paper's own model (flux block + temporal correction every
    fluxblock_kc steps, the forced-flow sizes of Table S3) is trained on the
    same labels and measured the same way; with deriv_iters so is the
    per-cell model with learned derivative stencils (a second network)."""
    log = progress or (lambda *a: None)
    phys = dict(nu=1e-3, forcing_amp=1.0, forcing_k=4.0, drag=0.1)
    dtf = 2.19e-4 * 2048 / fine_n
    r = fine_n // n
    dtc = r * dtf
    t0 = time.perf_counter()
    lab_tr = generate_labels(fine_n, n, train_batch, seeds[0], train_fine_steps // r, dtf, phys,
                             warmup_steps=warmup_fine, progress=log)
    lab_te, ics = generate_labels(fine_n, n, test_batch, seeds[1], horizon, dtf, phys,
                                  warmup_steps=warmup_fine, progress=log,
                                  ic_resolutions=tuple(N for N in sweep if N != n))
    log("labels ready (%.1f s)" % (time.perf_counter() - t0))
    net = init_network(seed=0)
    t_tr0 = time.perf_counter()
    st = ldsv.Solver(n, n, train_batch * windows)
    prm = ldsv.params(dt=dtc, k_c=1, fallback_enable=0, **phys)
    hist = train(st, net, lab_tr, prm, iters=iters, unroll=unroll, checkpoint_every=8, lr=lr,
                 progress=log, log_every=50, windows=windows)
    st.close()
    t_train = time.perf_counter() - t_tr0
    log("trained (%.1f s)" % (time.perf_counter() - t0))
    se = ldsv.Solver(n, n, test_batch)
    ev = evaluate(se, prm, lab_te, horizon, net=net)
    ev_plain = evaluate(se, prm, lab_te, horizon)
    se.close()
    hs = horizon * dtc
    spread = {"learned_%d" % n: t09_summary(ev["t09"], hs),
              "plain_%d" % n: t09_summary(ev_plain["t09"], hs)}
    for N in sweep:
        if N == n:
            continue
        pcc, _ = plain_sweep_pcc(N, n, ics[N], lab_te, dtc, phys, horizon)
        spread["plain_%d" % N] = t09_summary(first_drop(pcc.cpu(), dtc), hs)
        log("plain %d: T_0.9 = %.3f" % (N, spread["plain_%d" % N]["mean"]))
    t09 = {k: v["mean"] for k, v in spread.items()}
    target = t09["learned_%d" % n]
    match = None
    for N in sorted(sweep):
        if t09["plain_%d" % N] >= target:
            match = N
            break
    # throughput at the inference batch on device-resident state
    cs_l, st_l, ms_l = throughput(n, speed_batch, prm, speed_steps, net=net)
    out = {"workload": "forced Kolmogorov flow, nu=1e-3, drag 0.1; learned %d^2 trained on %d^2 "
                       "plain FV down-sampled %dx (%d trajectories, %d fine steps each)"
                       % (n, fine_n, r, train_batch, train_fine_steps),
           "horizon_s": horizon * dtc, "t09_s": t09, "t09_spread": spread,
           "test_trajectories": test_batch,
           "training": {"iters": iters, "unroll": unroll, "windows_per_iter": windows,
                        "lr": lr, "seconds": t_train},
           "final_train_loss": hist[-1][1], "initial_train_loss": hist[0][1],
           "learned": {"n": n, "batch": speed_batch, "cell_steps_per_s": cs_l,
                       "sim_time_per_s": st_l, "ms_per_step": ms_l},
           "mse_at_horizon": {"learned": ev["mse"][-1].item(), "plain_%d" % n: ev_plain["mse"][-1].item()}}
    if match is not None:
        pm = ldsv.params(dt=dtc * n / match, **phys)
        steps = max(10, speed_steps * n // match)
        cs_p, st_p, ms_p = throughput(match, speed_batch, pm, steps)
        out["plain_match"] = {"n": match, "batch": speed_batch, "cell_steps_per_s": cs_p,
                              "sim_time_per_s": st_p, "ms_per_step": ms_p}
        out["sim_time_speedup_at_equal_corr"] = st_l / st_p
    else:
        out["plain_match"] = "no plain resolution up to %d reached the learned T_0.9" % max(sweep)
    if fluxblock_iters:
        fnet, tc = init_fluxblock(seed=0, tc_kc=fluxblock_kc)
        prm_fb = ldsv.params(dt=dtc, k_c=fluxblock_kc, **phys)
        sf = ldsv.Solver(n, n, train_batch)
        t_fb0 = time.perf_counter()
        hist_fb = train_fluxblock(sf, fnet, lab_tr, prm_fb, iters=fluxblock_iters, unroll=unroll,
                                  lr=lr, tc=tc, progress=log, log_every=100)
        t_fb = time.perf_counter() - t_fb0
        sf.close()
        se = ldsv.Solver(n, n, test_batch)
        lu, lv = lab_te
        tu, tv = fluxblock_model_rollout(se, prm_fb, fnet, tc, lu[0], lv[0], horizon)
        pcc = vorticity_pcc_series(se, (tu, tv), (lu[1:horizon + 1], lv[1:horizon + 1]))
        se.close()
        fb_spread = t09_summary(first_drop(pcc.cpu(), dtc), hs)
        t09_fb = fb_spread["mean"]
        fb = {"model": "flux block (uniform 5x4 kernels + FNOs 6 layers / 32 modes / width 16) "
                       "+ temporal correction every %d steps (FNO 4 / 32 / 8)" % fluxblock_kc,
              "training": {"iters": fluxblock_iters, "unroll": unroll, "lr": lr,
                           "seconds": t_fb},
              "initial_train_loss": hist_fb[0][1], "final_train_loss": hist_fb[-1][1],
              "t09_s": t09_fb, "t09_spread": fb_spread}
        cs_f, st_f, ms_f = fluxblock_throughput(n, speed_batch, prm_fb, fnet, tc, speed_steps)
        fb["throughput"] = {"n": n, "batch": speed_batch, "cell_steps_per_s": cs_f,
                            "sim_time_per_s": st_f, "ms_per_step": ms_f}
        fmatch = None
        for N in sorted(sweep):
            if t09["plain_%d" % N] >= t09_fb:
                fmatch = N
                break
        if fmatch is not None:
            pm = ldsv.params(dt=dtc * n / fmatch, **phys)
            steps = max(10, speed_steps * n // fmatch)
            cs_p, st_p, ms_p = throughput(fmatch, speed_batch, pm, steps)
            fb["plain_match"] = {"n": fmatch, "sim_time_per_s": st_p, "ms_per_step": ms_p}
            fb["sim_time_speedup_at_equal_corr"] = st_f / st_p
        out["fluxblock_model"] = fb
        log("flux-block model: T_0.9 = %.3f (%.1f s)" % (t09_fb, time.perf_counter() - t0))
    if deriv_iters:
        net2 = init_network(seed=0)
        dnet = init_network(seed=1)
        st = ldsv.Solver(n, n, train_batch * windows)
        t_d0 = time.perf_counter()
        hist_d = train(st, net2, lab_tr, prm, iters=deriv_iters, unroll=unroll,
                       checkpoint_every=8, lr=lr, progress=log, log_every=250, windows=windows,
                       dnet=dnet)
        t_d = time.perf_counter() - t_d0
        st.close()
        se = ldsv.Solver(n, n, test_batch)
        ev_d = evaluate(se, prm, lab_te, horizon, net=net2, dnet=dnet)
        se.close()
        d_spread = t09_summary(ev_d["t09"], hs)
        t09_d = d_spread["mean"]
        dm = {"model": "per-cell learned interpolation and derivative stencils (two 6-layer "
                       "64-channel BF16 CNNs) + temporal correction every step",
              "training": {"iters": deriv_iters, "unroll": unroll, "windows_per_iter": windows,
                           "lr": lr, "seconds": t_d},
              "initial_train_loss": hist_d[0][1], "final_train_loss": hist_d[-1][1],
              "t09_s": t09_d, "t09_spread": d_spread, "fallbacks": ev_d["fallbacks"],
              "mse_at_horizon": ev_d["mse"][-1].item()}
        cs_d, st_d, ms_d = throughput(n, speed_batch, prm, speed_steps, net=net2, dnet=dnet)
        dm["throughput"] = {"n": n, "batch": speed_batch, "cell_steps_per_s": cs_d,
                            "sim_time_per_s": st_d, "ms_per_step": ms_d}
        dmatch = None
        for N in sorted(sweep):
            if t09["plain_%d" % N] >= t09_d:
                dmatch = N
                break
        if dmatch is not None:
            pm = ldsv.params(dt=dtc * n / dmatch, **phys)
            steps = max(10, speed_steps * n // dmatch)
            cs_p, st_p, ms_p = throughput(dmatch, speed_batch, pm, steps)
            dm["plain_match"] = {"n": dmatch, "sim_time_per_s": st_p, "ms_per_step": ms_p}
            dm["sim_time_speedup_at_equal_corr"] = st_d / st_p
        out["learned_deriv_model"] = dm
        log("learned-derivative model: T_0.9 = %.3f (%.1f s)" % (t09_d, time.perf_counter() - t0))
    log("corr metric done (%.1f s)" % (time.perf_counter() - t0))
    return out


def corr_shear(fine_n=1024, n=128, sweep=(128, 256, 512), train_batch=8, test_batch=16,
               train_steps=2048, horizon=4096, iters=600, unroll=16, windows=2, lr=1e-4,
               speed_batch=128, speed_steps=20, seeds=(1000, 0), progress=None):
    """The shear-flow measurement: doubly periodic shear layers (nu = 2e-4),
    the learned n^2 solver trained on fine plain FV down-sampled fine_n / n
    times (train_batch trajectories from seed seeds[0], train_steps coarse
    steps each), then on test_batch held-out trajectories (seed seeds[1])
    the time until the vorticity PCC against the down-sampled fine solve
    first drops below 0.9, for the learned solver and for plain FV at each
    sweep resolution; the fine solve itself is the last candidate (its
    correlation is 1 by construction).  Throughput of the learned step and
    of the coarsest plain resolution that lasts as long, at speed_batch."""
    log = progress or (lambda *a: None)
    phys = dict(nu=2e-4)
    lx = 2 * math.pi
    dtf = 0.1 * lx / fine_n
    r = fine_n // n
    dtc = r * dtf
    t0 = time.perf_counter()
    lab_tr = generate_labels(fine_n, n, train_batch, seeds[0], train_steps, dtf, phys,
                             ic=ldsv.IC_SHEAR_LAYER, progress=log)
    lab_te, ics = generate_labels(fine_n, n, test_batch, seeds[1], horizon, dtf, phys,
                                  ic=ldsv.IC_SHEAR_LAYER, progress=log,
                                  ic_resolutions=tuple(N for N in sweep if N != n))
    t_lab = time.perf_counter() - t0
    log("shear labels ready (%.1f s)" % t_lab)
    net = init_network(seed=0)
    st = ldsv.Solver(n, n, train_batch * windows)
    prm = ldsv.params(dt=dtc, k_c=1, fallback_enable=0, **phys)
    t_tr0 = time.perf_counter()
    hist = train(st, net, lab_tr, prm, iters=iters, unroll=unroll, checkpoint_every=8, lr=lr,
                 progress=log, log_every=100, windows=windows)
    st.close()
    t_train = time.perf_counter() - t_tr0
    log("shear model trained (%.1f s)" % (time.perf_counter() - t0))
    se = ldsv.Solver(n, n, test_batch)
    ev = evaluate(se, prm, lab_te, horizon, net=net)
    ev_plain = evaluate(se, prm, lab_te, horizon)
    se.close()
    hs = horizon * dtc
    spread = {"learned_%d" % n: t09_summary(ev["t09"], hs),
              "plain_%d" % n: t09_summary(ev_plain["t09"], hs)}
    for N in sweep:
        if N == n:
            continue
        pcc, _ = plain_sweep_pcc(N, n, ics[N], lab_te, dtc, phys, horizon)
        spread["plain_%d" % N] = t09_summary(first_drop(pcc.cpu(), dtc), hs)
        log("shear plain %d: T_0.9 = %.3f" % (N, spread["plain_%d" % N]["mean"]))
    t09 = {k: v["mean"] for k, v in spread.items()}
    target = t09["learned_%d" % n]
    match = fine_n
    for N in sorted(sweep):
        if t09["plain_%d" % N] >= target:
            match = N
            break
    cs_l, st_l, ms_l = throughput(n, speed_batch, prm, speed_steps, net=net,
                                  ic=ldsv.IC_SHEAR_LAYER)
    pm = ldsv.params(dt=dtc * n / match, **phys)
    cs_p, st_p, ms_p = throughput(match, speed_batch, pm, max(5, speed_steps * n // match),
                                  ic=ldsv.IC_SHEAR_LAYER)
    out = {"workload": "shear layers u = tanh((y - pi/2)/delta), -tanh((y - 3pi/2)/delta), "
                       "delta = 1/30, v = 0.05 sin 2x + divergence-free noise (rms 1e-3), "
                       "nu = 2e-4; learned %d^2 trained on %d^2 plain FV down-sampled %dx"
                       % (n, fine_n, r),
           "dt_fine": dtf, "dt_coarse": dtc, "horizon_steps": horizon, "horizon_s": hs,
           "t09_s": t09, "t09_spread": spread, "test_trajectories": test_batch,
           "test_trajectories_note": "%d held-out trajectories of the %d of the configuration "
                                     "(the fine %d^2 reference of all %d would take minutes of "
                                     "the bench); throughput is timed at batch %d"
                                     % (test_batch, speed_batch, fine_n, speed_batch,
                                        speed_batch),
           "training": {"trajectories": train_batch, "coarse_steps": train_steps,
                        "iters": iters, "unroll": unroll, "windows_per_iter": windows,
                        "lr": lr, "seconds": t_train, "labels_seconds": t_lab},
           "initial_train_loss": hist[0][1], "final_train_loss": hist[-1][1],
           "fallbacks": ev["fallbacks"],
           "mse_at_horizon": {"learned": ev["mse"][-1].item(),
                              "plain_%d" % n: ev_plain["mse"][-1].item()},
           "learned": {"n": n, "batch": speed_batch, "cell_steps_per_s": cs_l,
                       "sim_time_per_s": st_l, "ms_per_step": ms_l},
           "plain_match": {"n": match, "batch": speed_batch, "cell_steps_per_s": cs_p,
                           "sim_time_per_s": st_p, "ms_per_step": ms_p,
                           "note": ("the fine reference resolution itself" if match == fine_n
                                    else "coarsest plain resolution with mean T_0.9 >= the "
                                         "learned solver's")},
           "sim_time_speedup_at_equal_corr": st_l / st_p}
    log("shear corr done (%.1f s)" % (time.perf_counter() - t0))
    return out


def init_network(seed=0, last_scale=1e-3):
    """He-normal 3x3 kernels and zero biases, the last layer scaled by
    last_scale so that the learned correction starts small (Sec. 3.4: the
    learnable kernel starts from small random values)."""
    g = torch.Generator().manual_seed(seed)
    layers = ldsv.LAYERS
    ws, bs = [], []
    for li, (ci, co) in enumerate(layers):
        w = torch.randn(co, ci, 3, 3, generator=g) * math.sqrt(2.0 / (9 * ci))
        if li == len(layers) - 1:
            w = w * last_scale
        ws.append(w)
        bs.append(torch.zeros(co))
    return ldsv.NetParams(ws, bs)


def init_fno(width, layers, modes, n_in, n_out, g, out_scale=1e-2):
    """FNO parameters (the paper's frequency operator): complex spectral
    weights of scale 1/width^2 (Li et al.'s initialisation), pointwise
    weights N(0, 1/width), lift N(0, 1/n_in), a projection scaled by
    out_scale so the operator's first contribution is small, zero biases."""
    sc = 1.0 / (width * width)
    spec = [(torch.randn(2 * modes, modes, width, width, generator=g) * sc,
             torch.randn(2 * modes, modes, width, width, generator=g) * sc)
            for _ in range(layers)]
    return ldsv.FnoParams(torch.randn(width, n_in, generator=g) / math.sqrt(n_in),
                          torch.zeros(width), spec,
                          torch.randn(layers, width, width, generator=g) / math.sqrt(width),
                          torch.zeros(layers, width),
                          torch.randn(n_out, width, generator=g) / math.sqrt(width) * out_scale,
                          torch.zeros(n_out))


def init_fluxblock(seed=0, layers=6, modes=32, width=16, tc_kc=0, tc_sizes=(4, 32, 8)):
    """The paper's flux block with small random uniform kernels ("initialised
    with minor random values", Sec. 3.4) and two FNOs (Table S3 sizes; the
    forced-flow ones by default); with tc_kc > 0 also the temporal
    correction FNO over tc_kc states.  Returns (FluxNetParams, tc or None)."""
    g = torch.Generator().manual_seed(seed)
    w = torch.randn(2, 4, 20, generator=g) * 1e-2
    net = ldsv.FluxNetParams(w, init_fno(width, layers, modes, 2, 4, g),
                             init_fno(width, layers, modes, 2, 4, g))
    tc = None
    if tc_kc:
        tl, tm, tw = tc_sizes
        tc = init_fno(tw, tl, tm, 2 * tc_kc, 2, g)
    return net, tc


def fluxblock_model_rollout(solver, prm, net, tc, u0, v0, nsteps):
    """States u_1 .. u_nsteps [T, B, Ny, Nx] of the paper's model: the flux
    block every step and, with tc, the temporal correction every prm.k_c
    steps (Eq. 2)."""
    kc = prm.k_c
    tu = torch.empty((nsteps,) + tuple(u0.shape), dtype=u0.dtype, device=u0.device)
    tv = torch.empty_like(tu)
    states = [(u0.contiguous(), v0.contiguous())]
    for k in range(1, nsteps + 1):
        if tc is None:
            solver.fluxblock_step(prm, net, *states[-1], out=(tu[k - 1], tv[k - 1]))
        else:
            hu, hv = _history(states, k, kc)
            solver.fluxblock_tc_step(prm, net, tc, hu, hv, k, out=(tu[k - 1], tv[k - 1]))
        states.append((tu[k - 1], tv[k - 1]))
    return tu, tv


def fluxblock_throughput(n, B, prm, net, tc, steps, warmup=3, lx=2 * math.pi):
    """(cell-steps/s, sim-time/s per trajectory, ms/step) of the paper's model
    at n x n, batch B, device-resident state (history ring of k_c + 1)."""
    s = ldsv.Solver(n, n, B, lx=lx, ly=lx)
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=7)
    kc = prm.k_c
    ring = [(u.clone(), v.clone()) for _ in range(kc + 1)]

    def run(k0, k):
        for j in range(k0, k0 + k):
            i = j % (kc + 1)
            src = [(i - kc + q) % (kc + 1) for q in range(kc)]
            if tc is None:
                s.fluxblock_step(prm, net, *ring[src[-1]], out=ring[i])
            else:
                s.fluxblock_tc_step(prm, net, tc, [ring[q][0] for q in src],
                                    [ring[q][1] for q in src], j, out=ring[i])
    run(kc, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(kc + warmup, steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.close()
    return n * n * B * steps / t, prm.dt * steps / t, 1e3 * t / steps
