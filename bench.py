"""Benchmark of the FV hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (decaying 2D NS, the paper's decaying flow at 512^2): 512 x 512
MAC cells, batch 16 trajectories, FP32, nu = 1e-3, GRF initial vorticity
peaked at k = 4 with unit energy, RK4 with a spectral projection after every
sub-step, dt = 8.76e-4.  A step is one full RK4 time step of the batch (4
fused stage kernels and 4 three-pass projections), launched through the C
ABI on the current stream with the state already resident in HBM.  Prints
one JSON line on stdout; progress goes to stderr.

The line also carries
* roofline: the dominant kernel class's average launch duration (HIP events
  recorded around every launch on its stream, in a second pass of the same K
  steps right after the timed one, since the events themselves add gaps
  between launches), its algorithmic bytes per launch, achieved GB/s against
  8 TB/s;
* cpu_baseline: the FP64 CPU oracle timed on this host on a bounded sample
  of the same workload (the full batch, as many steps as fit in ~10 s), and
  the GPU step's error against it;
* fp64_errors: the learned step, the network output and the 200-step Burgers
  run against the FP64 oracle;
* learned: the learned step (64^2, batch 64, BF16 CNN on MFMA);
* streaming: the plain step at 1024^2 x 128 (a state far larger than the
  last-level cache) with its own roofline record;
* burgers64: microseconds per step of the FP64 Burgers configuration,
  eager and as a captured HIP graph;
* training: one Adam iteration of the 128^2 learned solver unrolled 32 steps
  through the hand-written adjoint (checkpoints every 8);
* corr_shear: the same comparison on the shear-layer flow (nu = 2e-4):
  learned 128^2 against plain FV at 128, 256, 512 and the 1024^2 fine solve,
  over 4096 coarse steps, throughput at batch 128;
* corr: the accuracy-matched comparison of the metric on forced Kolmogorov
  flow: the learned 64^2 solver is trained (Adam through the hand-written
  adjoint) on labels from 1024^2 plain FV down-sampled 16x; on held-out seeds
  the time until the vorticity correlation with the down-sampled 1024^2
  reference drops below 0.9 is measured for the learned solver and for plain
  FV at 64, 128, 256, 512; the coarsest plain resolution that lasts as long
  is timed at the same batch, giving the sim-time/s ratio at equal
  correlation.
"""
import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0

# algorithmic bytes per cell and launch (FP32, plain stencil), averaged over
# the four RK4 stage variants for the stage kernel
STAGE_BYTES = {0: (24 + 40 + 40 + 32) / 4.0, 1: 12.0, 2: 8.0, 3: 20.0}
CLASS_NAMES = {0: "k_stage_mac (fused residual + RK stage)", 1: "k_div_rowfft",
               2: "k_col_solve", 3: "k_rowifft_grad"}
KERNEL_KEYS = {0: "k_stage_mac", 1: "k_div_rowfft", 2: "k_col_solve", 3: "k_rowifft_grad"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(HERE, "profiles", "hbm_traffic_decaying512.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes, copy-calibrated), or None when the
    summary is missing or the kernel's sources changed since it was taken
    (the summary records a hash of those sources)."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)["kernels"][kernel]
    except (OSError, IndexError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["sources_sha256_16"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def _rel_l2(a, b):
    a = a.double().cpu()
    b = b.double().cpu()
    return float((a - b).norm() / b.norm().clamp_min(1e-300))


def cpu_baseline(w, u0, v0, u1_gpu, v1_gpu, budget_s=10.0):
    """The oracle as it stands on a bounded sample of the same workload: all
    16 trajectories at 512^2, RK4 steps until about budget_s of CPU time.
    The oracle's first step also gives the GPU step's error against FP64
    (same initial state)."""
    import torch
    from oracle import fv, timestep
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    u = u0.double().cpu()
    v = v0.double().cpu()
    prm = fv.grid_params(w["nx"], w["ny"], nu=w["nu"], dt=w["dt"])
    steps = 0
    err = None
    t0 = time.perf_counter()
    while True:
        u, v = timestep.fv_step(u, v, prm)
        steps += 1
        if steps == 1:
            t_err = time.perf_counter()
            err = max(_rel_l2(u1_gpu, u), _rel_l2(v1_gpu, v))
            t0 += time.perf_counter() - t_err
        t = time.perf_counter() - t0
        if t >= budget_s:
            break
    cells = w["nx"] * w["ny"] * u.shape[0] * steps
    rec = {"value": cells / t, "unit": "cell-steps/s", "cores": torch.get_num_threads(),
           "kind": "oracle", "sample": "%d RK4 steps of all 16 trajectories of the 512^2 "
           "workload (%.1f s, FP64 torch CPU)" % (steps, t),
           "gpu_step_rel_l2_vs_fp64": err}
    # the same oracle on one thread, on one trajectory of the workload
    torch.set_num_threads(1)
    u1 = u0[:1].double().cpu()
    v1 = v0[:1].double().cpu()
    steps1 = 0
    t0 = time.perf_counter()
    while True:
        u1, v1 = timestep.fv_step(u1, v1, prm)
        steps1 += 1
        t1 = time.perf_counter() - t0
        if t1 >= budget_s / 3:
            break
    torch.set_num_threads(cores)
    rec["one_thread"] = {"value": w["nx"] * w["ny"] * steps1 / t1, "unit": "cell-steps/s",
                         "cores": 1, "sample": "%d RK4 steps of trajectory 0 of the 512^2 "
                         "workload (%.1f s, FP64 torch CPU)" % (steps1, t1)}
    return rec


def copy_reference(nbytes):
    """Achieved rates of plain device-to-device copies (read + write) and
    fills (write) measured with HIP events over 20 repeats after warm-up:
    once with the dominant kernel's bytes per launch (the same working set,
    which like the kernel's own data can stay in the 256 MB last-level
    cache between repeats) and once with 1 GiB per buffer (beyond that
    cache: HBM).  The practical ceilings for mixed read/write traffic,
    reported beside the nominal 8 TB/s."""
    import torch
    out = {}
    for key, n in (("same_bytes", max(1 << 20, int(nbytes // 8))), ("1GiB", 1 << 28)):
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        rec = {"bytes_moved_by_copy": 8 * n}
        for name, fn, moved in (("copy_GBs", lambda: b.copy_(a), 8 * n),
                                ("fill_GBs", lambda: b.fill_(2.0), 4 * n)):
            for _ in range(3):
                fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                fn()
            e1.record()
            torch.cuda.synchronize()
            rec[name] = moved / (e0.elapsed_time(e1) / 20 * 1e-3) / 1e9
        out[key] = rec
        del a, b
    return out


def oracle_timed(call, cells_per_call, what, budget_s=2.0):
    """The oracle as it stands, timed on the host's cores on a bounded sample
    of a record's workload (for the records beside the headline one): `call`
    runs one oracle step of the sample, repeated until about budget_s."""
    import torch
    torch.set_num_threads(len(os.sched_getaffinity(0)))
    calls = 0
    t0 = time.perf_counter()
    while True:
        call()
        calls += 1
        t = time.perf_counter() - t0
        if t >= budget_s:
            break
    return {"value": cells_per_call * calls / t, "unit": "cell-steps/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": "%d call(s) of %s (%.1f s, FP64 torch CPU)" % (calls, what, t)}


def fp64_errors():
    """Errors of the other results against the FP64 oracle (the oracle is run
    here as the reference, outside every timed region): the learned step of the
    forced-flow workload (trajectory 0 of the batch of 64, bench network),
    its network output, the flux-block step of the same workload, and 200
    FP64 Burgers steps."""
    import torch
    import synthetic_inputs as si
    from oracle import fv as ofv, ic as oic, learned as olearned
    from oracle import timestep as ots
    from paper_2507_01975_amd import ldsv
    out = {}
    w = si.WORKLOADS["kolmogorov64"]
    n, B = w["nx"], w["batch"]
    s = ldsv.Solver(n, n, B)
    ws, bs = si.cnn_weights(0, ldsv.LAYERS)
    net = ldsv.NetParams([torch.tensor(x) for x in ws], [torch.tensor(x) for x in bs])
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=200)
    kw = dict(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"], forcing_k=w["forcing_k"],
              drag=w["drag"])
    uo, vo, no = s.learned_fv_step(ldsv.params(k_c=1, **kw), net, u, v, 1, want_net_out=True)
    prm = ofv.grid_params(n, n, k_c=1, **kw)
    wb = [x.double().cpu() for x in net.bf16_weights()]
    bb = [x.double().cpu() for x in net.b]
    u0, v0 = u[:1].double().cpu(), v[:1].double().cpu()
    eu, ev, eo = olearned.learned_fv_step(u0, v0, prm, wb, bb, 1, bf16=False)
    out["learned_step_rel_l2_vs_fp64"] = max(_rel_l2(uo[:1], eu), _rel_l2(vo[:1], ev))
    out["network_output_rel_l2_vs_fp64"] = _rel_l2(no[:1], eo)
    # with the derivative-stencil network beside it (trajectory 0)
    dws, dbs = si.cnn_weights(1, ldsv.LAYERS)
    dnet = ldsv.NetParams([torch.tensor(x) for x in dws], [torch.tensor(x) for x in dbs])
    du, dv = s.learned_d_fv_step(ldsv.params(k_c=1, **kw), net, dnet, u, v, 1)
    dwb = [x.double().cpu() for x in dnet.bf16_weights()]
    dbb = [x.double().cpu() for x in dnet.b]
    eu, ev, _ = olearned.learned_fv_step(u0, v0, prm, wb, bb, 1, bf16=False, dnet=(dwb, dbb))
    out["learned_deriv_step_rel_l2_vs_fp64"] = max(_rel_l2(du[:1], eu), _rel_l2(dv[:1], ev))
    # the flux-block model step of the same workload (trajectory 0)
    from oracle import fluxblock as ofb, fno as ofno
    fnet, (fw, a_i, a_d) = _fluxblock_net("forced", ldsv)
    fu, fv_ = s.fluxblock_step(ldsv.params(**kw), fnet, u, v)
    fparams = {"wi": torch.tensor(fw[0]), "wd": torch.tensor(fw[1]),
               "fno_i": ofno.from_arrays(a_i), "fno_d": ofno.from_arrays(a_d)}
    ru, rv = ofb.fluxblock_step(u0, v0, ofv.grid_params(n, n, **kw), fparams)
    out["fluxblock_step_rel_l2_vs_fp64"] = max(_rel_l2(fu[:1], ru), _rel_l2(fv_[:1], rv))
    s.close()
    wb_ = si.WORKLOADS["burgers64"]
    nb = wb_["nx"]
    s = ldsv.Solver(nb, nb, 1, dtype=torch.float64, layout=ldsv.COLLOCATED)
    gu, gv = s.init_state(ldsv.IC_FOURIER_MODES, seed=0)
    dt = s.cfl_dt(gu, gv, wb_["cfl"])
    gu, gv = s.fv_step(ldsv.params(nu=wb_["nu"], dt=dt, rk=ldsv.SSPRK3), gu, gv,
                       nsteps=wb_["steps"])
    bu, bv = oic.fourier_modes(1, nb, nb, 2 * math.pi, 2 * math.pi, seed=0)
    bprm = ofv.grid_params(nb, nb, nu=wb_["nu"], rk=ots.SSPRK3, layout=ots.COLLOCATED)
    bprm["dt"] = dt
    bu, bv = ots.fv_step(bu, bv, bprm, nsteps=wb_["steps"])
    out["burgers64_200_steps_fp64_rel_l2"] = max(_rel_l2(gu, bu), _rel_l2(gv, bv))
    s.close()
    return out


def learned_block(steps, warmup):
    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv
    w = si.WORKLOADS["kolmogorov64"]
    n, B = w["nx"], w["batch"]
    s = ldsv.Solver(n, n, B)
    ws, bs = si.cnn_weights(0, ldsv.LAYERS)
    net = ldsv.NetParams([torch.tensor(x) for x in ws], [torch.tensor(x) for x in bs])
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=200)
    prm = ldsv.params(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                      forcing_k=w["forcing_k"], drag=w["drag"], k_c=1)
    try:
        for k in range(warmup):
            s.learned_fv_step(prm, net, u, v, k + 1, out=(u, v))
    except ldsv.LdsvError as e:
        return {"status": "unavailable: %s" % e}
    # the rollout with its guard and plain-FV fallback on the device (the
    # way the learned solver runs), one snapshot at the end
    gprm = ldsv.params(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                       forcing_k=w["forcing_k"], drag=w["drag"], k_c=1, fallback_enable=1)
    flags = torch.zeros(B, dtype=torch.int32, device="cuda")

    def guarded():
        s.rollout(gprm, u, v, steps, save_every=steps, net=net, fallback_flags=flags)

    def bare():  # bare learned steps, for the guard's cost
        for k in range(steps):
            s.learned_fv_step(prm, net, u, v, k + 1, out=(u, v))

    def timed(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # both paths twice, alternating after the warm-up (the first timed region
    # of a process can run while the clocks still rise): the faster of each
    guarded()
    torch.cuda.synchronize()
    t, t_bare = float("inf"), float("inf")
    for _ in range(2):
        t = min(t, timed(guarded))
        t_bare = min(t_bare, timed(bare))
    # kernel durations from a second, instrumented pass (per-launch events
    # add several microseconds between launches, so the throughput above is
    # timed without them)
    s.timer_enable(True)
    for k in range(steps):
        s.learned_fv_step(prm, net, u, v, k + 1, out=(u, v))
    torch.cuda.synchronize()
    conv_ms, conv_n = s.timer_read(ldsv.TIMER_CONV)
    s.timer_enable(False)
    cells = n * n * B
    out = {"workload": "kolmogorov64 learned rollout (64^2, batch 64, 6-layer 64-channel BF16 "
                       "CNN, guard and plain-FV fallback on the device)",
           "cell_steps_per_s": cells * steps / t, "ms_per_step": 1e3 * t / steps,
           "sim_time_per_s": w["dt"] * steps / t,
           "bare_steps_ms_per_step": 1e3 * t_bare / steps,
           "guard_overhead": t / t_bare - 1.0, "fallbacks": int(flags.sum())}
    if conv_n:
        # the six layers on MFMA: 2 * 9 * 64 * Cout FLOP per cell for layers
        # 2..6, 2 * 18 * 64 for layer 1 (computed inside layer 2's launch)
        flop = (2 * 9 * 64 * (64 * 4 + 66) + 2 * 18 * 64) * cells
        per_launch_ms = conv_ms / conv_n
        launches_per_step = conv_n / steps
        out["mfma_conv"] = {"tflops": flop / launches_per_step / (per_launch_ms * 1e-3) / 1e12,
                            "peak": BF16_PEAK_TFLOPS, "avg_launch_ms": per_launch_ms}
        out["mfma_conv"]["frac"] = out["mfma_conv"]["tflops"] / BF16_PEAK_TFLOPS
    from oracle import fv as ofv, learned as olearned
    wb = [x.double().cpu() for x in net.bf16_weights()]
    bb = [x.double().cpu() for x in net.b]
    us, vs = u[:4].double().cpu(), v[:4].double().cpu()
    oprm = ofv.grid_params(n, n, k_c=1, nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                           forcing_k=w["forcing_k"], drag=w["drag"])
    out["cpu_oracle"] = oracle_timed(lambda: olearned.learned_fv_step(us, vs, oprm, wb, bb, 1),
                                     n * n * 4, "one learned step of 4 of the 64 trajectories")
    return out


def learned_deriv_block(steps, warmup):
    """The learned step with per-cell learned derivative stencils (the m = d
    operator in per-cell form, Sec. 3.4): a second network of the same shape
    beside the coefficient network, on the forced 64^2 workload (batch 64).
    The stage kernel then reads 64 BF16 interpolation and 64 BF16 derivative
    values per cell: 256 B/cell on top of the plain stage's 34 B/cell (and
    the correction's 8 B/cell in the last stage, 2 B/cell averaged)."""
    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv
    w = si.WORKLOADS["kolmogorov64"]
    n, B = w["nx"], w["batch"]
    s = ldsv.Solver(n, n, B)
    nets = []
    for seed in (0, 1):
        ws, bs = si.cnn_weights(seed, ldsv.LAYERS)
        nets.append(ldsv.NetParams([torch.tensor(x) for x in ws], [torch.tensor(x) for x in bs]))
    net, dnet = nets
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=200)
    prm = ldsv.params(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                      forcing_k=w["forcing_k"], drag=w["drag"], k_c=1)
    for k in range(warmup):
        s.learned_d_fv_step(prm, net, dnet, u, v, k + 1, out=(u, v))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        s.learned_d_fv_step(prm, net, dnet, u, v, k + 1, out=(u, v))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.timer_enable(True)
    for k in range(steps):
        s.learned_d_fv_step(prm, net, dnet, u, v, k + 1, out=(u, v))
    torch.cuda.synchronize()
    st_ms, st_n = s.timer_read(ldsv.TIMER_STAGE)
    conv_ms, conv_n = s.timer_read(ldsv.TIMER_CONV)
    s.timer_enable(False)
    diag = s.diagnostics(u, v).cpu()
    cells = n * n * B
    out = {"workload": "kolmogorov64 learned step with learned derivative stencils (64^2, "
                       "batch 64, two 6-layer 64-channel BF16 CNNs)",
           "cell_steps_per_s": cells * steps / t, "ms_per_step": 1e3 * t / steps,
           "sim_time_per_s": w["dt"] * steps / t, "finite": bool((diag[:, 5] == 1).all())}
    if st_n:
        alg = (34 + 256 + 2) * cells
        us = 1e3 * st_ms / st_n
        out["stage_hbm"] = {"kernel": "k_stage_mac<float, 5, ...> (fused residual + RK stage)", "avg_launch_us": us,
                            "alg_bytes_per_launch": alg, "achieved": alg / (us * 1e-6) / 1e9,
                            "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        out["stage_hbm"]["frac"] = out["stage_hbm"]["achieved"] / HBM_PEAK_GBS
    if conv_n:
        flop = 2 * (2 * 9 * 64 * (64 * 4 + 66) + 2 * 18 * 64) * cells
        per_launch_ms = conv_ms / conv_n
        out["mfma_conv"] = {"tflops": flop / (conv_n / steps) / (per_launch_ms * 1e-3) / 1e12,
                            "peak": BF16_PEAK_TFLOPS, "avg_launch_ms": per_launch_ms}
        out["mfma_conv"]["frac"] = out["mfma_conv"]["tflops"] / BF16_PEAK_TFLOPS
    from oracle import fv as ofv, learned as olearned
    wts = [([x.double().cpu() for x in m.bf16_weights()], [x.double().cpu() for x in m.b])
           for m in (net, dnet)]
    us, vs = u[:4].double().cpu(), v[:4].double().cpu()
    oprm = ofv.grid_params(n, n, k_c=1, nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                           forcing_k=w["forcing_k"], drag=w["drag"])
    out["cpu_oracle"] = oracle_timed(
        lambda: olearned.learned_fv_step(us, vs, oprm, wts[0][0], wts[0][1], 1, dnet=wts[1]),
        n * n * 4, "one two-network learned step of 4 of the 64 trajectories")
    s.close()
    return out


def _fluxblock_net(cfg, ldsv, seed=0):
    import numpy as np
    import synthetic_inputs as si
    layers, modes, width = si.FLUXBLOCK_FNO[cfg]
    w = np.stack([si.stencil_weights(seed, 0.01), si.stencil_weights(seed + 1, 0.01)])
    a_i = si.fno_weights(seed + 2, width, layers, modes)
    a_d = si.fno_weights(seed + 3, width, layers, modes)
    net = ldsv.FluxNetParams(w, ldsv.FnoParams.from_arrays(a_i), ldsv.FnoParams.from_arrays(a_d))
    return net, (w, a_i, a_d)


def fluxblock_block(steps, warmup):
    """The paper's own flux block (uniform 5x4 kernels + two FNOs, Sec. 3.4)
    as the learned model of the forced 64^2 configuration (batch 64, FNO: 6
    layers, 32 modes, width 16): throughput and per-class kernel time, and
    the HBM rate of the FNO transform kernels against their algorithmic
    bytes (per layer: the activation read and written once, the retained
    spectrum written and read once)."""
    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv
    w = si.WORKLOADS["kolmogorov64"]
    n, B = w["nx"], w["batch"]
    layers, modes, width = si.FLUXBLOCK_FNO["forced"]
    s = ldsv.Solver(n, n, B)
    net, (fw, a_i, a_d) = _fluxblock_net("forced", ldsv)
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=200)
    u2, v2 = torch.empty_like(u), torch.empty_like(v)
    prm = ldsv.params(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                      forcing_k=w["forcing_k"], drag=w["drag"])

    def run(k):
        nonlocal u, v, u2, v2
        for _ in range(k):
            s.fluxblock_step(prm, net, u, v, out=(u2, v2))
            u, v, u2, v2 = u2, v2, u, v
    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.timer_enable(True)
    run(steps)
    torch.cuda.synchronize()
    cls = {c: s.timer_read(c) for c in (ldsv.TIMER_STAGE, ldsv.TIMER_ROWFFT, ldsv.TIMER_COLSOLVE,
                                        ldsv.TIMER_ROWIFFT, ldsv.TIMER_FNO_FFT,
                                        ldsv.TIMER_FNO_MIX, ldsv.TIMER_OTHER)}
    s.timer_enable(False)
    diag = s.diagnostics(u, v).cpu()
    cells = n * n * B
    nm = 2 * modes * modes
    G = 2
    act = G * B * width * n * n * 4
    spec = G * B * width * nm * 8
    # spectral kernels per step: layer 0 reads (u, v) instead of an activation
    fft_bytes = layers * (2 * spec + 2 * act) - act + 2 * B * n * n * 4
    mix_bytes = layers * (2 * spec + G * width * width * nm * 8)
    out = {"workload": "kolmogorov64 flux-block step (64^2, batch 64, uniform 5x4 kernels + "
                       "2 FNOs of 6 layers, 32 modes, width 16)",
           "cell_steps_per_s": cells * steps / t, "ms_per_step": 1e3 * t / steps,
           "sim_time_per_s": w["dt"] * steps / t, "finite": bool((diag[:, 5] == 1).all()),
           "classes_ms_per_step": {k: cls[c][0] / steps for k, c in (
               ("stage", ldsv.TIMER_STAGE), ("project", ldsv.TIMER_COLSOLVE),
               ("fno_fft", ldsv.TIMER_FNO_FFT), ("fno_mix", ldsv.TIMER_FNO_MIX),
               ("fno_proj", ldsv.TIMER_OTHER))}}
    if cls[ldsv.TIMER_FNO_FFT][1]:
        tf = cls[ldsv.TIMER_FNO_FFT][0] * 1e-3 / steps
        out["fno_fft_hbm"] = {"achieved": fft_bytes / tf / 1e9, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": fft_bytes / tf / 1e9 / HBM_PEAK_GBS,
                              "alg_bytes_per_step": fft_bytes}
    if cls[ldsv.TIMER_FNO_MIX][1]:
        tm = cls[ldsv.TIMER_FNO_MIX][0] * 1e-3 / steps
        out["fno_mix_hbm"] = {"achieved": mix_bytes / tm / 1e9, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": mix_bytes / tm / 1e9 / HBM_PEAK_GBS,
                              "alg_bytes_per_step": mix_bytes}
    # the complete model: the same flux block plus the temporal correction
    # block every k_c = 4 steps (FNO over the 4 states since the last
    # correction: 4 layers, 32 modes, width 8)
    kc = 4
    tc = ldsv.FnoParams.from_arrays(si.fno_weights(9, 8, 4, 32, n_in=2 * kc, n_out=2))
    prm_tc = ldsv.params(nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                         forcing_k=w["forcing_k"], drag=w["drag"], k_c=kc)
    hu = [u.clone() for _ in range(kc + 1)]
    hv = [v.clone() for _ in range(kc + 1)]

    def run_tc(k0, k):
        for j in range(k0, k0 + k):
            i = j % (kc + 1)
            src = [(i - kc + q) % (kc + 1) for q in range(kc)]
            s.fluxblock_tc_step(prm_tc, net, tc, [hu[q] for q in src], [hv[q] for q in src], j,
                                out=(hu[i], hv[i]))
    run_tc(kc, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_tc(kc + warmup, steps)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out["complete_model"] = {"k_c": kc, "tc_fno": "4 layers, 32 modes, width 8",
                             "ms_per_step": 1e3 * t / steps,
                             "cell_steps_per_s": cells * steps / t}
    from oracle import fluxblock as ofb, fno as ofno, fv as ofv
    fparams = {"wi": torch.tensor(fw[0]), "wd": torch.tensor(fw[1]),
               "fno_i": ofno.from_arrays(a_i), "fno_d": ofno.from_arrays(a_d)}
    us, vs = u[:4].double().cpu(), v[:4].double().cpu()
    oprm = ofv.grid_params(n, n, nu=w["nu"], dt=w["dt"], forcing_amp=w["forcing_amp"],
                           forcing_k=w["forcing_k"], drag=w["drag"])
    out["cpu_oracle"] = oracle_timed(lambda: ofb.fluxblock_step(us, vs, oprm, fparams),
                                     n * n * 4, "one flux-block step of 4 of the 64 trajectories")
    return out


def shear_scalar_block(steps=10, warmup=2):
    """The shear-flow system with a passive scalar at the paper's fine
    resolution (2048 x 1024 on [0, 8] x [0, 4], batch 8, FP32): the plain
    DNS step of velocity and scalar together."""
    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv
    w = si.WORKLOADS["shear_scalar"]
    nx, ny, B = w["nx"], w["ny"], w["batch"]
    s = ldsv.Solver(nx, ny, B, lx=w["lx"], ly=w["ly"])
    u, v = s.init_state(ldsv.IC_SHEAR_LAYER, seed=1000, delta=w["delta"])
    c = s.init_scalar(delta=w["delta"])
    prm = ldsv.params(nu=w["nu"], dt=w["dt"])
    tot0 = c.double().sum().item()
    s.fv_step_scalar(prm, w["diffusivity"], u, v, c, nsteps=warmup, out=(u, v, c))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.fv_step_scalar(prm, w["diffusivity"], u, v, c, nsteps=steps, out=(u, v, c))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.timer_enable(True)
    s.fv_step_scalar(prm, w["diffusivity"], u, v, c, nsteps=steps, out=(u, v, c))
    torch.cuda.synchronize()
    sc_ms, sc_n = s.timer_read(ldsv.TIMER_OTHER)
    st_ms, st_n = s.timer_read(ldsv.TIMER_STAGE)
    s.timer_enable(False)
    cells = nx * ny * B
    # scalar stage: s_s, u_s, v_s, s_n, acc read, out and acc written (28 B/cell
    # in the middle stages, averaged over the four like the velocity's)
    sc_bytes = (16 + 28 + 28 + 24) / 4 * cells
    out = {"workload": "shear_scalar fine DNS (2048 x 1024 on [0,8] x [0,4], batch 8, FP32, "
                       "velocity + passive scalar, RK4 + projection per stage)",
           "cell_steps_per_s": cells * steps / t, "ms_per_step": 1e3 * t / steps,
           "scalar_total_rel_change": abs(c.double().sum().item() - tot0) / abs(tot0)}
    if sc_n:
        out["scalar_stage"] = {"avg_launch_us": 1e3 * sc_ms / sc_n,
                               "achieved_GBs": sc_bytes / (sc_ms * 1e-3 / sc_n) / 1e9,
                               "frac": sc_bytes / (sc_ms * 1e-3 / sc_n) / 1e9 / HBM_PEAK_GBS}
    if st_n:
        out["velocity_stage_avg_launch_us"] = 1e3 * st_ms / st_n
    from oracle import fv as ofv, scalar as oscalar
    us, vs, cs = u[:1].double().cpu(), v[:1].double().cpu(), c[:1].double().cpu()
    oprm = ofv.grid_params(nx, ny, lx=w["lx"], ly=w["ly"], nu=w["nu"], dt=w["dt"],
                           diffusivity=w["diffusivity"])
    out["cpu_oracle"] = oracle_timed(lambda: oscalar.fv_step_scalar(us, vs, cs, oprm),
                                     nx * ny, "one step of velocity and scalar of 1 of the 8 "
                                     "trajectories", budget_s=1.0)
    s.close()
    return out


def burgers_block(repeats=7):
    """The 2D viscous Burgers configuration (64^2, FP64, collocated, SSP-RK3,
    dt from CFL 0.5, 200 steps): microseconds per step, eager launches and a
    captured HIP graph of the whole 200-step call (median of `repeats`).  The
    state is 64 KB, so this is launch latency, not bandwidth."""
    import statistics
    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv
    w = si.WORKLOADS["burgers64"]
    n, steps = w["nx"], w["steps"]
    s = ldsv.Solver(n, n, 1, dtype=torch.float64, layout=ldsv.COLLOCATED)
    u0, v0 = s.init_state(ldsv.IC_FOURIER_MODES, seed=0)
    prm = ldsv.params(nu=w["nu"], dt=s.cfl_dt(u0, v0, w["cfl"]), rk=ldsv.SSPRK3)
    u, v = torch.empty_like(u0), torch.empty_like(v0)
    s.fv_step(prm, u0, v0, nsteps=steps, out=(u, v))
    torch.cuda.synchronize()
    ref = (u.clone(), v.clone())
    eager = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        s.fv_step(prm, u0, v0, nsteps=steps, out=(u, v))
        torch.cuda.synchronize()
        eager.append(time.perf_counter() - t0)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.fv_step(prm, u0, v0, nsteps=steps, out=(u, v))
    torch.cuda.synchronize()
    graph, same = [], True
    for _ in range(repeats):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        graph.append(time.perf_counter() - t0)
        same = same and torch.equal(u, ref[0]) and torch.equal(v, ref[1])
    from oracle import fv as ofv, timestep as ots
    bu, bv = u0.double().cpu(), v0.double().cpu()
    bprm = ofv.grid_params(n, n, nu=w["nu"], rk=ots.SSPRK3, layout=ots.COLLOCATED, dt=prm.dt)
    orc = oracle_timed(lambda: ots.fv_step(bu, bv, bprm, nsteps=20), n * n * 20,
                       "20 SSP-RK3 steps of the 64^2 state")
    orc["us_per_step"] = 1e6 * n * n / orc["value"]
    return {"cpu_oracle": orc,
            "workload": "burgers64 (64^2, FP64, collocated, SSP-RK3, 200 steps)",
            "us_per_step_eager": 1e6 * statistics.median(eager) / steps,
            "us_per_step_graph": 1e6 * statistics.median(graph) / steps,
            "graph_replays_match_eager": bool(same)}


def streaming_block(steps=10, warmup=2):
    """The plain step at a shape whose state does not fit the 256 MB
    last-level cache: 1024^2 x 128 trajectories (the fine grid of the shear
    configuration, 537 MB per field), FP32, RK4 with a projection per
    sub-step.  Throughput, then per-class event-timed launch durations and
    the dominant class against the HBM roofline."""
    import torch
    from paper_2507_01975_amd import ldsv
    n, B = 1024, 128
    s = ldsv.Solver(n, n, B)
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=0)
    prm = ldsv.params(nu=2e-4, dt=0.1 * 2 * math.pi / n)
    for _ in range(warmup):
        s.fv_step(prm, u, v, out=(u, v))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.fv_step(prm, u, v, out=(u, v))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.timer_enable(True)
    for _ in range(steps):
        s.fv_step(prm, u, v, out=(u, v))
    torch.cuda.synchronize()
    cls = {c: s.timer_read(c) for c in range(4)}
    s.timer_enable(False)
    cells = n * n * B
    dom = max(cls, key=lambda c: cls[c][0])
    avg_s = cls[dom][0] * 1e-3 / cls[dom][1]
    per_class = {}
    for c in cls:
        a = cls[c][0] * 1e-3 / cls[c][1]
        per_class[CLASS_NAMES[c]] = {"avg_launch_us": a * 1e6,
                                     "GB_per_s": STAGE_BYTES[c] * cells / a / 1e9}
    s.close()
    return {"workload": "1024^2 x 128 trajectories, FP32, RK4 + projection per sub-step",
            "cell_steps_per_s": cells * steps / t, "ms_per_step": 1e3 * t / steps,
            "roofline": {"bound": "hbm", "kernel": CLASS_NAMES[dom],
                         "achieved": STAGE_BYTES[dom] * cells / avg_s / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": STAGE_BYTES[dom] * cells / avg_s / 1e9 / HBM_PEAK_GBS},
            "classes": per_class}


def training_block(iters=5):
    """One training iteration of the decaying-flow configuration: the 128^2
    learned solver, batch 8, unrolled 32 steps with checkpoints every 8,
    forward + hand-written backward + Adam (labels: a plain-FV rollout of the
    same batch stands in for the down-sampled fine solution)."""
    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv, train as T
    w = si.WORKLOADS["decaying128_train"]
    n, B, unroll = w["nx"], w["batch"], w["unroll"]
    s = ldsv.Solver(n, n, B)
    prm = ldsv.params(nu=w["nu"], dt=w["dt"], k_c=1, fallback_enable=0)
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=300)
    tu, tv = s.rollout(prm, u, v, unroll + 8)
    lu, lv = torch.cat([u[None], tu]), torch.cat([v[None], tv])
    net = T.init_network(seed=0)
    T.train(s, net, (lu, lv), prm, iters=2, unroll=unroll,
            checkpoint_every=w["checkpoint_every"], log_every=10 ** 9)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T.train(s, net, (lu, lv), prm, iters=iters, unroll=unroll,
            checkpoint_every=w["checkpoint_every"], log_every=10 ** 9)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / iters
    s.close()
    return {"workload": "decaying128_train (128^2, batch 8, unroll 32, checkpoints every 8, "
                        "Adam)", "ms_per_iteration": 1e3 * t,
            "learned_steps_per_s": B * unroll / t}


def fluxblock_training_block(iters=3):
    """One training iteration of the paper's flux-block model on the
    decaying-flow configuration: 128^2, batch 8, FNOs of 4 layers, 16 modes,
    width 8, unrolled 32 steps (states kept, step adjoint backwards, Adam on
    every parameter); a plain-FV rollout stands in for the labels."""
    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv, train as T
    w = si.WORKLOADS["decaying128_train"]
    n, B, unroll = w["nx"], w["batch"], w["unroll"]
    s = ldsv.Solver(n, n, B)
    prm = ldsv.params(nu=w["nu"], dt=w["dt"])
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=300)
    tu, tv = s.rollout(prm, u, v, unroll + 8)
    labels = (torch.cat([u[None], tu]), torch.cat([v[None], tv]))
    net, _ = _fluxblock_net("decaying", ldsv)
    T.train_fluxblock(s, net, labels, prm, iters=1, unroll=unroll, log_every=10 ** 9)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T.train_fluxblock(s, net, labels, prm, iters=iters, unroll=unroll, log_every=10 ** 9)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / iters
    s.close()
    return {"workload": "decaying128_train with the flux-block model (128^2, batch 8, unroll 32, "
                        "FNOs 4 layers / 16 modes / width 8, Adam)", "ms_per_iteration": 1e3 * t,
            "learned_steps_per_s": B * unroll / t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-corr", action="store_true",
                    help="skip the corr>=0.9 comparison (training + resolution sweep, ~2 min)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the streaming-shape (1024^2 x 128) and Burgers latency records")
    ap.add_argument("--learned-only", action="store_true",
                    help="profiling aid: time only the learned 64^2 step and print its record")
    ap.add_argument("--training-only", action="store_true",
                    help="print only the training records (for kernel profiles)")
    ap.add_argument("--fluxblock-only", action="store_true",
                    help="profiling aid: time only the flux-block model (64^2 step, complete "
                    "model, 128^2 training iteration) and print its records")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="profiling aid: one device-to-device copy of this many MiB before the "
                    "timed loop, the known-size kernel that calibrates HBM byte counters")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs the batched step on a single MI355X "
              "(trajectories would shard across GPUs with no communication); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synthetic_inputs as si
    from paper_2507_01975_amd import ldsv

    if a.copy_probe_mib:
        src = torch.ones(a.copy_probe_mib << 18, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d MiB" % a.copy_probe_mib)
        del src, dst
    if a.learned_only:
        print(json.dumps({"learned": learned_block(a.steps, a.warmup),
                          "learned_deriv": learned_deriv_block(a.steps, a.warmup)}), flush=True)
        return
    if a.training_only:
        print(json.dumps({"training": training_block(),
                          "fluxblock_training": fluxblock_training_block()}), flush=True)
        return
    if a.fluxblock_only:
        print(json.dumps({"fluxblock": fluxblock_block(a.steps, a.warmup),
                          "fluxblock_training": fluxblock_training_block()}), flush=True)
        return

    w = si.WORKLOADS["decaying512"]
    n, B = w["nx"], w["batch"]
    log("workload decaying512: %dx%d, batch %d, fp32, rk4 + projection per stage" % (n, n, B))
    s = ldsv.Solver(n, n, B)
    u, v = s.init_state(ldsv.IC_GRF_PEAK, seed=0)
    u0, v0 = u.clone(), v.clone()
    prm = ldsv.params(nu=w["nu"], dt=w["dt"])
    # one step from the initial state, kept for the error against FP64
    u1, v1 = s.fv_step(prm, u0, v0)
    for _ in range(a.warmup):
        s.fv_step(prm, u, v, out=(u, v))
    torch.cuda.synchronize()
    log("warmup done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s.fv_step(prm, u, v, out=(u, v))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    log("timed %d steps in %.3f s" % (a.steps, t))
    # per-kernel durations: the same K steps again with a HIP event pair
    # recorded around every launch on the launch stream (the events add
    # several microseconds between launches, so the throughput above is
    # timed without them)
    s.timer_enable(True)
    t1 = time.perf_counter()
    for _ in range(a.steps):
        s.fv_step(prm, u, v, out=(u, v))
    torch.cuda.synchronize()
    t_inst = time.perf_counter() - t1
    cls = {c: s.timer_read(c) for c in range(4)}
    s.timer_enable(False)
    diag = s.diagnostics(u, v).cpu()
    assert bool((diag[:, 5] == 1).all()), "non-finite state after the timed steps"

    cells = n * n * B
    value = cells * a.steps / t
    dom = max(cls, key=lambda c: cls[c][0])
    ms, cnt = cls[dom]
    avg_s = ms * 1e-3 / cnt
    alg = STAGE_BYTES[dom] * cells
    achieved = alg / avg_s / 1e9
    roof = {"bound": "hbm", "kernel": CLASS_NAMES[dom], "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(KERNEL_KEYS[dom]), "traffic_unit": "bytes per launch",
            "alg_bytes_per_launch": alg, "avg_launch_us": avg_s * 1e6,
            "classes_ms_per_step": {CLASS_NAMES[c]: cls[c][0] / a.steps for c in cls},
            "instrumented_ms_per_step": 1e3 * t_inst / a.steps}
    roof["copy_reference"] = copy_reference(alg)
    roof["frac_of_copy"] = achieved / roof["copy_reference"]["same_bytes"]["copy_GBs"]
    line = {"metric": "cell-steps/s + sim-time/s at corr>=0.9: learned coarse FV vs plain fine FV",
            "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": 1e3 * t / a.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "decaying512", "nx": n, "ny": n, "batch": B, "nu": w["nu"],
                       "dt": w["dt"], "rk": "rk4", "projection": "every sub-step",
                       "ic": "GRF peaked at k=4, unit energy"},
            "sim_time_per_s": w["dt"] * a.steps / t,
            "roofline": roof}
    if not a.no_learned:
        log("learned step")
        line["learned"] = learned_block(max(10, a.steps // 4), 3)
        log("learned step with learned derivative stencils")
        line["learned_deriv"] = learned_deriv_block(max(10, a.steps // 4), 3)
        log("flux-block step")
        line["fluxblock"] = fluxblock_block(max(10, a.steps // 4), 3)
    if not a.no_extra:
        log("streaming shape 1024^2 x 128")
        line["streaming"] = streaming_block()
        log("burgers64 latency")
        line["burgers64"] = burgers_block()
        log("shear flow with a passive scalar, 2048 x 1024")
        line["shear_scalar"] = shear_scalar_block()
        log("training iteration 128^2")
        line["training"] = training_block()
        log("flux-block training iteration 128^2")
        line["fluxblock_training"] = fluxblock_training_block()
    if not a.no_corr:
        log("corr>=0.9 comparison: learned coarse vs plain FV resolution sweep")
        from paper_2507_01975_amd import train as T
        try:
            line["corr"] = T.corr_metric(progress=log)
        except Exception as e:  # report, do not lose the throughput line
            line["corr"] = {"status": "failed: %r" % (e,)}
        log("corr>=0.9 comparison on shear flow: learned 128^2 vs plain FV up to 1024^2")
        try:
            line["corr_shear"] = T.corr_shear(progress=log)
        except Exception as e:
            line["corr_shear"] = {"status": "failed: %r" % (e,)}
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(w, u0, v0, u1, v1)
        log("errors against the FP64 oracle")
        line["fp64_errors"] = fp64_errors()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
