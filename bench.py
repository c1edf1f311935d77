#!/usr/bin/env python3
"""Throughput benchmark of the gfx950 truncated-LJ MD hot path.

Workload (one GPU): single-species LJ fluid, N = 256,000 (FCC 40^3 start),
density 0.8442, T = 1.0 Maxwell-Boltzmann velocities, cutoff 2.5 sigma with
energy shift, skin 0.3, dt = 0.005, NVE velocity Verlet, list rebuilt on
half-skin displacement, space-filling-curve resort every 100 steps; FP32 pair
arithmetic with double-single positions/velocities (the plain FP64 GPU path
is timed on the same workload for comparison). Synthetic seeded inputs.

Metric: particle-steps/s = N * steps / wall time of the timed ljmd_run
(inputs resident in HBM, every rebuild, resort and per-step FP64 observable
reduction included).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s, LJ NVE N=256k on 1 GPU; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the FP32+DS step kernel on this workload, from two
# hardware counter passes (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0, the factors a
# 512 MiB copy reads), valid only for the kernel sources they were taken on.
STEP_KERNEL_SOURCES = ("k_step.hip", "step_common.h", "internal.h")
STEP_KERNEL_TRAFFIC = {
    "sources_sha256": "25fed7b0c7dd77b0ef3176e23e4fc6ca21da4fd1965334f8721c28c6047599e4",
    "fetch_bytes": 2.0 * 53446 * 1024,
    "write_bytes": 1.0 * 16035 * 1024,
}


def step_kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_04210_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Counter-measured bytes per step-kernel launch, or None once the kernel
    sources differ from those the counters were taken on."""
    try:
        if step_kernel_digest() != STEP_KERNEL_TRAFFIC["sources_sha256"]:
            return None
    except OSError:
        return None
    return STEP_KERNEL_TRAFFIC["fetch_bytes"] + STEP_KERNEL_TRAFFIC["write_bytes"]


def algorithmic_bytes_per_particle(mean_list: float) -> float:
    """HBM bytes one particle-step of the fused step kernel must move, as
    the method needs them: its list (4 B per entry) and length (4 B), its
    double-single position and velocity read and written (3 x 8 B each way
    for each), and its reference position (12 B) -- 4 n_L + 112 B. Neighbour
    records are re-reads of positions already counted (served by L2/MALL)
    and are not algorithmic traffic. The FP64 path needs the same bytes."""
    return 4.0 * mean_list + 4.0 + 2 * 24 + 2 * 24 + 12


def layout_bytes_per_particle(prec: int, mean_list: float) -> float:
    """Bytes the step kernel's data layout moves per particle-step: the list
    and its length, the own record, the state arrays as stored read and
    written (FP32+DS: double-single position and velocity in three float4
    words; FP64: the padded velocity), the new record, and the reference
    position."""
    if prec == 1:   # FP32 + double-single: three unpadded state words
        own_rec, state_rw, rec_out, xref = 16, 2 * 48, 16, 16
    else:           # FP64: the own record is the position
        own_rec, state_rw, rec_out, xref = 32, 2 * 32, 32, 16
    return 4.0 * mean_list + 4.0 + own_rec + state_rw + rec_out + xref


# The paper publishes no absolute throughput for this path; its relative
# figures, with the hardware they were measured on, as context.
PAPER_CONTEXT = {
    "absolute_throughput": "none published (the truncated-force performance figure is missing from the text)",
    "truncated_lj": {
        "workload": "N=100,000 LJ, 50,000 steps, several temperatures, GPU single precision",
        "hardware": "Nvidia A100 SXM4 80GB (CUDA 11.0.2 vs Intel LLVM SYCL 2022.12 on CUDA 11.7); A40 similar",
        "sycl_vs_cuda_runtime": "SYCL up to 1.8x slower",
        "force_kernel_slowdown": 1.8,
        "list_update_slowdown": 1.5,
        "runtime_share_force_list": [0.6, 0.3],
        "share_note": "list-update share grows with temperature",
    },
    "all_to_all": {
        "workload": "N=2,000, 20,000 steps (GPU, single precision); 5,000 steps FP64 on CPU",
        "sycl_vs_cuda": "SYCL about 1.3x faster (A40, A100)",
        "cpu": "Xeon W-2133: SYCL 1 thread 5.1x over sequential C++, 6 threads 21.9x (efficiency 0.84)",
        "mi210": "SYCL runs on MI210 (gfx90a, ROCm 5.0); no HIP baseline",
    },
}


def time_gpu(ljmd, torch, w, prec, steps, warmup, lanes, profile, cell_split=0):
    s = ljmd.System(w.n, w.box, w.params, precision=prec, sort_interval=100, lanes=lanes, cell_split=cell_split)
    s.set_state(w.x, w.v, w.species)
    if warmup:
        s.run(warmup)
    s.sync()
    obs = torch.empty((steps, ljmd.NOBS), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    if profile:
        s.set_profiling(True)
    start.record(stream)
    code = ljmd.lib.ljmd_run(s.ctx, steps, obs.data_ptr())
    stop.record(stream)
    torch.cuda.synchronize()
    if code != 0:
        raise ljmd.LJMDError(code, ljmd.last_error(s.ctx))
    s.sync()
    ms = start.elapsed_time(stop)
    kt = s.kernel_times() if profile else None
    o = obs.cpu().numpy()
    cnt, _ = s.neighbors(cap=1)
    mean_list = float(cnt.double().mean().item())
    info = s.observables()
    s.set_profiling(False)
    return {"ms": ms, "obs": o, "kt": kt, "mean_list": mean_list, "info": info}


def cpu_baseline(w, seconds_target: float = 15.0, one_core_seconds: float = 6.0):
    """The FP64 C oracle on the host cores: the step loop only (the initial
    list build and forces excluded), on all threads and on one."""
    import oracle
    threads = oracle.num_threads()
    # Calibrate on a few steps, then time a bounded sample of the same workload.
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, 3, want_obs=False)
    per_step = r["loop_seconds"] / 3.0
    steps = int(max(5, min(400, seconds_target / max(per_step, 1e-6))))
    r = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, steps, want_obs=False)
    value = w.n * steps / r["loop_seconds"]
    one = None
    if one_core_seconds > 0:
        steps1 = int(max(2, min(100, one_core_seconds / max(per_step * threads, 1e-6))))
        oracle.set_threads(1)
        try:
            r1 = oracle.run_nve(w.x, w.v, w.species, w.box, w.params, steps1, want_obs=False)
        finally:
            oracle.set_threads(threads)
        one = {"value": w.n * steps1 / r1["loop_seconds"], "cores": 1, "steps": steps1,
               "loop_seconds": r1["loop_seconds"]}
    return {
        "value": value,
        "unit": "particle-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"FP64 C oracle (OpenMP, {threads} threads), N={w.n} same workload, {steps} steps; "
                  f"step loop timed ({r['loop_seconds']:.1f} s), initial list build and forces excluded",
        "one_core": one,
    }


def time_adjoint(ljmd, torch, W, nsteps: int = 50, every: int = 10, reps: int = 3):
    """Differentiable workload: jittered FCC 40^3 (N=256,000), target
    parameters eps*, sigma* within 5%, loss
        L = |F(x_0; th) - F(x_0; th*)|^2 / 3N + U(x_N; th) / N,  N = 50 steps,
    a stored state every 10 steps. Forward = force evaluation at x_0 + the
    checkpointed rollout + the loss; backward = force VJP at x_0 + the reverse
    sweep (segment recompute, one VJP per frame) + dU/dtheta at x_N. Both
    timed with HIP events on the library's stream (FP32 pair math, DS state)."""
    import numpy as np
    wl, eps_t, sig_t = W.jittered_fcc(40)
    n = wl.n
    sp = torch.as_tensor(wl.species, device="cuda")
    x0 = torch.as_tensor(wl.x, device="cuda")
    v0 = torch.as_tensor(wl.v, device="cuda")
    sR = ljmd.System(n, wl.box, wl.params, precision=ljmd.FP32_DS)
    sF = ljmd.System(n, wl.box, wl.params, precision=ljmd.FP32_DS)
    sF.set_state(x0, torch.zeros_like(x0), sp)
    th = sF.theta()
    th_star = np.array([eps_t[0], eps_t[1], eps_t[3], sig_t[0], sig_t[1], sig_t[3]])
    sF.set_theta(th_star)
    F_star = sF.forces().clone()
    sF.set_theta(th)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd, bwd = [], []
    for r in range(reps + 1):
        sR.set_state(x0, v0, sp)
        torch.cuda.synchronize()
        ev[0].record(stream)
        sF.set_theta(th)                                   # forces at x_0 under theta
        F = sF.forces()
        obs = sR.vv_forward(nsteps, every)
        loss = ((F - F_star) ** 2).sum() / (3 * n) + obs[-1, 0] / n
        ev[1].record(stream)
        gF = 2.0 * (F - F_star) / (3 * n)
        gx_a, gth_a = sF.force_vjp(gF)
        zero = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        gx0, gv0, gth = sR.vv_backward(zero, zero, gU=1.0 / n)   # the U(x_N)/N term in the library
        gth = gth + gth_a
        gx0 = gx0 + gx_a
        ev[2].record(stream)
        torch.cuda.synchronize()
        sR.sync()
        if r > 0:                                          # the first pass is warmup
            fwd.append(ev[0].elapsed_time(ev[1]))
            bwd.append(ev[1].elapsed_time(ev[2]))
    f_ms, b_ms = float(np.median(fwd)), float(np.median(bwd))
    return {
        "workload": f"force-matching + final-energy loss, jittered FCC 40^3 N={n}, {nsteps} steps, "
                    f"checkpoint every {every}, FP32 pair math + DS state",
        "forward_ms": f_ms, "backward_ms": b_ms, "ratio": b_ms / f_ms,
        "loss": float(loss), "grad_norm_x0": float(gx0.norm()),
        "dL_deps": float(gth[0]), "dL_dsigma": float(gth[3]),
    }


def copy_bandwidth(torch, mib: int = 1024, reps: int = 5):
    """Achievable HBM bandwidth on this GPU: a device-to-device copy of
    mib MiB (read + write bytes over the best of reps event-timed copies)."""
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    stream = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        dst.copy_(src)
        b.record(stream)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    return 2.0 * n / (best * 1e-3) / 1e9


def time_mixture(ljmd, torch, W, copy_gbs, steps: int = 500, warmup: int = 20):
    """Binary 80:20 mixture, N = 4,000,000, rho = 1.2: uniform random
    positions relaxed by 200 steepest-descent steps (largest move 0.05 sigma
    per step, pair distances clamped at 0.6 sigma_ab), then velocities at
    T = 0.8 and NVE, FP32 pair math with double-single state, observables
    every step. Timed: steps NVE steps; then 100 more with per-kernel event
    brackets for the step kernel's average duration."""
    w = W.config_mixture()
    s = ljmd.System(w.n, w.box, w.params, precision=ljmd.FP32_DS, sort_interval=100)
    s.set_state(w.x, w.v, w.species)
    s.minimize_sd(200, 0.05, 0.6, record=False)
    x, _, _ = s.get_state()
    s.set_state(x, torch.as_tensor(w.v, device="cuda"), torch.as_tensor(w.species, device="cuda"))
    s.run(warmup)
    s.sync()
    obs = torch.empty((steps, ljmd.NOBS), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    code = ljmd.lib.ljmd_run(s.ctx, steps, obs.data_ptr())
    stop.record(stream)
    torch.cuda.synchronize()
    if code != 0:
        raise ljmd.LJMDError(code, ljmd.last_error(s.ctx))
    s.sync()
    ms = start.elapsed_time(stop)
    o = obs.cpu().numpy()
    E = (o[:, 0] + o[:, 1]) / w.n
    s.set_profiling(True)
    s.run(100, observe=True)
    s.sync()
    kt = s.kernel_times()
    s.set_profiling(False)
    cnt, _ = s.neighbors(cap=1)
    mean_list = float(cnt.double().mean().item())
    step_ms, step_n = kt["step"]
    avg_s = step_ms * 1e-3 / max(step_n, 1)
    bpp = algorithmic_bytes_per_particle(mean_list)
    achieved = bpp * w.n / avg_s / 1e9
    return {
        "workload": "binary 80:20 LJ mixture N=4000000, rho=1.2, eps_AB=1.5 sigma_AB=0.8 eps_BB=0.5 "
                    "sigma_BB=0.88, rc=2.5 sigma_ab, 200 steepest-descent steps then NVE at T=0.8, "
                    "dt=0.005, FP32 pair math + DS state",
        "value": w.n * steps / (ms * 1e-3), "unit": "particle-steps/s", "steps": steps,
        "ms_per_step": ms / steps, "rebuilds_in_timed_steps": int(o[:, 6].sum()),
        "energy_per_particle_first_last": [float(E[0]), float(E[-1])],
        "step_kernel_us": avg_s * 1e6, "mean_list_len": mean_list, "bytes_per_particle": bpp,
        "layout_bytes_per_particle": layout_bytes_per_particle(ljmd.FP32_DS, mean_list),
        "achieved_gbs": achieved, "frac_of_peak": achieved / HBM_PEAK_GBS,
        "frac_of_achievable": achieved / copy_gbs,
    }


def time_batch(ljmd, torch, W, steps: int = 1000, warmup: int = 50):
    """Batched replicas: 512 independent one-species LJ systems, N
    log-uniform in [500, 32000] (sum about 3.9 million), rho in [0.7, 1.2],
    T in [0.7, 1.5], FP32 pair math with double-single state, stepped
    together (every kernel spans all systems). Batched particle-steps/s =
    sum(N) * steps / wall time of the timed ljmd_batch_run."""
    import numpy as np
    ws = W.replica_draws(512)
    sizes, edges = [w.n for w in ws], [w.box[0] for w in ws]
    x, v, sp = (np.concatenate([w.x for w in ws]), np.concatenate([w.v for w in ws]),
                np.concatenate([w.species for w in ws]))
    # Lanes per particle and list capacity from the batch autotuner (not timed).
    tune = ljmd.autotune_batch(sizes, edges, ws[0].params, x, v, sp, steps=20)
    b = ljmd.Batch(sizes, edges, ws[0].params, sort_interval=100, lanes=tune["lanes"],
                   nbr_capacity=tune["nbr_capacity"], cell_split=tune["cell_split"])
    b.set_state(x, v, sp)
    b.run(warmup)
    b.sync()
    stream = torch.cuda.current_stream()

    def timed(n):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        b.run(n)
        stop.record(stream)
        torch.cuda.synchronize()
        b.sync()
        return start.elapsed_time(stop)

    # Graph replay of whole resort periods (the default), then every step
    # launched from the host for comparison.
    ms = timed(steps)
    obs = b.observables()
    b.use_graphs(False)
    ms_eager = timed(steps)
    ntot = sum(w.n for w in ws)
    return {
        "workload": f"512 replicas, sum N = {ntot}, N in [{min(w.n for w in ws)}, {max(w.n for w in ws)}], "
                    "rho U(0.7,1.2), T U(0.7,1.5), FP32 pair math + DS state",
        "value": ntot * steps / (ms * 1e-3), "unit": "particle-steps/s", "steps": steps,
        "ms_per_step": ms / steps, "launch": "HIP graph per 100-step resort period",
        "ms_per_step_eager_launches": ms_eager / steps,
        "autotuned": {"cell_split": tune["cell_split"], "lanes": tune["lanes"], "nbr_capacity": tune["nbr_capacity"],
                      "max_fill": tune["max_fill"], "ms_per_step_tuning": tune["ms_per_step"]},
        "rebuilds_per_system_mean": float(obs[:, 6].mean()),
    }


def time_allpairs(ljmd, torch, W, steps: int = 20000, warmup: int = 500):
    """The untruncated all-to-all interaction (every pair of the minimum
    image, no lists): N = 2,000 from a lattice with random vacancies at
    density 0.8442, T = 1.0, 20,000 NVE steps, in FP32 pair math with
    double-single state and in plain FP64 (the paper's all-to-all study
    size)."""
    w = W.all_pairs_fluid()
    out = {"workload": f"all-to-all LJ (no cutoff) N={w.n}, rho=0.8442, T=1.0, dt=0.005, {steps} NVE steps",
           "n": w.n, "steps": steps}
    stream = torch.cuda.current_stream()
    for name, prec in (("fp32_ds", ljmd.FP32_DS), ("fp64", ljmd.FP64)):
        s = ljmd.System(w.n, w.box, w.params, precision=prec, sort_interval=0)
        s.set_state(w.x, w.v, w.species)
        s.run(warmup, observe=False)
        s.sync()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        code = ljmd.lib.ljmd_run(s.ctx, steps, None)
        b.record(stream)
        torch.cuda.synchronize()
        if code != 0:
            raise ljmd.LJMDError(code, ljmd.last_error(s.ctx))
        s.sync()
        ms = a.elapsed_time(b)
        out[name] = {"value": w.n * steps / (ms * 1e-3), "unit": "particle-steps/s",
                     "ms_per_step": ms / steps,
                     "pair_interactions_per_s": w.n * (w.n - 1) * steps / (ms * 1e-3)}
        s.close()
    return out


def time_thermostat_sweep(ljmd, torch, W, temps=(0.7, 1.0, 1.5, 2.0, 3.0), steps: int = 2000,
                          warmup: int = 500, rate: float = 1.0):
    """The paper's truncated-force study shape: N = 100,000 at several
    temperatures under the Andersen-like thermostat (collision rate `rate`
    per unit time), FP32 pair math with double-single state. Per T: the
    throughput of `steps` timed steps, the mean steps between list builds,
    and the shares of the step kernel (forces) and of the list update
    (binning, canonical order, list build) in the kernel time of a
    profiled repeat."""
    rows = []
    stream = torch.cuda.current_stream()
    for T in temps:
        w = W.thermostat_fluid(temperature=T)
        s = ljmd.System(w.n, w.box, w.params, precision=ljmd.FP32_DS, sort_interval=100)
        s.set_state(w.x, w.v, w.species)
        s.set_thermostat(T, rate, seed=1234)
        s.run(warmup, observe=False)
        s.sync()
        r0 = s.observables()["rebuilds"]
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        code = ljmd.lib.ljmd_run(s.ctx, steps, None)
        b.record(stream)
        torch.cuda.synchronize()
        if code != 0:
            raise ljmd.LJMDError(code, ljmd.last_error(s.ctx))
        s.sync()
        ms = a.elapsed_time(b)
        o = s.observables()
        builds = o["rebuilds"] - r0
        s.set_profiling(True)
        s.run(steps, observe=False)
        s.sync()
        kt = s.kernel_times()
        s.set_profiling(False)
        tot = sum(v[0] for v in kt.values())
        rows.append({"T": T, "value": w.n * steps / (ms * 1e-3), "ms_per_step": ms / steps,
                     "steps_per_build": steps / max(builds, 1), "T_measured": o["T"],
                     "force_share": kt["step"][0] / tot,
                     "list_update_share": (kt["rebuild"][0] + kt["resort"][0]) / tot})
        s.close()
    return {"workload": f"LJ fluid N=100000 (FCC 30^3 sites, random vacancies), rho=0.8442, rc=2.5, "
                        f"skin=0.3, dt=0.005, Andersen-like thermostat rate {rate}, {steps} steps per T, "
                        "FP32 pair math + DS state",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--cell-split", type=int, default=0,
                    help="cells per list radius for the headline run (0: the library default, 1)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiable-workload timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-replica timing")
    ap.add_argument("--no-mixture", action="store_true", help="skip the 4M binary-mixture timing")
    ap.add_argument("--no-allpairs", action="store_true", help="skip the all-to-all (N=2000) timing")
    ap.add_argument("--no-tsweep", action="store_true", help="skip the thermostat temperature sweep")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--mixture-steps", type=int, default=500)
    ap.add_argument("--only-mixture", action="store_true",
                    help="time only the 4M binary mixture and print its JSON object (for profiling)")
    ap.add_argument("--only-allpairs", action="store_true",
                    help="time only the all-to-all workload and print its JSON object (for profiling)")
    ap.add_argument("--allpairs-steps", type=int, default=20000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device (a reference kernel of known "
                         "traffic for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library steps a system on one GPU (asked for --gpus {args.gpus}); "
              "there is no multi-GPU path to measure.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2406_04210_amd import ljmd
    from paper_2406_04210_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only_allpairs:
        print(json.dumps(time_allpairs(ljmd, torch, W, steps=args.allpairs_steps)), flush=True)
        return

    if args.only_mixture:
        print(json.dumps(time_mixture(ljmd, torch, W, copy_bandwidth(torch), steps=args.mixture_steps)), flush=True)
        return

    w = W.config_headline()
    print(f"bench: workload {w.name} N={w.n}", file=sys.stderr, flush=True)

    main_run = time_gpu(ljmd, torch, w, ljmd.FP32_DS, args.steps, args.warmup, args.lanes, False, args.cell_split)
    print(f"bench: fp32+ds {main_run['ms']:.2f} ms for {args.steps} steps", file=sys.stderr, flush=True)
    prof_run = time_gpu(ljmd, torch, w, ljmd.FP32_DS, args.steps, args.warmup, args.lanes, True, args.cell_split)
    ms_step = main_run["ms"] / args.steps
    value = w.n * args.steps / (main_run["ms"] * 1e-3)

    step_ms, step_n = prof_run["kt"]["step"]
    avg_step_kernel_s = step_ms * 1e-3 / max(step_n, 1)
    bpp = algorithmic_bytes_per_particle(prof_run["mean_list"])
    lbpp = layout_bytes_per_particle(ljmd.FP32_DS, prof_run["mean_list"])
    achieved = bpp * w.n / avg_step_kernel_s / 1e9
    copy_gbs = copy_bandwidth(torch)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                "achievable_copy_gbs": copy_gbs, "frac_of_achievable": achieved / copy_gbs,
                "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "algorithmic_bytes_per_launch": bpp * w.n,
                "algorithmic_bytes_per_particle": bpp,
                "layout_bytes_per_launch": lbpp * w.n,
                "layout_bytes_per_particle": lbpp,
                "kernel": "k_step_ds (forces + velocity Verlet + reductions)",
                "avg_kernel_us": avg_step_kernel_s * 1e6,
                "avg_kernel_us_source": "HIP events stamped by the kernel's own dispatch (extended launch) "
                                        "on the library's stream, every launch of the timed repeat",
                "mean_list_len": prof_run["mean_list"]}
    kernel_us = {k: (v[0] * 1e3 / v[1] if v[1] else 0.0) for k, v in prof_run["kt"].items()}

    obs = main_run["obs"]
    E = (obs[:, 0] + obs[:, 1]) / w.n
    rebuilds = int(obs[:, 6].sum())

    extra = {}
    if not args.no_fp64:
        r64 = time_gpu(ljmd, torch, w, ljmd.FP64, args.steps, args.warmup, args.lanes, False)
        extra["fp64_value"] = w.n * args.steps / (r64["ms"] * 1e-3)
        extra["fp64_ms_per_step"] = r64["ms"] / args.steps
        print(f"bench: fp64 {r64['ms']:.2f} ms", file=sys.stderr, flush=True)

    if not args.no_mixture:
        extra["mixture"] = time_mixture(ljmd, torch, W, copy_gbs, steps=args.mixture_steps)
        print(f"bench: mixture {extra['mixture']['value']:.3e} particle-steps/s", file=sys.stderr, flush=True)

    if not args.no_adjoint:
        extra["adjoint"] = time_adjoint(ljmd, torch, W)
        print(f"bench: adjoint/forward {extra['adjoint']['ratio']:.3f}", file=sys.stderr, flush=True)

    if not args.no_allpairs:
        extra["all_pairs"] = time_allpairs(ljmd, torch, W, steps=args.allpairs_steps)
        print(f"bench: all-pairs {extra['all_pairs']['fp32_ds']['value']:.3e} particle-steps/s",
              file=sys.stderr, flush=True)

    if not args.no_tsweep:
        extra["thermostat_sweep"] = time_thermostat_sweep(ljmd, torch, W)
        print("bench: T sweep " + " ".join(f"T={r['T']}:{r['list_update_share']:.2f}"
                                           for r in extra["thermostat_sweep"]["rows"]),
              file=sys.stderr, flush=True)

    if not args.no_batch:
        extra["batched"] = time_batch(ljmd, torch, W)
        print(f"bench: batched {extra['batched']['value']:.3e} particle-steps/s", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_seconds)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+ds",
        "data": "synthetic (seeded FCC 40^3 + Maxwell-Boltzmann T=1.0)",
        "config": {"workload": "LJ fluid N=256000 (FCC 40^3), rho=0.8442, T=1.0, rc=2.5 shifted, "
                               "skin=0.3, dt=0.005, NVE velocity Verlet, half-skin rebuild, "
                               "SFC resort every 100 steps",
                   "n": w.n, "precision": "fp32 pair math, double-single state",
                   "lanes": args.lanes or 2, "cell_split": args.cell_split or 1,
                   "nbr_capacity": prof_run["info"]["nbr_capacity"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernel_avg_us": kernel_us,
        "rebuilds_in_timed_steps": rebuilds,
        "paper_context": PAPER_CONTEXT,
        "energy_per_particle_first_last": [float(E[0]), float(E[-1])],
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
