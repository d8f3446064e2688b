"""Benchmark of the fused thermal two-component Shan-Chen LB step on one GPU.

A step is one pass of the whole update (pull streaming with bounce-back and
anti-bounce-back, moments, pseudopotentials, forces, collision, store) over
the lattice; the timed region runs --steps steps plus one FP64 observable
reduction at the end. Inputs are seeded synthetic emulsions (see
``workloads``), resident in HBM before timing starts.

Prints one JSON line with MLUPS (10^6 node updates per second), the HBM
roofline figures of the step kernel, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "MLUPS and % HBM roofline (FP32 vs FP16-storage); adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
ANALYSIS_CALLS = 5   # steady-state calls of the row averages and the droplet analysis
# Algorithmic bytes per node update: the 27 populations read once and
# written once (FP16 / BF16 deviations: 24 16-bit moving populations and 3
# FP32 rest populations), plus one byte of solid flag when the lattice has
# solid cells.
BYTES_PER_UPDATE = {"fp64": 432, "fp32": 216, "fp16dev": 120, "bf16dev": 120, "fix16dev": 108}
KERNEL_SOURCES = ("paper_2109_12565_amd/csrc/lb_kernels.hpp",
                  "paper_2109_12565_amd/csrc/lb_step2.hpp",
                  "paper_2109_12565_amd/csrc/launch_impl.hpp",
                  "paper_2109_12565_amd/csrc/tlb.hip")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash() or kernel not in rec.get("kernel", ""):
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w: dict, sample_steps: int, single_steps: int) -> dict:
    """FP64 oracle (C, OpenMP over rows) on the full lattice of the workload:
    `sample_steps` steps on all the threads the host gives the process, then
    `single_steps` on one thread; MLUPS over the step loop only."""
    from oracle.oracle import ModelParams, Oracle

    def run(steps, threads):
        ora = Oracle(ModelParams(**w["params"]), w["rho_a"], w["rho_b"], w["temp"],
                     solid=w["solid"], t_bottom=w["t_bottom"], threads=threads)
        t0 = time.perf_counter()
        ora.step(steps)
        dt = time.perf_counter() - t0
        return w["lx"] * w["ly"] * steps / dt / 1e6, dt, ora.threads

    mlups, dt, threads = run(sample_steps, None)
    out = {"value": mlups, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{sample_steps} steps of the full {w['lx']}x{w['ly']} lattice, FP64, "
                     f"{dt:.1f} s"}
    if single_steps > 0:
        m1, dt1, _ = run(single_steps, 1)
        out["single_thread"] = {"value": m1, "unit": "MLUPS", "cores": 1,
                                "sample": f"{single_steps} steps of the same lattice, {dt1:.1f} s"}
    return out


def adjoint_ratio(steps: int, ckpt: int, precision: str, config: str = "mid") -> dict:
    """Time of the taped forward plus the reverse sweep (checkpoint segment
    recompute included) over the time of the plain forward, for the same
    `steps` steps of an emulsion with a noisy bottom temperature: the
    1024x512 lattice (its gradient is zero: in 500 steps no signal crosses
    512 rows), the 1024x64 strip (a live gradient) or the 4096x2048 lattice
    with flat walls. ckpt = 1 keeps the
    moments of every step's pulled state in HBM (no recompute); tape_gib is
    the device memory of the tape (moments, checkpoints, recompute buffers). Steady state: a first taped run and
    reverse sweep on the handle (from the initial state; their loss and
    gradient are reported, and their time, allocation of the checkpoints and
    the tape included, as first_call_ms) precede the timed calls."""
    import torch

    from paper_2109_12565_amd import Simulation

    w = workloads.CONFIGS[config]()
    tb = workloads.bottom_temperature_noise(w["lx"], 5)

    def make():
        return Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], t_bottom=tb,
                          precision=precision)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    with make() as sim:  # load the code of every kernel once
        sim.step(10)
        warm = max(2 * ckpt, 10)
        sim.forward_taped(warm, ckpt)
        sim.adjoint(warm)
    # device memory of the tape (without row padding): at tau = tau_g = 1 the
    # moments of every step (K = 1), or checkpoints, two segments' moments
    # and two scratch states; else states
    elem = 8 if precision == "fp64" else 4
    state_bytes = 27 * w["lx"] * w["ly"] * elem
    moment_bytes = 5 * w["lx"] * w["ly"] * elem
    tau_one = w["params"]["tau"] == 1.0 and w["params"]["tau_g"] == 1.0
    with make() as sim:
        t_first_tape, loss = timed(lambda: sim.forward_taped(steps, ckpt))
        t_first_adj, g = timed(lambda: sim.adjoint(steps))
        t_tape, _ = timed(lambda: sim.forward_taped(steps, ckpt))
        t_adj, _ = timed(lambda: sim.adjoint(steps))
        t_fwd, _ = timed(lambda: sim.step(steps))
    nck = -(-steps // ckpt)
    if tau_one:
        tape = steps * moment_bytes if ckpt == 1 else (nck + 2) * state_bytes + 2 * ckpt * moment_bytes
    else:
        tape = (nck + ckpt - 1) * state_bytes
    tape_gib = tape / 2**30
    return {"workload": w["name"], "storage": precision, "steps": steps, "ckpt_every": ckpt,
            "tape_gib": round(tape_gib, 2),
            "forward_ms": round(t_fwd * 1e3, 2), "taped_forward_ms": round(t_tape * 1e3, 2),
            "reverse_ms": round(t_adj * 1e3, 2),
            "ratio": round((t_tape + t_adj) / t_fwd, 2),
            "first_call_ms": round((t_first_tape + t_first_adj) * 1e3, 2), "loss": loss,
            "grad_max_abs": float(np.abs(g).max())}


def precision_study(steps: int, every: int, storages) -> dict:
    """Errors of each storage against the FP64 oracle on the 512x256 crop of
    the large recipe: max relative error of rho_A, rho_B, T (over max|field|)
    and of u^H (over the largest oracle velocity) after `steps` steps, the
    relative error of the time-averaged Nusselt number (sampled every
    `every` steps), and the per-component mass drift."""
    from oracle.oracle import ModelParams, Oracle
    from paper_2109_12565_amd import Simulation

    w = workloads.crop()
    ora = Oracle(ModelParams(**w["params"]), w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                 t_bottom=w["t_bottom"])
    sims = {pr: Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                           t_bottom=w["t_bottom"], precision=pr) for pr in storages}
    nu = {k: [] for k in ["oracle", *storages]}
    m0 = {pr: s.observables() for pr, s in sims.items()}
    t0 = time.perf_counter()
    for t in range(every, steps + 1, every):
        ora.step(every)
        nu["oracle"].append(ora.observables()["nu"])
        for pr, sim in sims.items():
            sim.step(every)
            nu[pr].append(sim.observables()["nu"])
    ref = ora.fields()
    umax = max(np.abs(ref["ux"]).max(), np.abs(ref["uy"]).max())
    nu_ref = float(np.mean(nu["oracle"]))
    out = {"study": "precision", "workload": w["name"], "steps": steps, "nu_every": every,
           "oracle_threads": ora.threads, "nu_mean_oracle": nu_ref, "storages": {}}
    for pr, sim in sims.items():
        f = sim.fields()
        obs = sim.observables()
        e = {k: float(np.abs(f[k] - ref[k]).max() / np.abs(ref[k]).max())
             for k in ("rho_a", "rho_b", "temp")}
        e["u"] = float(max(np.abs(f["ux"] - ref["ux"]).max(), np.abs(f["uy"] - ref["uy"]).max()) / umax)
        e["nu_mean"] = float(np.mean(nu[pr]))
        e["nu_mean_rel_err"] = abs(e["nu_mean"] - nu_ref) / abs(nu_ref)
        e["mass_a_drift"] = (obs["mass_a"] - m0[pr]["mass_a"]) / m0[pr]["mass_a"]
        e["mass_b_drift"] = (obs["mass_b"] - m0[pr]["mass_b"]) / m0[pr]["mass_b"]
        info = sim.launch_info()
        e["launch"] = ("fused two-step, %d lanes, %d-row chunks" % (info["fused_lanes"], info["fused_rows"])
                       if info["fused_rows"] > 0 else "single steps")
        out["storages"][pr] = e
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    return out


def companion_runs(config: str, precision: str) -> dict:
    """Throughput of the storages and lattice the headline metric compares
    with, measured in the same process: FP16 deviations on the benchmark
    lattice (FP32 if the main run used another storage) and FP32 on the
    1024x512 lattice; HIP events around tlb_step(K) plus one observables
    call, as in the main measurement."""
    import torch

    from paper_2109_12565_amd import Simulation

    def run(name, prec, steps, warmup):
        w = workloads.CONFIGS[name]()
        with Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                        t_bottom=w["t_bottom"], precision=prec) as sim:
            sim.step(warmup)
            sim.observables()
            e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            torch.cuda.synchronize()
            e0.record()
            sim.step(steps)
            sim.observables()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            launch = sim.launch_info()
        return {"workload": w["name"], "storage": prec, "steps": steps,
                "mlups": round(w["lx"] * w["ly"] * steps / (ms * 1e-3) / 1e6, 1),
                "ms_per_step": round(ms / steps, 4), "fused": launch["fused_rows"] > 0}

    other = "fp16dev" if precision != "fp16dev" else "fp32"
    return {"other_storage": run(config, other, 300, 20),
            "fp32_1024x512": run("mid", "fp32", 2000, 50)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="large", choices=sorted(workloads.CONFIGS))
    ap.add_argument("--precision", default="fp32", choices=sorted(BYTES_PER_UPDATE))
    ap.add_argument("--cpu-steps", type=int, default=40,
                    help="oracle steps for the CPU baseline on all host threads (0 to skip)")
    ap.add_argument("--cpu-steps-1t", type=int, default=2,
                    help="oracle steps for the one-thread CPU baseline (0 to skip)")
    ap.add_argument("--study", choices=["precision"], default=None,
                    help="instead of the benchmark, print the precision study (storages vs the "
                         "FP64 oracle on the 512x256 crop)")
    ap.add_argument("--adjoint-large-steps", type=int, default=0,
                    help="also time the adjoint on the 4096x2048 lattice with flat walls over "
                         "this many steps, moment tape and checkpoints every 25 (0 to skip)")
    ap.add_argument("--adjoint-steps", type=int, default=500,
                    help="steps of the adjoint/forward time ratio on the 1024x512 emulsion "
                         "(FP32, checkpoints every 25; 0 to skip)")
    ap.add_argument("--u-wall", type=float, nargs=2, default=(0.0, 0.0), metavar=("UB", "UT"),
                    help="x-velocity of the bottom and top walls (Couette walls)")
    ap.add_argument("--companions", type=int, default=1,
                    help="also time the other storage on the same lattice and FP32 on the "
                         "1024x512 lattice (0 to skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before warmup, run 3 plain device copies of this many MiB (a known "
                         "traffic reference for hardware counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU only (no multi-GPU halo exchange); --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import torch

    from paper_2109_12565_amd import Simulation

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.study == "precision":
        print(json.dumps(precision_study(args.steps, 50, ["fp32", "fp16dev", "bf16dev", "fix16dev"])),
              flush=True)
        return 0
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = workloads.CONFIGS[args.config]()
    print(f"# bench: {w['name']} {args.precision} warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
    params = dict(w["params"], u_wall=tuple(args.u_wall))
    sim = Simulation(params, w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision=args.precision)
    sim.step(args.warmup)
    sim.observables()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    obs = sim.observables()   # FP64 reductions (synchronises the stream)
    e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    # The first calls of the two analyses below allocate their buffers: one
    # call each (the droplets' one timed as first_call_ms), then the
    # steady-state calls, best of ANALYSIS_CALLS wall-clock times each.
    sim.row_averages()
    t_drop_first = time.perf_counter()
    sim.droplets(0.8)
    t_drop_first = time.perf_counter() - t_drop_first

    def best_of(fn):
        best, out = float("inf"), None
        for _ in range(ANALYSIS_CALLS):
            t = time.perf_counter()
            out = fn()
            best = min(best, time.perf_counter() - t)
        return best, out

    # stress fields + row averages of the same time level (Couette rheology
    # observables): one pass of the step kernel without store, then the row
    # reduction and the copy of 2 * ly doubles (synchronising)
    t_rows, rows = best_of(sim.row_averages)
    # droplet detection of the same time level: fields pass, labelling,
    # exact per-droplet sums, droplet Nusselt numbers, copy of the results
    t_drop, drops = best_of(lambda: sim.droplets(0.8))
    total_ms = e0.elapsed_time(e2)         # whole job: steps + observables

    # Launch durations, measured directly with HIP events on the library's
    # stream (torch's current stream): tlb_step(n) with fused launches runs
    # (n - 1) // 2 of them and one or two single steps, so two calls whose
    # step counts differ by 2 (b - a) differ by exactly b - a fused launches;
    # without the fused kernel they differ by that many single steps.
    launch = sim.launch_info()
    fused = launch["fused_rows"] > 0

    def call_ms(n, reps=3):
        best = float("inf")
        for _ in range(reps):
            ea, eb = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            ea.record(stream)
            sim.step(n)
            eb.record(stream)
            torch.cuda.synchronize()
            best = min(best, ea.elapsed_time(eb))
        return best

    ka, kb = 2, 12
    per_launch_s = (call_ms(2 * kb + 1) - call_ms(2 * ka + 1)) * 1e-3 / (2 * (kb - ka) if not fused
                                                                         else (kb - ka))
    # the single step that ends every call (it also forms the observable sums)
    n_one = 20
    e3, e4 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    e3.record(stream)
    for _ in range(n_one):
        sim.step(1)
    e4.record(stream)
    torch.cuda.synchronize()
    single_s = e3.elapsed_time(e4) * 1e-3 / n_one

    n_fused = (args.steps - 1) // 2 if fused and args.steps >= 3 else 0
    n_single = args.steps - 2 * n_fused
    nodes = w["lx"] * w["ly"]
    mlups = nodes * args.steps / (total_ms * 1e-3) / 1e6
    bpn = BYTES_PER_UPDATE[args.precision] + (1 if w["solid"] is not None else 0)
    kernel, updates = ("lb_step2_kernel", 2) if n_fused > 0 else ("lb_step_kernel", 1)
    if fused and n_fused == 0:  # fused kernel chosen, but too few steps to use it
        per_launch_s = single_s
    # algorithmic bytes per launch: the method's bytes per lattice update
    # (27 populations read and written once, plus the solid flag) times the
    # updates one launch performs; the fused kernel moves its populations
    # once for two updates, so the bytes it must move per launch are half of
    # that (hbm_bytes_per_launch_min); `traffic` is the counted HBM rate
    achieved = bpn * nodes * updates / per_launch_s / 1e9
    moved = bpn * nodes / per_launch_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": kernel, "bytes_per_lattice_update": bpn, "nodes_per_launch": nodes,
            "updates_per_node": updates, "launch_us": round(per_launch_s * 1e6, 2),
            "launch_timing": f"HIP events: tlb_step({2 * kb + 1}) minus tlb_step({2 * ka + 1}), "
                             f"best of 3 each, over {kb - ka if fused else 2 * (kb - ka)} launches",
            "hbm_bytes_per_launch_min": bpn * nodes,
            "frac_of_min_bytes": round(moved / HBM_PEAK_GBS, 4),
            "launches": {"fused": n_fused, "single": n_single},
            # what the counters show limits the kernel: the fused kernel does two
            # steps' arithmetic per pass over HBM at 8 wavefronts per CU (LDS
            # caps it) and is bound by latency and instruction issue, as is the
            # 16-bit single step; the 4- and 8-byte single step by HBM
            "limiter": "latency-issue" if n_fused > 0 or BYTES_PER_UPDATE[args.precision] <= 120
                       else "hbm"}
    traffic = measured_traffic(w["name"], args.precision, kernel)
    if traffic is not None:
        # counted HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated) over the
        # launch time measured here, and that rate as a fraction of peak
        roof["traffic"] = round(traffic / per_launch_s / 1e9, 1)
        roof["traffic_bytes_per_launch"] = traffic
        roof["traffic_frac"] = round(traffic / per_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    # measured device-copy ceiling (1 GiB read + 1 GiB written, best of 3),
    # the practical bound beside the nominal peak
    cbuf = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    csrc, cdst = cbuf[: 1 << 30], cbuf[1 << 30:]
    best = float("inf")
    for _ in range(4):
        ea, eb = (torch.cuda.Event(enable_timing=True) for _ in range(2))
        ea.record(stream)
        cdst.copy_(csrc)
        eb.record(stream)
        torch.cuda.synchronize()
        best = min(best, ea.elapsed_time(eb))
    del cbuf, csrc, cdst
    copy_gbs = 2.0 * (1 << 30) / (best * 1e-3) / 1e9
    # achieved over it can exceed 1 for the fused kernel (two updates per
    # pass over HBM); the counted traffic over it cannot
    roof["copy_ceiling"] = {
        "GBps": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
        "how": "torch device copy of 1 GiB, HIP events, best of 4",
        "achieved_over_copy": round(achieved / copy_gbs, 4),
        "traffic_over_copy": None if roof["traffic"] is None else round(roof["traffic"] / copy_gbs, 4)}
    single_gbs = bpn * nodes / single_s / 1e9
    roof["single_step_kernel"] = {"kernel": "lb_step_kernel (with the observable sums)",
                                  "launch_us": round(single_s * 1e6, 2),
                                  "achieved": round(single_gbs, 1),
                                  "frac": round(single_gbs / HBM_PEAK_GBS, 4),
                                  "mlups": round(nodes / single_s / 1e6, 1)}

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        # the paper's own figure (Sec. 2.5), other hardware, lattice and
        # precision not stated: context, not a baseline for this workload
        "paper_context": {"mlups": 525, "hardware": "NVIDIA Titan V", "lattice": "not stated",
                          "precision": "not stated"},
        "dtype": {"fp32": "f32", "fp64": "f64", "fp16dev": "f16-storage/f32",
                  "bf16dev": "bf16-storage/f32", "fix16dev": "i16-storage/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w["name"], "lx": w["lx"], "ly": w["ly"], "storage": args.precision,
                   "droplets": int(w["n_droplets"]), "solid_cells": 0 if w["solid"] is None
                   else int((w["solid"] != 0).sum()), "observables": "once at the end",
                   "u_wall": list(args.u_wall), "seed": w["seed"]},
        "roofline": roof,
        "check": {"mass_a": obs["mass_a"], "mass_b": obs["mass_b"], "nu": obs["nu"],
                  "wall_s": round(wall, 3)},
        "row_averages": {"ms": round(t_rows * 1e3, 3), "calls": ANALYSIS_CALLS, "pxy_av_mean": float(np.mean(rows["pxy_av"])),
                         "u_av_top": float(rows["u_av"][-1])},
        "droplets": {"ms": round(t_drop * 1e3, 3), "calls": ANALYSIS_CALLS,
                     "first_call_ms": round(t_drop_first * 1e3, 3),
                     "count": int(len(drops["root"])),
                     "threshold": 0.8, "nu_mean": float(np.mean(drops["nu"])) if len(drops["nu"]) else None},
    }
    sim.close()
    if args.companions:
        out["companions"] = companion_runs(args.config, args.precision)
    if args.adjoint_steps > 0:
        # the moments of every step kept (4.9 GiB at 1024x512 over 500
        # steps), then checkpoints every 25 steps with segment recompute
        out["adjoint"] = adjoint_ratio(args.adjoint_steps, 1, "fp32")
        out["adjoint_ckpt"] = adjoint_ratio(args.adjoint_steps, 25, "fp32")
        out["adjoint_strip"] = adjoint_ratio(args.adjoint_steps, 1, "fp32", "strip")
    if args.adjoint_large_steps > 0:
        out["adjoint_large"] = adjoint_ratio(args.adjoint_large_steps, 1, "fp32", "large-flat")
        out["adjoint_large_ckpt"] = adjoint_ratio(args.adjoint_large_steps, 25, "fp32", "large-flat")
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, args.cpu_steps_1t)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
