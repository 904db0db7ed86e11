#!/usr/bin/env python
"""Benchmark of the adjoint-FDTD hot path on one MI355X.

Headline (default, `--workload multiport`): the 600x400x120 1-to-4
splitter-like device, 5 wavelengths x (1 forward + 4 adjoint port sources) =
25 right-hand sides batched in the same launches, 20 000 Yee steps each.
One bench step is a fixed block of `--block` (200) whole Yee steps of all 25
right-hand sides of that solve (the interior and CPML-shell step launches,
the source injection, and in the last four periods the running DFT): W
warm-up blocks, then K timed blocks, all inside one forward+adjoint solve
that then runs to its end and is finished with the modal coefficients and
the Eq. (1) gradient pulled back to dF/dC.  That whole gradient, from
set_design to dF/dC, is timed too (gradients/hour).  The 320x240x96
realistic device's whole gradients (6 right-hand sides, 10 000 steps) are
timed after it and reported as extra keys.  Inputs are seeded synthetic
SOI-like devices, resident on the GPU before timing starts.

Prints ONE JSON line on stdout.  Diagnostics go to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s + % HBM peak; adjoint gradients/hour; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2505_03352_amd/csrc/yo_step.hip", "paper_2505_03352_amd/csrc/yo_internal.h"]
PROFILES = os.path.join(ROOT, "profiles")
PART_NAMES = ("interior", "shell", "two_step", "frame", "zslab_two_step", "shell_paired")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# yo_set_tiling flag bits that change each launch's work split: the interior
# (x-shell layouts 1, 128 and 256, 8 waves per block, cooperative interior
# blocks, no interior prefetch), the CPML shell (the x-shell layouts, 8 waves
# per block, cooperative shell blocks, per-class code, no shell prefetch),
# the two-step launch (x-shell layouts, 8 waves per block) and the interior
# around it (the same and no prefetch), the z-slabs' two-step launch and the
# shell of paired steps (2048 decides which tiles each holds; 4096 and 8192
# the two-step tiles' rows and blocks; 16384 the shell tiles' rows); 512
# (two steps per launch) in all
SPLIT_BITS = (1 | 2 | 16 | 32 | 128 | 256 | 512, 1 | 2 | 4 | 8 | 64 | 128 | 256 | 512 | 2048 | 16384,
              1 | 2 | 128 | 256 | 512 | 4096 | 8192, 1 | 2 | 32 | 128 | 256 | 512,
              1 | 2 | 128 | 256 | 512 | 2048, 1 | 2 | 4 | 8 | 64 | 128 | 256 | 512 | 2048 | 16384)


def part_split(tiling, part: int) -> str:
    """rows,z-chunk,flag bits of a (rows, zchunk, flags) tiling that shape
    launch `part` (see PART_NAMES)."""
    rows, zc, flags = tiling
    return f"{rows},{zc},{flags & SPLIT_BITS[part]}"


def traffic_file(part: int, workload: str) -> str:
    return os.path.join(PROFILES, f"yee_step_{PART_NAMES[part]}_{workload}_traffic.txt")


def read_traffic(path: str, sha: str, split) -> float:
    """HBM bytes per launch from a committed counter summary, or None if the
    file is missing, the kernel changed since the counters were taken, or the
    launch is split differently from the run they were taken on."""
    try:
        kv = {}
        with open(path) as f:
            for line in f:
                if "=" in line and not line.startswith("#"):
                    k, v = line.strip().split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_sha") != sha or split is None or kv.get("split") != split:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def lscpu_summary() -> dict:
    """Model, sockets and physical cores of this host (lscpu), and the CPUs
    this process may run on."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass

    def num(k):
        try:
            return int(info.get(k, ""))
        except ValueError:
            return None
    sockets, per = num("Socket(s)"), num("Core(s) per socket")
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"model": info.get("Model name"), "sockets": sockets, "cores_per_socket": per,
            "threads_per_core": num("Thread(s) per core"),
            "physical_cores": sockets * per if sockets and per else None,
            "logical_cpus": num("CPU(s)"), "cpus_allowed": allowed,
            "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(dev, target_s: float):
    """The FP64 oracle on this host's cores: one right-hand side of the same
    grid (CPML, source, no DFT window) for a bounded number of steps, at one
    thread and at all the physical cores this process may use."""
    from oracle import adjoint, chain, fdtd, ports
    kap, _ = chain.kappa(dev)
    lam = dev.wavelengths[len(dev.wavelengths) // 2]
    src = dev.sources[0]
    J = ports.source_current(src.h)

    def run(n):
        prm = adjoint.sim_params(dev, lam, n_steps=n)
        t = time.perf_counter()
        fdtd.run(prm, kap, src_plane=src.plane, src_j=J)
        return time.perf_counter() - t

    cpu = lscpu_summary()
    phys = cpu["physical_cores"] or cpu["cpus_allowed"]
    # all physical cores, but no more than this process's CPU share
    cap = int(os.environ.get("OMP_NUM_THREADS") or cpu["cpus_allowed"])
    full = max(1, min(phys, cpu["cpus_allowed"], cap))

    def measure(threads, budget):
        used = fdtd.set_threads(threads)
        # the per-step cost from two short runs (their difference drops the
        # set-up every run pays), then one run sized to about `budget`
        t2, t6 = run(2), run(6)
        per_step = max((t6 - t2) / 4.0, 1e-4)
        n = int(max(6, min(5000, (budget - t2) / per_step)))
        t = run(n)
        return {"value": dev.cells * n / t / 1e9, "unit": "Gcell-updates/s", "cores": used,
                "kind": "oracle",
                "sample": f"{dev.nx}x{dev.ny}x{dev.nz} grid, 1 right-hand side, {n} steps, FP64 "
                          f"(CPML, source, no DFT window), {t:.1f} s on {used} thread(s)"}

    one = measure(1, 0.4 * target_s)
    out = measure(full, 0.6 * target_s)
    fdtd.set_threads(cap)
    out["one_thread"] = one
    out["host"] = cpu
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--chunk", type=int, default=100)
    ap.add_argument("--block", type=int, default=200,
                    help="multiport: Yee steps per bench step (an even divisor of 20000)")
    ap.add_argument("--cpu-seconds", type=float, default=24.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-realistic", action="store_true",
                    help="multiport: leave out the realistic device's whole gradients")
    ap.add_argument("--realistic-only", action="store_true",
                    help="the realistic device's whole gradients alone, as their own line "
                         "(a short run for counter collection)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="multi-port and realistic: sweep the splits instead of applying the shipped ones")
    ap.add_argument("--tiling", default=None,
                    help="multi-port: rows,zchunk,flags of the step launches instead of the autotuner's")
    ap.add_argument("--eager", action="store_true",
                    help="plain launches instead of HIP-graph replays (for counter collection)")
    ap.add_argument("--workload", choices=("multiport", "batch", "serving", "optimize", "broadband",
                                           "batch-fd"),
                    default="multiport",
                    help="multiport: the headline line; batch / serving: the batched and served "
                         "forms against one-at-a-time solves (their own JSON line)")
    ap.add_argument("--requests", type=int, default=12, help="serving: first N requests of the trace")
    ap.add_argument("--sides", default="served,plain",
                    help="serving: which of served (continuous batching), plain (one request at "
                         "a time, plain forward-then-adjoint solves per wavelength) and same (the "
                         "served executor with one slot) to run, comma-separated")
    ap.add_argument("--iters", type=int, default=5, help="optimize: optimizer iterations")
    ap.add_argument("--pulse", action="store_true",
                    help="optimize: gradients from pulse runs; serving: pulse runs for "
                         "multi-wavelength requests in the served loop")
    ap.add_argument("--pulse-steps", type=int, default=None,
                    help="steps of the pulse runs (broadband: 7000 realistic, 12000 multi-port; "
                         "optimize: 12000)")
    ap.add_argument("--device", choices=("realistic", "multiport"), default="realistic",
                    help="broadband: the device (multiport: 600x400x120, 5 wavelengths, 4 ports)")
    ap.add_argument("--pulse-k", type=float, default=None,
                    help="band edges in spectral widths of the pulse (broadband: 0.4, "
                         "optimize: 1.0)")
    ap.add_argument("--dft-stride", type=int, default=4,
                    help="pulse runs: the DFT samples every n-th step (the library checks that "
                         "the pulse spectrum vanishes at the aliases)")
    ap.add_argument("--slots", type=int, default=8, help="serving: concurrent requests")
    ap.add_argument("--rate", type=float, default=4.0, help="serving: arrival rate, requests/s")
    ap.add_argument("--max-cells", type=float, default=4.5e7,
                    help="serving: cap on cell-updates per step of the admitted requests")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the right-hand sides shard across GPUs without exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "optimize":
        return bench_optimize(args)
    if args.workload == "broadband":
        return bench_broadband(args)
    if args.workload == "batch-fd":
        return bench_batch_fd(args)
    if args.realistic_only:
        return bench_realistic_only(args)

    return bench_headline(args)


def bench_realistic_only(args):
    """The realistic device's whole gradients (the headline line's extra
    keys) without the multi-port solve, after the same calibration copy."""
    import torch
    torch.cuda.set_device(0)
    calibration_copy(torch)
    res = realistic_gradients(args, torch)
    _line("Gcell-updates/s (realistic device, whole gradients)", res["gcell_updates_per_s"],
          "Gcell-updates/s", res["s_per_gradient"] * 1e3, args,
          {"workload": res["workload"], "tiling": res["tiling"]}, {"realistic": res})


def calibration_copy(torch):
    """A plain 1 GiB device copy, its source pushed out of the 256 MB
    last-level cache first: the reference the HBM counters are scaled by."""
    cal_bytes = 1 << 30
    cal_src = torch.ones(cal_bytes // 4, dtype=torch.float32, device="cuda:0")
    evict = torch.zeros((512 << 20) // 4, dtype=torch.float32, device="cuda:0")
    cal_dst = torch.empty_like(cal_src)
    torch.cuda.synchronize()
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    log(f"calibration copy: {cal_bytes} bytes read, {cal_bytes} bytes written")
    del cal_src, cal_dst, evict


KERNEL_OF_PART = ("k_yee_step interior tiles", "k_yee_step CPML shell tiles",
                  "k_yee_step2 two-step region (two steps per launch)",
                  "k_yee_step interior tiles around the two-step region",
                  "k_yee_step2 z-slabs under the two-step region (two steps per launch)",
                  "k_yee_step CPML shell tiles of the steps in pairs")


def part_rooflines(plan, timed, tiling, workload, sha):
    """Per launch part that ran in the timed region: HIP-event duration, the
    part's algorithmic bytes per launch (the two-step launch counts both of
    its steps), the share of the timed kernels' time, and the committed
    counter figure when it belongs to this kernel and split."""
    out = []
    total = sum(ms * n for ms, n in timed)
    for part, (ms, n) in enumerate(timed):
        if n == 0:
            continue
        _, b, cells = plan.time_kernel(part, 1)
        ach = b / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        out.append({"kernel": KERNEL_OF_PART[part], "part": PART_NAMES[part],
                    "ms_per_launch": round(ms, 4), "launches_timed": n,
                    "time_share": round(ms * n / total, 4) if total > 0 else None,
                    "bytes_per_launch": b, "cell_updates_per_launch": cells,
                    "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": read_traffic(traffic_file(part, workload), sha,
                                            part_split(tiling, part))})
    return out


def roofline_of(parts):
    """The bench line's roofline object: the launch part that takes the most
    of the timed kernel time (launches times mean duration), with the others
    beside it."""
    dom = max(parts, key=lambda q: q["ms_per_launch"] * q["launches_timed"])
    return {"bound": "hbm", "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["frac"], "traffic": dom["traffic"], "kernel": dom["kernel"],
            "bytes_per_launch": dom["bytes_per_launch"], "ms_per_launch": dom["ms_per_launch"],
            "launches_timed": dom["launches_timed"], "parts": parts}


def realistic_gradients(args, torch, n_timed=1):
    """Whole gradients of the 320x240x96 realistic device (6 right-hand
    sides x 10 000 steps): set_design, forward+adjoint runs, alpha, dF/dC."""
    from paper_2505_03352_amd import YO_BOTH, autotune
    from paper_2505_03352_amd.plan import plan_for
    from workloads import configs
    dev = configs.realistic()
    plan = plan_for(dev, device="cuda:0", time_blocking=2)
    tuned = autotune.tune(plan, YO_BOTH, use_cache=False, shipped=not args.retune)
    tiling = (tuned["rows"], tuned["zchunk"], tuned["flags"])
    C = torch.as_tensor(dev.C, dtype=torch.float32, device="cuda:0")

    from paper_2505_03352_amd.plan import advance_many
    mid = dev.n_steps // 2

    def grad(timing):
        # one solve as yo_run does it (reset, chunked steps, finalize), its
        # middle 100 steps, before the DFT window, in a call of their own with
        # HIP events around every launch part (those steps run as plain
        # launches)
        plan.set_design(C, dev.beta)
        plan.reset(YO_BOTH)
        g = not args.eager
        advance_many([plan], [YO_BOTH], mid, chunk=args.chunk, use_graph=g)
        if timing:
            plan.set_timing(2, 100)
        advance_many([plan], [YO_BOTH], 100, chunk=args.chunk, use_graph=g)
        plan.set_timing(2, 0)          # off; what was recorded stays
        advance_many([plan], [YO_BOTH], dev.n_steps - mid - 100, chunk=args.chunk, use_graph=g)
        plan.finalize(YO_BOTH)
        a = plan.alpha()
        return plan.gradient(torch.conj(a))

    grad(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_timed):
        grad(True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n_timed
    timed = [plan.timing(q) for q in range(6)]
    plan.set_timing(0, 0)
    plan.reset(YO_BOTH)
    plan.advance(YO_BOTH, 4)
    parts = part_rooflines(plan, timed, tiling, "realistic", kernel_sha())
    cells = plan.n_rhs * dev.cells * dev.n_steps
    plan.close()
    log(f"realistic: {dt:.2f} s per gradient, {cells / dt / 1e9:.1f} Gcell-updates/s; " +
        "; ".join(f"{q['part']} {q['ms_per_launch']:.4f} ms/launch {q['achieved']:.0f} GB/s"
                  for q in parts))
    return {"workload": "realistic: 320x240x96 cells at 20 nm (CPML 8), 100x100 design/controls, "
                        "r=3, beta=8, 1.50/1.55/1.60 um, 1 forward + 1 adjoint each (6 right-hand "
                        "sides), 10000 steps; whole gradient (set_design, runs, alpha, dF/dC)",
            "gcell_updates_per_s": round(cells / dt / 1e9, 3), "s_per_gradient": round(dt, 3),
            "gradients_per_hour": round(3600.0 / dt, 1), "gradients_timed": n_timed,
            "tiling": list(tiling), "roofline": roofline_of(parts)}


def bench_headline(args):
    import numpy as np
    import torch
    from paper_2505_03352_amd import YO_BOTH, autotune
    from paper_2505_03352_amd.plan import advance_many, plan_for
    from workloads import configs

    torch.cuda.set_device(0)
    dev = configs.multiport()
    block = args.block
    tail = 8                        # timed plain-launch steps at the end of each block
    chunk = (block - tail) // 2     # two graph replays per block
    if block < 2 * tail or (block - tail) % 2 or dev.n_steps % block:
        raise SystemExit(f"--block must be an even divisor of {dev.n_steps} of at least {2 * tail}")
    n_blocks = dev.n_steps // block
    log(f"workload {dev.name}: {dev.nx}x{dev.ny}x{dev.nz}, {dev.n_freq} wavelengths, "
        f"{len(dev.ports)} ports, {dev.n_steps} steps; bench step = {block} Yee steps of all "
        f"right-hand sides ({n_blocks} per solve)")
    plan = plan_for(dev, device="cuda:0", time_blocking=2)
    calibration_copy(torch)
    tuned = None
    if args.tiling:
        tiling = tuple(int(v) for v in args.tiling.split(","))
        plan.set_tiling(*tiling)
        log(f"tiling (given): rows {tiling[0]} zchunk {tiling[1]} flags {tiling[2]}")
    else:
        if not args.no_autotune:
            tuned = autotune.tune(plan, YO_BOTH, use_cache=False, shipped=not args.retune)
            log(f"autotune{' (shipped split)' if tuned.get('shipped') else ''}: rows {tuned['rows']} "
                f"zchunk {tuned['zchunk']} flags {tuned['flags']} ({tuned['ms_per_step']:.3f} ms per step)")
        tiling = (tuned["rows"], tuned["zchunk"], tuned["flags"]) if tuned else (4, 16, 0)
    C = torch.as_tensor(dev.C, dtype=torch.float32, device="cuda:0")
    state = {"block": 0, "grads": []}

    def begin():
        torch.cuda.synchronize()
        state["t_grad"] = time.perf_counter()
        plan.set_design(C, dev.beta)
        plan.reset(YO_BOTH)
        state["block"] = 0

    def finish():
        # the rest of the solve in pieces of 2000 steps, a progress line after each
        done = state["block"] * block
        while done < dev.n_steps:
            k = min(2000, dev.n_steps - done)
            advance_many([plan], [YO_BOTH], k, chunk=args.chunk, use_graph=not args.eager)
            done += k
            torch.cuda.synchronize()
            log(f"  solve: {done}/{dev.n_steps} steps")
        plan.finalize(YO_BOTH)
        a = plan.alpha()
        g = plan.gradient(torch.conj(a))
        torch.cuda.synchronize()
        state["grads"].append(time.perf_counter() - state["t_grad"])
        state["alpha"] = a
        state["g"] = g

    def bench_step():
        if state["block"] == n_blocks:       # past the end of a solve: the next one
            finish()
            begin()
        advance_many([plan], [YO_BOTH], block, chunk=chunk, use_graph=not args.eager)
        state["block"] += 1

    begin()
    for _ in range(args.warmup):
        bench_step()
    torch.cuda.synchronize()
    # HIP events around every launch part's launches of the last `tail` steps of each block
    plan.set_timing(2, tail)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bench_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = [plan.timing(q) for q in range(6)]
    plan.set_timing(0, 0)
    ms = (t1 - t0) / args.steps * 1e3
    cells_per_step = plan.n_rhs * dev.cells * block
    value = cells_per_step / (ms / 1e3) / 1e9
    log(f"{ms:.1f} ms per block of {block} steps, {value:.2f} Gcell-updates/s")
    finish()
    s_grad = state["grads"][0]
    alpha = state["alpha"].abs().cpu().numpy()
    log(f"whole gradient {s_grad:.2f} s ({3600.0 / s_grad:.1f}/h); |alpha| "
        f"{np.round(alpha.ravel(), 4).tolist()}")
    bytes_model, _ = plan.model_bytes(YO_BOTH)
    eff_gbs = bytes_model * block / (ms / 1e3) / 1e9
    plan.reset(YO_BOTH)
    plan.advance(YO_BOTH, 4)
    sha = kernel_sha()
    parts = part_rooflines(plan, timed, tiling, "multiport", sha)
    for q in parts:
        log(f"{q['part']}: {q['ms_per_launch']:.4f} ms/launch over {q['launches_timed']} launches, "
            f"{q['bytes_per_launch'] / 1e9:.3f} GB algorithmic, {q['achieved']:.0f} GB/s "
            f"({q['frac']:.3f} of peak)")
    plan.close()
    del plan
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "multi-port: 600x400x120 cells at 20 nm (CPML 8), 1-to-4 "
                               "splitter-like SOI device, 250x150 design/controls, r=4, beta=16, "
                               "5 wavelengths 1.500-1.600 um x (1 forward + 4 adjoint port "
                               "sources) = 25 right-hand sides in the same launches, 20000 Yee "
                               f"steps per solve; one bench step = {block} whole Yee steps of all "
                               "25 right-hand sides (step launches, sources, DFT in the window), "
                               "inside a forward+adjoint solve that is run to its end and turned "
                               "into alpha and dF/dC",
                   "cells": dev.cells, "rhs": int(plan_rhs(dev)), "time_steps_per_solve": dev.n_steps,
                   "yee_steps_per_bench_step": block, "graph_chunk": chunk,
                   "tiling": list(tiling)},
        "gradients_per_hour": round(3600.0 / s_grad, 2),
        "s_per_gradient": round(s_grad, 2),
        "hbm_frac_model_bytes_whole_step": round(eff_gbs / HBM_PEAK_GBS, 4),
        "roofline": roofline_of(parts),
    }
    if not args.no_realistic:
        out["realistic"] = realistic_gradients(args, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)...")
        out["cpu_baseline"] = cpu_baseline(dev, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def plan_rhs(dev) -> int:
    return (len(dev.sources) + len(dev.ports)) * dev.n_freq


def _line(metric, value, unit, ms, args, cfg, extra, steps=1, warmup=0):
    out = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": cfg}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """8 designs of uneven size (1 wavelength, forward + adjoint each):
    shared launches with graph replays against one design at a time, (a)
    with the same graph replays and chunk (the gain of shared launches
    alone) and (b) as plain solves: the forward run, then the adjoint run,
    plain launches, no graph (no right-hand-side sharing); equal steps and
    windows, so equal accuracy."""
    import numpy as np
    import torch
    from paper_2505_03352_amd import batch
    from paper_2505_03352_amd.plan import plan_for
    from workloads import configs
    torch.cuda.set_device(0)
    devs = configs.batch(8)
    log("batch: " + ", ".join(f"{d.nx}x{d.ny}x{d.nz}/{d.n_steps}" for d in devs))
    cells = sum(2 * d.cells * d.n_steps for d in devs)
    plans = [plan_for(d, device="cuda:0", time_blocking=2) for d in devs]
    batch.shared_tiling(plans, 4, batch.DEFAULT_FLAGS_PAIRS, zchunk=batch.DEFAULT_ZCHUNK)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.solve(plans, chunk=args.chunk, use_graph=True)
    res_b = [(a.cpu().numpy(), g.cpu().numpy()) for a, g in batch.gradients(plans)]
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batched: {t_batch:.2f} s")

    def one_at_a_time(plain):
        torch.cuda.synchronize()
        t = time.perf_counter()
        same, worst = True, 0.0
        for p, (a0, g0) in zip(plans, res_b):
            if plain:
                p.run(1, chunk=args.chunk, use_graph=False)
                p.run(2, chunk=args.chunk, use_graph=False)
            else:
                p.run(3, chunk=args.chunk, use_graph=True)
            a = p.alpha()
            g = p.gradient(torch.conj(a)).cpu().numpy()
            a = a.cpu().numpy()
            same &= bool((a == a0).all() and (g == g0).all())
            worst = max(worst, float(np.abs(g - g0).max() / np.abs(g0).max()))
        torch.cuda.synchronize()
        return time.perf_counter() - t, same, worst

    t_seq, same, _ = one_at_a_time(False)
    log(f"one at a time, graph replays: {t_seq:.2f} s, identical results: {same}")
    t_plain, same_plain, worst_plain = one_at_a_time(True)
    log(f"one at a time, plain forward then adjoint runs: {t_plain:.2f} s, identical results: "
        f"{same_plain} (largest gradient difference {worst_plain:.1e} of its maximum)")
    for p in plans:
        p.close()

    def rec(t):
        return {"designs_per_h": round(3600 * len(devs) / t, 1),
                "gcell_updates_per_s": round(cells / t / 1e9, 3), "seconds": round(t, 3)}
    _line("designs/hour (batched, 8 uneven designs)", 3600 * len(devs) / t_batch, "designs/h",
          t_batch * 1e3, args,
          {"workload": "batch: 8 designs, axes uniform in 128..320 x 96..240 x 64..96 at 20 nm, "
                       "1 wavelength, forward + adjoint + gradient each, seeds 100..107"},
          {"gcell_updates_per_s": round(cells / t_batch / 1e9, 3),
           "one_at_a_time_graph": dict(rec(t_seq), identical_results=same),
           "one_at_a_time_plain": dict(rec(t_plain), identical_results=same_plain,
                                       max_gradient_diff_over_max=worst_plain,
                                       how="forward run then adjoint run per design, plain "
                                           "launches, no graph"),
           "speedup_vs_graph": round(t_seq / t_batch, 3),
           "speedup_vs_plain": round(t_plain / t_batch, 3)})


class PlainOneAtATime:
    """The serving baseline of plain solves: requests in arrival order, one
    at a time; each wavelength of a request is its own plan (one forward and
    one adjoint right-hand side, the request's steps and windows), run as a
    forward solve and then an adjoint solve with plain launches and no graph,
    with the served side's split and two steps per launch; the request's
    gradient is the sum over its wavelengths."""

    def __init__(self, torch, chunk):
        self.torch = torch
        self.chunk = chunk

    def run(self, trace, on_done=None):
        from paper_2505_03352_amd.plan import plan_for
        from paper_2505_03352_amd.serve import ServeStats, percentile
        from workloads import configs
        torch = self.torch
        t0 = time.perf_counter()
        lat, results, cu = [], [], 0.0
        for i, (arr, cls, lams) in enumerate(trace):
            now = time.perf_counter() - t0
            if now < arr:
                time.sleep(arr - now)
            n_steps = configs.serving_request(i, cls, lams).n_steps
            alphas, g_sum = [], None
            for lam in lams:
                dev = configs.serving_request(i, cls, [lam], n_steps=n_steps)
                p = plan_for(dev, device="cuda:0", time_blocking=2)
                p.set_tiling(4, 10, 200 | 512)      # the served side's split
                p.run(1, chunk=self.chunk, use_graph=False)
                p.run(2, chunk=self.chunk, use_graph=False)
                a = p.alpha()
                g = p.gradient(torch.conj(a))
                alphas.append(a.cpu().numpy())
                g_sum = g if g_sum is None else g_sum + g
                cu += 2 * dev.cells * dev.n_steps
                p.close()
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            lat.append(t - arr)
            results.append((alphas, g_sum.cpu().numpy()))
            if on_done is not None:
                on_done(i, t)
        makespan = (time.perf_counter() - t0) - min(t for t, _, _ in trace)
        import numpy as np
        st = ServeStats(n_done=len(lat), n_rejected=0, makespan_s=makespan, p50_s=percentile(lat, 50),
                        p99_s=percentile(lat, 99), mean_s=float(np.mean(lat)),
                        throughput_per_h=3600.0 * len(lat) / makespan, max_active=1, peak_bytes=0,
                        cell_updates=cu, latencies=lat)
        return st, results


def bench_serving(args):
    """The first N requests of the Poisson trace: continuous batching with
    `--slots` concurrent requests against (plain) one request at a time with
    plain forward-then-adjoint solves per wavelength, and (same) the served
    loop's own executor with one slot and the same route; `--sides` picks
    which of the three run."""
    import numpy as np
    import torch
    from paper_2505_03352_amd.serve import GpuExecutor, Request, Scheduler
    from workloads import configs
    torch.cuda.set_device(0)
    trace = [(t * 4.0 / args.rate, cls, lams)
             for t, cls, lams in configs.serving_trace()[:args.requests]]

    def build(p):
        i, cls, lams = p
        return configs.serving_request(i, cls, lams)

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    sides = [x for x in args.sides.split(",") if x]
    out, res = {}, {}
    for name in sides:
        t_start = time.perf_counter()

        def done(rid, t=None, name=name):
            if rid % 10 == 9:
                log(f"{name}: request {rid} done at {time.perf_counter() - t_start:.1f} s")

        if name == "plain":
            st, res[name] = PlainOneAtATime(torch, args.chunk).run(trace, on_done=done)
        else:
            slots = args.slots if name == "served" else 1
            # --pulse: multi-wavelength requests from pulse runs where cheaper
            ex = GpuExecutor(build, device="cuda:0", chunk=args.chunk, pulse_multi=args.pulse,
                             dft_stride=args.dft_stride)
            reqs = [Request(i, t, (i, cls, lams)) for i, (t, cls, lams) in enumerate(trace)]
            cap = args.max_cells if slots > 1 else None
            st = Scheduler(ex, max_slots=slots, hbm_budget=budget, chunk=args.chunk,
                           max_active_cells=cap, on_done=lambda r: done(r.rid)).run(reqs)
            res[name] = [(None, r.result["grad"]) for r in sorted(reqs, key=lambda r: r.rid)]
        torch.cuda.synchronize()
        out[name] = st
        log(f"{name}: {st.as_dict()}")
    diffs = {}
    if len(res) > 1:
        names = list(res)
        for other in names[1:]:
            d = max(float(np.abs(a[1] - b[1]).max() / np.abs(b[1]).max())
                    for a, b in zip(res[names[0]], res[other]))
            diffs[f"{names[0]}_vs_{other}_max_gradient_diff"] = d
            log(f"gradients {names[0]} vs {other}: largest difference {d:.1e} of the maximum")

    def rec(st):
        return {"designs_per_h": round(st.throughput_per_h, 1), "p50_s": round(st.p50_s, 3),
                "p99_s": round(st.p99_s, 3), "mean_s": round(st.mean_s, 3),
                "makespan_s": round(st.makespan_s, 2),
                "gcell_updates_per_s": round(st.cell_updates / st.makespan_s / 1e9, 3)}
    head = out.get("served") or next(iter(out.values()))
    extra = {k: rec(v) for k, v in out.items()}
    if "served" in out:
        for k in out:
            if k != "served":
                extra[f"speedup_vs_{k}"] = round(out["served"].throughput_per_h / out[k].throughput_per_h, 3)
    extra.update(diffs)
    _line("p50/p99 request latency and designs/hour (continuous batching)", head.throughput_per_h,
          "designs/h", head.makespan_s * 1e3, args,
          {"workload": f"serving: first {args.requests} of 200 Poisson arrivals at {args.rate:g} req/s, "
                       "sizes 96^3+-8 / 200x160x80 / 320x240x96, 1-3 wavelengths, forward + "
                       "adjoint + gradient, seed 200" + (
                           "; multi-wavelength requests from pulse runs where cheaper (served "
                           "and same)" if args.pulse else "; time-harmonic runs"),
           "sides": sides, "slots": args.slots,
           "max_active_cell_updates_per_step": args.max_cells,
           "hbm_budget_bytes": budget},
          extra)


def bench_batch_fd(args):
    """The differentiable batch's check: for each of the 8 batch designs, the
    autograd Function's gradient of sum |alpha|^2 against central
    differences (h = 1e-3) on 16 random control entries, the 32 perturbed
    forward runs of a design advancing together in shared launches."""
    import numpy as np
    import torch
    from paper_2505_03352_amd import YO_BOTH, YO_FORWARD, batch, fn
    from paper_2505_03352_amd.plan import plan_for
    from workloads import configs
    torch.cuda.set_device(0)
    h = 1e-3
    worst, rows = 0.0, []
    t0 = time.perf_counter()
    for d, dev in enumerate(configs.batch(8)):
        rng = np.random.default_rng(500 + d)
        flat = rng.choice(dev.C.size, size=16, replace=False)
        idx = [np.unravel_index(k, dev.C.shape) for k in flat]
        p = plan_for(dev, device="cuda:0")
        batch.shared_tiling([p], 4, batch.DEFAULT_FLAGS, zchunk=batch.DEFAULT_ZCHUNK)
        C = torch.as_tensor(dev.C, dtype=torch.float32, device="cuda:0").requires_grad_(True)
        a = fn.modal_coefficients(C, p, dev.beta, chunk=args.chunk)
        (a.abs() ** 2).sum().backward()
        g = C.grad.detach().cpu().numpy()
        p.close()
        plans = []
        for k in idx:
            for sgn in (1.0, -1.0):
                Cp = dev.C.copy()
                Cp[k] += sgn * h
                plans.append(plan_for(dev, device="cuda:0", C=Cp))
        batch.shared_tiling(plans, 4, batch.DEFAULT_FLAGS, zchunk=batch.DEFAULT_ZCHUNK)
        batch.solve(plans, which=YO_FORWARD, chunk=args.chunk)
        vals = [float((q.alpha().abs() ** 2).sum()) for q in plans]
        for q in plans:
            q.close()
        fd = np.array([(vals[2 * i] - vals[2 * i + 1]) / (2 * h) for i in range(16)])
        ga = np.array([g[k] for k in idx])
        err = float(np.max(np.abs(fd - ga)) / np.abs(g).max())
        rel = float(np.linalg.norm(fd - ga) / np.linalg.norm(ga))
        worst = max(worst, err)
        rows.append({"grid": [dev.nx, dev.ny, dev.nz], "steps": dev.n_steps,
                     "max_err_over_max_grad": err, "rel_l2_16": rel})
        log(f"design {d} {dev.nx}x{dev.ny}x{dev.nz}/{dev.n_steps}: max |fd - autograd| / max|g| "
            f"{err:.2e}, rel L2 over the 16 entries {rel:.2e} ({time.perf_counter() - t0:.0f} s)")
    out = {"metric": "autograd gradient vs central differences (batch designs)", "value": worst,
           "unit": "max |fd - autograd| / max |gradient|", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": round((time.perf_counter() - t0) * 1e3, 1), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch: 8 designs, axes uniform in 128..320 x 96..240 x 64..96 at "
                                  "20 nm, 1 wavelength, F = sum |alpha|^2; central differences "
                                  "h = 1e-3 on 16 random controls per design (seeds 500..507)"},
           "designs": rows}
    print(json.dumps(out), flush=True)


def bench_broadband(args):
    """Gradients of the realistic device's three wavelengths from pulse runs
    (one per source and per port, every wavelength's DFT accumulated in the
    same run) against the time-harmonic runs (one per source or port and
    wavelength): gradients per hour of each, and how far apart the two
    gradients and modal coefficients are."""
    import numpy as np
    import torch
    from paper_2505_03352_amd import YO_BOTH, autotune
    from paper_2505_03352_amd.plan import plan_for
    from workloads import configs
    torch.cuda.set_device(0)
    make = configs.multiport if args.device == "multiport" else configs.realistic
    dev = make()
    C = torch.as_tensor(dev.C, dtype=torch.float32, device="cuda:0")

    from paper_2505_03352_amd.plan import advance_many

    def grad(plan):
        # the run in pieces of 2500 steps with a progress line after each
        # (the same launches as one yo_run: reset, chunked graph replays,
        # finalize)
        plan.set_design(C, dev.beta)
        plan.reset(YO_BOTH)
        done = 0
        while done < plan.n_steps:
            k = min(2500, plan.n_steps - done)
            advance_many([plan], [YO_BOTH], k, chunk=args.chunk, use_graph=not args.eager)
            done += k
            if args.device == "multiport":
                torch.cuda.synchronize()
                log(f"  {done}/{plan.n_steps} steps")
        plan.finalize(YO_BOTH)
        a = plan.alpha()
        return a, plan.gradient(torch.conj(a))

    def timed(plan, n):
        if args.warmup > 0:
            grad(plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            a, g = grad(plan)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n, a.cpu().numpy(), g.cpu().numpy()

    ph = plan_for(dev, device="cuda:0", time_blocking=2)
    th = autotune.tune(ph, YO_BOTH, use_cache=False)
    s_h, a_h, g_h = timed(ph, args.steps)
    ph.close()
    log(f"time-harmonic: {s_h * 1e3:.1f} ms per gradient ({ph.n_rhs} runs x {dev.n_steps} steps)")
    n_h = ph.n_rhs
    dp = make(n_steps=args.pulse_steps or (7000 if args.device == "realistic" else 12000))
    w0, sig, t0 = dp.pulse(k=0.4 if args.pulse_k is None else args.pulse_k)
    pp = plan_for(dp, device="cuda:0", pulse=(w0 / dp.dt(), sig, t0, args.dft_stride), time_blocking=2)
    tp = autotune.tune(pp, YO_BOTH, use_cache=False)
    s_p, a_p, g_p = timed(pp, args.steps)
    ea = float(np.abs(a_p - a_h).max() / np.abs(a_h).max())
    eg = float(np.linalg.norm(g_p - g_h) / np.linalg.norm(g_h))
    cells = pp.n_stepped * dp.cells * dp.n_steps
    log(f"pulse: {s_p * 1e3:.1f} ms per gradient ({pp.n_stepped} runs x {dp.n_steps} steps, sigma "
        f"{sig:.0f}, t0 {t0:.0f}); alpha max diff {ea:.2e}, gradient rel L2 diff {eg:.2e}")
    pp.close()
    if args.device == "multiport":
        what = ("multi-port: 600x400x120 cells at 20 nm (CPML 8), 250x150 design/controls, r=4, "
                "beta=16, 5 wavelengths 1.500-1.600 um, 4 output ports")
    else:
        what = ("realistic: 320x240x96 cells at 20 nm (CPML 8), 100x100 design/controls, r=3, "
                "beta=8, wavelengths 1.50/1.55/1.60 um")
    _line(f"adjoint gradients/hour, {dev.n_freq} wavelengths (pulse excitation)", 3600.0 / s_p,
          "gradients/h", s_p * 1e3, args,
          {"workload": f"{what}; pulse runs (1 forward + {len(dev.ports)} adjoint, {dp.n_steps} "
                       f"steps, carrier mid-band, sigma {sig:.0f} steps, t0 {t0:.0f}) against "
                       f"time-harmonic runs ({n_h} runs, {dev.n_steps} steps)",
           "tiling_pulse": [tp["rows"], tp["zchunk"], tp["flags"]],
           "tiling_harmonic": [th["rows"], th["zchunk"], th["flags"]]},
          {"gcell_updates_per_s": round(cells / s_p / 1e9, 3),
           "time_harmonic_gradients_per_hour": round(3600.0 / s_h, 1),
           "speedup_vs_time_harmonic": round(s_h / s_p, 3),
           "alpha_max_rel_diff": ea, "gradient_rel_l2_diff": eg}, steps=args.steps,
          warmup=min(args.warmup, 1))


def bench_optimize(args):
    """The Sec. 4 optimizer loop on the two-wavelength demultiplexer analogue
    (1.30 um to output 1, 1.55 um to output 2): iterations per hour, with
    the objective, grey fraction and projection strength of each iteration.
    With --pulse the gradients come from pulse runs (one per source and per
    port for both wavelengths, --pulse-steps steps); one gradient of each
    kind at the same controls is compared first."""
    import numpy as np
    import torch
    from paper_2505_03352_amd import YO_BOTH, autotune, optimize
    from paper_2505_03352_amd.plan import plan_for
    from workloads import configs
    torch.cuda.set_device(0)
    dev = configs.demux()
    T = np.array([[[1.0, 0.0], [0.0, 1.0]]])     # [source][port][wavelength]: demux, no crosstalk
    log(f"demux: {dev.nx}x{dev.ny}x{dev.nz}, {dev.n_steps} steps, {dev.mc}x{dev.nc} controls")
    plan = plan_for(dev, device="cuda:0", time_blocking=2)
    tuned = autotune.tune(plan, YO_BOTH, use_cache=False)
    extra = {}
    run_dev, how = dev, f"1 forward + 2 adjoint per wavelength, {dev.n_steps} steps"
    if args.pulse:
        Tt = torch.as_tensor(T, dtype=torch.float32, device="cuda:0")
        Cc = torch.as_tensor(np.random.default_rng(3).uniform(0.3, 0.7, dev.C.shape),
                             dtype=torch.float32, device="cuda:0")

        def one(p):
            torch.cuda.synchronize()
            t = time.perf_counter()
            p.set_design(Cc, dev.beta)
            p.run(YO_BOTH, chunk=args.chunk)
            a = p.alpha()
            g = p.gradient(2.0 * (a.abs() ** 2 - Tt) * torch.conj(a))
            torch.cuda.synchronize()
            return time.perf_counter() - t, a.cpu().numpy(), g.cpu().numpy()

        s_h, a_h, g_h = one(plan)
        plan.close()
        run_dev = configs.demux(n_steps=args.pulse_steps or 12000)
        w0, sig, t0 = run_dev.pulse(k=1.0 if args.pulse_k is None else args.pulse_k)
        plan = plan_for(run_dev, device="cuda:0", pulse=(w0 / run_dev.dt(), sig, t0, args.dft_stride),
                        time_blocking=2)
        tuned = autotune.tune(plan, YO_BOTH, use_cache=False)
        s_p, a_p, g_p = one(plan)
        ea = float(np.abs(a_p - a_h).max() / np.abs(a_h).max())
        eg = float(np.linalg.norm(g_p - g_h) / np.linalg.norm(g_h))
        log(f"one gradient: time-harmonic {s_h:.2f} s, pulse {s_p:.2f} s; alpha max diff {ea:.2e}, "
            f"gradient rel L2 diff {eg:.2e}")
        how = (f"pulse runs: 1 forward + 2 adjoint for both wavelengths, {run_dev.n_steps} steps "
               f"(sigma {sig:.0f}, t0 {t0:.0f})")
        extra = {"time_harmonic_s_per_gradient": round(s_h, 3), "pulse_s_per_gradient": round(s_p, 3),
                 "alpha_max_rel_diff_vs_time_harmonic": ea, "gradient_rel_l2_diff_vs_time_harmonic": eg}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C, h = optimize.optimize(plan, dev.C, T, n_iter=args.iters, iters_total=100, chunk=args.chunk)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = plan.n_stepped * run_dev.cells * run_dev.n_steps * args.iters
    for i, (F, u, b) in enumerate(zip(h.F, h.u, h.beta)):
        log(f"iter {i}: F {F:.5f} u {u:.4f} beta {b:.2f} ({h.seconds[i]:.2f} s)")
    plan.close()
    extra.update({"gcell_updates_per_s": round(cells / dt / 1e9, 3),
                  "F": [round(x, 6) for x in h.F], "unbinarity": [round(x, 5) for x in h.u],
                  "beta": [round(x, 3) for x in h.beta]})
    _line("optimizer iterations/hour (demux analogue)", 3600.0 * args.iters / dt, "iterations/h",
          dt / args.iters * 1e3, args,
          {"workload": "demux analogue: 430x450x64 cells at 25 nm (CPML 8), 210x210-pixel design, "
                       f"36x36 controls from C = 1/2, 1.30/1.55 um, {how}; Adam lr 1e-3, "
                       "beta_min 10, gamma 0.95, u0 0.01, schedule length 100",
           "iterations": args.iters, "tiling": [tuned["rows"], tuned["zchunk"], tuned["flags"]]},
          extra, steps=args.iters)


if __name__ == "__main__":
    main()
