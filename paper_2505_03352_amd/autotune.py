"""Autotuner for the time-stepping kernel's work split.

Each step runs two launches, the interior tiles and the CPML shell; their
layout choices are independent except for what the two share (z-planes per
tile, waves per block, how the x-shell strips are cut).  For
each shared setting the tuner times every interior choice (cooperative
blocks or not, prefetch or not) with the interior launch alone and every
shell choice (cooperative, per-class code, prefetch) with the shell launch
alone, on the real grid with HIP events (the kernel-timing entry point
re-runs one step without advancing), and keeps the fastest sum.  Results are
cached in a JSON file keyed by the shape class (architecture, padded x
extent, ny, nz, number of right-hand sides, CPML width, time blocking), so
plans of the same class reuse the choice.  For a plan with time blocking it
also times two steps per launch (the two-step region's launch, with flag
2048 the z-slabs' two-step launch, the interior around them and the shell of
the paired steps, each with its own best choice) and keeps that when it is
faster per step; with two steps per launch chosen, it then times whole
steps with the two-step launch on a second stream beside the first step's
other launches (flag 1024) against the same launches in one stream, and keeps
the faster.  Every split gives bitwise the same fields, so tuning only
changes speed.

`tuned_splits.json` beside this file ships splits the tuner chose on an
MI355X for the benchmark devices, keyed the same way; `tune(...,
shipped=True)` applies a shipped split when the key matches instead of
sweeping (so a run and the hardware counters taken of that split agree).
"""
from __future__ import annotations

import json
import os
import threading
from typing import Iterable, Optional, Tuple

import torch

from ._abi import YO_BOTH

ROWS = 4
# shared settings: (z-planes per tile, flags from {1: full 62-cell x-shell strips,
# 128: x-shell strips sized so the interior strips are whole, 2: 8 waves per
# block}).  10 planes split the 79 planes between the z-slabs of a 96-plane
# grid with an 8-cell CPML into 8 tiles instead of 5: more, shorter tiles,
# 0.950 against 0.969 ms per step for 16 on the 320x240x96 device.  (Flag 256, the x-slab tiles in the interior launch,
# measured 6-10 % slower per step there and is left out of the sweep.)
SHARED: Tuple[Tuple[int, int], ...] = tuple((z, a | b) for z in (8, 10, 16, 32) for a in (0, 1, 128)
                                            for b in (0, 2))
INTERIOR_FLAGS = (0, 16, 32, 16 | 32)          # cooperative, no prefetch
# settings swept for two steps per launch (plans with time blocking): z-planes
# per tile and flags from {1, 128: x-shell cuts as above (with two steps per
# launch, 128 cuts whole 60-cell two-step strips); 2: 8 waves per block;
# 2048: the z-slabs under the two-step region take two steps per launch
# too}; for each, the two-step launch is timed with 4- and 6-row tiles
# (flag 4096), independent or cooperative (8192), and the fastest kept.  (Flag 256, the tiles that meet only the
# x-slabs run with the interior around the two-step region, measured slower
# and is left out.)
PAIR_SHARED: Tuple[Tuple[int, int], ...] = tuple((z, a | b | c) for z in (8, 10, 16) for a in (0, 1, 128)
                                                 for b in (0, 2) for c in (0, 2048))
# shell choices: cooperative blocks (4), per-class code (8), no prefetch
# (64), 6-row tiles (16384; not cooperative)
SHELL_FLAGS = tuple(a | b | c | d for a in (0, 4) for b in (0, 8) for c in (0, 64) for d in (0, 16384)
                    if not (a and d))
_lock = threading.Lock()


SHIPPED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_splits.json")


def shipped_splits() -> dict:
    try:
        with open(SHIPPED_PATH) as f:
            return {k: v for k, v in json.load(f).items() if not k.startswith("_")}
    except (OSError, ValueError):
        return {}


def cache_path() -> str:
    return os.environ.get("YEEOPT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "yeeopt", "autotune.json"))


def shape_key(plan, which: int) -> str:
    g = plan.grid
    tb = getattr(plan, "time_blocking", 1)
    nxp = (g["nx"] + 31) // 32 * 32
    nf, nr = plan.n_stepped_fwd, plan.n_stepped
    r = nf if which == 1 else (nr - nf if which == 2 else nr)
    arch = "gfx950"
    try:
        arch = torch.cuda.get_device_properties(plan.device).gcnArchName.split(":")[0]
    except Exception:
        pass
    return f"{arch}|nx{nxp}|ny{g['ny']}|nz{g['nz']}|R{r}|pml{max(g['npml'])}" + ("|tb2" if tb == 2 else "")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time(plan, zc, flags, part, which, n_launch, stream) -> float:
    plan.set_tiling(ROWS, zc, flags)
    plan.reset(which, stream)
    plan.time_kernel(part, 1, stream)                 # warm-up
    ms, _, _ = plan.time_kernel(part, n_launch, stream)
    return ms


def _time_steps(plan, zc, flags, which, n_steps, stream) -> float:
    """ms per step of `n_steps` whole steps as plain launches (HIP events
    on the plan's stream)."""
    from .plan import advance_many
    plan.set_tiling(ROWS, zc, flags)
    plan.reset(which, stream)
    advance_many([plan], [which], 2, chunk=2, use_graph=False, stream=stream)   # warm-up
    s = torch.cuda.current_stream() if stream is None else stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    advance_many([plan], [which], n_steps, chunk=n_steps, use_graph=False, stream=stream)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / n_steps


def tune(plan, which: int = YO_BOTH, shared: Optional[Iterable] = None, n_launch: int = 5,
         use_cache: bool = True, stream=None, pair_shared: Optional[Iterable] = None,
         shipped: bool = False) -> dict:
    """Pick and apply the fastest split for `plan`; returns the record.
    shipped: apply the shipped split of the plan's shape class when there
    is one (before the user cache and the sweep).

    Leaves the plan reset (fields zero) for `which`."""
    key = shape_key(plan, which)
    if shipped:
        rec = shipped_splits().get(key)
        if rec:
            plan.set_tiling(rec["rows"], rec["zchunk"], rec["flags"])
            plan.reset(which, stream)
            return dict(rec, cached=True, shipped=True)
    if use_cache:
        with _lock:
            rec = _load().get(key)
        if rec:
            plan.set_tiling(rec["rows"], rec["zchunk"], rec.get("flags", 0))
            plan.reset(which, stream)
            return dict(rec, cached=True)
    nz = plan.grid["nz"]
    timings = {}
    best = None
    for zc, base in (shared or SHARED):
        if zc > nz and zc != 8:
            continue
        ti = {f: _time(plan, zc, base | f, 0, which, n_launch, stream) for f in INTERIOR_FLAGS}
        ts = {f: _time(plan, zc, base | f, 1, which, n_launch, stream) for f in SHELL_FLAGS}
        fi = min(ti, key=ti.get)
        fs = min(ts, key=ts.get)
        total = ti[fi] + ts[fs]
        flags = base | fi | fs
        timings[f"z{zc}f{base}"] = dict(interior={str(k): round(v, 4) for k, v in ti.items()},
                                        shell={str(k): round(v, 4) for k, v in ts.items()},
                                        best=flags, ms=round(total, 4))
        if best is None or total < best[0]:
            best = (total, zc, flags)
    total, zc, flags = best
    if getattr(plan, "time_blocking", 1) == 2 and plan.n_steps >= 2:
        # two steps per launch over the two-step region: per step, half the
        # two-step launch, the interior around it and the shell (one launch
        # each per step), each with its own best choice; kept when it beats
        # the best single-step split
        for zc2, base in (pair_shared or PAIR_SHARED):
            if zc2 > nz and zc2 != 8:
                continue
            fl0 = base | 512
            t2 = _time(plan, zc2, fl0, 2, which, n_launch, stream)
            if t2 <= 0.0:
                break               # no two-step region on this grid
            # 6-row two-step tiles (flag 4096) and cooperative two-step
            # blocks (8192) where that launch runs faster
            for v in (4096, 8192, 4096 | 8192):
                t2b = _time(plan, zc2, (base | 512) | v, 2, which, n_launch, stream)
                if t2b < t2:
                    fl0, t2 = (base | 512) | v, t2b
            # the z-slabs' two-step launch (0: none, without 2048 or where
            # planes cut the region) and the shell of the paired steps
            t4 = _time(plan, zc2, fl0, 4, which, n_launch, stream)
            tf = {f: _time(plan, zc2, fl0 | f, 3, which, n_launch, stream) for f in (0, 32)}
            ts = {f: _time(plan, zc2, fl0 | f, 5, which, n_launch, stream) for f in SHELL_FLAGS}
            ff = min(tf, key=tf.get)
            fs = min(ts, key=ts.get)
            per_step = 0.5 * (t2 + t4) + tf[ff] + ts[fs]
            fl = fl0 | ff | fs
            timings[f"pairs_z{zc2}f{base}"] = dict(two_step=round(t2, 4), zslab_two_step=round(t4, 4),
                                                   frame={str(k): round(v, 4) for k, v in tf.items()},
                                                   shell={str(k): round(v, 4) for k, v in ts.items()},
                                                   best=fl, ms=round(per_step, 4))
            if per_step < total:
                total, zc, flags = per_step, zc2, fl
    overlap = None
    n_ov = 4 * n_launch
    if flags & 512 and plan.n_steps >= n_ov + 2:
        # the two-step launch beside the first step's frame and shell: the
        # parts' separate timings cannot tell, so whole steps are timed
        t_one = _time_steps(plan, zc, flags, which, n_ov, stream)
        t_two = _time_steps(plan, zc, flags | 1024, which, n_ov, stream)
        overlap = dict(one_stream=round(t_one, 4), two_streams=round(t_two, 4))
        if t_two < 0.99 * t_one:
            flags |= 1024
            total *= t_two / t_one
    plan.set_tiling(ROWS, zc, flags)
    plan.reset(which, stream)
    rec = dict(rows=ROWS, zchunk=zc, flags=flags, ms_per_step=total, timings=timings)
    if overlap:
        rec["overlap"] = overlap
    if use_cache:
        with _lock:
            d = _load()
            d[key] = rec
            _store(d)
    return dict(rec, cached=False)
