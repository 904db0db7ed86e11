"""Autotuner for the time-stepping kernel's tile shape.

For a plan it times every candidate (rows per wave, z-planes per wave, layout flags) on
the real grid with HIP events, using the kernel-timing entry point (which
re-runs one step without advancing), and keeps the fastest.  Results are
cached in a JSON file keyed by the shape class (architecture, padded x
extent, ny, nz, number of right-hand sides, CPML width), so plans of the
same class reuse the choice.  Any tile shape gives bitwise the same fields,
so tuning only changes speed.
"""
from __future__ import annotations

import json
import os
import threading
from typing import Iterable, Optional, Tuple

import torch

from ._abi import YO_BOTH

# (rows per wave, z-planes per wave, flags): flag 1 = full-width CPML x-strips,
# flag 2 = 8 waves per block, flag 4 = cooperative blocks (waves stacked in y),
# flag 8 / 16 = one launch for all CPML classes (per-class code / code of all
# axes).  Eight-row tiles run two waves per SIMD; only a few are tried.
CANDIDATES: Tuple[Tuple[int, int, int], ...] = tuple(
    [(4, z, a | b | c | d) for z in (8, 16, 32) for a in (0, 1) for b in (0, 2) for c in (0, 4)
     for d in (0, 8, 16)]
    + [(8, z, f) for z in (8, 16) for f in (1, 9, 17)])
# what one step launches: the interior class and the CPML classes
TIMED_CLASSES = (0, 8)
_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("YEEOPT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "yeeopt", "autotune.json"))


def shape_key(plan, which: int) -> str:
    g = plan.grid
    nxp = (g["nx"] + 31) // 32 * 32
    r = plan.n_fwd if which == 1 else (plan.n_rhs - plan.n_fwd if which == 2 else plan.n_rhs)
    arch = "gfx950"
    try:
        arch = torch.cuda.get_device_properties(plan.device).gcnArchName.split(":")[0]
    except Exception:
        pass
    return f"{arch}|nx{nxp}|ny{g['ny']}|nz{g['nz']}|R{r}|pml{max(g['npml'])}"


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


def tune(plan, which: int = YO_BOTH, candidates: Optional[Iterable] = None, n_launch: int = 5,
         use_cache: bool = True, stream=None) -> dict:
    """Pick and apply the fastest tiling for `plan`; returns the record.

    Leaves the plan reset (fields zero) for `which`."""
    key = shape_key(plan, which)
    if use_cache:
        with _lock:
            rec = _load().get(key)
        if rec:
            plan.set_tiling(rec["rows"], rec["zchunk"], rec.get("flags", 0))
            return dict(rec, cached=True)
    timings = {}
    nz = plan.grid["nz"]
    for rows, zc, fl in (candidates or CANDIDATES):
        if zc > nz and zc != 8:
            continue
        plan.set_tiling(rows, zc, fl)
        plan.reset(which, stream)
        t0 = 0.0
        for cls in TIMED_CLASSES:
            plan.time_kernel(cls, 1, stream)          # warm-up
            ms, _, _ = plan.time_kernel(cls, n_launch, stream)
            t0 += ms
        timings[f"{rows}x{zc}x{fl}"] = t0
    best = min(timings, key=timings.get)
    rows, zc, fl = (int(v) for v in best.split("x"))
    plan.set_tiling(rows, zc, fl)
    plan.reset(which, stream)
    rec = dict(rows=rows, zchunk=zc, flags=fl, ms_per_step=timings[best], timings=timings)
    if use_cache:
        with _lock:
            d = _load()
            d[key] = rec
            _store(d)
    return dict(rec, cached=False)
