"""Batched solves: many plans (designs of uneven size, each with its own
wavelengths, sources and ports) advanced in the same launches.

Every step launch covers every tile of every right-hand side of every plan
in the batch (the library's multi-plan entry point, ``yo_advance_many``);
chunks of steps are captured once as a HIP graph and replayed.  Plans keep
their own step counters and step counts: a plan whose run is complete
drops out at the next chunk boundary, so the batch shrinks instead of
idling.  The paper runs independent channels one after another (Sec. 5);
this is the same work sharing the GPU.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from ._abi import YO_BOTH
from .plan import Plan, advance_many


# Split for shared launches of uneven designs: x-shell strips that leave
# whole interior strips, CPML shell with per-class code and no prefetch, 10
# z-planes per tile (8 designs of 128..320 x 96..240 x 64..96 cells: 9.74 s
# against 9.91 s with 16 planes and 10.02 s with flags 73)
DEFAULT_FLAGS = 200
DEFAULT_ZCHUNK = 10
# the same with two steps per launch over each plan's interior (plans made
# with time_blocking=2; bitwise the same results)
DEFAULT_FLAGS_PAIRS = 200 | 512


def shared_tiling(plans: Sequence[Plan], rows: int = 4, flags: int = DEFAULT_FLAGS,
                  zchunk: Optional[int] = None):
    """Give every plan the same split flags (required to share launches);
    the z-chunk stays per plan unless given."""
    for p in plans:
        zc = zchunk if zchunk is not None else getattr(p, "tiling", (rows, 16, flags))[1]
        p.set_tiling(rows, zc, flags)


def solve(plans: Sequence[Plan], which: int = YO_BOTH, chunk: int = 100, use_graph: bool = True,
          stream=None, reset: bool = True) -> None:
    """Run every plan of the list to its own step count in shared launches,
    then finalize them (the steps are asynchronous on `stream`; finalize
    synchronises it to read the watchdog and raises YeeOptError(YO_EUNSTABLE)
    for a plan whose fields diverged)."""
    plans = list(plans)
    if reset:
        for p in plans:
            p.reset(which, stream)
    done = {id(p): 0 for p in plans}
    active: List[Plan] = [p for p in plans if p.n_steps > 0]
    while active:
        left = min(p.n_steps - done[id(p)] for p in active)
        # whole chunks where possible (graph replays), the remainder eagerly
        n = left if left < chunk else (left // chunk) * chunk
        advance_many(active, [which] * len(active), n, chunk=chunk, use_graph=use_graph,
                     stream=stream)
        for p in active:
            done[id(p)] += n
        active = [p for p in active if done[id(p)] < p.n_steps]
    for p in plans:
        p.finalize(which, stream)


def gradients(plans: Sequence[Plan], objective="abs2", stream=None):
    """alpha and dF/dC of F = sum |alpha|^2 for each plan of a finished
    YO_BOTH batch."""
    out = []
    for p in plans:
        a = p.alpha(stream)
        if objective != "abs2":
            raise ValueError("only the |alpha|^2 objective is built in")
        g = p.gradient(torch.conj(a), stream)
        out.append((a, g))
    return out
