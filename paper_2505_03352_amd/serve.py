"""Continuous-batching request loop for design evaluations.

A request is one design evaluation: forward and adjoint runs over its
wavelengths, alpha and the gradient dF/dC.  Requests arrive over time
(their arrival times are given); the loop

  * prepares each arrived request on the host (geometry, plan descriptors)
    in a worker thread, in arrival order;
  * admits the request at the head of the queue when a slot is free, its
    device footprint fits in the free part of the HBM budget and, if a work
    cap is set, the cell-updates per step of everything admitted stay under
    it (more resident work than saturates the GPU's bandwidth only stretches
    every latency; FIFO: a request that does not fit yet holds back the ones
    behind it);
  * advances every admitted request together, in shared launches, one chunk
    of steps at a time; new requests join and finished ones leave at chunk
    boundaries, so requests that arrive while others run overlap with them
    on the GPU;
  * on completion, enqueues finalize, alpha and the gradient, and releases
    the request's memory once they are done; a request whose solve fails
    (e.g. fields that diverged) leaves with its `error` set and no result,
    and the others go on.

Each request keeps its own fields, counters and results, and a right-hand
side's update does not depend on what else shares the launch, so a result
is the same alone and in a mix.

A request with several wavelengths may instead be evaluated from pulse
runs (one per source and per port for all its wavelengths, Sec. 2's
Fourier-transform route) when that takes fewer cell-updates than one
time-harmonic run per wavelength (`GpuExecutor(pulse_multi=True)`).

The scheduler is independent of the GPU: it drives an executor (prepare,
start, advance, finish, ready, collect, release) and a clock, so the
admission logic runs on the CPU with a simulated executor in the tests.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time
from dataclasses import dataclass, field
from typing import Any, Callable, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float                     # seconds from the start of the run
    payload: Any                       # what the executor's prepare() turns into a job
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Any = None
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


@dataclass
class Job:
    req: Request
    footprint: int                     # device bytes held while admitted
    n_steps: int
    state: Any = None
    steps_done: int = 0
    handle: Any = None


class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        dt = t - self.now()
        if dt > 0:
            time.sleep(min(dt, 0.05))


def percentile(values: Sequence[float], q: float) -> float:
    """Linear-interpolation percentile (q in [0, 100])."""
    v = np.sort(np.asarray(values, np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, q))


@dataclass
class ServeStats:
    n_done: int
    n_rejected: int
    makespan_s: float
    p50_s: float
    p99_s: float
    mean_s: float
    throughput_per_h: float
    max_active: int
    peak_bytes: int
    cell_updates: float = 0.0
    n_failed: int = 0
    latencies: List[float] = field(default_factory=list)

    def as_dict(self) -> dict:
        d = dict(self.__dict__)
        d.pop("latencies")
        return d


class Scheduler:
    """FIFO admission by slot and HBM footprint; chunked shared stepping."""

    def __init__(self, executor, max_slots: int = 8, hbm_budget: int = 64 << 30, chunk: int = 100,
                 clock=None, prep_workers: int = 2, max_active_cells: Optional[float] = None,
                 on_done: Optional[Callable] = None):
        if max_slots < 1 or chunk < 1:
            raise ValueError("max_slots and chunk must be >= 1")
        self.ex = executor
        self.max_slots = int(max_slots)
        self.budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.clock = clock or RealClock()
        self.prep_workers = prep_workers
        self.max_active_cells = max_active_cells
        self.on_done = on_done               # called with each finished request
        self.events: List[tuple] = []      # (time, kind, rid) for inspection

    def _log(self, kind, rid):
        self.events.append((self.clock.now(), kind, rid))

    def run(self, requests: Sequence[Request]) -> ServeStats:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: collections.deque = collections.deque()     # (req, future)
        active: List[Job] = []
        retiring: List[Job] = []
        used = 0
        max_active = 0
        peak = 0
        cell_updates = 0.0
        done: List[Request] = []
        rejected: List[Request] = []
        failed: List[Request] = []
        pool = cf.ThreadPoolExecutor(max_workers=max(1, self.prep_workers)) if self.prep_workers else None
        self.ex.begin(self.clock)

        def prepare(req):
            return self.ex.prepare(req)

        try:
            while pending or queue or active or retiring:
                now = self.clock.now()
                # arrivals
                while pending and pending[0].arrival <= now:
                    r = pending.popleft()
                    fut = pool.submit(prepare, r) if pool else _Done(prepare, r)
                    queue.append((r, fut))
                    self._log("arrive", r.rid)
                # retire finished work whose results are ready
                for j in list(retiring):
                    if self.ex.ready(j):
                        try:
                            j.req.result = self.ex.collect(j)
                        except Exception as e:      # noqa: BLE001  (a solve that failed)
                            j.req.result = None
                            j.req.error = f"solve: {e}"
                        t = self.ex.done_time(j)
                        j.req.t_done = t if t is not None else self.clock.now()
                        self.ex.release(j)
                        used -= j.footprint
                        retiring.remove(j)
                        (failed if j.req.error else done).append(j.req)
                        if self.on_done is not None:
                            self.on_done(j.req)
                        self._log("fail" if j.req.error else "done", j.req.rid)
                # admissions, FIFO
                while queue and len(active) + len(retiring) < self.max_slots:
                    r, fut = queue[0]
                    if not fut.done():
                        break
                    try:
                        job = fut.result()
                    except Exception as e:          # a request that cannot be built
                        queue.popleft()
                        r.error = f"prepare: {e}"
                        rejected.append(r)
                        self._log("reject", r.rid)
                        continue
                    if job.footprint > self.budget:
                        queue.popleft()
                        r.error = f"footprint {job.footprint} B exceeds the budget {self.budget} B"
                        self.ex.release(job)
                        rejected.append(r)
                        self._log("reject", r.rid)
                        continue
                    if used + job.footprint > self.budget:
                        break
                    if self.max_active_cells is not None and active:
                        work = sum(self.ex.cells_per_step(j) for j in active)
                        if work + self.ex.cells_per_step(job) > self.max_active_cells:
                            break
                    queue.popleft()
                    used += job.footprint
                    peak = max(peak, used)
                    self.ex.start(job)
                    r.t_admit = self.clock.now()
                    active.append(job)
                    self._log("admit", r.rid)
                max_active = max(max_active, len(active) + len(retiring))
                if active:
                    n = min(self.chunk, min(j.n_steps - j.steps_done for j in active))
                    self.ex.advance(active, n)
                    for j in active:
                        j.steps_done += n
                        cell_updates += n * self.ex.cells_per_step(j)
                    for j in [j for j in active if j.steps_done >= j.n_steps]:
                        active.remove(j)
                        self.ex.finish(j)
                        retiring.append(j)
                    continue
                # nothing to step: wait for results, a preparation or an arrival
                if retiring:
                    self.ex.wait_any(retiring)
                elif queue:
                    r, fut = queue[0]
                    if not fut.done():
                        cf.wait([fut], timeout=0.05)
                elif pending:
                    self.clock.sleep_until(pending[0].arrival)
        finally:
            if pool:
                pool.shutdown(wait=True)
        lat = [r.latency for r in done]
        makespan = max([r.t_done for r in done], default=0.0) - min(
            [r.arrival for r in requests], default=0.0)
        return ServeStats(
            n_done=len(done), n_rejected=len(rejected), makespan_s=makespan,
            p50_s=percentile(lat, 50), p99_s=percentile(lat, 99),
            mean_s=float(np.mean(lat)) if lat else float("nan"),
            throughput_per_h=3600.0 * len(done) / makespan if makespan > 0 else float("nan"),
            max_active=max_active, peak_bytes=peak, cell_updates=cell_updates, n_failed=len(failed),
            latencies=lat)


class _Done:
    """Synchronous stand-in for a future."""

    def __init__(self, fn, *a):
        try:
            self._v, self._e = fn(*a), None
        except Exception as e:   # noqa: BLE001
            self._v, self._e = None, e

    def done(self):
        return True

    def result(self):
        if self._e:
            raise self._e
        return self._v


# ---------------------------------------------------------------- GPU executor
def pulse_plan(dev, periods: float = 2.0, m: float = 4.5, frac: float = 1.0, tail: int = 1000):
    """Pulse excitation for a multi-wavelength device, or None when one
    time-harmonic run per wavelength is cheaper.  The carrier sits mid-band,
    sigma is `periods` carrier periods (its spectrum stays within a few per
    cent of flat over a 1.50-1.60 um band), the centre m sigma from the
    start; the run lasts `frac` of the time-harmonic run, at least the pulse
    (2 m sigma) plus `tail` steps for the field to die away.  Returns
    (omega0 rad/s, sigma, t0, n_steps) with times in steps."""
    if dev.n_freq < 2:
        return None
    w = [dev.omega_dt(lam) for lam in dev.wavelengths]
    w0 = 0.5 * (min(w) + max(w))
    sigma = periods * 2.0 * np.pi / w0
    t0 = m * sigma
    n = int(max(frac * dev.n_steps, 2 * t0 + tail))
    if n >= dev.n_freq * dev.n_steps:
        return None
    dt = dev.courant * dev.dx / 299792458.0
    return w0 / dt, sigma, t0, n


class GpuExecutor:
    """Runs jobs through the library.  Set-up (workspace, background,
    modes, design) is enqueued on a set-up stream so it overlaps the
    stepping of admitted work on the compute stream; the compute stream
    waits for a job's set-up before its first chunk.  At most two chunks
    are in flight, which keeps admission decisions close to the GPU's
    progress.  The default split is the batch executor's (rows 4, 10
    z-planes per tile, flags 200), since admitted requests share launches."""

    def __init__(self, build: Callable, device="cuda:0", tiling=None, use_graph=False,
                 chunk: int = 100, pulse_multi: bool = False, dft_stride: int = 4,
                 time_blocking: int = 2):
        import torch
        from . import _abi  # noqa: F401  (fails loudly without the library)
        self.torch = torch
        self.build = build                 # payload -> workloads.Device-like description
        self.device = torch.device(device)
        # plans take two steps per launch over their interior by default
        # (bitwise the same results); the split: whole interior x-strips,
        # per-class shell code without prefetch, 10-plane tiles
        self.time_blocking = int(time_blocking)
        self.tiling = tiling if tiling is not None else (4, 10, 200 | (512 if self.time_blocking == 2 else 0))
        self.use_graph = use_graph
        self.chunk = chunk
        self.pulse_multi = pulse_multi
        self.dft_stride = dft_stride       # pulse runs: the DFT samples every dft_stride-th step
        self.compute = torch.cuda.Stream(self.device)
        self.setup = torch.cuda.Stream(self.device)
        self._inflight = collections.deque()
        self.start_event = None
        self.anchor = 0.0

    def begin(self, clock):
        """Tie GPU event times to the scheduler's clock: an event recorded on
        the idle compute stream marks clock time `anchor`."""
        self.compute.synchronize()
        self.start_event = self.torch.cuda.Event(enable_timing=True)
        self.start_event.record(self.compute)
        self.start_event.synchronize()
        self.anchor = clock.now()

    def prepare(self, req: Request) -> Job:
        from .plan import Plan, freqs_of, grid_design_of
        dev = self.build(req.payload)
        pulse = pulse_plan(dev) if self.pulse_multi else None
        if pulse is not None:
            dev.n_steps = pulse[3]
        grid, design = grid_design_of(dev)
        plan = Plan(grid, design, dev.n_steps, freqs_of(dev), [m.plane for m in dev.sources],
                    [m.plane for m in dev.ports], device=self.device,
                    pulse=None if pulse is None else tuple(pulse[:3]) + (self.dft_stride,),
                    time_blocking=self.time_blocking)
        plan.set_tiling(*self.tiling)
        host = dict(kappa=self.torch.as_tensor(dev.kappa_bg, dtype=self.torch.float32),
                    mask=self.torch.as_tensor(dev.mask_hr, dtype=self.torch.float32),
                    C=self.torch.as_tensor(dev.C, dtype=self.torch.float32))
        # workspace, plus the dense background copy the plan holds and the
        # design inputs and outputs
        extra = 4 * (3 * dev.cells + plan.canvas_shape[0] * plan.canvas_shape[1]
                     + 2 * dev.mc * dev.nc) + 8 * plan.n_rhs + 4096
        job = Job(req, plan.workspace_bytes + 256 + extra, dev.n_steps)
        job.state = dict(plan=plan, dev=dev, host=host, cells=dev.cells * plan.n_stepped)
        return job

    def start(self, job: Job):
        torch = self.torch
        st = job.state
        plan, dev, host = st["plan"], st["dev"], st["host"]
        with torch.cuda.stream(self.setup):
            plan.bind(None, self.setup)
            plan.set_background(host["kappa"], host["mask"], self.setup)
            for s, m in enumerate(dev.sources):
                plan.set_source_mode(s, m.h, self.setup)
            for q, m in enumerate(dev.ports):
                plan.set_port_mode(q, m.e, m.h, self.setup)
            plan.set_design(host["C"], dev.beta, self.setup)
            plan.reset(3, self.setup)
            ev = torch.cuda.Event()
            ev.record(self.setup)
        self.compute.wait_event(ev)
        st["host"] = None

    def cells_per_step(self, job: Job) -> float:
        return float(job.state["cells"])

    def advance(self, jobs: Sequence[Job], n: int):
        from .plan import advance_many
        plans = [j.state["plan"] for j in jobs]
        advance_many(plans, [3] * len(plans), n, chunk=self.chunk, use_graph=self.use_graph,
                     stream=self.compute)
        ev = self.torch.cuda.Event()
        ev.record(self.compute)
        self._inflight.append(ev)
        while len(self._inflight) > 2:
            self._inflight.popleft().synchronize()

    def finish(self, job: Job):
        from ._abi import YeeOptError
        torch = self.torch
        plan = job.state["plan"]
        with torch.cuda.stream(self.compute):
            try:
                plan.finalize(3, self.compute)
                a = plan.alpha(self.compute)
                g = plan.gradient(torch.conj(a), self.compute)
                job.state["out"] = (a, g)
            except YeeOptError as e:         # e.g. the watchdog: the fields diverged
                job.state["error"] = e
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(self.compute)
        job.handle = ev

    def ready(self, job: Job) -> bool:
        return job.handle.query()

    def wait_any(self, jobs: Sequence[Job]):
        jobs[0].handle.synchronize()

    def done_time(self, job: Job) -> float:
        return self.anchor + self.start_event.elapsed_time(job.handle) / 1e3

    def collect(self, job: Job):
        if job.state.get("error") is not None:
            raise job.state["error"]
        a, g = job.state["out"]
        return dict(alpha=a.cpu().numpy(), grad=g.cpu().numpy())

    def release(self, job: Job):
        job.state["plan"].close()
        job.state = None
