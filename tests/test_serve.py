"""Scheduler of the serving loop on the CPU, with a simulated executor and
clock: FIFO admission by slot and memory, continuous batching (work that
arrives while others run joins them at the next chunk), rejection of work
that can never fit, latency percentiles."""
import numpy as np
import pytest

from paper_2505_03352_amd.serve import Job, Request, Scheduler, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


class FakeExecutor:
    """A chunk of n steps over jobs J costs n * (launch + sum cells / rate):
    a fixed per-step overhead shared by everything in the launch."""

    def __init__(self, clock, launch=1e-4, rate=1e9, tail=0.01):
        self.clock, self.launch, self.rate, self.tail = clock, launch, rate, tail
        self.calls = []          # job ids per advance call
        self.started = []
        self.released = []

    def begin(self, clock):
        pass

    def prepare(self, req):
        cells, steps, nbytes = req.payload
        if cells <= 0:
            raise ValueError("empty grid")
        return Job(req, nbytes, steps, state=dict(cells=cells))

    def start(self, job):
        self.started.append(job.req.rid)

    def cells_per_step(self, job):
        return job.state["cells"]

    def advance(self, jobs, n):
        self.calls.append(tuple(j.req.rid for j in jobs))
        self.clock.t += n * (self.launch + sum(j.state["cells"] for j in jobs) / self.rate)

    def finish(self, job):
        job.handle = self.clock.t + self.tail

    def ready(self, job):
        return self.clock.t >= job.handle

    def wait_any(self, jobs):
        self.clock.t = max(self.clock.t, min(j.handle for j in jobs))

    def done_time(self, job):
        return job.handle

    def collect(self, job):
        return job.req.rid

    def release(self, job):
        self.released.append(job.req.rid)


def make(reqs):
    return [Request(i, t, p) for i, (t, p) in enumerate(reqs)]


def run(reqs, **kw):
    clk = FakeClock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, clock=clk, prep_workers=0, **kw)
    st = sch.run(reqs)
    return st, sch, ex


def test_everything_completes_in_fifo_order():
    rng = np.random.default_rng(5)
    t = np.cumsum(rng.exponential(0.05, 30))
    reqs = make([(float(t[i]), (int(rng.integers(1e5, 1e6)), int(rng.integers(50, 400)), 1 << 20))
                 for i in range(30)])
    st, sch, ex = run(reqs, max_slots=4, chunk=50)
    assert st.n_done == 30 and st.n_rejected == 0
    assert ex.started == sorted(ex.started)               # admitted in arrival order
    for r in reqs:
        assert r.t_admit >= r.arrival
        assert r.t_done > r.t_admit
        assert r.result == r.rid
    assert st.max_active <= 4
    assert sorted(ex.released) == list(range(30))


def test_late_arrival_joins_running_work():
    # A long request starts alone; a short one arrives while it runs and is
    # admitted at the next chunk boundary, finishing long before A.
    reqs = make([(0.0, (1_000_000, 2000, 1 << 20)), (0.05, (100_000, 100, 1 << 20))])
    st, sch, ex = run(reqs, max_slots=4, chunk=10)
    a, b = reqs
    assert b.t_admit < a.t_done
    assert b.t_done < a.t_done
    assert any(len(c) == 2 for c in ex.calls)              # shared launches
    # B waits at most one chunk of A's stepping before it is admitted
    one_chunk = 10 * (1e-4 + 1_000_000 / 1e9)
    assert b.t_admit - b.arrival <= one_chunk + 1e-12


def test_memory_budget_limits_admission():
    reqs = make([(0.0, (100_000, 200, 600)) for _ in range(6)])
    st, sch, ex = run(reqs, max_slots=8, hbm_budget=1300, chunk=20)
    assert st.n_done == 6
    assert st.peak_bytes <= 1300
    assert st.max_active == 2                              # two of 600 B fit in 1300 B
    # two at a time: admissions come in pairs
    admits = [t for t, k, _ in sch.events if k == "admit"]
    assert len(set(np.round(admits, 12))) == 3


def test_slot_cap():
    reqs = make([(0.0, (50_000, 100, 1)) for _ in range(10)])
    st, sch, ex = run(reqs, max_slots=3, chunk=25)
    assert st.max_active == 3
    assert max(len(c) for c in ex.calls) == 3


def test_oversize_and_broken_requests_are_rejected():
    reqs = make([(0.0, (100_000, 100, 10)), (0.0, (100_000, 100, 10_000)), (0.0, (0, 100, 10)),
                 (0.01, (100_000, 100, 10))])
    st, sch, ex = run(reqs, max_slots=2, hbm_budget=1000, chunk=20)
    assert st.n_done == 2 and st.n_rejected == 2
    assert "exceeds the budget" in reqs[1].error
    assert "prepare" in reqs[2].error
    assert reqs[3].t_done is not None


def test_idle_gaps_wait_for_arrivals():
    reqs = make([(0.0, (10_000, 10, 1)), (5.0, (10_000, 10, 1))])
    st, sch, ex = run(reqs, max_slots=2, chunk=10)
    assert reqs[1].t_admit >= 5.0
    assert st.makespan_s >= 5.0


def test_percentiles_and_stats():
    rng = np.random.default_rng(1)
    t = np.cumsum(rng.exponential(0.2, 40))
    reqs = make([(float(t[i]), (200_000, 300, 1)) for i in range(40)])
    st, sch, ex = run(reqs, max_slots=4, chunk=30)
    lat = [r.latency for r in reqs]
    assert st.p50_s == pytest.approx(np.percentile(lat, 50))
    assert st.p99_s == pytest.approx(np.percentile(lat, 99))
    assert st.p50_s <= st.p99_s
    assert st.throughput_per_h == pytest.approx(3600 * 40 / st.makespan_s)
    assert st.cell_updates == pytest.approx(40 * 200_000 * 300)
    assert percentile([], 50) != percentile([], 50)        # nan


def test_bad_parameters():
    with pytest.raises(ValueError):
        Scheduler(FakeExecutor(FakeClock()), max_slots=0)


def test_work_cap_limits_concurrency_but_not_progress():
    # each request steps 300k cells; a cap of 700k cells admits two at a time,
    # and a single request above the cap still runs (alone)
    reqs = make([(0.0, (300_000, 100, 1)) for _ in range(5)] + [(0.0, (900_000, 50, 1))])
    st, sch, ex = run(reqs, max_slots=8, chunk=20, max_active_cells=700_000)
    assert st.n_done == 6
    assert max(len(c) for c in ex.calls) == 2
    assert any(c == (5,) for c in ex.calls)               # the big one ran alone


def test_completion_callback_sees_every_finished_request():
    reqs = make([(0.01 * i, (200000, 100, 1 << 20)) for i in range(6)])
    seen = []
    clock = FakeClock()
    ex = FakeExecutor(clock)
    sch = Scheduler(ex, max_slots=3, hbm_budget=1 << 30, chunk=50, clock=clock, prep_workers=0,
                    on_done=lambda r: seen.append((r.rid, r.t_done is not None)))
    st = sch.run(reqs)
    assert st.n_done == 6
    assert sorted(rid for rid, _ in seen) == list(range(6))
    assert all(ok for _, ok in seen)


def test_failed_solve_is_reported_and_the_others_finish():
    """A request whose solve fails (the library's watchdog raises from
    finalize when the fields diverged) leaves with its error, frees its
    memory, and does not count as done; the rest complete."""
    class Failing(FakeExecutor):
        def collect(self, job):
            if job.req.rid == 2:
                raise RuntimeError("YO_EUNSTABLE: non-finite phasors")
            return job.req.rid

    reqs = make([(0.0, (200_000, 100, 10)) for _ in range(5)])
    clock = FakeClock()
    ex = Failing(clock)
    seen = []
    sch = Scheduler(ex, max_slots=2, hbm_budget=25, chunk=20, clock=clock, prep_workers=0,
                    on_done=lambda r: seen.append(r.rid))
    st = sch.run(reqs)
    assert st.n_done == 4 and st.n_failed == 1 and st.n_rejected == 0
    assert "solve" in reqs[2].error and "EUNSTABLE" in reqs[2].error
    assert reqs[2].result is None
    assert [r.result for r in reqs if r.rid != 2] == [0, 1, 3, 4]
    assert sorted(ex.released) == list(range(5))
    assert sorted(seen) == list(range(5))
    assert len(st.latencies) == 4
