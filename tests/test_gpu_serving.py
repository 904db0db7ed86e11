"""Batched and served solves on the GPU: every result equals the same
request solved alone (the stepping of one right-hand side does not depend
on what shares its launches)."""
import sys

import numpy as np
import pytest
import torch

from workloads import configs

pytestmark = [pytest.mark.gpu]

UM = 1e-6


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03352_amd import _abi
    _abi.lib()


def test_batch_solve_matches_individual_runs():
    from paper_2505_03352_amd import batch
    from paper_2505_03352_amd.plan import plan_for
    devs = [configs.micro(n_steps=530, seed=11), configs.micro(n_steps=700, seed=12, nx=34, ny=28),
            configs.micro(n_steps=610, seed=13, nz=20, wavelengths=[0.8 * UM, 0.85 * UM])]
    alone = []
    for d in devs:
        say(f"alone {d.nx}x{d.ny}x{d.nz} steps {d.n_steps}")
        p = plan_for(d)
        p.set_tiling(4, 8, 1)
        p.run(3, chunk=64, use_graph=False)
        a = p.alpha()
        g = p.gradient(torch.conj(a))
        alone.append((a.cpu().numpy(), g.cpu().numpy()))
        p.close()
    say("batch.solve with graphs, chunk 64")
    plans = [plan_for(d) for d in devs]
    batch.shared_tiling(plans, 4, 1, zchunk=8)
    batch.solve(plans, chunk=64, use_graph=True)
    for p, (a0, g0), (a, g) in zip(plans, alone, batch.gradients(plans)):
        assert np.array_equal(a.cpu().numpy(), a0)
        assert np.array_equal(g.cpu().numpy(), g0)
        p.close()
    say("batch.solve with two steps per launch (the bench's batch split)")
    plans = [plan_for(d, time_blocking=2) for d in devs]
    batch.shared_tiling(plans, 4, batch.DEFAULT_FLAGS_PAIRS, zchunk=8)
    batch.solve(plans, chunk=64, use_graph=True)
    for p, (a0, g0), (a, g) in zip(plans, alone, batch.gradients(plans)):
        assert np.array_equal(a.cpu().numpy(), a0)
        assert np.array_equal(g.cpu().numpy(), g0)
        p.close()


def _serve(payloads, arrivals, max_slots, chunk=100, pulse=False):
    from paper_2505_03352_amd.serve import GpuExecutor, Request, Scheduler

    def build(p):
        i, cls, lams, steps = p
        return configs.serving_request(i, cls, lams, n_steps=steps)

    # two steps per launch over each request's interior (the executor's default)
    ex = GpuExecutor(build, tiling=(4, 16, 1 | 512), chunk=chunk, pulse_multi=pulse)
    reqs = [Request(i, t, p) for i, (t, p) in enumerate(zip(arrivals, payloads))]
    st = Scheduler(ex, max_slots=max_slots, chunk=chunk, prep_workers=2).run(reqs)
    torch.cuda.synchronize()
    return reqs, st


def test_served_results_equal_alone_results():
    payloads = [(0, "small", [1.55 * UM], 900), (1, "small", [1.50 * UM, 1.60 * UM], 1200),
                (2, "small", [1.55 * UM], 700), (3, "small", [1.50 * UM], 1000)]
    say("one at a time")
    alone, st1 = _serve(payloads, [0.0] * 4, max_slots=1)
    assert st1.n_done == 4 and st1.max_active == 1
    say("in a mix, staggered arrivals")
    mixed, st2 = _serve(payloads, [0.0, 0.0, 0.02, 0.04], max_slots=4, chunk=50)
    assert st2.n_done == 4 and st2.max_active >= 2
    for a, m in zip(alone, mixed):
        assert np.isfinite(a.result["grad"]).all()
        assert np.abs(a.result["alpha"]).max() > 0
        assert np.array_equal(a.result["alpha"], m.result["alpha"])
        assert np.array_equal(a.result["grad"], m.result["grad"])
    say(f"alone makespan {st1.makespan_s:.3f} s, mixed {st2.makespan_s:.3f} s, "
        f"p50 {st2.p50_s:.3f} p99 {st2.p99_s:.3f}")


def test_served_pulse_results_equal_alone_results():
    """With pulse runs for multi-wavelength requests: the 3-wavelength
    request runs as pulses, the others time-harmonic; each result is the
    same alone and in the mix."""
    from paper_2505_03352_amd.serve import pulse_plan
    payloads = [(0, "small", [1.55 * UM], 900),
                (1, "small", [1.50 * UM, 1.55 * UM, 1.60 * UM], 2000),
                (2, "small", [1.50 * UM], 1000)]
    assert pulse_plan(configs.serving_request(*payloads[1])) is not None
    assert pulse_plan(configs.serving_request(*payloads[0])) is None
    alone, st1 = _serve(payloads, [0.0] * 3, max_slots=1, pulse=True)
    mixed, st2 = _serve(payloads, [0.0, 0.01, 0.02], max_slots=3, chunk=50, pulse=True)
    assert st1.n_done == 3 and st2.n_done == 3 and st2.max_active >= 2
    for a, m in zip(alone, mixed):
        assert np.abs(a.result["alpha"]).max() > 0
        assert np.array_equal(a.result["alpha"], m.result["alpha"])
        assert np.array_equal(a.result["grad"], m.result["grad"])


@pytest.mark.parametrize("i", [0, 2, 8])
def test_pulse_requests_match_time_harmonic(i):
    """The serving trace's multi-wavelength requests evaluated from pulse
    runs (the executor's choice of pulse and run length) against one
    time-harmonic run per wavelength: gradients within the gradient
    tolerance (1e-3 relative L2), alpha within 1e-3 of its largest entry."""
    from paper_2505_03352_amd.plan import plan_for
    from paper_2505_03352_amd.serve import pulse_plan
    _, cls, lams = configs.serving_trace()[i]
    dev = configs.serving_request(i, cls, lams)
    pp = pulse_plan(dev)
    assert pp is not None
    say(f"request {i} ({cls}, {len(lams)} wavelengths): time-harmonic {dev.n_steps} steps")
    ph = plan_for(dev)
    ph.run(3)
    ah = ph.alpha()
    gh = ph.gradient(torch.conj(ah)).cpu().numpy()
    ah = ah.cpu().numpy()
    ph.close()
    dp = configs.serving_request(i, cls, lams, n_steps=pp[3])
    say(f"  pulse {pp[3]} steps (sigma {pp[1]:.0f}, t0 {pp[2]:.0f})")
    q = plan_for(dp, pulse=pp[:3])
    q.run(3)
    ap = q.alpha()
    gp = q.gradient(torch.conj(ap)).cpu().numpy()
    ap = ap.cpu().numpy()
    q.close()
    ea = np.abs(ap - ah).max() / np.abs(ah).max()
    eg = np.linalg.norm(gp - gh) / np.linalg.norm(gh)
    say(f"  alpha max diff {ea:.2e}, gradient rel L2 diff {eg:.2e}")
    assert ea < 1e-3
    assert eg < 1e-3
