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


def _serve(payloads, arrivals, max_slots, chunk=100):
    from paper_2505_03352_amd.serve import GpuExecutor, Request, Scheduler

    def build(p):
        i, cls, lams, steps = p
        return configs.serving_request(i, cls, lams, n_steps=steps)

    ex = GpuExecutor(build, tiling=(4, 16, 1), chunk=chunk)
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
