"""Temporal blocking (two steps per launch over the two-step region, tiling
flag 512 after yo_set_time_blocking(plan, 2)) against single steps, through
the C ABI: every field value, phasor, alpha and gradient bitwise equal, with
CPML and a source plane, with several right-hand sides and wavelengths (the
DFT window runs single steps), under a pulse whose DFT samples every fourth
step, for plans stepped together in shared launches, and with odd step
counts (a run's last step alone); also with the two-step launch on a second
stream beside the first step's other launches (flag 1024), eager and in
graphs."""
import sys

import numpy as np
import pytest
import torch

from workloads import Plane, configs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03352_amd import _abi
    _abi.lib()


def _box_plan(steps, tb, nx=150, ny=40, nz=34, npml=6, seed=5):
    """Random medium, CPML on all faces, a random plane source 10 cells in."""
    from paper_2505_03352_amd.plan import FreqSpec, Plan
    rng = np.random.default_rng(seed)
    kap = np.full((3, nz, ny, nx), 1.0 / 2.085)
    kap[:, 10:24, 9:30, 14:130] = 1.0 / rng.uniform(2.085, 12.11, size=(3, 14, 21, 116))
    pl = Plane(0, 16, 12, 11, 16, 12)
    h = rng.standard_normal((2, 12, 16)) + 1j * rng.standard_normal((2, 12, 16))
    grid = dict(nx=nx, ny=ny, nz=nz, dx=40e-9, dy=40e-9, dz=40e-9, courant=0.5, npml=(npml,) * 6)
    design = dict(i0=30, j0=15, md=4, nd=4, k_lo=15, k_hi=16, mc=2, nc=2, filter_r=1.0,
                  supersample=2, eps_core=12.11, eps_clad=2.085, sobel_delta=1e-6)
    dt = 0.5 * 40e-9 / 299792458.0
    f = FreqSpec(2 * np.pi / 31.0 / dt, 40.0, steps - 60, 60)
    p = Plan(grid, design, steps, [f], [pl], [], device="cuda", time_blocking=tb)
    p.bind()
    p.set_background(torch.as_tensor(kap, dtype=torch.float32), torch.zeros(p.canvas_shape))
    p.set_source_mode(0, h)
    return p


@pytest.mark.parametrize("steps", [200, 201])
def test_pairs_bitwise_equal_single_steps_with_cpml_and_source(steps):
    outs = {}
    for tb, zc, fl, graph in [(1, 16, 0, False), (2, 16, 512, False), (2, 8, 512 | 2, True),
                              (2, 10, 512 | 1 | 64 | 8, True), (2, 10, 512 | 128, False),
                              (2, 4, 512 | 32, True), (2, 10, 512 | 256 | 1 | 64, True),
                              (2, 8, 512 | 256 | 128 | 2, False), (2, 10, 512 | 1024 | 1 | 8, True),
                              (2, 8, 512 | 1024 | 128, False), (2, 10, 512 | 2048 | 128 | 8, True),
                              (2, 4, 512 | 2048 | 128, False), (2, 16, 512 | 2048 | 1024 | 128 | 2, True),
                              (2, 8, 512 | 4096 | 128 | 8, True), (2, 10, 512 | 4096 | 2048 | 128, False),
                              (2, 8, 512 | 8192 | 128 | 8, True), (2, 10, 512 | 8192 | 2, False),
                              (2, 8, 512 | 8192 | 4096 | 2048 | 128, True),
                              (2, 16, 512 | 16384 | 4096 | 1 | 2 | 8 | 64, True), (2, 10, 512 | 16384 | 128, False),
                              (2, 10, 512 | 16384 | 2048 | 128 | 8, True)]:
        say(f"pairs box steps={steps} tb={tb} tiling=(4,{zc},{fl}) graph={graph}")
        p = _box_plan(steps, tb)
        p.set_tiling(4, zc, fl)
        p.reset(1)
        from paper_2505_03352_amd.plan import advance_many
        advance_many([p], [1], steps, chunk=50, use_graph=graph)
        E, H = p.get_fields(0)
        outs[(tb, zc, fl)] = (E.cpu().numpy(), H.cpu().numpy())
        p.close()
    ref = outs[(1, 16, 0)]
    assert np.abs(ref[0]).max() > 0
    for k, v in outs.items():
        assert np.array_equal(v[0], ref[0]) and np.array_equal(v[1], ref[1]), k


def test_two_step_region_is_used():
    """The two-step launch has tiles (the region is not empty) and times;
    with flag 2048 (and the two-step strips cut clear of the source plane by
    flag 128) the z-slabs under it take two steps too, and the pair-step
    shell launch holds the rest of the shell."""
    p = _box_plan(100, 2)
    p.set_tiling(4, 16, 512)
    p.reset(1)
    p.advance(1, 4)
    ms, b, c = p.time_kernel(2, 2)
    ms3, b3, c3 = p.time_kernel(3, 2)
    say(f"two-step launch {ms:.4f} ms for {c:.0f} cell-updates; frame {ms3:.4f} ms, {c3:.0f}")
    assert c > 0 and ms > 0 and c3 > 0
    assert p.time_kernel(4, 1)[2] == 0.0
    p.set_tiling(4, 16, 512 | 2048 | 128)
    p.reset(1)
    p.advance(1, 4)
    c1 = p.time_kernel(1, 1)[2]
    ms4, b4, c4 = p.time_kernel(4, 2)
    ms5, b5, c5 = p.time_kernel(5, 2)
    say(f"z-slab two-step launch {ms4:.4f} ms for {c4:.0f}; pair-step shell {ms5:.4f} ms, {c5:.0f}")
    assert c4 > 0 and ms4 > 0 and c5 > 0
    assert c4 / 2 + c5 == pytest.approx(c1)       # the z-slabs' cells move from the shell
    assert p.time_kernel(3, 1)[2] == 0.0           # R2 is the whole interior: no frame
    p.close()


def test_pairs_bitwise_equal_with_window_and_several_wavelengths():
    """Forward and adjoint right-hand sides, three wavelengths: the run goes in
    pairs outside the DFT window; phasors, alpha and the gradient are bitwise
    those of single steps."""
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=400, nx=150, ny=40, nz=30, md=10, nd=10, mc=5, nc=5,
                        wavelengths=[0.78e-6, 0.8e-6, 0.82e-6])
    res = {}
    for tb, fl in [(1, 0), (2, 512), (2, 512 | 73), (2, 512 | 1024 | 73), (2, 512 | 2048 | 128 | 8),
                   (2, 512 | 4096 | 128 | 8), (2, 512 | 8192 | 73), (2, 512 | 16384 | 73)]:
        say(f"pairs micro tb={tb} flags={fl}")
        p = plan_for(dev, time_blocking=tb)
        p.set_tiling(4, 10, fl)
        p.run(3, chunk=50, use_graph=True)
        a = p.alpha()
        g = p.gradient(torch.conj(a).resolve_conj().contiguous())
        res[(tb, fl)] = [p.get_dft(r, 0).cpu().numpy() for r in range(p.n_rhs)] + \
                        [p.get_dft(0, 1).cpu().numpy(), a.cpu().numpy(), g.cpu().numpy()]
        p.close()
    ref = res[(1, 0)]
    for k, v in res.items():
        for x, y in zip(v, ref):
            assert np.array_equal(x, y), k


def test_pairs_bitwise_equal_under_a_pulse_and_in_shared_launches():
    """A pulse whose DFT samples every fourth step (pairs start on the sampled
    steps) and two plans of different sizes and step counts stepped together:
    bitwise the results of single steps."""
    from paper_2505_03352_amd.plan import advance_many, plan_for
    devs = [configs.micro_demux(n_steps=2600), configs.micro(n_steps=1300, nx=90, ny=34, nz=24)]
    res = {}
    for tb, fl in ((1, 0), (2, 512), (2, 512 | 1024), (2, 512 | 2048 | 128), (2, 512 | 4096),
                   (2, 512 | 8192), (2, 512 | 16384)):
        say(f"pairs pulse + shared launches tb={tb} flags={fl}")
        plans = []
        for d in devs:
            w0, sig, t0 = d.pulse()
            p = plan_for(d, pulse=(w0 / d.dt(), sig, t0, 4), time_blocking=tb)
            p.set_tiling(4, 8, fl)
            plans.append(p)
        for p in plans:
            p.reset(3)
        advance_many(plans, [3, 3], max(d.n_steps for d in devs), chunk=40, use_graph=True)
        out = []
        for p in plans:
            p.finalize(3)
            a = p.alpha()
            out += [p.get_dft(r, 0).cpu().numpy() for r in range(p.n_rhs)] + [a.cpu().numpy()]
            p.close()
        res[fl] = out
    for fl in (512, 512 | 1024, 512 | 2048 | 128, 512 | 4096, 512 | 8192, 512 | 16384):
        for x, y in zip(res[fl], res[0]):
            assert np.array_equal(x, y), fl


def test_autotuner_times_pairs_and_keeps_results():
    """For a plan with time blocking the tuner times two steps per launch
    beside the single-step splits, applies the fastest per step, and the
    fields after it are bitwise those of single steps."""
    from paper_2505_03352_amd import autotune
    from paper_2505_03352_amd.plan import advance_many
    ref = _box_plan(120, 1)
    ref.set_tiling(4, 16, 0)
    ref.reset(1)
    advance_many([ref], [1], 120, chunk=40, use_graph=True)
    E0, H0 = (x.cpu().numpy() for x in ref.get_fields(0))
    ref.close()
    p = _box_plan(120, 2)
    say("pairs autotune")
    rec = autotune.tune(p, 1, shared=[(10, 1)], pair_shared=[(10, 1), (10, 257), (8, 128)],
                        n_launch=2, use_cache=False)
    assert {"pairs_z10f1", "pairs_z10f257", "pairs_z8f128"} <= set(rec["timings"])
    for k in ("pairs_z10f1", "pairs_z10f257", "pairs_z8f128"):
        t = rec["timings"][k]
        assert t["two_step"] > 0 and min(t["shell"].values()) > 0
    best = min(rec["timings"].values(), key=lambda t: t["ms"])
    # flag 1024 (the two-step launch on a second stream) is decided on whole
    # steps after the split, when the split has two steps per launch
    assert rec["flags"] & ~1024 == best["best"]
    if rec["flags"] & 512:
        ov = rec["overlap"]
        assert ov["one_stream"] > 0 and ov["two_streams"] > 0
        assert bool(rec["flags"] & 1024) == (ov["two_streams"] < 0.99 * ov["one_stream"])
    else:
        assert rec["ms_per_step"] == pytest.approx(best["ms"], abs=1e-4)
    advance_many([p], [1], 120, chunk=40, use_graph=True)
    E, H = (x.cpu().numpy() for x in p.get_fields(0))
    assert np.array_equal(E, E0) and np.array_equal(H, H0)
    p.close()


def test_pairs_bitwise_equal_with_two_term_ports():
    """The two-term coefficient's adjoint currents touch each port plane and
    the plane after it; the two-step region keeps clear of both, also in the
    split of whole 60-cell two-step strips (flag 128), so alpha and the
    gradient are bitwise those of single steps."""
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=400, nx=150, ny=40, nz=30, md=10, nd=10, mc=5, nc=5)
    res = {}
    for tb, fl in [(1, 0), (2, 512 | 128), (2, 512 | 73), (2, 512 | 1024 | 128 | 8), (2, 512 | 2048 | 128)]:
        say(f"pairs two-term tb={tb} flags={fl}")
        p = plan_for(dev, two_term=True, time_blocking=tb)
        p.set_tiling(4, 10, fl)
        p.run(3, chunk=50, use_graph=True)
        a = p.alpha()
        g = p.gradient(torch.conj(a).resolve_conj().contiguous())
        res[(tb, fl)] = [p.get_dft(r, 0).cpu().numpy() for r in range(p.n_rhs)] + \
                        [a.cpu().numpy(), g.cpu().numpy()]
        p.close()
    ref = res[(1, 0)]
    assert np.abs(ref[-1]).max() > 0
    for k, v in res.items():
        for x, y in zip(v, ref):
            assert np.array_equal(x, y), k
