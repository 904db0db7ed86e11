"""Parity of the HIP path (through the C ABI) with the FP64 oracle and with
closed forms.  Tolerances: DFT phasors relative L2 <= 1e-4, gradients
relative L2 <= 1e-3 (FP32 kernels against the FP64 oracle)."""
import sys

import numpy as np
import pytest
import torch

from oracle import adjoint, chain, fdtd
from workloads import Plane, cavity, configs

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03352_amd import _abi
    _abi.lib()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def closed_box_plan(nx, ny, nz, kappa, n_steps, courant=0.5):
    """A plan whose grid is a bare PEC box (no CPML, no design, no source set)."""
    from paper_2505_03352_amd.plan import FreqSpec, Plan
    grid = dict(nx=nx, ny=ny, nz=nz, dx=40e-9, dy=40e-9, dz=40e-9, courant=courant,
                npml=(0,) * 6)
    design = dict(i0=2, j0=2, md=2, nd=2, k_lo=2, k_hi=2, mc=1, nc=1, filter_r=1.0,
                  supersample=2, eps_core=12.11, eps_clad=2.085, sobel_delta=1e-6)
    f = FreqSpec(2 * np.pi * 299792458.0 / 1.55e-6, 0.0, n_steps - 2, 2)
    p = Plan(grid, design, n_steps, [f], [Plane(0, 1, 1, 1, 1, 1)], [], device="cuda")
    p.bind()
    mask = torch.zeros(p.canvas_shape)
    p.set_background(torch.as_tensor(kappa, dtype=torch.float32), mask)
    return p


# work splits (rows per wave, z-planes, flags); a closed box has no CPML
# shell, so only the interior choices matter: 16 cooperative, 32 no prefetch
@pytest.mark.parametrize("rows,zchunk,flags", [(4, 16, 0), (4, 8, 32), (4, 16, 16), (4, 8, 50)])
@pytest.mark.parametrize("mnp,eps", [((2, 3, 0), 2.085), ((1, 2, 1), 12.11), ((0, 2, 1), 1.0)])
def test_cavity_eigenmode(mnp, eps, rows, zchunk, flags):
    nx, ny, nz = 70, 44, 36
    m, n, p_ = mnp
    steps = 2000
    say(f"cavity {mnp} eps={eps} tiling=({rows},{zchunk},{flags})")
    kap = np.full((3, nz, ny, nx), 1.0 / eps)
    E0, H0 = cavity.pec_standing_wave(nx, ny, nz, m, n, p_,
                                      cavity.divergence_free_amplitudes(nx, ny, nz, m, n, p_))
    plan = closed_box_plan(nx, ny, nz, kap, steps)
    plan.set_tiling(rows, zchunk, flags)
    plan.reset(1)
    plan.set_fields(0, torch.as_tensor(E0, dtype=torch.float32), torch.as_tensor(H0, dtype=torch.float32))
    plan.advance(1, steps)
    E, H = plan.get_fields(0)
    torch.cuda.synchronize()
    k32 = float(np.float32(1.0 / eps))
    r = (0.25 * k32) * (np.sin(0.5 * m * np.pi / nx) ** 2 + np.sin(0.5 * n * np.pi / ny) ** 2
                        + np.sin(0.5 * p_ * np.pi / nz) ** 2)
    phi = 2 * np.arcsin(np.sqrt(r))
    err = np.abs(E.cpu().numpy() - E0 * np.cos(steps * phi)).max() / np.abs(E0).max()
    say(f"  max err {err:.2e}")
    assert err < 1e-4
    plan.close()


def test_energy_conservation_random_medium():
    rng = np.random.default_rng(3)
    nx, ny, nz = 75, 40, 33
    kap = (1.0 / rng.uniform(1.0, 12.0, size=(3, nz, ny, nx))).astype(np.float32).astype(np.float64)
    E0 = rng.standard_normal((3, nz, ny, nx))
    H0 = rng.standard_normal((3, nz, ny, nx))
    E0[0, :, 0, :] = 0; E0[0, 0] = 0
    E0[1, :, :, 0] = 0; E0[1, 0] = 0
    E0[2, :, :, 0] = 0; E0[2, :, 0, :] = 0
    E0 = E0.astype(np.float32).astype(np.float64)
    H0 = H0.astype(np.float32).astype(np.float64)
    steps = 1000
    say("energy conservation")
    plan = closed_box_plan(nx, ny, nz, kap, steps + 1)
    plan.reset(1)
    plan.set_fields(0, torch.as_tensor(E0, dtype=torch.float32), torch.as_tensor(H0, dtype=torch.float32))

    def energy_now():
        E, Hm = plan.get_fields(0)
        plan.advance(1, 1)
        _, Hp = plan.get_fields(0)
        E, Hm, Hp = (t.double().cpu().numpy() for t in (E, Hm, Hp))
        return np.sum(E * E / kap) + np.sum(Hm * Hp)

    w0 = energy_now()
    plan.advance(1, steps - 1)
    w1 = energy_now()
    say(f"  energy drift {abs(w1 - w0) / w0:.2e}")
    assert abs(w1 - w0) / abs(w0) < 1e-4
    plan.close()


def _sourced_box(nx=72, ny=40, nz=34, npml=6, seed=5):
    """Random medium, CPML on all faces, one random plane source."""
    from paper_2505_03352_amd.plan import FreqSpec, Plan
    rng = np.random.default_rng(seed)
    kap = np.full((3, nz, ny, nx), 1.0 / 2.085)
    kap[:, 10:24, 9:30, 14:60] = 1.0 / rng.uniform(2.085, 12.11, size=(3, 14, 21, 46))
    kap = kap.astype(np.float32).astype(np.float64)
    pl = Plane(0, 10, 12, 11, 16, 12)
    h = (rng.standard_normal((2, 12, 16)) + 1j * rng.standard_normal((2, 12, 16)))
    h = (h.astype(np.complex64)).astype(np.complex128)
    w_dt = 2 * np.pi / 31.0
    return kap, pl, h, w_dt, npml


def test_whole_interior_strip_tilings_bitwise_equal():
    """Tilings that cut the x-shell so the interior strips are whole (flag
    128) or run the x-slab tiles in the interior launch (flag 256), on a
    grid wide enough for them, give bitwise the fields of the plain tiling
    (which the test below checks against the oracle)."""
    kap, pl, h, w_dt, npml = _sourced_box(nx=150)
    _, nz, ny, nx = kap.shape
    steps = 200
    from paper_2505_03352_amd.plan import FreqSpec, Plan
    grid = dict(nx=nx, ny=ny, nz=nz, dx=40e-9, dy=40e-9, dz=40e-9, courant=0.5, npml=(npml,) * 6)
    design = dict(i0=30, j0=15, md=4, nd=4, k_lo=15, k_hi=16, mc=2, nc=2, filter_r=1.0,
                  supersample=2, eps_core=12.11, eps_clad=2.085, sobel_delta=1e-6)
    dt = 0.5 * 40e-9 / 299792458.0
    f = FreqSpec(w_dt / dt, 40.0, steps - 60, 60)
    outs = {}
    for rows, zc, fl in [(4, 16, 0), (4, 16, 128), (4, 16, 201), (4, 8, 178), (4, 16, 129),
                         (4, 4, 232), (4, 16, 329), (4, 16, 456), (4, 8, 256), (4, 16, 304)]:
        say(f"whole-strip tiling=({rows},{zc},{fl})")
        p = Plan(grid, design, steps, [f], [pl], [], device="cuda")
        p.bind()
        p.set_background(torch.as_tensor(kap, dtype=torch.float32), torch.zeros(p.canvas_shape))
        p.set_source_mode(0, h)
        p.set_tiling(rows, zc, fl)
        p.reset(1)
        p.advance(1, steps)
        E, H = p.get_fields(0)
        outs[(rows, zc, fl)] = (E.cpu().numpy(), H.cpu().numpy())
        p.close()
    ref = outs[(4, 16, 0)]
    assert np.abs(ref[0]).max() > 0
    for k, v in outs.items():
        assert np.array_equal(v[0], ref[0]) and np.array_equal(v[1], ref[1]), k


def test_fields_match_oracle_with_cpml_and_source():
    kap, pl, h, w_dt, npml = _sourced_box()
    _, nz, ny, nx = kap.shape
    steps = 300
    from paper_2505_03352_amd.plan import FreqSpec, Plan
    grid = dict(nx=nx, ny=ny, nz=nz, dx=40e-9, dy=40e-9, dz=40e-9, courant=0.5, npml=(npml,) * 6)
    design = dict(i0=30, j0=15, md=4, nd=4, k_lo=15, k_hi=16, mc=2, nc=2, filter_r=1.0,
                  supersample=2, eps_core=12.11, eps_clad=2.085, sobel_delta=1e-6)
    dt = 0.5 * 40e-9 / 299792458.0
    f = FreqSpec(w_dt / dt, 40.0, steps - 60, 60)
    outs = {}
    # every interior and shell choice (see yo_set_tiling); cooperative shell
    # blocks on the y-slabs of 7 rows leave idle waves
    for rows, zc, fl in [(4, 16, 0), (4, 8, 1), (4, 4, 2), (4, 48, 3), (4, 16, 4), (4, 16, 13),
                         (4, 8, 70), (4, 4, 23), (4, 16, 45), (4, 8, 122), (4, 16, 77),
                         (4, 8, 53), (4, 16, 16384 | 73), (4, 10, 16384 | 2)]:
        say(f"cpml+source fields tiling=({rows},{zc},{fl})")
        p = Plan(grid, design, steps, [f], [pl], [], device="cuda")
        p.bind()
        p.set_background(torch.as_tensor(kap, dtype=torch.float32), torch.zeros(p.canvas_shape))
        p.set_source_mode(0, h)
        p.set_tiling(rows, zc, fl)
        p.reset(1)
        p.advance(1, steps)
        E, H = p.get_fields(0)
        outs[(rows, zc, fl)] = (E.cpu().numpy(), H.cpu().numpy())
        p.close()
    # every tiling gives bitwise the same fields
    ref = outs[(4, 16, 0)]
    for k, v in outs.items():
        assert np.array_equal(v[0], ref[0]) and np.array_equal(v[1], ref[1]), k
    # against the FP64 oracle
    J = np.empty_like(h)
    J[0] = -h[1]
    J[1] = h[0]
    prm = fdtd.SimParams(nx, ny, nz, npml=(npml,) * 6, n_steps=steps, omega_dt=w_dt,
                         ramp_steps=40.0, win_start=steps - 60, win_len=60)
    r = fdtd.run(prm, kap, src_plane=pl, src_j=J)
    eE = np.abs(ref[0] - r.E).max() / np.abs(r.E).max()
    eH = np.abs(ref[1] - r.H).max() / np.abs(r.H).max()
    say(f"  max rel err E {eE:.2e} H {eH:.2e}")
    assert eE < 1e-4 and eH < 1e-4


@pytest.fixture(scope="module")
def tiny_results():
    """cfg tiny: forward + adjoint + gradient on the GPU and in the oracle."""
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.tiny()
    say("tiny device: oracle")
    ref = adjoint.forward_adjoint(dev)
    say("tiny device: GPU run")
    p = plan_for(dev)
    p.run(3, chunk=100, use_graph=True)
    alpha = p.alpha()
    coef = torch.conj(alpha)
    g = p.gradient(coef)
    gk = p.gradient_kappa(coef)
    fwd_box = p.get_dft(0, 0)
    adj_box = p.get_dft(1, 0)
    fwd_mon = p.get_dft(0, 1)
    kap = p.get_kappa()
    torch.cuda.synchronize()
    out = dict(dev=dev, ref=ref, alpha=alpha.cpu().numpy(), g=g.cpu().numpy(),
               gk=gk.cpu().numpy(), fwd_box=fwd_box.cpu().numpy(), adj_box=adj_box.cpu().numpy(),
               fwd_mon=fwd_mon.cpu().numpy(), kappa=kap.cpu().numpy())
    p.close()
    return out


def test_tiny_kappa_matches_oracle_chain(tiny_results):
    t = tiny_results
    err = np.abs(t["kappa"] - t["ref"].kappa).max() / np.abs(t["ref"].kappa).max()
    say(f"tiny kappa max rel err {err:.2e}")
    assert err < 1e-5


def test_tiny_dft_fields_match_oracle(tiny_results):
    t = tiny_results
    ref = t["ref"]
    e1 = rel_l2(t["fwd_box"], ref.fwd[0][0].box)
    e2 = rel_l2(t["adj_box"], ref.adj[0][0].box)
    e3 = rel_l2(t["fwd_mon"], ref.fwd[0][0].mon[0])
    say(f"tiny DFT rel L2: fwd box {e1:.2e} adj box {e2:.2e} fwd port {e3:.2e}")
    assert e1 < 1e-4 and e2 < 1e-4 and e3 < 1e-4


def test_tiny_alpha_and_gradient_match_oracle(tiny_results):
    t = tiny_results
    ref = t["ref"]
    ea = np.abs(t["alpha"] - ref.alpha).max() / np.abs(ref.alpha).max()
    _, cref = adjoint.objective_abs2(ref.alpha)
    gref = adjoint.grad_C(t["dev"], ref, cref)
    gkref = adjoint.grad_kappa(t["dev"], ref, cref)
    eg = rel_l2(t["g"], gref)
    egk = rel_l2(t["gk"], gkref)
    say(f"tiny alpha err {ea:.2e}, dF/dkappa rel L2 {egk:.2e}, dF/dC rel L2 {eg:.2e}")
    assert ea < 1e-4
    assert egk < 1e-3
    assert eg < 1e-3


def test_two_ports_two_wavelengths_eq9_gradient():
    from paper_2505_03352_amd.plan import plan_for
    from workloads import devices
    base = configs.micro(n_steps=900, ny=30)
    dev = devices.soi_device("micro2", base.nx, base.ny, base.nz, base.dx, base.npml[0],
                             md=base.md, nd=base.nd, slab_layers=3, mc=base.mc, nc=base.nc,
                             filter_r=base.filter_r, beta=base.beta,
                             wavelengths=[0.8e-6, 0.85e-6], n_steps=900, seed=base.seed,
                             mode_w=(3.0, 1.5), ramp_periods=3.0, strip_width=240e-9,
                             src_inset=3, out_offsets=(-0.12e-6, 0.12e-6))
    T = np.array([[[0.3, 0.2], [0.1, 0.4]]])
    say("two ports x two wavelengths: oracle")
    ref = adjoint.forward_adjoint(dev)
    cref = 2 * np.conj(ref.alpha) * (np.abs(ref.alpha) ** 2 - T)
    gref = adjoint.grad_C(dev, ref, cref)
    say("two ports x two wavelengths: GPU")
    p = plan_for(dev)
    p.run(3, chunk=50, use_graph=False)
    a = p.alpha().cpu().numpy()
    coef = 2 * np.conj(a) * (np.abs(a) ** 2 - T)
    g = p.gradient(torch.as_tensor(coef, dtype=torch.complex64)).cpu().numpy()
    ea = np.abs(a - ref.alpha).max() / np.abs(ref.alpha).max()
    eg = rel_l2(g, gref)
    say(f"  alpha err {ea:.2e} gradient rel L2 {eg:.2e}")
    assert ea < 1e-4 and eg < 1e-3
    p.close()


@pytest.mark.parametrize("name", ["tiny", "realistic", "multiport"])
def test_chain_and_vjp_match_oracle_full_size(name):
    from paper_2505_03352_amd.plan import plan_for
    dev = {"tiny": configs.tiny, "realistic": configs.realistic,
           "multiport": configs.multiport}[name]()
    dev = _light(dev)
    say(f"chain parity {name}")
    ops = chain.make_ops(dev)
    kref, st = chain.kappa(dev, ops=ops)
    p = plan_for(dev)
    kap = p.get_kappa().cpu().numpy()
    ek = np.abs(kap - kref).max() / np.abs(kref).max()
    rng = np.random.default_rng(0)
    x0, y0, z0, bx, by, bz = dev.dft_box()
    g3 = rng.standard_normal((3, bz, by, bx))
    gC = p.chain_vjp(torch.as_tensor(g3, dtype=torch.float32)).cpu().numpy()
    gref = chain.vjp(dev, st, dev.beta, *chain.zsum(dev, g3), ops)
    eg = rel_l2(gC, gref)
    say(f"  kappa max rel err {ek:.2e}, VJP rel L2 {eg:.2e}")
    assert ek < 1e-5
    assert eg < 1e-4
    p.close()


def _light(dev):
    """Same geometry with one wavelength and a short run (the chain tests do
    not step)."""
    dev.wavelengths = dev.wavelengths[:1]
    dev.n_steps = 400
    return dev


def test_graph_and_eager_bitwise_equal_and_deterministic():
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=600)
    res = []
    for graph, chunk in [(False, 600), (True, 64), (True, 64), (False, 7)]:
        say(f"determinism graph={graph} chunk={chunk}")
        p = plan_for(dev)
        p.run(3, chunk=chunk, use_graph=graph)
        res.append((p.get_dft(0, 0).cpu().numpy(), p.get_dft(1, 0).cpu().numpy(),
                    p.alpha().cpu().numpy()))
        p.close()
    for r in res[1:]:
        for a, b in zip(r, res[0]):
            assert np.array_equal(a, b)


def test_batched_advance_matches_individual_runs():
    from paper_2505_03352_amd import plan as P
    devs = [configs.micro(n_steps=500, seed=1), configs.micro(n_steps=700, seed=2, nx=34, ny=28),
            configs.micro(n_steps=600, seed=3, nz=20)]
    alone = []
    for d in devs:
        say(f"batch reference {d.nx}x{d.ny}x{d.nz}")
        p = P.plan_for(d)
        p.run(3, chunk=50, use_graph=False)
        alone.append(p.get_dft(0, 0).cpu().numpy())
        p.close()
    say("batched run")
    plans = [P.plan_for(d) for d in devs]
    for p in plans:
        p.reset(3)
    P.advance_many(plans, [3] * 3, max(d.n_steps for d in devs), chunk=50, use_graph=True)
    for p, ref in zip(plans, alone):
        p.finalize(3)
        assert np.array_equal(p.get_dft(0, 0).cpu().numpy(), ref)
        p.close()


def test_realistic_full_size_short_run_fields_match_oracle():
    """The 320x240x96 grid one step per launch (rows 4, 10 z-planes per
    tile, flags 73: strips, 8-wave blocks, per-class shell code), 150 steps
    from rest with the input source on: every field value against the
    oracle.  (The bench's two-steps-per-launch split of this grid is
    checked end to end in test_gpu_fullsize.py.)"""
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.realistic(n_steps=150, wavelengths=[1.55e-6])
    say("realistic full-size fields: GPU")
    p = plan_for(dev)
    p.set_tiling(4, 10, 73)
    p.reset(1)
    p.advance(1, 150)
    E, H = p.get_fields(0)
    E, H = E.cpu().numpy(), H.cpu().numpy()
    kap = p.get_kappa().cpu().numpy().astype(np.float64)
    p.close()
    say("realistic full-size fields: oracle")
    from oracle import ports
    lam = dev.wavelengths[0]
    prm = adjoint.sim_params(dev, lam)
    r = fdtd.run(prm, kap, src_plane=dev.sources[0].plane,
                 src_j=ports.source_current(dev.sources[0].h))
    eE = np.abs(E - r.E).max() / np.abs(r.E).max()
    eH = np.abs(H - r.H).max() / np.abs(r.H).max()
    say(f"  max rel err E {eE:.2e} H {eH:.2e}")
    assert eE < 1e-4 and eH < 1e-4


def shipped_split(shape: str) -> dict:
    """The shipped two-steps-per-launch split of a grid shape (the one the
    bench applies), e.g. shape "ny400|nz120"."""
    from paper_2505_03352_amd import autotune
    recs = [v for k, v in autotune.shipped_splits().items() if f"|{shape}|" in k and k.endswith("|tb2")]
    assert len(recs) == 1, shape
    return recs[0]


def test_multiport_full_size_short_run_fields_match_oracle():
    """The 600x400x120 multi-port grid (1 wavelength: 1 forward + 4 adjoint
    right-hand sides), 101 steps from rest with the input source on, in the
    headline bench's launch configuration (two steps per launch, its shipped
    split: 6-row two-step and shell tiles, 16 z-planes per tile; the odd
    last step and the DFT window one step per launch): every field value
    of the forward right-hand side against the oracle."""
    from paper_2505_03352_amd.plan import plan_for
    from oracle import ports
    dev = configs.multiport(n_steps=101, wavelengths=[1.55e-6])
    rec = shipped_split("ny400|nz120")
    say(f"multi-port full-size fields: GPU, split {rec}")
    p = plan_for(dev, time_blocking=2)
    p.set_tiling(rec["rows"], rec["zchunk"], rec["flags"])
    p.reset(3)
    p.advance(3, 101)
    E, H = p.get_fields(0)
    E, H = E.cpu().numpy(), H.cpu().numpy()
    kap = p.get_kappa().cpu().numpy().astype(np.float64)
    p.close()
    say("multi-port full-size fields: oracle")
    prm = adjoint.sim_params(dev, dev.wavelengths[0])
    r = fdtd.run(prm, kap, src_plane=dev.sources[0].plane,
                 src_j=ports.source_current(dev.sources[0].h))
    eE = np.abs(E - r.E).max() / np.abs(r.E).max()
    eH = np.abs(H - r.H).max() / np.abs(r.H).max()
    say(f"  max rel err E {eE:.2e} H {eH:.2e}")
    assert eE < 1e-4 and eH < 1e-4


@pytest.mark.parametrize("c_value,beta", [(0.0, 8.0), (1.0, 8.0), (0.5, 1000.0)])
def test_degenerate_designs_match_oracle(c_value, beta):
    """Uniform controls (all cladding, all core, and exactly grey under a
    near-step projection): kappa equals the oracle's, alpha and the gradient
    stay finite and match it."""
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.tiny()
    dev.C = np.full_like(dev.C, c_value)
    dev.beta = beta
    say(f"degenerate design C={c_value} beta={beta}")
    p = plan_for(dev)
    p.run(3, chunk=100, use_graph=True)
    a = p.alpha()
    g = p.gradient(torch.conj(a)).cpu().numpy()
    kap = p.get_kappa().cpu().numpy()
    a = a.cpu().numpy()
    p.close()
    say("  oracle")
    res = adjoint.forward_adjoint(dev)
    assert np.abs(kap - res.kappa).max() < 1e-5 * np.abs(res.kappa).max()
    ao = res.alpha[0, 0, 0]
    go = adjoint.grad_C(dev, res, np.conj(res.alpha))
    assert np.isfinite(g).all() and np.isfinite(a).all()
    assert abs(a[0, 0, 0] - ao) < 1e-4 * abs(ao)
    scale = np.abs(go).max()
    if scale > 0:
        assert rel_l2(g, go) < 1e-3
    else:
        assert np.abs(g).max() == 0.0


def test_autograd_function_matches_library_and_finite_differences():
    """torch conventions: L = sum |alpha|^2 gives C.grad = the library's
    gradient with coef = conj(alpha); and it matches central differences of
    forward-only runs."""
    from paper_2505_03352_amd import fn
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=1200)
    p = plan_for(dev)
    C = torch.as_tensor(dev.C, dtype=torch.float32, device="cuda").requires_grad_(True)
    say("autograd forward/backward")
    a = fn.modal_coefficients(C, p, dev.beta, chunk=100)
    L = (a.abs() ** 2).sum()
    L.backward()
    g_auto = C.grad.detach().cpu().numpy()
    g_lib = p.gradient(torch.conj(a.detach())).cpu().numpy()
    assert np.allclose(g_auto, g_lib, rtol=1e-6, atol=1e-9 * np.abs(g_lib).max())
    # central differences on a few controls (forward-only runs)
    q = plan_for(dev)
    h = 1e-2
    gmax = np.abs(g_auto).max()
    for idx in [(1, 2), (3, 4), (2, 1)]:
        vals = []
        for sgn in (1, -1):
            Cp = dev.C.copy()
            Cp[idx] += sgn * h
            q.set_design(torch.as_tensor(Cp, dtype=torch.float32), dev.beta)
            q.run(1, chunk=100)
            vals.append(float((q.alpha().abs() ** 2).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        say(f"  FD {idx}: autograd {g_auto[idx]:.5e} fd {fd:.5e}")
        assert abs(fd - g_auto[idx]) < 2e-2 * gmax
    p.close()
    q.close()


def test_conjugate_views_are_resolved():
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=400)
    p = plan_for(dev)
    p.run(3, chunk=100)
    a = p.alpha()
    g1 = p.gradient(torch.conj(a)).cpu().numpy()                 # lazy view
    g2 = p.gradient(torch.conj(a).resolve_conj()).cpu().numpy()  # materialised
    assert np.array_equal(g1, g2)
    p.close()


def test_launch_timing_keeps_results_and_counts_launches():
    """Timing the last steps' launches (plain launches with events) leaves
    the fields bitwise unchanged."""
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=500)
    res = []
    for timed in (False, True):
        say(f"launch timing {timed}")
        p = plan_for(dev)
        if timed:
            p.set_timing(0, 64)
        p.run(3, chunk=50, use_graph=True)
        res.append((p.get_dft(0, 0).cpu().numpy(), p.alpha().cpu().numpy()))
        if timed:
            ms, n = p.timing()
            assert n == 64 and ms > 0
        p.close()
    for a, b in zip(*res):
        assert np.array_equal(a, b)


def test_largest_grid_random_fields_match_oracle():
    """A grid at the size limit (one right-hand side's 6-component state
    just under 2 GiB, so the kernels' 32-bit buffer offsets reach their
    largest values): random fields everywhere, CPML on every face, random
    kappa in a block; two steps against the oracle, every value."""
    from paper_2505_03352_amd.plan import FreqSpec, Plan
    nx, ny, nz, npml = 640, 480, 270, 8
    nxp = (nx + 2 + 31) // 32 * 32
    state = 6 * 4 * (nz + 2) * (ny + 2) * nxp
    assert 0.98 * 2 ** 31 < state < 2 ** 31
    rng = np.random.default_rng(70)
    kap = np.full((3, nz, ny, nx), 1.0 / 2.085, np.float32)
    kap[:, 100:180, 150:350, 200:500] = (1.0 / rng.uniform(2.085, 12.11, (3, 80, 200, 300))).astype(np.float32)
    E0 = rng.standard_normal((3, nz, ny, nx), dtype=np.float32)
    H0 = rng.standard_normal((3, nz, ny, nx), dtype=np.float32)
    # tangential E on the PEC planes i = 0, j = 0, k = 0 starts at zero, as the scheme keeps it
    E0[0, 0, :, :] = E0[0, :, 0, :] = 0.0
    E0[1, 0, :, :] = E0[1, :, :, 0] = 0.0
    E0[2, :, 0, :] = E0[2, :, :, 0] = 0.0
    grid = dict(nx=nx, ny=ny, nz=nz, dx=40e-9, dy=40e-9, dz=40e-9, courant=0.5, npml=(npml,) * 6)
    design = dict(i0=300, j0=220, md=4, nd=4, k_lo=130, k_hi=131, mc=2, nc=2, filter_r=1.0,
                  supersample=2, eps_core=12.11, eps_clad=2.085, sobel_delta=1e-6)
    f = FreqSpec(2 * np.pi * 299792458.0 / 1.55e-6, 0.0, 0, 2)
    say(f"largest grid {nx}x{ny}x{nz}: GPU")
    p = Plan(grid, design, 2, [f], [Plane(0, 20, 20, 20, 4, 4)], [], device="cuda")
    p.bind()
    p.set_background(torch.as_tensor(kap), torch.zeros(p.canvas_shape))
    p.set_tiling(4, 16, 200)
    p.reset(1)
    p.set_fields(0, torch.as_tensor(E0), torch.as_tensor(H0))
    p.advance(1, 2)
    E, H = p.get_fields(0)
    E, H = E.cpu().numpy(), H.cpu().numpy()
    p.close()
    say("largest grid: oracle")
    prm = fdtd.SimParams(nx, ny, nz, npml=(npml,) * 6, n_steps=2, omega_dt=0.1, win_start=0, win_len=2)
    r = fdtd.run(prm, kap.astype(np.float64), E0=E0.astype(np.float64), H0=H0.astype(np.float64))
    eE = np.abs(E - r.E).max() / np.abs(r.E).max()
    eH = np.abs(H - r.H).max() / np.abs(r.H).max()
    say(f"  max rel err E {eE:.2e} H {eH:.2e}")
    assert eE < 1e-5 and eH < 1e-5
