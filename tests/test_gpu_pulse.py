"""Pulse excitation (paper Sec. 2's Fourier-transform-of-transients route) on
the GPU against the FP64 oracle's pulse route, through the C ABI: the
phasors of every wavelength from one run per source and per port, alpha and
the Eq. (9) gradient; and the GPU's pulse phasors against its own
time-harmonic ones.  Tolerances are those of the time-harmonic path (DFT
fields and alpha <= 1e-4 relative, gradients <= 1e-3 relative L2)."""
import sys

import numpy as np
import pytest
import torch

from oracle import adjoint
from workloads import configs

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


def pulse_args(dev):
    w0, sig, t0 = dev.pulse()
    return (w0 / dev.dt(), sig, t0), adjoint.Pulse(w0, sig, t0, dev.n_steps, tail=dev.n_steps // 8)


@pytest.mark.parametrize("name,stride", [("micro_demux", 1), ("tiny", 1), ("micro_demux", 4),
                                         ("tiny", 4)])
def test_pulse_phasors_alpha_gradient_match_oracle(name, stride):
    """stride 4: the GPU's DFT samples every fourth step (the oracle every
    step); the pulse spectrum vanishes at the aliases, so the phasors stay
    within the same tolerances."""
    from paper_2505_03352_amd.plan import plan_for
    if name == "micro_demux":
        dev = configs.micro_demux(n_steps=2600)
        dev.C = np.random.default_rng(41).uniform(0.3, 0.7, dev.C.shape)
        T = np.array([[[1.0, 0.0], [0.0, 1.0]]])
    else:
        dev = configs.tiny(n_steps=2400)
        T = np.array([[[0.8]]])
    gpu_pulse, P = pulse_args(dev)
    gpu_pulse = gpu_pulse + (stride,)
    say(f"pulse {name} (DFT stride {stride}): oracle (sigma {P.sigma:.1f}, t0 {P.t0:.1f}, "
        f"{dev.n_steps} steps)")
    ref = adjoint.forward_adjoint_pulse(dev, P)
    cref = 2.0 * (np.abs(ref.alpha) ** 2 - T) * np.conj(ref.alpha)
    gref = adjoint.grad_C(dev, ref, cref)
    say(f"pulse {name}: GPU")
    p = plan_for(dev, pulse=gpu_pulse)
    assert p.n_stepped == len(dev.sources) + len(dev.ports)
    p.run(3)
    ns, npo, nf = len(dev.sources), len(dev.ports), dev.n_freq
    worst = 0.0
    for f in range(nf):
        for s in range(ns):
            e = rel_l2(p.get_dft(f * ns + s).cpu().numpy(), ref.fwd[s][f].box)
            worst = max(worst, e)
        for q in range(npo):
            e = rel_l2(p.get_dft(ns * nf + f * npo + q).cpu().numpy(), ref.adj[q][f].box)
            worst = max(worst, e)
    a = p.alpha().cpu().numpy()
    ea = np.abs(a - ref.alpha).max() / np.abs(ref.alpha).max()
    coef = torch.as_tensor(cref, dtype=torch.complex64, device="cuda")
    g = p.gradient(coef).cpu().numpy()
    eg = rel_l2(g, gref)
    p.close()
    say(f"  DFT worst rel L2 {worst:.2e}, alpha err {ea:.2e}, gradient rel L2 {eg:.2e}, "
        f"tail residual {max(r.resid for r in ref.fwd[0]):.1e}")
    assert worst < 1e-4
    assert ea < 1e-4
    assert eg < 1e-3


def test_pulse_and_time_harmonic_runs_agree_on_the_gpu():
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro_demux(n_steps=2600)
    gpu_pulse, _ = pulse_args(dev)
    p = plan_for(dev, pulse=gpu_pulse)
    p.run(3)
    ap = p.alpha().cpu().numpy()
    bp = [p.get_dft(r).cpu().numpy() for r in range(p.n_rhs)]
    p.close()
    dh = configs.micro_demux(n_steps=4000)
    q = plan_for(dh)
    q.run(3)
    ah = q.alpha().cpu().numpy()
    bh = [q.get_dft(r).cpu().numpy() for r in range(q.n_rhs)]
    q.close()
    e = max(rel_l2(x, y) for x, y in zip(bp, bh))
    say(f"pulse vs time-harmonic on the GPU: DFT worst rel L2 {e:.2e}, "
        f"alpha {np.abs(ap - ah).max() / np.abs(ah).max():.2e}")
    assert e < 1e-4
    assert np.abs(ap - ah).max() < 1e-4 * np.abs(ah).max()


def test_realistic_full_size_pulse_dft_matches_oracle():
    """The 320x240x96 grid with its three wavelengths under a pulse, in the
    broadband benchmark's launch configuration (the split its autotuner
    picks for the pulse plan: rows 4, 10 z-planes per tile, flags 75): 500
    steps of the forward run (pulse centred at step 250, so the front
    crosses the design box), every box phasor of every wavelength against
    the oracle."""
    from paper_2505_03352_amd.plan import plan_for
    from oracle import ports
    dev = configs.realistic(n_steps=500)
    w0, sig, _ = dev.pulse(k=0.4)
    t0 = 250.0
    say("realistic full-size pulse: GPU")
    p = plan_for(dev, pulse=(w0 / dev.dt(), sig, t0))
    p.set_tiling(4, 10, 75)
    p.run(1)
    boxes = [p.get_dft(f * len(dev.sources)).cpu().numpy() for f in range(dev.n_freq)]
    kap = p.get_kappa().cpu().numpy().astype(np.float64)
    p.close()
    say("realistic full-size pulse: oracle")
    P = adjoint.Pulse(w0, sig, t0, dev.n_steps, tail=dev.n_steps // 8)
    ref = adjoint.solve_pulse(dev, kap, dev.sources[0].plane, ports.source_current(dev.sources[0].h), P)
    eb = [rel_l2(b, r.box) for b, r in zip(boxes, ref)]
    say(f"  box phasors rel L2 per wavelength {', '.join(f'{e:.2e}' for e in eb)}")
    assert max(eb) < 1e-4


def test_autograd_function_with_pulse_plan_matches_oracle():
    """The torch.autograd.Function over a pulse plan: C.grad of the Eq. (9)
    objective against the oracle's pulse-route gradient."""
    from paper_2505_03352_amd import fn
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro_demux(n_steps=2600)
    dev.C = np.random.default_rng(42).uniform(0.3, 0.7, dev.C.shape)
    gpu_pulse, P = pulse_args(dev)
    T = np.array([[[1.0, 0.0], [0.0, 1.0]]])
    ref = adjoint.forward_adjoint_pulse(dev, P)
    cref = 2.0 * (np.abs(ref.alpha) ** 2 - T) * np.conj(ref.alpha)
    gref = adjoint.grad_C(dev, ref, cref)
    p = plan_for(dev, pulse=gpu_pulse)
    C = torch.tensor(dev.C, dtype=torch.float32, device="cuda", requires_grad=True)
    a = fn.modal_coefficients(C, p, dev.beta)
    loss = fn.transmission_objective(a, torch.as_tensor(T, dtype=torch.float32, device="cuda"))
    loss.backward()
    g = C.grad.cpu().numpy()
    p.close()
    eg = rel_l2(g, gref)
    say(f"autograd over a pulse plan: dL/dC rel L2 {eg:.2e}")
    assert eg < 1e-3
