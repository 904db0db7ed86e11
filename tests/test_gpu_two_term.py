"""The two-term modal coefficient (paper Appendix A) on the GPU against the
FP64 oracle, through the C ABI.  The library evaluates the H term on E sites
through the Yee update's H step and injects the same weights as electric
adjoint currents; the oracle reads H phasors on the port planes and drives
the adjoint with electric plus magnetic currents, so agreement also checks
the two routes against each other.  Tolerances: alpha <= 1e-4 relative,
gradients <= 1e-3 relative L2 (the time-harmonic fits of the two routes
differ by the runs' steady-state residual, a few 1e-6 here)."""
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


@pytest.mark.parametrize("name", ["micro", "micro_demux"])
def test_two_term_alpha_and_gradient_match_oracle(name):
    from paper_2505_03352_amd.plan import plan_for
    if name == "micro":
        dev = configs.micro(n_steps=1600)
        T = np.array([[[0.5]]])
    else:
        dev = configs.micro_demux(n_steps=1600)
        T = np.array([[[1.0, 0.0], [0.0, 1.0]]])
    dev.C = np.random.default_rng(60).uniform(0.3, 0.7, dev.C.shape)
    say(f"two-term {name}: oracle")
    ref = adjoint.forward_adjoint(dev, two_term=True)
    cref = 2.0 * (np.abs(ref.alpha) ** 2 - T) * np.conj(ref.alpha)
    gref = adjoint.grad_C(dev, ref, cref)
    say(f"two-term {name}: GPU")
    p = plan_for(dev, two_term=True)
    p.run(3)
    a = p.alpha().cpu().numpy()
    g = p.gradient(torch.as_tensor(cref, dtype=torch.complex64, device="cuda")).cpu().numpy()
    mon = p.get_dft(0, 1).cpu().numpy()
    p.close()
    assert mon.shape[0] == 5
    ea = np.abs(a - ref.alpha).max() / np.abs(ref.alpha).max()
    eg = rel_l2(g, gref)
    say(f"  alpha {a.ravel()} oracle {ref.alpha.ravel()}; alpha err {ea:.2e}, gradient rel L2 {eg:.2e}")
    assert ea < 1e-4
    assert eg < 1e-3


def test_one_term_path_unchanged_next_to_two_term_plan():
    """An E-only plan gives bitwise the same results whether or not a
    two-term plan of the same device ran before it."""
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=600)
    p = plan_for(dev)
    p.run(3)
    a0 = p.alpha().cpu().numpy()
    p.close()
    q = plan_for(dev, two_term=True)
    q.run(3)
    q.close()
    p = plan_for(dev)
    p.run(3)
    a1 = p.alpha().cpu().numpy()
    p.close()
    assert np.array_equal(a0, a1)


@pytest.mark.parametrize("two", [True, False])
@pytest.mark.parametrize("axis", [1, 2])
def test_ports_normal_to_y_and_z(axis, two):
    """Ports normal to y and to z (whose in-plane storage order differs from
    the (t1, t2) order for y), with random mode profiles: alpha and the
    gradient of the two-term (and of the E-only) coefficient against the
    oracle."""
    from paper_2505_03352_amd.plan import plan_for
    from workloads import Mode, Plane
    dev = configs.micro(n_steps=1600)
    dev.C = np.random.default_rng(61).uniform(0.3, 0.7, dev.C.shape)
    rng = np.random.default_rng(62 + axis)
    # a plane clear of the CPML, the source and the design, crossed by the field
    pl = {1: Plane(1, 17, 9, 5, 12, 8), 2: Plane(2, 11, 9, 6, 12, 10)}[axis]
    shape = (2, pl.n1, pl.n0)
    e = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    h = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    dev.ports = [Mode(pl, e, h)]
    ref = adjoint.forward_adjoint(dev, two_term=two)
    cref = np.conj(ref.alpha)
    gref = adjoint.grad_C(dev, ref, cref)
    p = plan_for(dev, two_term=two)
    p.run(3)
    a = p.alpha().cpu().numpy()
    g = p.gradient(torch.as_tensor(cref, dtype=torch.complex64, device="cuda")).cpu().numpy()
    p.close()
    ea = np.abs(a - ref.alpha).max() / np.abs(ref.alpha).max()
    eg = rel_l2(g, gref)
    say(f"{'two-term' if two else 'E-only'}, port normal to axis {axis}: alpha err {ea:.2e}, "
        f"gradient rel L2 {eg:.2e}")
    assert ea < 1e-4
    assert eg < 1e-3
