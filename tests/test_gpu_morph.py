"""Morphological filters (paper Sec. 3, Eqs. 4-6) on the GPU against the FP64
oracle, through the C ABI: kappa and the chain's transpose with filters at
the tiny and realistic sizes, the unbinarity of the filtered design, and
forward + adjoint + gradient on a micro device.

Tolerances: kappa max error <= 5e-5 of max |kappa| (FP32 sums of up to a few
hundred exponentials per stage, then Eq. (6) scales an error in the filtered
density by beta/2 before the density mix); the chain's transpose <= 1e-4
relative L2; alpha <= 1e-4 and dF/dC <= 1e-3 as for the unfiltered chain."""
import sys

import numpy as np
import pytest
import torch

from oracle import adjoint, chain
from oracle import optimize as O
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


def with_filters(dev, ops, d, alpha=20.0):
    dev.morph_ops, dev.morph_d, dev.morph_alpha = ops, d, alpha
    return dev


def light(dev):
    dev.wavelengths = dev.wavelengths[:1]
    dev.n_steps = 400
    return dev


@pytest.mark.parametrize("name,ops,d,beta", [("tiny", "edde", 3.0, None), ("tiny", "d", 2.0, None),
                                             ("tiny", "e", 2.5, 30.0), ("tiny", "de", 7.5, None),
                                             ("realistic", "edde", 5.0, None)])
def test_chain_and_vjp_with_filters_match_oracle(name, ops, d, beta):
    from paper_2505_03352_amd.plan import plan_for
    dev = with_filters(light({"tiny": configs.tiny, "realistic": configs.realistic}[name]()), ops, d)
    if beta is not None:
        dev.beta = beta
    say(f"filtered chain {name} ops={ops} d={d}: oracle")
    o = chain.make_ops(dev)
    kref, st = chain.kappa(dev, ops=o)
    say(f"filtered chain {name} ops={ops} d={d}: GPU")
    p = plan_for(dev)
    kap = p.get_kappa().cpu().numpy()
    ek = np.abs(kap - kref).max() / np.abs(kref).max()
    rng = np.random.default_rng(1)
    x0, y0, z0, bx, by, bz = dev.dft_box()
    g3 = rng.standard_normal((3, bz, by, bx))
    gC = p.chain_vjp(torch.as_tensor(g3, dtype=torch.float32)).cpu().numpy()
    gref = chain.vjp(dev, st, dev.beta, *chain.zsum(dev, g3), o)
    eg = rel_l2(gC, gref)
    u = float(p.unbinarity()[0])
    uo = O.unbinarity(O.design_rho(dev, st))
    say(f"  kappa max rel err {ek:.2e}, VJP rel L2 {eg:.2e}, u {u:.5f} / {uo:.5f}")
    p.close()
    assert ek < 5e-5
    assert eg < 1e-4
    assert abs(u - uo) < 1e-3
    # the filters changed the design
    plain = light({"tiny": configs.tiny, "realistic": configs.realistic}[name]())
    plain.beta = dev.beta
    k0, _ = chain.kappa(plain, ops=chain.make_ops(plain))
    assert np.abs(k0 - kref).max() > 1e-3


def test_gradient_with_filters_matches_oracle():
    from paper_2505_03352_amd.plan import plan_for
    dev = with_filters(configs.micro(n_steps=700, md=10, nd=9, mc=7, nc=6), "edde", 1.5)
    say("filtered micro device: oracle")
    ref = adjoint.forward_adjoint(dev)
    _, cref = adjoint.objective_abs2(ref.alpha)
    gref = adjoint.grad_C(dev, ref, cref)
    say("filtered micro device: GPU")
    p = plan_for(dev)
    p.run(3)
    a = p.alpha().cpu().numpy()
    g = p.gradient(torch.conj(p.alpha())).cpu().numpy()
    p.close()
    ea = np.abs(a - ref.alpha).max() / np.abs(ref.alpha).max()
    eg = rel_l2(g, gref)
    say(f"  alpha err {ea:.2e} gradient rel L2 {eg:.2e}")
    assert ea < 1e-4
    assert eg < 1e-3


def test_filters_off_again_gives_the_plain_chain():
    from paper_2505_03352_amd.plan import plan_for
    dev = light(configs.tiny())
    p0 = plan_for(dev)
    k0 = p0.get_kappa().cpu().numpy()
    p0.close()
    dev.morph_ops = ""
    dev.morph_d = 3.0
    p1 = plan_for(dev)
    k1 = p1.get_kappa().cpu().numpy()
    p1.close()
    assert np.array_equal(k0, k1)
