"""Plans with no output ports (forward fields only) or no sources (adjoint
fields only), through the C ABI: alpha and the coefficient array are empty
(null device pointers), the gradient is exactly zero, and every right-hand
side's DFT box is bitwise the one the full plan computes for it."""
import sys

import numpy as np
import pytest
import torch

from workloads import configs

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


def test_forward_only_and_adjoint_only_plans():
    from paper_2505_03352_amd.plan import plan_for
    n_steps = 900
    dev = configs.micro_demux(n_steps=n_steps)
    ns, npo, nf = len(dev.sources), len(dev.ports), dev.n_freq
    assert ns == 1 and npo == 2 and nf == 2
    say("empty plans: full plan")
    full = plan_for(dev)
    full.run(3)
    fwd = [full.get_dft(f * ns).cpu() for f in range(nf)]
    adj = [full.get_dft(ns * nf + f * npo + q).cpu() for f in range(nf) for q in range(npo)]
    full.close()

    say("empty plans: no ports")
    d1 = configs.micro_demux(n_steps=n_steps)
    d1.ports = []
    p1 = plan_for(d1)
    assert p1.n_rhs == ns * nf
    p1.run(3)
    a1 = p1.alpha()
    assert tuple(a1.shape) == (ns, 0, nf)
    g1 = p1.gradient(torch.zeros((ns, 0, nf), dtype=torch.complex64, device="cuda"))
    gk1 = p1.gradient_kappa(torch.zeros((ns, 0, nf), dtype=torch.complex64, device="cuda"))
    for f in range(nf):
        assert torch.equal(p1.get_dft(f).cpu(), fwd[f])
    p1.close()
    assert torch.count_nonzero(g1).item() == 0 and torch.count_nonzero(gk1).item() == 0

    say("empty plans: no sources")
    d2 = configs.micro_demux(n_steps=n_steps)
    d2.sources = []
    p2 = plan_for(d2)
    assert p2.n_rhs == npo * nf
    p2.run(3)
    assert tuple(p2.alpha().shape) == (0, npo, nf)
    g2 = p2.gradient(torch.zeros((0, npo, nf), dtype=torch.complex64, device="cuda"))
    for r in range(npo * nf):
        assert torch.equal(p2.get_dft(r).cpu(), adj[r])
    p2.close()
    assert torch.count_nonzero(g2).item() == 0
    assert np.isfinite(torch.stack(adj).numpy()).all()
