"""Order checks of the C ABI that need a bound workspace: alpha and the
Eq. (1) gradient of a run are refused once the permittivity they were
computed for has been replaced (yo_set_design or yo_set_background after the
run's reset), and accepted again after a new run."""
import sys

import numpy as np
import pytest
import torch

from paper_2505_03352_amd import YO_BOTH, _abi
from paper_2505_03352_amd.plan import plan_for
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _abi.lib()


def test_results_of_a_replaced_design_are_refused():
    print("[gpu] stale-design guard on micro", flush=True)
    sys.stdout.flush()
    dev = configs.micro(n_steps=400)
    p = plan_for(dev, device="cuda:0")
    p.run(YO_BOTH, chunk=100, use_graph=False)
    a = p.alpha()
    coef = torch.conj(a).resolve_conj().contiguous()
    g1 = p.gradient(coef)
    C2 = torch.as_tensor(np.clip(dev.C[::-1].copy(), 0, 1), dtype=torch.float32)
    p.set_design(C2, dev.beta)
    for fn in (p.alpha, lambda: p.gradient(coef), lambda: p.gradient_kappa(coef)):
        with pytest.raises(_abi.YeeOptError) as e:
            fn()
        assert e.value.status == _abi.YO_ESTATE
    p.run(YO_BOTH, chunk=100, use_graph=False)
    a2 = p.alpha()
    g2 = p.gradient(torch.conj(a2).resolve_conj().contiguous())
    torch.cuda.synchronize()
    assert torch.isfinite(g2).all() and not torch.equal(g1, g2)
    # a new background invalidates the run too
    p.set_background(torch.as_tensor(dev.kappa_bg, dtype=torch.float32),
                     torch.as_tensor(dev.mask_hr, dtype=torch.float32))
    with pytest.raises(_abi.YeeOptError) as e:
        p.alpha()
    assert e.value.status == _abi.YO_ESTATE
    p.close()


def test_forward_then_adjoint_equals_both_together():
    """Separate forward and adjoint runs (the paper's order: forward, then
    adjoint) give bitwise the phasors, alpha and gradient of one run of both
    sides in shared launches; resetting one side leaves the other's alone."""
    print("[gpu] forward then adjoint on micro", flush=True)
    dev = configs.micro(n_steps=500)
    p = plan_for(dev, device="cuda:0")
    p.run(YO_BOTH, chunk=100, use_graph=True)
    a3 = p.alpha()
    g3 = p.gradient(torch.conj(a3).resolve_conj().contiguous()).cpu().numpy()
    b3 = (p.get_dft(0, 0).cpu().numpy(), p.get_dft(1, 0).cpu().numpy())
    q = plan_for(dev, device="cuda:0")
    q.run(1, chunk=100, use_graph=False)
    with pytest.raises(_abi.YeeOptError) as e:       # no adjoint phasors yet
        q.gradient(torch.conj(a3).resolve_conj().contiguous())
    assert e.value.status == _abi.YO_ESTATE
    q.run(2, chunk=100, use_graph=False)
    a = q.alpha()
    g = q.gradient(torch.conj(a).resolve_conj().contiguous()).cpu().numpy()
    assert np.array_equal(a.cpu().numpy(), a3.cpu().numpy())
    assert np.array_equal(q.get_dft(0, 0).cpu().numpy(), b3[0])
    assert np.array_equal(q.get_dft(1, 0).cpu().numpy(), b3[1])
    assert np.array_equal(g, g3)
    p.close()
    q.close()
