"""The non-finite watchdog of the C ABI on the GPU: a run whose fields
diverged reports YO_EUNSTABLE from finalize, alpha and the gradient refuse
until the next reset, the phasors stay readable, and the next clean run of
the same plan gives bitwise the results it gave before."""
import sys

import numpy as np
import pytest
import torch

from workloads import configs

pytestmark = pytest.mark.gpu

YO_EUNSTABLE = -5


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_03352_amd import _abi
    _abi.lib()


@pytest.mark.parametrize("bad", ["nan", "inf"])
def test_diverged_run_is_reported_and_cleared_by_reset(bad):
    from paper_2505_03352_amd import YeeOptError
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=600)
    p = plan_for(dev)
    say(f"watchdog ({bad}): clean run")
    p.run(3)
    a0 = p.alpha().cpu().numpy()
    g0 = p.gradient(torch.conj(p.alpha())).cpu().numpy()
    assert np.isfinite(a0).all() and np.isfinite(g0).all()

    say(f"watchdog ({bad}): run from non-finite forward fields")
    p.reset(3)
    E, H = p.get_fields(0)
    E.fill_(float(bad))
    p.set_fields(0, E, H)
    p.advance(3, dev.n_steps)
    with pytest.raises(YeeOptError) as e:
        p.finalize(3)
    assert e.value.status == YO_EUNSTABLE
    with pytest.raises(YeeOptError) as e:
        p.alpha()
    assert e.value.status == YO_EUNSTABLE
    with pytest.raises(YeeOptError) as e:
        p.gradient(torch.as_tensor(np.conj(a0), device="cuda"))
    assert e.value.status == YO_EUNSTABLE
    # the phasors stay readable: the forward box is non-finite, the adjoint
    # right-hand sides (clean fields) are not
    assert not np.isfinite(p.get_dft(0).cpu().numpy()).all()
    assert np.isfinite(p.get_dft(p.n_rhs - 1).cpu().numpy()).all()

    say(f"watchdog ({bad}): clean run again")
    p.run(3)
    a1 = p.alpha().cpu().numpy()
    g1 = p.gradient(torch.conj(p.alpha())).cpu().numpy()
    p.close()
    assert np.array_equal(a0, a1)
    assert np.array_equal(g0, g1)


def test_forward_only_run_that_diverged_is_reported():
    from paper_2505_03352_amd import YO_FORWARD, YeeOptError
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=400)
    p = plan_for(dev)
    p.reset(YO_FORWARD)
    E, H = p.get_fields(0)
    H.fill_(float("nan"))
    p.set_fields(0, E, H)
    p.advance(YO_FORWARD, dev.n_steps)
    with pytest.raises(YeeOptError) as e:
        p.finalize(YO_FORWARD)
    assert e.value.status == YO_EUNSTABLE
    with pytest.raises(YeeOptError) as e:
        p.alpha()
    assert e.value.status == YO_EUNSTABLE
    p.run(YO_FORWARD)
    assert np.isfinite(p.alpha().cpu().numpy()).all()
    p.close()


def test_diverged_plan_in_a_shared_launch_leaves_the_others_alone():
    """Two plans stepped in the same launches, one from NaN fields: only
    that plan's finalize reports YO_EUNSTABLE, and the clean plan's alpha
    and gradient are bitwise those of its run alone."""
    from paper_2505_03352_amd import YeeOptError
    from paper_2505_03352_amd.plan import advance_many, plan_for
    dev = configs.micro(n_steps=500)
    a = plan_for(dev)
    b = plan_for(dev)
    a.run(3)
    a0 = a.alpha().cpu().numpy()
    g0 = a.gradient(torch.conj(a.alpha())).cpu().numpy()
    say("watchdog: clean and diverged plan in shared launches")
    a.reset(3)
    b.reset(3)
    E, H = b.get_fields(0)
    E.fill_(float("nan"))
    b.set_fields(0, E, H)
    advance_many([a, b], [3, 3], dev.n_steps, chunk=100, use_graph=True)
    a.finalize(3)
    with pytest.raises(YeeOptError) as e:
        b.finalize(3)
    assert e.value.status == YO_EUNSTABLE
    a1 = a.alpha().cpu().numpy()
    g1 = a.gradient(torch.conj(a.alpha())).cpu().numpy()
    a.close()
    b.close()
    assert np.array_equal(a0, a1)
    assert np.array_equal(g0, g1)


def test_negative_background_kappa_diverges_and_is_reported():
    """A block of negative kappa (negative permittivity, no dispersion) next
    to the source makes the scheme grow without bound (the FP64 oracle's
    fields on this device reach 1e28 after 100 steps and 1e64 after 200);
    the run returns YO_EUNSTABLE instead of NaN coefficients."""
    from paper_2505_03352_amd import YeeOptError
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.micro(n_steps=600)
    kb = dev.kappa_bg.copy()
    x0, y0, z0, bx, by, bz = dev.dft_box()
    assert 8 <= x0                      # the block [6, 8) lies before the design box in x
    kb[:, 7:11, 8:13, 6:8] = -0.3
    dev.kappa_bg = kb
    p = plan_for(dev)
    say("watchdog: negative background kappa")
    with pytest.raises(YeeOptError) as e:
        p.run(3)
    assert e.value.status == YO_EUNSTABLE
    with pytest.raises(YeeOptError) as e:
        p.alpha()
    assert e.value.status == YO_EUNSTABLE
    p.close()
