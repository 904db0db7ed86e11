"""End-to-end parity at full size: the 320x240x96 realistic device at one
wavelength (1.55 um: one forward and one adjoint right-hand side, 10 000
steps), run through the C ABI in the bench's launch configuration for this
grid (two steps per launch with its shipped split: cooperative two-step
blocks, 16 z-planes per tile; hipGraph chunks of 100 steps), and
the FP64 oracle computing everything from the same controls (its own chain,
its own kappa): DFT phasors of the design box and the port plane (relative
L2 <= 1e-4), alpha (<= 1e-4) and dF/dC (relative L2 <= 1e-3)."""
import os
import sys
import time

import numpy as np
import pytest
import torch

from oracle import adjoint, chain, ports
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


@pytest.mark.timeout(900)
def test_realistic_one_wavelength_end_to_end_matches_oracle():
    from paper_2505_03352_amd import YO_BOTH
    from paper_2505_03352_amd.plan import plan_for
    dev = configs.realistic(wavelengths=[1.55e-6])
    assert dev.n_steps == 10000
    from paper_2505_03352_amd import autotune
    recs = [v for k, v in autotune.shipped_splits().items() if "|ny240|nz96|" in k and k.endswith("|tb2")]
    assert len(recs) == 1
    rec = recs[0]
    say(f"realistic end to end: GPU (2 right-hand sides x 10000 steps), split {rec}")
    p = plan_for(dev, time_blocking=2)
    p.set_tiling(rec["rows"], rec["zchunk"], rec["flags"])
    p.run(YO_BOTH, chunk=100, use_graph=True)
    alpha = p.alpha()
    g = p.gradient(torch.conj(alpha).resolve_conj().contiguous())
    got = dict(alpha=alpha.cpu().numpy(), g=g.cpu().numpy(),
               fbox=p.get_dft(0, 0).cpu().numpy(), abox=p.get_dft(1, 0).cpu().numpy(),
               fmon=p.get_dft(0, 1).cpu().numpy(), amon=p.get_dft(1, 1).cpu().numpy(),
               kappa=p.get_kappa().cpu().numpy())
    p.close()
    torch.cuda.synchronize()
    # the oracle: its own chain from the controls, then the two runs
    os.environ.setdefault("ORC_PROGRESS_STEPS", "1000")
    t0 = time.time()
    kap, st = chain.kappa(dev)
    ek = np.abs(got["kappa"] - kap).max() / np.abs(kap).max()
    say(f"  kappa max rel err {ek:.2e}; oracle forward run")
    lam = dev.wavelengths[0]
    W = ports.monitor_weights(dev.ports[0].e, dev.ports[0].h)
    fwd = adjoint.solve(dev, kap, dev.sources[0].plane, ports.source_current(dev.sources[0].h), lam)
    say(f"  oracle adjoint run ({time.time() - t0:.0f} s so far)")
    adj = adjoint.solve(dev, kap, dev.ports[0].plane, W, lam)
    say(f"  oracle done in {time.time() - t0:.0f} s; residuals {fwd.resid:.1e} {adj.resid:.1e}")
    a_ref = np.array([[[ports.alpha(W, fwd.mon[0])]]])
    res = adjoint.Result(a_ref, [[fwd]], [[adj]], kap, st, [W], dev.beta)
    g_ref = adjoint.grad_C(dev, res, np.conj(a_ref))
    e = dict(fbox=rel_l2(got["fbox"], fwd.box), abox=rel_l2(got["abox"], adj.box),
             fmon=rel_l2(got["fmon"], fwd.mon[0]), amon=rel_l2(got["amon"], adj.mon[0]),
             alpha=float(np.abs(got["alpha"] - a_ref).max() / np.abs(a_ref).max()),
             g=rel_l2(got["g"], g_ref))
    say("  " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert ek < 1e-5
    assert e["fbox"] < 1e-4 and e["abox"] < 1e-4
    assert e["fmon"] < 1e-4 and e["amon"] < 1e-4
    assert e["alpha"] < 1e-4
    assert e["g"] < 1e-3
