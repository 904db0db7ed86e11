"""The allocation-free binding (yo_bind_static_workspace) against the
caller-workspace binding (yo_bind_workspace): the same forward and adjoint
runs, alpha and Eq. (1) gradient through the C ABI, twice in a row on the
device's static workspace, the second time with a smaller device."""
import sys

import numpy as np
import pytest
import torch

from paper_2505_03352_amd import YO_BOTH, _abi
from paper_2505_03352_amd.plan import plan_for
from workloads import configs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _abi.lib()


def _solve(dev, static):
    p = plan_for(dev, device="cuda:0", static_workspace=static)
    p.run(YO_BOTH, chunk=100, use_graph=True)
    alpha = p.alpha()
    g = p.gradient(torch.conj(alpha).resolve_conj().contiguous())
    box = p.get_dft(0, 0)
    torch.cuda.synchronize()
    return p, alpha.cpu().numpy(), g.cpu().numpy(), box.cpu().numpy()


def test_static_workspace_matches_caller_workspace_twice():
    # first call: the tiny 56x56x36 device (about 21 MiB of workspace); second:
    # the micro device (under 3 MiB), on the array the first call left dirty
    devs = [configs.tiny(), configs.micro(n_steps=800)]
    first = None
    for i, dev in enumerate(devs):
        say(f"static workspace call {i}: {dev.name} {dev.nx}x{dev.ny}x{dev.nz}, {dev.n_steps} steps")
        ps, a_s, g_s, b_s = _solve(dev, static=True)
        pr, a_r, g_r, b_r = _solve(dev, static=False)
        pr.close()
        # same kernels on the same inputs: identical bits
        assert np.array_equal(a_s, a_r), np.abs(a_s - a_r).max()
        assert np.array_equal(g_s, g_r), np.abs(g_s - g_r).max()
        assert np.array_equal(b_s, b_r), np.abs(b_s - b_r).max()
        assert np.abs(a_s).max() > 0 and np.abs(g_s).max() > 0
        if first is not None:
            # the second static binding took the memory over from the first plan
            with pytest.raises(_abi.YeeOptError) as e:
                first.alpha()
            assert e.value.status == _abi.YO_EWORKSPACE
            first.close()
        first = ps
    first.close()
