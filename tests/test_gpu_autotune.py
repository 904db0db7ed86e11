"""The work-split autotuner on the GPU: it times exactly the settings it is
given, applies the fastest, leaves alpha and the gradient bitwise unchanged
(every split computes the same fields), and a second plan of the same shape
class takes the cached choice without timing."""
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


def test_tuner_choice_cache_and_unchanged_results(tmp_path, monkeypatch):
    from paper_2505_03352_amd import autotune
    from paper_2505_03352_amd.plan import plan_for
    monkeypatch.setenv("YEEOPT_AUTOTUNE_CACHE", str(tmp_path / "autotune.json"))
    dev = configs.tiny(n_steps=400)
    p = plan_for(dev)
    p.run(3)
    a0 = p.alpha().cpu().numpy()
    g0 = p.gradient(torch.conj(p.alpha())).cpu().numpy()
    shared = [(8, 0), (10, 1), (16, 128)]
    say("autotune: sweep")
    rec = autotune.tune(p, 3, shared=shared, n_launch=2, use_cache=True)
    assert not rec["cached"]
    assert set(rec["timings"]) == {"z8f0", "z10f1", "z16f128"}
    best = min(rec["timings"].values(), key=lambda t: t["ms"])
    assert rec["flags"] == best["best"] and rec["ms_per_step"] == pytest.approx(best["ms"], abs=1e-4)
    assert p.tiling == (rec["rows"], rec["zchunk"], rec["flags"])
    for t in rec["timings"].values():
        assert min(t["shell"].values()) > 0
    assert min(rec["timings"]["z8f0"]["interior"].values()) > 0
    # on this 56-cell-wide grid the two full 62-cell x-shell strips take every
    # column: the interior launch has no tiles and times zero
    assert max(rec["timings"]["z10f1"]["interior"].values()) == 0.0
    p.run(3)
    a1 = p.alpha().cpu().numpy()
    g1 = p.gradient(torch.conj(p.alpha())).cpu().numpy()
    p.close()
    assert np.array_equal(a0, a1) and np.array_equal(g0, g1)

    say("autotune: cached choice")
    q = plan_for(dev)
    rec2 = autotune.tune(q, 3, use_cache=True)
    assert rec2["cached"]
    assert q.tiling == (rec["rows"], rec["zchunk"], rec["flags"])
    q.close()
