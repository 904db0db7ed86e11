"""The shipped split table (paper_2505_03352_amd/tuned_splits.json): every
entry is a split yo_set_tiling accepts for a plan with two steps per launch,
and the benchmark devices' shape-class keys (as autotune.shape_key builds
them for a gfx950 device) are in it."""
import types

from paper_2505_03352_amd import autotune
from workloads import configs


def _fake_plan(dev):
    n_src, n_ports, n_freq = len(dev.sources), len(dev.ports), dev.n_freq
    n_fwd = n_src * n_freq
    from paper_2505_03352_amd.plan import grid_design_of
    g, _ = grid_design_of(dev)
    return types.SimpleNamespace(grid=g, n_stepped_fwd=n_fwd, n_stepped=(n_src + n_ports) * n_freq,
                                 time_blocking=2, device="cpu")


def test_shipped_splits_are_valid_and_cover_the_benchmark_devices():
    table = autotune.shipped_splits()
    assert table
    for key, rec in table.items():
        assert key.startswith("gfx950|") and key.endswith("|tb2")
        assert rec["rows"] == 4 and 4 <= rec["zchunk"] <= 63
        assert rec["flags"] & 512 and not rec["flags"] & ~32767
        assert not (rec["flags"] & 16)            # 512 does not combine with 16
        assert rec["ms_per_step"] > 0
    for dev in (configs.multiport(), configs.realistic()):
        assert autotune.shape_key(_fake_plan(dev), 3) in table
