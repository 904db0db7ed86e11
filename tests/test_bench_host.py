"""Host-side bookkeeping of bench.py (no GPU): the flag bits that shape
each launch part, and the rule that a committed counter summary only
counts for the kernel sources and split it was taken on."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_part_split_keeps_only_the_bits_that_shape_the_part():
    t = (4, 16, 21067)                 # 16384|4096|512|64|8|2|1
    assert bench.part_split(t, 2) == "4,16,4611"       # two-step: 4096|512|2|1
    assert bench.part_split(t, 5) == "4,16,16971"      # paired shell: 16384|512|64|8|2|1
    # bits that do not shape a launch leave its split unchanged
    assert bench.part_split((4, 16, 21067 | 1024), 2) == bench.part_split(t, 2)
    assert bench.part_split((4, 16, 21067 & ~16384), 2) == bench.part_split(t, 2)
    assert bench.part_split((4, 16, 21067 & ~16384), 5) != bench.part_split(t, 5)


def _summary(tmp_path, sha, split, b=123456789):
    p = tmp_path / "t.txt"
    p.write_text(f"# header line with = in it\nkernel_sha={sha}\nsplit={split}\n"
                 f"hbm_bytes_per_launch={b}\nfetch_kib=1\nwrite_kib=1\n")
    return str(p)


def test_read_traffic_needs_the_same_kernel_and_split(tmp_path):
    path = _summary(tmp_path, "abc", "4,16,4611")
    assert bench.read_traffic(path, "abc", "4,16,4611") == 123456789.0
    assert bench.read_traffic(path, "abd", "4,16,4611") is None
    assert bench.read_traffic(path, "abc", "4,10,4611") is None
    assert bench.read_traffic(path, "abc", None) is None
    assert bench.read_traffic(str(tmp_path / "missing.txt"), "abc", "4,16,4611") is None


def test_committed_summaries_parse_and_are_plausible():
    """Every committed traffic summary names a kernel hash and a split and
    gives a per-launch byte count between half and three times the
    launch's one-step algorithmic bytes stated in it."""
    import re
    found = 0
    for name in os.listdir(bench.PROFILES):
        if not name.endswith("_traffic.txt"):
            continue
        txt = open(os.path.join(bench.PROFILES, name)).read()
        kv = dict(line.split("=", 1) for line in txt.splitlines() if "=" in line and not line.startswith("#"))
        assert re.fullmatch(r"[0-9a-f]{16}", kv["kernel_sha"]), name
        assert re.fullmatch(r"4,\d+,\d+", kv["split"]), name
        m = re.search(r"traffic / algorithmic = ([0-9.]+)", txt)
        assert m and 0.5 < float(m.group(1)) < 3.0, name
        assert bench.read_traffic(os.path.join(bench.PROFILES, name), kv["kernel_sha"], kv["split"]) > 0
        found += 1
    assert found >= 2
