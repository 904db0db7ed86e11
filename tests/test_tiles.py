"""The work split on the host (yo_tile_table, no GPU): for every tiling
choice the launches of a single step own every cell of the grid exactly
once, and so do the launches of a pair of steps (the two-step region, the
interior around it, the z-slabs under it and the paired steps' shell); the
two-step region keeps two cells clear of every absorbing slab and clear of
the source and port planes; tile classes say which slabs a tile meets."""
import numpy as np
import pytest

from paper_2505_03352_amd.plan import Plan, freqs_of, grid_design_of
from workloads import configs

SINGLE = [0, 1, 128, 2 | 4, 16 | 32, 256, 8 | 64, 1 | 2 | 8 | 64, 16384 | 1 | 8]
PAIRS = [512, 512 | 128, 512 | 1, 512 | 2048 | 128, 512 | 4096 | 128, 512 | 8192 | 2, 512 | 256,
         512 | 1024 | 8, 512 | 4096 | 8192 | 1 | 2, 512 | 2048 | 16384 | 128]


def _plan(dev, tb):
    grid, design = grid_design_of(dev)
    return Plan(grid, design, dev.n_steps, freqs_of(dev), [m.plane for m in dev.sources],
                [m.plane for m in dev.ports], device="cpu", time_blocking=tb)


def _cover(p, parts, shape):
    cov = np.zeros(shape, dtype=np.int16)
    for part in parts:
        for x0, x1, y0, y1, z0, z1, _ in p.tile_table(part):
            assert x0 < x1 and y0 < y1 and z0 < z1
            cov[z0:z1, y0:y1, x0:x1] += 1
    return cov


def _slabs(dev):
    g, _ = grid_design_of(dev)
    return g["npml"], (dev.nx, dev.ny, dev.nz)


@pytest.mark.parametrize("name", ["micro", "realistic", "multiport"])
def test_every_split_owns_every_cell_once(name):
    dev = getattr(configs, name)()
    shape = (dev.nz, dev.ny, dev.nx)
    npml, n = _slabs(dev)
    plo, phi = npml[0::2], npml[1::2]
    planes = [m.plane for m in dev.sources] + [m.plane for m in dev.ports]
    for tb, flag_sets in ((1, SINGLE), (2, SINGLE + PAIRS)):
        p = _plan(dev, tb)
        for zc in (8, 10, 16):
            for fl in flag_sets:
                p.set_tiling(4, zc, fl)
                cov = _cover(p, (0, 1), shape)
                assert cov.min() == 1 and cov.max() == 1, (name, tb, zc, fl, "single")
                if not fl & 512:
                    continue
                r2 = p.tile_table(2)
                if len(r2) == 0:
                    continue
                cov = _cover(p, (2, 3, 4, 5), shape)
                assert cov.min() == 1 and cov.max() == 1, (name, zc, fl, "pairs")
                lo = r2[:, [0, 2, 4]].min(axis=0)
                hi = r2[:, [1, 3, 5]].max(axis=0)
                for a in range(3):
                    assert lo[a] >= plo[a] + 2 and hi[a] <= n[a] - phi[a] - 1, (fl, a)
                # no source or port plane where the region computes step
                # n+1's E (one cell around it along the plane's normal)
                for pl in planes:
                    a = pl.axis
                    assert pl.index < lo[a] - 1 or pl.index > hi[a], (fl, pl)
                assert (r2[:, 1] - r2[:, 0]).max() <= 60
                rows = 6 if fl & 4096 else 4
                waves = (8 if fl & 2 else 4) if fl & 8192 else 1
                assert (r2[:, 3] - r2[:, 2]).max() <= rows * waves
                z2 = p.tile_table(4)
                if len(z2):
                    assert (z2[:, 6] == 4).all()
                    assert ((z2[:, 5] <= plo[2] + 2) | (z2[:, 4] >= n[2] - phi[2] - 1)).all()
        p.close()


def test_tile_classes_name_the_slabs_a_tile_meets():
    dev = configs.realistic()
    npml, n = _slabs(dev)
    plo, phi = npml[0::2], npml[1::2]
    p = _plan(dev, 2)
    for fl in (0, 1, 128, 512 | 128):
        p.set_tiling(4, 10, fl)
        for part in (0, 1):
            for t in p.tile_table(part):
                cls = 0
                for a in range(3):
                    if t[2 * a] < plo[a] + 1 or t[2 * a + 1] > n[a] - phi[a]:
                        cls |= 1 << a
                if part == 0:
                    assert t[6] == 0 and cls == 0, (fl, t)
                else:
                    # a shell tile's class holds every slab it meets (it may
                    # hold more: strips cut wider than the slab run its code)
                    assert t[6] != 0 and (t[6] & cls) == cls, (fl, t)
    p.close()


@pytest.mark.parametrize("zc", [4, 63])
def test_extreme_z_chunks_still_own_every_cell_once(zc):
    """The shortest and longest z-chunks the library accepts, with the
    shipped splits' other choices: the launches of one step and of a pair
    of steps still cover the realistic grid once."""
    dev = configs.realistic()
    shape = (dev.nz, dev.ny, dev.nx)
    p = _plan(dev, 2)
    for fl in (8777, 21067, 16384 | 1 | 8):
        p.set_tiling(4, zc, fl)
        cov = _cover(p, (0, 1), shape)
        assert cov.min() == 1 and cov.max() == 1, (zc, fl, "single")
        if fl & 512:
            cov = _cover(p, (2, 3, 4, 5), shape)
            assert cov.min() == 1 and cov.max() == 1, (zc, fl, "pairs")
            z = p.tile_table(2)[:, 5] - p.tile_table(2)[:, 4]
            assert z.max() <= zc
    p.close()


def _tuner_space():
    """Every (z-chunk, flags) the autotuner can apply: the single-step
    sweep (shared choice | interior flags | shell flags) and the pairs
    sweep (shared choice | 512 | two-step variant | frame flag | shell
    flags, with or without the side stream)."""
    from paper_2505_03352_amd import autotune as at
    out = set()
    for zc, base in at.SHARED:
        for fi in at.INTERIOR_FLAGS:
            for fs in at.SHELL_FLAGS:
                out.add((zc, base | fi | fs))
    for zc, base in at.PAIR_SHARED:
        for v in (0, 4096, 8192, 4096 | 8192):
            for ff in (0, 32):
                for fs in at.SHELL_FLAGS:
                    for ov in (0, 1024):
                        out.add((zc, base | 512 | v | ff | fs | ov))
    return sorted(out)


def test_every_split_the_tuner_can_pick_is_valid_and_owns_every_cell_once():
    """The library accepts every split in the tuner's search space (no
    YO_EINVAL mid-sweep), and each owns every cell once: all of them on
    the micro device, a seeded sample of 60 on the realistic one."""
    import random
    from paper_2505_03352_amd import autotune as at
    space = _tuner_space()
    assert len(space) > 1000
    for name, n in (("micro", None), ("realistic", 60)):
        dev = getattr(configs, name)()
        shape = (dev.nz, dev.ny, dev.nx)
        p = _plan(dev, 2)
        for zc, fl in space:
            p.set_tiling(at.ROWS, zc, fl)
        for zc, fl in (space if n is None else random.Random(0).sample(space, n)):
            p.set_tiling(at.ROWS, zc, fl)
            cov = _cover(p, (0, 1), shape)
            assert cov.min() == 1 and cov.max() == 1, (name, zc, fl, "single")
            if fl & 512:
                cov = _cover(p, (2, 3, 4, 5), shape)
                assert cov.min() == 1 and cov.max() == 1, (name, zc, fl, "pairs")
        p.close()
