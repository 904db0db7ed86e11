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
