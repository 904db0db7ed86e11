"""The benchmark workloads as seeded synthetic devices.

* ``tiny()``       40x40x20 cells at 40 nm plus an 8-cell CPML outside
                   (56x56x36 allocated), 24x24x6 design, 24x24 controls,
                   Gaussian filter r=2, beta=4, 1.55 um, 2000 steps.
* ``realistic()``  320x240x96 at 20 nm (CPML included), 220 nm Si slab in
                   SiO2, 2x2 um design (100x100 px), 100x100 controls, r=3,
                   beta=8, 10 000 steps, 1.50/1.55/1.60 um.
* ``batch()``      8 designs, each axis drawn uniformly between 128x96x64 and
                   320x240x96, one wavelength, seeds 100+d.
* ``serving_trace()`` 200 Poisson arrivals at 4 req/s, sizes from a 3-way
                   mixture, 1-3 wavelengths each.
* ``multiport()``  600x400x120 1-to-4 splitter-like grid, 250x150 controls,
                   r=4, beta=16, 5 wavelengths 1.50-1.60 um, 20 000 steps.
* ``demux()``      two-wavelength demultiplexer analogue (optimizer loop).
* ``micro()``, ``micro_demux()``  very small devices for tests.
"""
from __future__ import annotations

import math

import numpy as np

from .devices import soi_device

UM = 1e-6


def steps_rule(nx: int, ny: int, dx: float, lam: float, courant: float = 0.5,
               minimum: int = 2000) -> int:
    """31 * max(nx, ny) steps rounded up to whole periods, at least ``minimum``."""
    period = lam / (courant * dx)
    n = max(31 * max(nx, ny), minimum)
    return int(math.ceil(math.ceil(n / period) * period))


def tiny(seed: int = 0, n_steps: int = 2000):
    npml = 8
    return soi_device("tiny", 40 + 2 * npml, 40 + 2 * npml, 20 + 2 * npml, 40e-9, npml,
                      md=24, nd=24, slab_layers=6, mc=24, nc=24, filter_r=2.0, beta=4.0,
                      wavelengths=[1.55 * UM], n_steps=n_steps, seed=seed,
                      mode_w=(5.0, 3.0), ramp_periods=5.0)


def realistic(seed: int = 1, n_steps: int = 10000, wavelengths=None):
    wl = [1.50 * UM, 1.55 * UM, 1.60 * UM] if wavelengths is None else wavelengths
    return soi_device("realistic", 320, 240, 96, 20e-9, 8, md=100, nd=100, slab_layers=11,
                      mc=100, nc=100, filter_r=3.0, beta=8.0, wavelengths=wl,
                      n_steps=n_steps, seed=seed)


def batch_member(d: int, n_steps=None, wavelength=1.55 * UM):
    rng = np.random.default_rng(100 + d)
    nx = int(rng.integers(128, 321))
    ny = int(rng.integers(96, 241))
    nz = int(rng.integers(64, 97))
    md, nd = nx // 2, ny // 2
    steps = steps_rule(nx, ny, 20e-9, wavelength) if n_steps is None else n_steps
    return soi_device(f"batch{d}", nx, ny, nz, 20e-9, 8, md=md, nd=nd, slab_layers=11,
                      mc=md, nc=nd, filter_r=3.0, beta=8.0, wavelengths=[wavelength],
                      n_steps=steps, seed=100 + d)


def batch(n_designs: int = 8, n_steps=None):
    return [batch_member(d, n_steps) for d in range(n_designs)]


SERVING_CLASSES = ("small", "medium", "large")


def serving_request(i: int, cls: str, wavelengths, n_steps=None):
    rng = np.random.default_rng(1000 + i)
    if cls == "small":
        nx, ny, nz = (96 + int(rng.integers(-8, 9)) for _ in range(3))
    elif cls == "medium":
        nx, ny, nz = 200, 160, 80
    else:
        nx, ny, nz = 320, 240, 96
    md, nd = nx // 2, ny // 2
    lam_max = max(wavelengths)
    steps = steps_rule(nx, ny, 20e-9, lam_max) if n_steps is None else n_steps
    return soi_device(f"req{i}", nx, ny, nz, 20e-9, 8, md=md, nd=nd, slab_layers=11,
                      mc=md, nc=nd, filter_r=3.0, beta=8.0, wavelengths=list(wavelengths),
                      n_steps=steps, seed=1000 + i)


def serving_trace(n_requests: int = 200, rate: float = 4.0, seed: int = 200):
    """(arrival_time_s, size class, wavelengths) for each request."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    grid = [1.50 * UM, 1.55 * UM, 1.60 * UM]
    out = []
    for i in range(n_requests):
        cls = SERVING_CLASSES[int(rng.integers(0, 3))]
        nw = int(rng.integers(1, 4))
        lams = sorted(rng.choice(grid, size=nw, replace=False).tolist())
        out.append((float(t[i]), cls, lams))
    return out


def multiport(seed: int = 300, n_steps: int = 20000, wavelengths=None):
    wl = ([1.500 * UM, 1.525 * UM, 1.550 * UM, 1.575 * UM, 1.600 * UM]
          if wavelengths is None else wavelengths)
    offs = (-1.125 * UM, -0.375 * UM, 0.375 * UM, 1.125 * UM)
    return soi_device("multiport", 600, 400, 120, 20e-9, 8, md=250, nd=150, slab_layers=11,
                      mc=250, nc=150, filter_r=4.0, beta=16.0, wavelengths=wl,
                      n_steps=n_steps, seed=seed, out_offsets=offs)


def micro(seed: int = 7, n_steps: int = 600, nx: int = 30, ny: int = 26, nz: int = 18,
          npml: int = 5, md: int = 8, nd: int = 8, mc: int = 6, nc: int = 5,
          wavelengths=None, beta: float = 4.0, filter_r: float = 1.5, layers: int = 3,
          out_offsets=(0.0,)):
    """A few-thousand-cell device for CPU tests of the oracle (40 nm cells,
    shorter wavelength so a few periods fit)."""
    wl = [0.8 * UM] if wavelengths is None else wavelengths
    return soi_device("micro", nx, ny, nz, 40e-9, npml, md=md, nd=nd, slab_layers=layers,
                      mc=mc, nc=nc, filter_r=filter_r, beta=beta, wavelengths=wl,
                      n_steps=n_steps, seed=seed, mode_w=(3.0, 1.5), ramp_periods=3.0,
                      strip_width=240e-9, src_inset=3, out_offsets=out_offsets)


def demux(seed: int = 400, n_steps=None):
    """Two-wavelength demultiplexer analogue of the paper's Sec. 4 example:
    1.30 um to output 1, 1.55 um to output 2; 430x450x64 cells (the
    example's 12.38 M) at a uniform 25 nm (CPML 8), a 210x210-pixel design
    (5.25 um) with 36x36 controls, one input stub and two output stubs
    1.5 um apart.  The controls start grey (C = 1/2, the uniform average
    material)."""
    wl = [1.30 * UM, 1.55 * UM]
    steps = steps_rule(430, 450, 25e-9, max(wl)) if n_steps is None else n_steps
    dev = soi_device("demux", 430, 450, 64, 25e-9, 8, md=210, nd=210, slab_layers=9, mc=36, nc=36,
                     filter_r=2.0, beta=10.0, wavelengths=wl, n_steps=steps, seed=seed,
                     out_offsets=(-0.75 * UM, 0.75 * UM))
    dev.C = np.full_like(dev.C, 0.5)
    return dev


def micro_demux(n_steps: int = 700):
    """A few-thousand-cell two-port, two-wavelength device for tests of the
    optimizer loop."""
    dev = micro(seed=9, n_steps=n_steps, nx=32, ny=28, nz=18, md=10, nd=10, mc=5, nc=5,
                wavelengths=[0.78 * UM, 0.86 * UM], out_offsets=(-0.16 * UM, 0.16 * UM))
    dev.C = np.full_like(dev.C, 0.5)
    return dev
