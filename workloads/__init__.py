"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the oracle.

This package only *describes* problems: grid sizes, material layouts (which
cells are silicon), synthetic waveguide mode profiles, control variables and
time-stepping lengths.  It performs none of the method's arithmetic (no
filtering, projection, averaging, FDTD, modal overlaps or gradients), so both
implementations can consume the same inputs without sharing any computation.
"""
from .devices import Plane, Mode, Device, soi_device, vacuum_box  # noqa: F401
from . import configs  # noqa: F401
