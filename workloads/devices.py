"""Synthetic SOI-like devices: geometry, mode profiles, controls and time lengths.

Conventions shared by every consumer (they are descriptions, not arithmetic):

* Grid: ``nx x ny x nz`` cells (CPML included), cubic spacing ``dx`` metres,
  Courant number ``courant = c*dt/dx``.  Yee positions in cell units:
  E_x(i+1/2, j, k), E_y(i, j+1/2, k), E_z(i, j, k+1/2).  Arrays are
  ``[3][nz][ny][nx]`` (x fastest).
* Design: in-plane design area of ``md x nd`` FDTD pixels whose lower corner
  pixel is ``(i0, j0)``; the slab holds E_x/E_y planes ``k_lo..k_hi``.  The
  high-resolution canvas is the design plus a 2-pixel margin on every side,
  ``S`` sub-pixels per FDTD pixel, stored ``[S*(nd+4)][S*(md+4)]``; canvas
  sub-pixel ``(v, u)`` covers x in ``[i0-2.5+u/S, i0-2.5+(u+1)/S)`` (and the
  same in y), so the design area itself is ``x in [i0-1/2, i0+md-1/2)``.
* Controls ``C``: ``[nc][mc]`` (y rows, x fastest), uniform on [0, 1].
* Planes: normal ``axis`` at cell ``index``; ``(c0, c1)`` are the two other
  axes in increasing order, extents ``[lo0, lo0+n0) x [lo1, lo1+n1)``; plane
  arrays are ``[2][n1][n0]`` with the two tangential components ordered
  cyclically (axis x -> (y, z), axis y -> (z, x), axis z -> (x, y)).
* Mode profiles: ``e[t]`` is sampled at the E_{t} sites of the plane;
  ``h[0]`` (= h_t1) is sampled at the E_t2 sites and ``h[1]`` (= h_t2) at the
  E_t1 sites, i.e. each h sample sits where it pairs with E in E x h*.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

C0 = 299792458.0


@dataclass
class Plane:
    axis: int
    index: int
    lo0: int
    lo1: int
    n0: int
    n1: int


@dataclass
class Mode:
    plane: Plane
    e: np.ndarray  # complex128 [2][n1][n0]
    h: np.ndarray  # complex128 [2][n1][n0]


@dataclass
class Device:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    courant: float
    npml: tuple
    i0: int
    j0: int
    md: int
    nd: int
    k_lo: int
    k_hi: int
    mc: int
    nc: int
    filter_r: float
    supersample: int
    beta: float
    eps_core: float
    eps_clad: float
    sobel_delta: float
    wavelengths: List[float]
    n_steps: int
    ramp_periods: float
    window_periods: float
    kappa_bg: np.ndarray          # float64 [3][nz][ny][nx]
    mask_hr: np.ndarray           # float64 [S(nd+4)][S(md+4)] background fill of the canvas
    sources: List[Mode]
    ports: List[Mode]
    C: np.ndarray                 # float64 [nc][mc]
    seed: int = 0
    pml_m: float = 3.0
    pml_sigma_scale: float = 1.0
    pml_kappa_max: float = 1.0
    pml_a_max: float = 0.0
    morph_ops: str = ""           # morphological operations, 'd'/'e' left to right ('' = none)
    morph_d: float = 0.0          # disc diameter, design pixels
    morph_alpha: float = 20.0     # sharpness of the soft dilation/erosion
    extra: dict = field(default_factory=dict)

    # ---- time lengths (descriptions of the run, per wavelength) ----
    def period_steps(self, lam: float) -> float:
        """Optical period in time steps: lambda / (c dt)."""
        return lam / (self.courant * self.dx)

    def omega_dt(self, lam: float) -> float:
        return 2.0 * np.pi / self.period_steps(lam)

    def ramp_steps(self, lam: float) -> float:
        return self.ramp_periods * self.period_steps(lam)

    def pulse(self, k: float = 1.5, m: float = 4.5, single_periods: float = 3.0):
        """Pulse excitation covering the device's wavelengths, in steps:
        (carrier omega dt, sigma, t0).  The carrier sits mid-band; the
        Gaussian's spectral width 1/sigma puts the band edges k widths away
        (one wavelength: sigma = `single_periods` periods); the centre is m
        sigma after the start."""
        w = [self.omega_dt(lam) for lam in self.wavelengths]
        w0 = 0.5 * (min(w) + max(w))
        half = 0.5 * (max(w) - min(w))
        sigma = k / half if half > 0 else single_periods * 2.0 * np.pi / w0
        return w0, sigma, m * sigma

    def dt(self) -> float:
        return self.courant * self.dx / 299792458.0

    def window(self, lam: float):
        wl = int(round(self.window_periods * self.period_steps(lam)))
        wl = max(2, min(wl, self.n_steps))
        return self.n_steps - wl, wl

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_freq(self) -> int:
        return len(self.wavelengths)

    def dft_box(self):
        """Region whose E is kept in the frequency domain: the 1-pixel ring
        around the design area (its averaging windows see the design) times
        the slab plus its two E_z interface planes.  (x0, y0, z0, bx, by, bz)."""
        return (self.i0 - 1, self.j0 - 1, self.k_lo - 1,
                self.md + 2, self.nd + 2, self.k_hi - self.k_lo + 3)


def _quasi_te_mode(plane: Plane, yc: float, zc: float, wy: float, wz: float,
                   neff: float) -> Mode:
    """Separable Gaussian quasi-TE profile (E along y) on an x-normal plane.

    t1 = y, t2 = z.  E_y sites are at (j+1/2, k); h_z pairs with E_y there.
    """
    assert plane.axis == 0
    j = plane.lo0 + np.arange(plane.n0)
    k = plane.lo1 + np.arange(plane.n1)
    yy = (j + 0.5)[None, :]
    zz = k.astype(np.float64)[:, None]
    g = np.exp(-((yy - yc) / wy) ** 2 - ((zz - zc) / wz) ** 2)
    e = np.zeros((2, plane.n1, plane.n0), np.complex128)
    h = np.zeros((2, plane.n1, plane.n0), np.complex128)
    e[0] = g
    h[1] = neff * g
    return Mode(plane, e, h)


def soi_device(name: str, nx: int, ny: int, nz: int, dx: float, npml: int,
               md: int, nd: int, slab_layers: int, mc: int, nc: int,
               filter_r: float, beta: float, wavelengths: Sequence[float],
               n_steps: int, seed: int, *, supersample: int = 4,
               out_offsets: Sequence[float] = (0.0,), strip_width: float = 500e-9,
               mode_w: Optional[tuple] = None, ramp_periods: float = 10.0,
               window_periods: float = 4.0, courant: float = 0.5,
               eps_core: float = 12.11, eps_clad: float = 2.085,
               sobel_delta: float = 1e-6, neff: float = 2.4,
               src_inset: int = 10) -> Device:
    """A design box in an SiO2 cladding joined by Si strip stubs.

    One input stub on -x at the centre in y; one output stub per entry of
    ``out_offsets`` (metres from the centre in y) on +x.  Stubs are
    ``strip_width`` wide and ``slab_layers`` cells thick.  The design box is
    centred.  Source and monitor planes sit ``src_inset`` cells (at most half
    the gap) inside the CPML's inner edge.
    """
    rng = np.random.default_rng(seed)
    S = supersample
    i0 = (nx - md) // 2
    j0 = (ny - nd) // 2
    k_lo = (nz - slab_layers) // 2
    k_hi = k_lo + slab_layers - 1
    yc = ny / 2.0 + 0.25           # keeps stub edges off every Yee site
    half_w = 0.5 * strip_width / dx
    zc = 0.5 * (k_lo + k_hi)
    z_bot, z_top = k_lo - 0.5, k_hi + 0.5
    x_in_end = i0 - 0.5            # design area edges
    x_out_start = i0 + md - 0.5
    out_yc = [yc + o / dx for o in out_offsets]

    def in_strip_xy(x, y):
        inside = (x < x_in_end) & (np.abs(y - yc) < half_w)
        for c in out_yc:
            inside = inside | ((x > x_out_start) & (np.abs(y - c) < half_w))
        return inside

    k_core, k_clad = 1.0 / eps_core, 1.0 / eps_clad
    kappa = np.full((3, nz, ny, nx), k_clad)
    ii = np.arange(nx, dtype=np.float64)
    jj = np.arange(ny, dtype=np.float64)
    kk = np.arange(nz, dtype=np.float64)
    # E_x at (i+1/2, j, k), E_y at (i, j+1/2, k): point-sampled in-plane
    sx_ = in_strip_xy((ii + 0.5)[None, :], jj[:, None])
    sy_ = in_strip_xy(ii[None, :], (jj + 0.5)[:, None])
    sz_ = in_strip_xy(ii[None, :], jj[:, None])
    slab_xy = (kk >= z_bot) & (kk <= z_top)
    for k in range(nz):
        if slab_xy[k]:
            kappa[0, k][sx_] = k_core
            kappa[1, k][sy_] = k_core
    # E_z at k+1/2: inside planes fully filled, the two face planes half filled
    for k in range(nz):
        z = k + 0.5
        if z_bot < z < z_top:
            kappa[2, k][sz_] = k_core
        elif z == z_bot or z == z_top:
            kappa[2, k][sz_] = 0.5 * (k_core + k_clad)

    # canvas background fill (sub-pixel centres)
    U, V = S * (md + 4), S * (nd + 4)
    xu = (i0 - 2.5) + (np.arange(U) + 0.5) / S
    yv = (j0 - 2.5) + (np.arange(V) + 0.5) / S
    mask_hr = in_strip_xy(xu[None, :], yv[:, None]).astype(np.float64)

    gap = i0 - npml
    inset = max(1, min(src_inset, gap // 2))
    if mode_w is None:
        mode_w = (0.24e-6 / dx, 0.1e-6 / dx)
    wy, wz = mode_w
    py = int(np.ceil(3 * wy)) + 1
    pz = int(np.ceil(3 * wz)) + 1

    def port_plane(x, ycen):
        lo0 = max(npml + 1, int(np.floor(ycen - py)))
        hi0 = min(ny - npml - 1, int(np.ceil(ycen + py)))
        lo1 = max(npml + 1, int(np.floor(zc - pz)))
        hi1 = min(nz - npml - 1, int(np.ceil(zc + pz)))
        return Plane(0, x, lo0, lo1, hi0 - lo0, hi1 - lo1)

    src_x = npml + inset
    mon_x = nx - npml - 1 - inset
    sources = [_quasi_te_mode(port_plane(src_x, yc), yc, zc, wy, wz, neff)]
    ports = [_quasi_te_mode(port_plane(mon_x, c), c, zc, wy, wz, neff) for c in out_yc]

    C = rng.uniform(0.0, 1.0, size=(nc, mc))
    npml6 = (npml,) * 6
    return Device(name=name, nx=nx, ny=ny, nz=nz, dx=dx, courant=courant, npml=npml6,
                  i0=i0, j0=j0, md=md, nd=nd, k_lo=k_lo, k_hi=k_hi, mc=mc, nc=nc,
                  filter_r=filter_r, supersample=S, beta=beta, eps_core=eps_core,
                  eps_clad=eps_clad, sobel_delta=sobel_delta,
                  wavelengths=list(wavelengths), n_steps=n_steps,
                  ramp_periods=ramp_periods, window_periods=window_periods,
                  kappa_bg=kappa, mask_hr=mask_hr, sources=sources, ports=ports,
                  C=C, seed=seed)


def vacuum_box(nx: int, ny: int, nz: int, eps=1.0):
    """Homogeneous closed box (no design, no PML) used by the cavity tests."""
    return np.full((3, nz, ny, nx), 1.0 / eps)
