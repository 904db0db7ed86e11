"""ctypes front end of the FP64 C FDTD (test infrastructure only).

Adds the steady-state amplitude/phase extraction (paper Sec. 2: the
frequency-domain field is read as the amplitude and phase of a time-harmonic
steady state): over the window the field is modelled as
E^n = a cos(w t_n) + b sin(w t_n), t_n = n dt, and (a, b) solve the 2x2 normal
equations of that least-squares fit.  Then Ehat = a + i b, which is the phasor
of E(t) = Re(Ehat exp(-i w t)).  The fit is exact for a pure sinusoid at any
window length.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import build as _build

_LIB = None


class _Sim(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("sx", ct.c_double), ("sy", ct.c_double), ("sz", ct.c_double),
                ("npml", ct.c_int * 6),
                ("pml_m", ct.c_double), ("pml_sigma_scale", ct.c_double),
                ("pml_kappa_max", ct.c_double), ("pml_a_max", ct.c_double),
                ("n_steps", ct.c_int), ("omega_dt", ct.c_double), ("ramp_steps", ct.c_double),
                ("win_start", ct.c_int), ("win_len", ct.c_int),
                ("pulse_sigma", ct.c_double), ("pulse_t0", ct.c_double),
                ("n_dft", ct.c_int), ("dft_omega_dt", ct.POINTER(ct.c_double))]


class _Plane(ct.Structure):
    _fields_ = [("axis", ct.c_int), ("index", ct.c_int), ("lo0", ct.c_int),
                ("lo1", ct.c_int), ("n0", ct.c_int), ("n1", ct.c_int)]


class _Ext(ct.Structure):
    _fields_ = [("n_hmon", ct.c_int), ("hmon", ct.c_void_p), ("hmon_acc", ct.c_void_p),
                ("msrc", ct.c_void_p), ("msrc_m", ct.c_void_p)]


class _Box(ct.Structure):
    _fields_ = [("x0", ct.c_int), ("y0", ct.c_int), ("z0", ct.c_int),
                ("bx", ct.c_int), ("by", ct.c_int), ("bz", ct.c_int)]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _LIB = ct.CDLL(path)
        _LIB.orc_run.restype = ct.c_int
        _LIB.orc_set_threads.argtypes = [ct.c_int]
        _LIB.orc_set_threads.restype = None
        _LIB.orc_max_threads.restype = ct.c_int
    return _LIB


def set_threads(n: int) -> int:
    """Thread count of the oracle's OpenMP loops (for timing it at a chosen
    core count); returns the count now in effect."""
    lib().orc_set_threads(int(n))
    return int(lib().orc_max_threads())


@dataclass
class SimParams:
    nx: int
    ny: int
    nz: int
    sx: float = 0.5
    sy: float = 0.5
    sz: float = 0.5
    npml: Sequence[int] = (0, 0, 0, 0, 0, 0)
    pml_m: float = 3.0
    pml_sigma_scale: float = 1.0
    pml_kappa_max: float = 1.0
    pml_a_max: float = 0.0
    n_steps: int = 0
    omega_dt: float = 0.0
    ramp_steps: float = 0.0
    win_start: int = 0
    win_len: int = 0
    pulse_sigma: float = 0.0          # > 0: Gaussian pulse on the carrier omega_dt
    pulse_t0: float = 0.0
    dft_omega_dt: Sequence[float] = ()   # pulse excitation: DFT frequencies (every step)


@dataclass
class RunResult:
    E: np.ndarray
    H: np.ndarray
    box_sums: Optional[np.ndarray]      # complex [2 halves][3][bz][by][bx]
    mon_sums: List[np.ndarray]          # per plane complex [2 halves][2][n1][n0]
    # (pulse excitation: [2 parts][n_dft][...] with the part split at win_start)
    energy: Optional[np.ndarray]
    hmon_sums: List[np.ndarray] = None  # per H plane complex [2 halves][2][n1][n0] (t = n + 1/2)


def _pd(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def run(p: SimParams, kappa: np.ndarray, E0=None, H0=None, src_plane=None, src_j=None,
        box=None, mon_planes=(), energy=False, hmon_planes=(), msrc_plane=None,
        msrc_m=None) -> RunResult:
    """Advance the Yee scheme ``p.n_steps`` steps from (E0, H0) (zero if None)."""
    nx, ny, nz = p.nx, p.ny, p.nz
    shape = (3, nz, ny, nx)
    kappa = np.ascontiguousarray(kappa, dtype=np.float64).reshape(shape)
    E = np.zeros(shape) if E0 is None else np.array(E0, dtype=np.float64, order="C").reshape(shape)
    H = np.zeros(shape) if H0 is None else np.array(H0, dtype=np.float64, order="C").reshape(shape)
    pulse = p.pulse_sigma > 0
    wdft = np.ascontiguousarray(np.asarray(p.dft_omega_dt if pulse else [0.0], np.float64))
    nd = len(wdft) if pulse else 0
    sim = _Sim(nx, ny, nz, p.sx, p.sy, p.sz, (ct.c_int * 6)(*p.npml), p.pml_m,
               p.pml_sigma_scale, p.pml_kappa_max, p.pml_a_max, p.n_steps, p.omega_dt,
               p.ramp_steps, p.win_start, p.win_len, p.pulse_sigma, p.pulse_t0, nd, _pd(wdft))
    sp = None
    sj = None
    if src_plane is not None:
        sp = _Plane(src_plane.axis, src_plane.index, src_plane.lo0, src_plane.lo1,
                    src_plane.n0, src_plane.n1)
        sj = np.ascontiguousarray(np.asarray(src_j, np.complex128).reshape(
            2, src_plane.n1, src_plane.n0)).view(np.float64)
    bx = None
    box_acc = None
    if box is not None:
        bx = _Box(*box)
        box_acc = np.zeros((2, max(nd, 1), 3, box[5], box[4], box[3]), np.complex128)
    planes = list(mon_planes)
    n_mon = len(planes)
    mons = (_Plane * max(1, n_mon))()
    tot = 0
    for q, pl in enumerate(planes):
        mons[q] = _Plane(pl.axis, pl.index, pl.lo0, pl.lo1, pl.n0, pl.n1)
        tot += 2 * pl.n0 * pl.n1
    mon_acc = np.zeros((2, max(nd, 1), max(tot, 1)), np.complex128)
    en = np.zeros(max(p.n_steps, 1)) if energy else None
    hplanes = list(hmon_planes)
    ext = None
    keep = []
    if hplanes or msrc_plane is not None:
        hp = (_Plane * max(1, len(hplanes)))()
        htot = 0
        for q, pl in enumerate(hplanes):
            hp[q] = _Plane(pl.axis, pl.index, pl.lo0, pl.lo1, pl.n0, pl.n1)
            htot += 2 * pl.n0 * pl.n1
        hacc = np.zeros((2, max(htot, 1)), np.complex128)
        mp = None
        mm = None
        if msrc_plane is not None:
            mp = _Plane(msrc_plane.axis, msrc_plane.index, msrc_plane.lo0, msrc_plane.lo1,
                        msrc_plane.n0, msrc_plane.n1)
            mm = np.ascontiguousarray(np.asarray(msrc_m, np.complex128).reshape(
                2, msrc_plane.n1, msrc_plane.n0)).view(np.float64)
        keep = [hp, hacc, mp, mm]
        ext = _Ext(len(hplanes), ct.addressof(hp), hacc.ctypes.data,
                   ct.addressof(mp) if mp is not None else None,
                   mm.ctypes.data if mm is not None else None)
    rc = lib().orc_run(ct.byref(sim), _pd(kappa), _pd(E), _pd(H),
                       ct.byref(sp) if sp is not None else None,
                       _pd(sj) if sj is not None else None,
                       ct.byref(bx) if bx is not None else None,
                       _pd(box_acc.view(np.float64)) if box_acc is not None else None,
                       n_mon, mons, _pd(mon_acc.view(np.float64)),
                       _pd(en) if en is not None else None,
                       ct.byref(ext) if ext is not None else None)
    if rc != 0:
        raise MemoryError("oracle FDTD failed to allocate")
    mon_sums = []
    off = 0
    for pl in planes:
        n = 2 * pl.n0 * pl.n1
        m = mon_acc[:, :, off:off + n].reshape(2, max(nd, 1), 2, pl.n1, pl.n0)
        mon_sums.append(m if pulse else m[:, 0])
        off += n
    if box_acc is not None and not pulse:
        box_acc = box_acc[:, 0]
    hmon_sums = []
    if ext is not None:
        off = 0
        for pl in hplanes:
            n = 2 * pl.n0 * pl.n1
            hmon_sums.append(keep[1][:, off:off + n].reshape(2, 2, pl.n1, pl.n0).copy())
            off += n
    return RunResult(E, H, box_acc, mon_sums, en[:p.n_steps] if energy else None, hmon_sums)


def gram(omega_dt: float, n0: int, n1: int) -> np.ndarray:
    """Sum over n in [n0, n1) of [[c^2, c s], [c s, s^2]], c=cos(w n dt), s=sin(w n dt)."""
    n = np.arange(n0, n1, dtype=np.float64)
    c, s = np.cos(omega_dt * n), np.sin(omega_dt * n)
    return np.array([[np.sum(c * c), np.sum(c * s)], [np.sum(c * s), np.sum(s * s)]])


def gram_half(omega_dt: float, n0: int, n1: int) -> np.ndarray:
    """gram() at the half-step times t = n + 1/2 of the H samples."""
    t = np.arange(n0, n1, dtype=np.float64) + 0.5
    c, s = np.cos(omega_dt * t), np.sin(omega_dt * t)
    return np.array([[np.sum(c * c), np.sum(c * s)], [np.sum(c * s), np.sum(s * s)]])


def extract(sums: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Least-squares phasor from DFT sums S = sum E^n exp(+i w n dt)."""
    Gi = np.linalg.inv(G)
    a = Gi[0, 0] * sums.real + Gi[0, 1] * sums.imag
    b = Gi[1, 0] * sums.real + Gi[1, 1] * sums.imag
    return a + 1j * b


def extract_halves(sums2: np.ndarray, omega_dt: float, win_start: int, win_len: int):
    """(Ehat over the whole window, steady-state residual) from half-window sums."""
    half = win_len // 2
    G1 = gram(omega_dt, win_start, win_start + half)
    G2 = gram(omega_dt, win_start + half, win_start + win_len)
    full = extract(sums2[0] + sums2[1], G1 + G2)
    e1 = extract(sums2[0], G1)
    e2 = extract(sums2[1], G2)
    nrm = np.linalg.norm(full)
    resid = float(np.linalg.norm(e2 - e1) / nrm) if nrm > 0 else 0.0
    return full, resid


def pulse_samples(n_steps: int, omega_dt: float, sigma: float, t0: float) -> np.ndarray:
    """The complex pulse signal s(t) = g(t) exp(-i w t) at t = n + 1/2 (in
    steps) for n in [0, n_steps): the source current is Re(jhat s(t))."""
    t = np.arange(n_steps, dtype=np.float64) + 0.5
    return np.exp(-0.5 * ((t - t0) / sigma) ** 2) * np.exp(-1j * omega_dt * t)


def pulse_spectrum(s: np.ndarray, omega_dt: float) -> complex:
    """Discrete-time Fourier transform of the source signal at its sample
    times: S(w) = sum_m s_m exp(+i w (m + 1/2))."""
    t = np.arange(len(s), dtype=np.float64) + 0.5
    return complex(np.sum(s * np.exp(1j * omega_dt * t)))


def extract_pulse(sums: np.ndarray, S: complex) -> np.ndarray:
    """Phasor from the DFT of a pulse response.  The response to the real
    source Re(jhat s) is the real part of the response to jhat s, whose DFT
    is S(w) Ehat(w); the conjugate half sits at -w and is negligible for a
    smooth envelope, so Ehat(w) = 2 sum_n E^n exp(+i w n) / S(w)."""
    return 2.0 * sums / S

