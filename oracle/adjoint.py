"""Forward run, adjoint run and the Eq. (1) gradient.  TEST INFRASTRUCTURE ONLY.

With E^n = Re(Ehat e^{-i w n dt}), Ht^{n+1/2} = Re(Hhat e^{-i w (n+1/2) dt}) and
the same for the source current, the Yee updates become A Ehat = b with
    A = S^2 curl_h curl_e - 4 sin^2(theta) diag(eps),   b = 2 i sin(theta) jhat,
theta = w dt / 2 (the CPML only stretches the differences and keeps A
symmetric outside the absorbing layers).  For alpha = w^T Ehat:
    d alpha / d eps_j = 4 sin^2(theta) (A^{-1} w)_j Ehat_j .
The adjoint run uses the source jhat_A = w, whose phasor is
Ehat_A = A^{-1} (2 i sin(theta) w), so
    d alpha / d eps_j = -2 i sin(theta) Ehat_A,j Ehat_F,j ,
an unconjugated element-wise product of the two fields on the design region,
which is the form of the paper's Eq. (1).  For a real objective F(alpha) with
coef = dF/dalpha (holomorphic Wirtinger derivative, e.g. conj(alpha) for
F = |alpha|^2),
    dF/d eps_j = sum 2 Re( coef * d alpha / d eps_j ),
    dF/d kappa_j = -eps_j^2 dF/d eps_j .
The adjoint sources are unit-amplitude; the coefficient enters afterwards,
which is the same as scaling the adjoint source by dF/dalpha (Appendix A).

Pulse excitation (the other route of Sec. 2: Fourier transforms of field
transients): each source and each port is excited once with a Gaussian pulse
on a carrier, and the phasors of every wavelength come from the DFT of the
whole run divided by the pulse's own spectrum (``fdtd.extract_pulse``).  Once
the field has died away the DFT obeys the same frequency-domain equations,
so alpha, the adjoint fields and Eq. (1) are used exactly as above.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from . import chain, fdtd, ports


def sim_params(dev, lam: float, n_steps: int = None) -> fdtd.SimParams:
    n = dev.n_steps if n_steps is None else n_steps
    ws, wl = dev.window(lam)
    if n_steps is not None:
        wl = min(wl, n)
        ws = n - wl
    return fdtd.SimParams(dev.nx, dev.ny, dev.nz, dev.courant, dev.courant, dev.courant,
                          tuple(dev.npml), dev.pml_m, dev.pml_sigma_scale, dev.pml_kappa_max,
                          dev.pml_a_max, n, dev.omega_dt(lam), dev.ramp_steps(lam), ws, wl)


@dataclass
class Solve:
    box: np.ndarray          # complex [3][bz][by][bx]
    mon: List[np.ndarray]    # per port plane complex [2][n1][n0]
    resid: float
    hmon: List[np.ndarray] = None   # per port plane, tangential Hhat [2][n1][n0] (two-term)


def solve(dev, kap, src_plane, src_j, lam, n_steps=None, hmon=False, m_plane=None,
          m_src=None) -> Solve:
    """One time-harmonic run: an electric current on src_plane, optionally a
    magnetic current m_src on the H sites of m_plane, optionally recording
    the tangential H of the port planes."""
    p = sim_params(dev, lam, n_steps)
    planes = [m.plane for m in dev.ports]
    r = fdtd.run(p, kap, src_plane=src_plane, src_j=src_j, box=dev.dft_box(), mon_planes=planes,
                 hmon_planes=planes if hmon else (), msrc_plane=m_plane, msrc_m=m_src)
    box, res = fdtd.extract_halves(r.box_sums, p.omega_dt, p.win_start, p.win_len)
    mons = [fdtd.extract_halves(s, p.omega_dt, p.win_start, p.win_len)[0] for s in r.mon_sums]
    hm = None
    if hmon:
        G = fdtd.gram_half(p.omega_dt, p.win_start, p.win_start + p.win_len)
        hm = [fdtd.extract(s[0] + s[1], G) for s in r.hmon_sums]
    return Solve(box, mons, res, hm)


@dataclass
class Result:
    alpha: np.ndarray        # complex [n_src][n_ports][n_freq]
    fwd: list                # [s][f] Solve
    adj: list                # [p][f] Solve
    kappa: np.ndarray
    state: chain.ChainState
    weights: list            # per port w
    beta: float


def forward_adjoint(dev, C=None, beta=None, n_steps=None, ops=None, kap=None,
                    two_term: bool = False) -> Result:
    """Forward and unit adjoint runs.  two_term: the Appendix A coefficient
    with both terms, alpha = wE . Ehat + u . Hhat, read from the E and H
    phasors of the port planes; the adjoint of port p then carries the
    electric current wE on the plane's E sites and the magnetic current -u
    on its H sites (a magnetic current m enters the E equation as the
    electric current -curl_h m / (2 i sin theta) and curl_h is the transpose
    of curl_e, so -u reproduces the H term's weights on E sites)."""
    if two_term:
        return _forward_adjoint_two_term(dev, C, beta, n_steps, ops, kap)
    C = dev.C if C is None else C
    beta = dev.beta if beta is None else beta
    st = None
    if kap is None:
        kap, st = chain.kappa(dev, C, beta, ops)
    W = [ports.monitor_weights(m.e, m.h) for m in dev.ports]
    J = [ports.source_current(s.h) for s in dev.sources]
    ns, npo, nf = len(dev.sources), len(dev.ports), dev.n_freq
    alpha = np.zeros((ns, npo, nf), np.complex128)
    fwd = [[None] * nf for _ in range(ns)]
    adj = [[None] * nf for _ in range(npo)]
    for f, lam in enumerate(dev.wavelengths):
        for s in range(ns):
            r = solve(dev, kap, dev.sources[s].plane, J[s], lam, n_steps)
            fwd[s][f] = r
            for p in range(npo):
                alpha[s, p, f] = ports.alpha(W[p], r.mon[p])
        for p in range(npo):
            adj[p][f] = solve(dev, kap, dev.ports[p].plane, W[p], lam, n_steps)
    return Result(alpha, fwd, adj, kap, st, W, beta)


def _forward_adjoint_two_term(dev, C, beta, n_steps, ops, kap) -> Result:
    C = dev.C if C is None else C
    beta = dev.beta if beta is None else beta
    st = None
    if kap is None:
        kap, st = chain.kappa(dev, C, beta, ops)
    WU = [ports.two_term_weights(m.e, m.h, m.plane.axis) for m in dev.ports]
    J = [ports.source_current(s.h) for s in dev.sources]
    ns, npo, nf = len(dev.sources), len(dev.ports), dev.n_freq
    alpha = np.zeros((ns, npo, nf), np.complex128)
    fwd = [[None] * nf for _ in range(ns)]
    adj = [[None] * nf for _ in range(npo)]
    for f, lam in enumerate(dev.wavelengths):
        for s in range(ns):
            r = solve(dev, kap, dev.sources[s].plane, J[s], lam, n_steps, hmon=True)
            fwd[s][f] = r
            for p in range(npo):
                alpha[s, p, f] = ports.alpha_two_term(WU[p][0], WU[p][1], r.mon[p], r.hmon[p])
        for p in range(npo):
            pl = dev.ports[p].plane
            adj[p][f] = solve(dev, kap, pl, WU[p][0], lam, n_steps, m_plane=pl, m_src=-WU[p][1])
    return Result(alpha, fwd, adj, kap, st, WU, beta)


@dataclass
class Pulse:
    """Gaussian pulse exp(-(t - t0)^2 / (2 sigma^2)) on the carrier omega_dt
    (t in steps), run for n_steps; the last `tail` steps' DFT is also kept
    apart to show how much the late field still contributes."""
    omega_dt: float
    sigma: float
    t0: float
    n_steps: int
    tail: int = 0


def solve_pulse(dev, kap, src_plane, src_j, pulse: Pulse) -> List[Solve]:
    """Phasors at every wavelength of the device from one pulse run; the
    residual of each is |DFT of the tail| / |DFT of the whole run|."""
    wf = [dev.omega_dt(lam) for lam in dev.wavelengths]
    n = pulse.n_steps
    p = fdtd.SimParams(dev.nx, dev.ny, dev.nz, dev.courant, dev.courant, dev.courant,
                       tuple(dev.npml), dev.pml_m, dev.pml_sigma_scale, dev.pml_kappa_max,
                       dev.pml_a_max, n, pulse.omega_dt, 0.0, n - pulse.tail, n,
                       pulse.sigma, pulse.t0, wf)
    r = fdtd.run(p, kap, src_plane=src_plane, src_j=src_j, box=dev.dft_box(),
                 mon_planes=[m.plane for m in dev.ports])
    sig = fdtd.pulse_samples(n, pulse.omega_dt, pulse.sigma, pulse.t0)
    out = []
    for f, w in enumerate(wf):
        S = fdtd.pulse_spectrum(sig, w)
        box = fdtd.extract_pulse(r.box_sums[0, f] + r.box_sums[1, f], S)
        late = fdtd.extract_pulse(r.box_sums[1, f], S)
        mons = [fdtd.extract_pulse(m[0, f] + m[1, f], S) for m in r.mon_sums]
        nrm = np.linalg.norm(box)
        out.append(Solve(box, mons, float(np.linalg.norm(late) / nrm) if nrm > 0 else 0.0))
    return out


def forward_adjoint_pulse(dev, pulse: Pulse, C=None, beta=None, ops=None, kap=None) -> Result:
    """forward_adjoint with one pulse run per source and per port."""
    C = dev.C if C is None else C
    beta = dev.beta if beta is None else beta
    st = None
    if kap is None:
        kap, st = chain.kappa(dev, C, beta, ops)
    W = [ports.monitor_weights(m.e, m.h) for m in dev.ports]
    J = [ports.source_current(s.h) for s in dev.sources]
    ns, npo, nf = len(dev.sources), len(dev.ports), dev.n_freq
    alpha = np.zeros((ns, npo, nf), np.complex128)
    fwd = [solve_pulse(dev, kap, dev.sources[s].plane, J[s], pulse) for s in range(ns)]
    adj = [solve_pulse(dev, kap, dev.ports[p].plane, W[p], pulse) for p in range(npo)]
    for s in range(ns):
        for f in range(nf):
            for p in range(npo):
                alpha[s, p, f] = ports.alpha(W[p], fwd[s][f].mon[p])
    return Result(alpha, fwd, adj, kap, st, W, beta)


def grad_eps(dev, res: Result, coef) -> np.ndarray:
    """dF/d eps on the DFT box, [3][bz][by][bx]."""
    g = np.zeros(res.fwd[0][0].box.shape)
    for f, lam in enumerate(dev.wavelengths):
        theta = 0.5 * dev.omega_dt(lam)
        for s in range(len(dev.sources)):
            for p in range(len(dev.ports)):
                dad = -2j * np.sin(theta) * res.fwd[s][f].box * res.adj[p][f].box
                g += 2.0 * np.real(coef[s, p, f] * dad)
    return g


def box_kappa(dev, kap):
    x0, y0, z0, bx, by, bz = dev.dft_box()
    return kap[:, z0:z0 + bz, y0:y0 + by, x0:x0 + bx]


def grad_kappa(dev, res: Result, coef) -> np.ndarray:
    ge = grad_eps(dev, res, coef)
    kb = box_kappa(dev, res.kappa)
    return -ge / kb ** 2


def grad_C(dev, res: Result, coef, ops=None) -> np.ndarray:
    gk = grad_kappa(dev, res, coef)
    gx, gy, gzi, gzf = chain.zsum(dev, gk)
    return chain.vjp(dev, res.state, res.beta, gx, gy, gzi, gzf, ops)


def objective_abs2(alpha):
    """F = sum |alpha|^2 and coef = dF/dalpha = conj(alpha)."""
    return float(np.sum(np.abs(alpha) ** 2)), np.conj(alpha)
