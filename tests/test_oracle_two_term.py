"""Pins of the oracle's two-term modal coefficient (paper Appendix A): the H
term read from H phasors equals its rewrite on E sites through the discrete
Faraday law, on planes of every orientation; the two-term coefficient of a
field that is the port's own mode profile; and the adjoint gradient (electric
plus magnetic adjoint currents) against finite differences."""
import numpy as np
import pytest

from oracle import adjoint, chain, fdtd, ports
from workloads import configs
from workloads.devices import Plane

pytestmark = pytest.mark.usefixtures("oracle_built")


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_h_term_equals_its_rewrite_on_e_sites(axis):
    dev = configs.micro(n_steps=2400)
    kap, _ = chain.kappa(dev)
    lam = dev.wavelengths[0]
    # a plane of H sites inside the domain, clear of the CPML and the source
    idx = {0: 20, 1: 14, 2: 10}[axis]
    lo = {0: (8, 6), 1: (8, 6), 2: (8, 8)}[axis]
    n = (9, 6)
    pl = Plane(axis, idx, lo[0], lo[1], n[0], n[1])
    rng = np.random.default_rng(50 + axis)
    u = rng.standard_normal((2, n[1], n[0])) + 1j * rng.standard_normal((2, n[1], n[0]))
    t1 = (axis + 1) % 3
    if t1 == min(t1, (axis + 2) % 3):
        u[0][-1, :] = 0.0
        u[1][:, -1] = 0.0
    else:
        u[0][:, -1] = 0.0
        u[1][-1, :] = 0.0
    # E phasors of every component on the plane and the next one
    c0, c1 = [a for a in range(3) if a != axis]
    start = [0, 0, 0]
    size = [0, 0, 0]
    start[axis], size[axis] = idx, 2
    start[c0], size[c0] = lo[0], n[0]
    start[c1], size[c1] = lo[1], n[1]
    box = (start[0], start[1], start[2], size[0], size[1], size[2])
    p = adjoint.sim_params(dev, lam)
    r = fdtd.run(p, kap, src_plane=dev.sources[0].plane,
                 src_j=ports.source_current(dev.sources[0].h), box=box, hmon_planes=[pl])
    E, _ = fdtd.extract_halves(r.box_sums, p.omega_dt, p.win_start, p.win_len)   # [3][z][y][x]
    G = fdtd.gram_half(p.omega_dt, p.win_start, p.win_start + p.win_len)
    H = fdtd.extract(r.hmon_sums[0][0] + r.hmon_sums[0][1], G)                  # [2][n1][n0]

    def plane_of(comp, k):
        # [n1][n0] slice of component comp at offset k along the normal: the
        # box is [z][y][x], so dropping the normal axis leaves (c1, c0)
        sl = [slice(None)] * 3
        sl[2 - axis] = k
        return E[comp][tuple(sl)]

    t2 = (axis + 2) % 3
    Et_i = np.stack([plane_of(t1, 0), plane_of(t2, 0)])
    Et_i1 = np.stack([plane_of(t1, 1), plane_of(t2, 1)])
    En = plane_of(axis, 0)
    S = dev.courant
    q_i, q_n, q_i1 = ports.h_term_on_e_sites(u, axis, S, S, S, 0.5 * p.omega_dt)
    via_h = np.sum(u * H)
    via_e = np.sum(q_i * Et_i) + np.sum(q_n * En) + np.sum(q_i1 * Et_i1)
    assert abs(via_h) > 1e-8
    # equal for pure sinusoids; what the two fits leave of the start-up
    # transient is the difference (its size is the run's steady-state residual)
    _, resid = fdtd.extract_halves(r.box_sums, p.omega_dt, p.win_start, p.win_len)
    assert abs(via_e - via_h) <= max(1e-6, 10 * resid) * abs(via_h)


def test_two_term_coefficient_of_the_mode_itself():
    # a field equal to the mode on the plane (E = e, H = h) gives alpha = 1,
    # the same as the E-only coefficient
    dev = configs.micro()
    m = dev.ports[0]
    wE, u = ports.two_term_weights(m.e, m.h, m.plane.axis)
    # h at the H sites: the mode's h stored at the E sites it shares (h_t1 at
    # the E_t2 sites, h_t2 at the E_t1 sites)
    H = np.stack([m.h[0], m.h[1]])
    a = ports.alpha_two_term(wE, u, m.e, H)
    # the edge trim of u takes away a negligible part of the profile
    assert abs(a - 1.0) < 1e-3
    assert abs(ports.alpha(ports.monitor_weights(m.e, m.h), m.e) - 1.0) < 1e-12


def test_two_term_gradient_matches_finite_differences():
    # (the steady-state fit of a finite run limits the finite differences to
    # a few parts in 1e3, the same as for the E-only coefficient)
    dev = configs.micro(n_steps=2400)
    dev.C = np.random.default_rng(51).uniform(0.3, 0.7, dev.C.shape)

    def F(C):
        a = adjoint.forward_adjoint(dev, C=C, two_term=True).alpha
        return float(np.sum(np.abs(a) ** 2))

    res = adjoint.forward_adjoint(dev, two_term=True)
    g = adjoint.grad_C(dev, res, np.conj(res.alpha))
    h = 1e-4
    for (b, a) in [(0, 0), (2, 3), (4, 1)]:
        Cp, Cm = dev.C.copy(), dev.C.copy()
        Cp[b, a] += h
        Cm[b, a] -= h
        fd = (F(Cp) - F(Cm)) / (2 * h)
        assert g[b, a] == pytest.approx(fd, rel=5e-3, abs=2e-4 * np.abs(g).max())
