"""Pins of the FP64 oracle's time stepping against facts that do not come
from the oracle itself: exact eigenmodes of the closed Yee cavity (the Yee
dispersion relation), exact discrete energy conservation, exact recovery of
a pure sinusoid by the amplitude/phase fit, Lorentz reciprocity, and the
smallness of the CPML reflection."""
import numpy as np
import pytest

from oracle import fdtd
from workloads import cavity

pytestmark = pytest.mark.usefixtures("oracle_built")

S = 0.5


def yee_phase(eps, nx, ny, nz, m, n, p, s=S):
    """Yee dispersion: sin^2(w dt/2) = (s^2/eps) sum_a sin^2(k_a/2)."""
    r = (s * s / eps) * (np.sin(0.5 * m * np.pi / nx) ** 2 + np.sin(0.5 * n * np.pi / ny) ** 2
                         + np.sin(0.5 * p * np.pi / nz) ** 2)
    return 2.0 * np.arcsin(np.sqrt(r))


@pytest.mark.parametrize("eps", [1.0, 2.085, 12.11])
@pytest.mark.parametrize("mnp", [(2, 3, 0), (0, 2, 1), (1, 0, 2), (1, 2, 1), (2, 1, 3)])
def test_pec_cavity_eigenmode(eps, mnp):
    nx, ny, nz = 14, 12, 10
    m, n, p = mnp
    amps = cavity.divergence_free_amplitudes(nx, ny, nz, m, n, p)
    E0, H0 = cavity.pec_standing_wave(nx, ny, nz, m, n, p, amps, S)
    kap = np.full((3, nz, ny, nx), 1.0 / eps)
    steps = 3000
    r = fdtd.run(fdtd.SimParams(nx, ny, nz, S, S, S, n_steps=steps), kap, E0, H0)
    phi = yee_phase(eps, nx, ny, nz, m, n, p)
    ref = E0 * np.cos(steps * phi)
    assert np.max(np.abs(r.E - ref)) < 1e-10


def test_dispersion_phase_slope():
    """Frequency read off the phase of a probe, compared with the closed form."""
    nx, ny, nz = 16, 12, 10
    m, n, p = 3, 2, 1
    eps = 2.085
    amps = cavity.divergence_free_amplitudes(nx, ny, nz, m, n, p)
    E0, H0 = cavity.pec_standing_wave(nx, ny, nz, m, n, p, amps, S)
    kap = np.full((3, nz, ny, nx), 1.0 / eps)
    probe = (2, 3, 4, 5)   # component, k, j, i
    vals = []
    E, H = E0, H0
    for _ in range(400):
        r = fdtd.run(fdtd.SimParams(nx, ny, nz, S, S, S, n_steps=1), kap, E, H)
        E, H = r.E, r.H
        vals.append(E[probe] / E0[probe])
    vals = np.array(vals)
    # least-squares frequency from cos(n phi): use arccos on the first samples
    n_idx = np.arange(1, 401)
    phi_ref = yee_phase(eps, nx, ny, nz, m, n, p)
    assert np.max(np.abs(vals - np.cos(n_idx * phi_ref))) < 1e-11
    # a 1e-5 relative frequency error would be visible
    assert np.max(np.abs(vals - np.cos(n_idx * phi_ref * (1 + 1e-5)))) > 1e-4


def test_energy_conserved_random_anisotropic():
    rng = np.random.default_rng(3)
    nx, ny, nz = 13, 11, 9
    kap = 1.0 / rng.uniform(1.0, 12.0, size=(3, nz, ny, nx))
    E0 = rng.standard_normal((3, nz, ny, nx))
    H0 = rng.standard_normal((3, nz, ny, nx))
    # the PEC walls hold tangential E at zero: start from an admissible state
    E0[0, :, 0, :] = 0; E0[0, 0] = 0
    E0[1, :, :, 0] = 0; E0[1, 0] = 0
    E0[2, :, :, 0] = 0; E0[2, :, 0, :] = 0
    r = fdtd.run(fdtd.SimParams(nx, ny, nz, 0.5, 0.45, 0.4, n_steps=4000), kap, E0, H0,
                 energy=True)
    w = r.energy
    assert np.max(np.abs(w - w[0])) / abs(w[0]) < 1e-12
    assert np.max(np.abs(r.E)) > 1e-3          # the fields did evolve


def test_energy_detects_wrong_kappa_weight():
    """Planted mistake: weighting |E|^2 by kappa instead of eps breaks the
    invariant, so the energy test can fail."""
    rng = np.random.default_rng(4)
    nx, ny, nz = 9, 8, 7
    kap = 1.0 / rng.uniform(1.0, 12.0, size=(3, nz, ny, nx))
    E0 = rng.standard_normal((3, nz, ny, nx))
    E0[0, :, 0, :] = 0; E0[0, 0] = 0
    E0[1, :, :, 0] = 0; E0[1, 0] = 0
    E0[2, :, :, 0] = 0; E0[2, :, 0, :] = 0
    H0 = np.zeros_like(E0)
    E, H = E0, H0
    bad = []
    for _ in range(50):
        bad.append(np.sum(kap * E ** 2))
        r = fdtd.run(fdtd.SimParams(nx, ny, nz, n_steps=1), kap, E, H)
        E, H = r.E, r.H
    assert np.ptp(bad) / bad[0] > 1e-3


@pytest.mark.parametrize("wl", [37, 64, 155, 311])
def test_amplitude_phase_fit_exact(wl):
    w_dt = 2 * np.pi / 77.5
    n0 = 1000
    ehat = 0.7 - 1.3j
    n = np.arange(n0, n0 + wl)
    e_n = np.real(ehat * np.exp(-1j * w_dt * n))
    sums = np.sum(e_n * np.exp(1j * w_dt * n))
    got = fdtd.extract(np.array(sums), fdtd.gram(w_dt, n0, n0 + wl))
    assert abs(got - ehat) < 1e-12


def _point_source(axis_c, pos):
    """A single-component current at cell pos=(i,j,k) on a plane normal to an
    axis other than the component, so the component is tangential."""
    normal = (axis_c + 2) % 3          # then t1 = (normal+1)%3 = axis_c
    i, j, k = pos
    c = [i, j, k]
    others = [a for a in range(3) if a != normal]
    plane = fdtd_plane(normal, c[normal], c[others[0]], c[others[1]], 1, 1)
    jv = np.zeros((2, 1, 1), np.complex128)
    t1 = (normal + 1) % 3
    jv[0 if t1 == axis_c else 1, 0, 0] = 1.0
    return plane, jv


def fdtd_plane(axis, index, lo0, lo1, n0, n1):
    from workloads import Plane
    return Plane(axis, index, lo0, lo1, n0, n1)


def test_reciprocity_random_medium():
    rng = np.random.default_rng(11)
    nx, ny, nz, npml = 26, 24, 22, 6
    kap = np.full((3, nz, ny, nx), 1.0 / 2.085)
    kap[:, 8:14, 8:16, 8:18] = 1.0 / rng.uniform(2.085, 12.11, size=(3, 6, 8, 10))
    w_dt = 2 * np.pi / 20.0
    steps, wl = 2400, 200
    p = fdtd.SimParams(nx, ny, nz, npml=(npml,) * 6, n_steps=steps, omega_dt=w_dt,
                       ramp_steps=60.0, win_start=steps - wl, win_len=wl)
    a_pos, a_c = (8, 9, 10), 1      # E_y near one corner of the inhomogeneity
    b_pos, b_c = (17, 15, 12), 2    # E_z near the other
    pa, ja = _point_source(a_c, a_pos)
    pb, jb = _point_source(b_c, b_pos)

    def probe(plane, jv, pos, c):
        box = (pos[0], pos[1], pos[2], 1, 1, 1)
        r = fdtd.run(p, kap, src_plane=plane, src_j=jv, box=box)
        e, res = fdtd.extract_halves(r.box_sums, w_dt, p.win_start, p.win_len)
        return e[c, 0, 0, 0], res

    e_ab, r1 = probe(pa, ja, b_pos, b_c)     # source at a, field at b
    e_ba, r2 = probe(pb, jb, a_pos, a_c)     # source at b, field at a
    assert abs(e_ab) > 1e-4
    assert abs(e_ab - e_ba) / abs(e_ab) < 1e-5


def test_cpml_reflection_small():
    """A point source near a CPML face; the steady field at a probe between
    source and face, compared with the same geometry whose boundary is moved
    far away.  The difference is the reflection from the absorbing layer."""
    w_dt = 2 * np.pi / 20.0
    steps, wl = 1600, 200
    eps = 2.085
    npml = 8

    def run(nx, ny, nz, src, probe, layers=npml):
        kap = np.full((3, nz, ny, nx), 1.0 / eps)
        p = fdtd.SimParams(nx, ny, nz, npml=(layers,) * 6, n_steps=steps, omega_dt=w_dt,
                           ramp_steps=60.0, win_start=steps - wl, win_len=wl)
        pl, jv = _point_source(1, src)
        r = fdtd.run(p, kap, src_plane=pl, src_j=jv, box=probe + (1, 1, 1))
        e, _ = fdtd.extract_halves(r.box_sums, w_dt, p.win_start, p.win_len)
        return e[1, 0, 0, 0]

    def run_pec(n, src, probe):
        return run(n, n, n, src, probe, layers=0)

    small = run(30, 30, 30, (15, 15, 15), (10, 15, 15))
    big = run(70, 70, 70, (35, 35, 35), (30, 35, 35))
    assert abs(small - big) / abs(big) < 1e-3
    # the same probe in a box with bare PEC walls differs by far more
    pec = run_pec(30, (15, 15, 15), (10, 15, 15))
    assert abs(pec - big) / abs(big) > 1e-1
