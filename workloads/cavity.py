"""Closed-form initial states for the PEC-cavity tests.

A standing wave in the closed box [0,nx]x[0,ny]x[0,nz] (cell units) with
wavenumbers k_a = m_a pi / n_a:
    E_x(i+1/2, j, k)   = A cos(k_x (i+1/2)) sin(k_y j) sin(k_z k)
    E_y(i, j+1/2, k)   = B sin(k_x i) cos(k_y (j+1/2)) sin(k_z k)
    E_z(i, j, k+1/2)   = C sin(k_x i) sin(k_y j) cos(k_z (k+1/2))
The magnetic state one half step earlier is the standing wave's partner,
written in closed form with the lattice wavenumbers q_a = 2 sin(k_a/2):
    Ht_x(i, j+1/2, k+1/2) = 1/2 (s q_y C - s q_z B) sin(k_x i) cos(k_y (j+1/2)) cos(k_z (k+1/2))
    Ht_y(i+1/2, j, k+1/2) = 1/2 (s q_z A - s q_x C) cos(k_x (i+1/2)) sin(k_y j) cos(k_z (k+1/2))
    Ht_z(i+1/2, j+1/2, k) = 1/2 (s q_x B - s q_y A) cos(k_x (i+1/2)) cos(k_y (j+1/2)) sin(k_z k)
with s the Courant number.  When (A, B, C) . (q_x, q_y, q_z) = 0 the wave
is an exact eigenmode of the leapfrog scheme.
"""
import numpy as np


def lattice_q(m, n):
    return 2.0 * np.sin(0.5 * m * np.pi / n)


def divergence_free_amplitudes(nx, ny, nz, m, n, p, rng=None):
    """A unit (A, B, C) orthogonal to (q_x, q_y, q_z).  If one index is zero
    the wave is uniform along that axis and only that axis' component
    survives; it is set to one."""
    idx = (m, n, p)
    if 0 in idx:
        v = np.zeros(3)
        v[idx.index(0)] = 1.0
        return v
    q = np.array([lattice_q(m, nx), lattice_q(n, ny), lattice_q(p, nz)])
    rng = np.random.default_rng(0) if rng is None else rng
    v = rng.standard_normal(3)
    v = v - q * (v @ q) / (q @ q)
    return v / np.linalg.norm(v)


def pec_standing_wave(nx, ny, nz, m, n, p, amps, s=0.5):
    A, B, C = amps
    kx, ky, kz = m * np.pi / nx, n * np.pi / ny, p * np.pi / nz
    qx, qy, qz = lattice_q(m, nx), lattice_q(n, ny), lattice_q(p, nz)
    i = np.arange(nx, dtype=np.float64)[None, None, :]
    j = np.arange(ny, dtype=np.float64)[None, :, None]
    k = np.arange(nz, dtype=np.float64)[:, None, None]
    E = np.zeros((3, nz, ny, nx))
    H = np.zeros((3, nz, ny, nx))
    E[0] = A * np.cos(kx * (i + 0.5)) * np.sin(ky * j) * np.sin(kz * k)
    E[1] = B * np.sin(kx * i) * np.cos(ky * (j + 0.5)) * np.sin(kz * k)
    E[2] = C * np.sin(kx * i) * np.sin(ky * j) * np.cos(kz * (k + 0.5))
    H[0] = 0.5 * (s * qy * C - s * qz * B) * np.sin(kx * i) * np.cos(ky * (j + 0.5)) * np.cos(kz * (k + 0.5))
    H[1] = 0.5 * (s * qz * A - s * qx * C) * np.cos(kx * (i + 0.5)) * np.sin(ky * j) * np.cos(kz * (k + 0.5))
    H[2] = 0.5 * (s * qx * B - s * qy * A) * np.cos(kx * (i + 0.5)) * np.cos(ky * (j + 0.5)) * np.sin(kz * k)
    return E, H
