"""FP64 parametrization chain C -> rho -> eps -> kappa on the Yee grid, and its
vector-Jacobian product (paper Sec. 3).  TEST INFRASTRUCTURE ONLY.

Every linear stage is an explicit dense operator (a matrix built entry by
entry from its definition) applied with matmuls, and its VJP is the same
matrix transposed.  Pointwise stages use closed-form derivatives.

Stages (in the paper's order):
  * level-set function, Eq. (2): Phi = sum_ij C_ij b(x - x_i, y - y_j) with b a
    truncated Gaussian (support |d| <= r control pixels per axis, sigma = r/2),
    separable, renormalised to unit sum for every sub-pixel and with
    edge-replicated controls; the threshold 1/2 of Eq. (6) is subtracted so
    that C = 1/2 everywhere is the uniform average material;
  * tanh projection, Eq. (3)/(6): rho = (1 + tanh(beta Phi)) / 2 on the
    design area of the high-resolution canvas, fixed background elsewhere;
  * density mix: eps = eps_clad + rho (eps_core - eps_clad);
  * averages over a Yee-cell-sized window centred on each E component,
    Eq. (8), as S x S box means of the canvas (x window shifted by half a
    cell for E_x, y window for E_y), giving <1/eps>, <eps> and <rho>;
  * normals from a Sobel edge detector on <rho>, n_a^2 = G_a^2 / (|G|^2 + delta);
  * anisotropic smoothing, Eq. (7): 1/eps_ii = n_i^2 <1/eps> + (1 - n_i^2)/<eps>
    for i = x, y; E_z sees vertical sidewalls only (n_z = 0) so kappa_z = 1/<eps>;
  * extrusion along z through the slab; E_z planes on the two slab faces are
    half filled with normal z, kappa_z = (<1/eps> + 1/eps_clad) / 2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------- operators
def filter_matrix(n_sub: int, n_ctl: int, n_px: int, S: int, r: float) -> np.ndarray:
    """W[u, a]: weight of control a at design sub-pixel u (u in [0, S*n_px)).

    Sub-pixel u is centred at design coordinate (u + 1/2)/S pixels, i.e. at
    x = ((u + 1/2)/S) * n_ctl/n_px - 1/2 in control-pixel units (control a is
    centred at a).  Taps i with |x - i| <= r; out-of-range taps fall back on
    the nearest control (edge replicate); weights sum to one per sub-pixel.
    """
    assert n_sub == S * n_px
    sigma = r / 2.0
    W = np.zeros((n_sub, n_ctl))
    for u in range(n_sub):
        x = ((u + 0.5) / S) * n_ctl / n_px - 0.5
        lo = int(np.ceil(x - r))
        hi = int(np.floor(x + r))
        taps = []
        for i in range(lo, hi + 1):
            d = x - i
            if abs(d) <= r:
                taps.append((i, np.exp(-d * d / (2.0 * sigma * sigma))))
        z = sum(g for _, g in taps)
        for i, g in taps:
            W[u, min(max(i, 0), n_ctl - 1)] += g / z
    return W


def box_matrix(n_px: int, S: int, shift: int, n_hr: int) -> np.ndarray:
    """B[m, u]: S-wide window starting at sub-pixel S*m + shift (clamped into
    [0, n_hr)), each sub-pixel weighted 1/S."""
    B = np.zeros((n_px, n_hr))
    for m in range(n_px):
        for a in range(S):
            u = min(max(S * m + shift + a, 0), n_hr - 1)
            B[m, u] += 1.0 / S
    return B


def diff_matrix(n: int) -> np.ndarray:
    """D[m, q]: central difference f[m+1] - f[m-1] with edge replication."""
    D = np.zeros((n, n))
    for m in range(n):
        D[m, min(m + 1, n - 1)] += 1.0
        D[m, max(m - 1, 0)] -= 1.0
    return D


def smooth_matrix(n: int) -> np.ndarray:
    """M[m, q]: [1, 2, 1] smoothing with edge replication."""
    M = np.zeros((n, n))
    for m in range(n):
        M[m, max(m - 1, 0)] += 1.0
        M[m, m] += 2.0
        M[m, min(m + 1, n - 1)] += 1.0
    return M


@dataclass
class ChainOps:
    S: int
    md: int
    nd: int
    Wx: np.ndarray      # [S*md][mc]
    Wy: np.ndarray      # [S*nd][nc]
    Bx: list            # per component [(md+4)][U]
    By: list            # per component [(nd+4)][V]
    Dx: np.ndarray
    Dy: np.ndarray
    Mx: np.ndarray
    My: np.ndarray


def make_ops(dev) -> ChainOps:
    S, md, nd = dev.supersample, dev.md, dev.nd
    U, V = S * (md + 4), S * (nd + 4)
    Wx = filter_matrix(S * md, dev.mc, md, S, dev.filter_r)
    Wy = filter_matrix(S * nd, dev.nc, nd, S, dev.filter_r)
    half = S // 2
    shifts_x = (half, 0, 0)   # E_x window shifted half a cell in x
    shifts_y = (0, half, 0)   # E_y window shifted half a cell in y
    Bx = [box_matrix(md + 4, S, shifts_x[c], U) for c in range(3)]
    By = [box_matrix(nd + 4, S, shifts_y[c], V) for c in range(3)]
    return ChainOps(S, md, nd, Wx, Wy, Bx, By, diff_matrix(md + 4), diff_matrix(nd + 4),
                    smooth_matrix(md + 4), smooth_matrix(nd + 4))


# ----------------------------------------------------------------- forward
@dataclass
class ChainState:
    phi: np.ndarray
    t: np.ndarray           # tanh(beta*phi) on the design area
    rho: np.ndarray         # canvas [V][U]
    eps: np.ndarray
    P: list
    Q: list
    R: list
    Gx: list
    Gy: list
    n2: list                # n_x^2 (from R_x), n_y^2 (from R_y)
    kx: np.ndarray          # 2-D maps on the (md+4) x (nd+4) component grids
    ky: np.ndarray
    kz_in: np.ndarray
    kz_face: np.ndarray


def design_slices(dev):
    S = dev.supersample
    return (slice(2 * S, 2 * S + S * dev.nd), slice(2 * S, 2 * S + S * dev.md))


def smooth_kappa(dev, rho: np.ndarray, ops: ChainOps):
    """Averages, Sobel normals and Eq. (7) for a canvas rho [V][U].
    Returns (eps, P, Q, R, Gx, Gy, [nx2, ny2], kx, ky, kz_in, kz_face)."""
    eps = dev.eps_clad + (dev.eps_core - dev.eps_clad) * rho
    inv = 1.0 / eps
    P, Q, R, Gx, Gy = [], [], [], [], []
    for c in range(3):
        By, Bx = ops.By[c], ops.Bx[c]
        P.append(By @ inv @ Bx.T)
        Q.append(By @ eps @ Bx.T)
        R.append(By @ rho @ Bx.T)
        Gx.append(ops.My @ R[c] @ ops.Dx.T / 8.0)
        Gy.append(ops.Dy @ R[c] @ ops.Mx.T / 8.0)
    d = dev.sobel_delta
    nx2 = Gx[0] ** 2 / (Gx[0] ** 2 + Gy[0] ** 2 + d)
    ny2 = Gy[1] ** 2 / (Gx[1] ** 2 + Gy[1] ** 2 + d)
    kx = nx2 * P[0] + (1.0 - nx2) / Q[0]
    ky = ny2 * P[1] + (1.0 - ny2) / Q[1]
    kz_in = 1.0 / Q[2]
    kz_face = 0.5 * (P[2] + 1.0 / dev.eps_clad)
    return eps, P, Q, R, Gx, Gy, [nx2, ny2], kx, ky, kz_in, kz_face


def project(dev, C, beta, ops: ChainOps):
    """(phi, tanh(beta phi), canvas rho): Eq. (2) then Eq. (3)/(6)."""
    phi = ops.Wy @ np.asarray(C, np.float64) @ ops.Wx.T - 0.5
    t = np.tanh(beta * phi)
    rho = np.array(dev.mask_hr, np.float64, copy=True)
    sv, su = design_slices(dev)
    rho[sv, su] = 0.5 * (1.0 + t)
    return phi, t, rho


def forward(dev, C, beta, ops: ChainOps = None) -> ChainState:
    ops = ops or make_ops(dev)
    phi, t, rho = project(dev, C, beta, ops)
    return ChainState(phi, t, rho, *smooth_kappa(dev, rho, ops))


def written_region(dev):
    """(slice in y, slice in x) of the component grids whose kappa is written:
    the design area plus a one-pixel ring."""
    return (slice(1, dev.nd + 3), slice(1, dev.md + 3))


def extrude(dev, st: ChainState, kappa_bg: np.ndarray) -> np.ndarray:
    """Write the design kappa into a copy of the 3-D background."""
    kap = np.array(kappa_bg, np.float64, copy=True)
    wy, wx = written_region(dev)
    y0, x0 = dev.j0 - 1, dev.i0 - 1
    ys = slice(y0, y0 + dev.nd + 2)
    xs = slice(x0, x0 + dev.md + 2)
    for k in range(dev.k_lo, dev.k_hi + 1):
        kap[0, k, ys, xs] = st.kx[wy, wx]
        kap[1, k, ys, xs] = st.ky[wy, wx]
    for k in range(dev.k_lo, dev.k_hi):
        kap[2, k, ys, xs] = st.kz_in[wy, wx]
    for k in (dev.k_lo - 1, dev.k_hi):
        kap[2, k, ys, xs] = st.kz_face[wy, wx]
    return kap


def kappa(dev, C=None, beta=None, ops=None):
    C = dev.C if C is None else C
    beta = dev.beta if beta is None else beta
    st = forward(dev, C, beta, ops)
    return extrude(dev, st, dev.kappa_bg), st


# ----------------------------------------------------------------- VJP
def zsum(dev, g3: np.ndarray):
    """Transpose of the extrusion: dF/dkappa on the DFT box [3][bz][by][bx]
    (box = ring x slab planes k_lo-1 .. k_hi) -> 2-D maps on the component
    grids (zero outside the written region)."""
    shape = (dev.nd + 4, dev.md + 4)
    gx, gy, gzi, gzf = (np.zeros(shape) for _ in range(4))
    wy, wx = written_region(dev)
    z0 = dev.k_lo - 1
    for k in range(dev.k_lo, dev.k_hi + 1):
        gx[wy, wx] += g3[0, k - z0]
        gy[wy, wx] += g3[1, k - z0]
    for k in range(dev.k_lo, dev.k_hi):
        gzi[wy, wx] += g3[2, k - z0]
    for k in (dev.k_lo - 1, dev.k_hi):
        gzf[wy, wx] += g3[2, k - z0]
    return gx, gy, gzi, gzf


def vjp(dev, st: ChainState, beta, gx, gy, gzi, gzf, ops: ChainOps = None):
    """dF/dC from dF/dkappa maps (the z-summed gradients)."""
    ops = ops or make_ops(dev)
    d = dev.sobel_delta
    gP = [None] * 3
    gQ = [None] * 3
    gR = [None] * 3
    for c, g in ((0, gx), (1, gy)):
        n2 = st.n2[c]
        Gx, Gy = st.Gx[c], st.Gy[c]
        D = Gx ** 2 + Gy ** 2 + d
        gP[c] = g * n2
        gQ[c] = -g * (1.0 - n2) / st.Q[c] ** 2
        gn = g * (st.P[c] - 1.0 / st.Q[c])
        if c == 0:
            gGx = gn * 2.0 * Gx * (Gy ** 2 + d) / D ** 2
            gGy = -gn * 2.0 * Gy * Gx ** 2 / D ** 2
        else:
            gGy = gn * 2.0 * Gy * (Gx ** 2 + d) / D ** 2
            gGx = -gn * 2.0 * Gx * Gy ** 2 / D ** 2
        gR[c] = ops.My.T @ gGx @ ops.Dx / 8.0 + ops.Dy.T @ gGy @ ops.Mx / 8.0
    gP[2] = 0.5 * gzf
    gQ[2] = -gzi / st.Q[2] ** 2
    gR[2] = np.zeros_like(gzi)
    g_inv = sum(ops.By[c].T @ gP[c] @ ops.Bx[c] for c in range(3))
    g_eps = sum(ops.By[c].T @ gQ[c] @ ops.Bx[c] for c in range(3))
    g_rho = sum(ops.By[c].T @ gR[c] @ ops.Bx[c] for c in range(3))
    de = dev.eps_core - dev.eps_clad
    g_rho_tot = g_inv * (-de / st.eps ** 2) + g_eps * de + g_rho
    sv, su = design_slices(dev)
    g_phi = g_rho_tot[sv, su] * 0.5 * beta * (1.0 - st.t ** 2)
    return ops.Wy.T @ g_phi @ ops.Wx
