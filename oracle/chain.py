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

Optional morphological filtering (Eqs. 4-5, then Eq. 6), when the device
names a sequence of operations (``dev.morph_ops``, 'd' dilate, 'e' erode,
applied left to right): the projected density rho_0 of Eq. (3) goes through
soft dilations rho~ = (1/a) log sum K exp(a rho) and erosions
rho~ = 1 - (1/a) log sum K exp(a (1 - rho)) with the disc kernel K_m of
diameter d (``dev.morph_d`` design pixels: the sub-pixel offsets whose
length is at most d S / 2), normalised to unit sum, and sharpness a
(``dev.morph_alpha``); then rho = (1 + tanh(beta (rho~ - 1/2))) / 2.  Each
stage is evaluated on the design area of the canvas; kernel taps that fall
in the margin read the fixed background there, and taps beyond the canvas
read its nearest edge sub-pixel.  Without operations rho = rho_0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

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


def disc_taps(d: float, S: int):
    """Sub-pixel offsets (dy, dx) of the disc kernel K_m of diameter d design
    pixels: every offset of length at most d S / 2."""
    R = d * S / 2.0
    n = int(np.floor(R))
    return [(dy, dx) for dy in range(-n, n + 1) for dx in range(-n, n + 1)
            if dx * dx + dy * dy <= R * R]


def morph_operator(dev, taps):
    """Sparse K[x, q]: x runs over the design sub-pixels ([S nd][S md], row
    major), q over the canvas ([V][U]); each tap adds 1/len(taps) at the canvas
    sub-pixel x + delta, clamped into the canvas."""
    from scipy import sparse
    S, md, nd = dev.supersample, dev.md, dev.nd
    U, V = S * (md + 4), S * (nd + 4)
    vd, ud = np.meshgrid(np.arange(S * nd), np.arange(S * md), indexing="ij")
    rows, cols = [], []
    for dy, dx in taps:
        v = np.clip(vd + 2 * S + dy, 0, V - 1)
        u = np.clip(ud + 2 * S + dx, 0, U - 1)
        rows.append((vd * (S * md) + ud).ravel())
        cols.append((v * U + u).ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.full(rows.size, 1.0 / len(taps))
    return sparse.csr_matrix((vals, (rows, cols)), shape=(S * S * md * nd, U * V))


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
    K: object = None    # morphological operator (None without operations)


def morph_ops_of(dev) -> str:
    return getattr(dev, "morph_ops", "") or ""


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
    K = morph_operator(dev, disc_taps(dev.morph_d, S)) if morph_ops_of(dev) else None
    return ChainOps(S, md, nd, Wx, Wy, Bx, By, diff_matrix(md + 4), diff_matrix(nd + 4),
                    smooth_matrix(md + 4), smooth_matrix(nd + 4), K)


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
    stages: list = field(default_factory=list)   # per morphological stage: (input canvas, sums)
    t2: np.ndarray = None                        # tanh of the Eq. (6) projection after them


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


def morph_stage(dev, canvas: np.ndarray, op: str, alpha: float, K):
    """One soft dilation (Eq. 4, op 'd') or erosion (Eq. 5, op 'e') of a
    canvas; returns (output canvas, the kernel sums on the design area)."""
    sv, su = design_slices(dev)
    if op == "d":
        sums = K @ np.exp(alpha * canvas).ravel()
        y = np.log(sums) / alpha
    elif op == "e":
        sums = K @ np.exp(alpha * (1.0 - canvas)).ravel()
        y = 1.0 - np.log(sums) / alpha
    else:
        raise ValueError(f"unknown morphological operation {op!r}")
    out = canvas.copy()
    out[sv, su] = y.reshape(out[sv, su].shape)
    return out, sums


def morph_stage_vjp(dev, canvas: np.ndarray, op: str, alpha: float, K, sums, g):
    """Transpose of one stage's Jacobian: g on the design area of its output
    -> gradient on the design area of its input.  Both operations have
    d rho~(x) / d rho(q) = K[x, q] e(q) / sums(x) with e the exponential the
    stage sums."""
    sv, su = design_slices(dev)
    e = np.exp(alpha * canvas) if op == "d" else np.exp(alpha * (1.0 - canvas))
    gc = e.ravel() * (K.T @ (np.asarray(g).ravel() / sums))
    return gc.reshape(canvas.shape)[sv, su]


def forward(dev, C, beta, ops: ChainOps = None) -> ChainState:
    ops = ops or make_ops(dev)
    phi, t, rho = project(dev, C, beta, ops)
    stages, t2 = [], None
    seq = morph_ops_of(dev)
    if seq:
        for op in seq:
            out, sums = morph_stage(dev, rho, op, dev.morph_alpha, ops.K)
            stages.append((rho, sums))
            rho = out
        sv, su = design_slices(dev)
        t2 = np.tanh(beta * (rho[sv, su] - 0.5))           # Eq. (6)
        rho = rho.copy()
        rho[sv, su] = 0.5 * (1.0 + t2)
    return ChainState(phi, t, rho, *smooth_kappa(dev, rho, ops), stages=stages, t2=t2)


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
    g_d = g_rho_tot[sv, su]
    seq = morph_ops_of(dev)
    if seq:
        g_d = g_d * 0.5 * beta * (1.0 - st.t2 ** 2)
        for op, (canvas, sums) in zip(reversed(seq), reversed(st.stages)):
            g_d = morph_stage_vjp(dev, canvas, op, dev.morph_alpha, ops.K, sums, g_d)
    g_phi = g_d * 0.5 * beta * (1.0 - st.t ** 2)
    return ops.Wy.T @ g_phi @ ops.Wx
