"""Pins of the oracle's parametrization chain (paper Sec. 3): closed forms of
the filter and projection, exact fill fractions of straight edges, the Sobel
normalisation, the special cases of Eq. (7), transpose identities, and the
VJP against finite differences."""
import numpy as np
import pytest

from oracle import chain
from workloads import configs


@pytest.fixture(scope="module")
def dev():
    return configs.micro(md=10, nd=9, mc=7, nc=6, filter_r=1.5)


@pytest.fixture(scope="module")
def ops(dev):
    return chain.make_ops(dev)


def test_filter_partition_of_unity_and_support(dev, ops):
    for W, n_px, n_ctl in ((ops.Wx, dev.md, dev.mc), (ops.Wy, dev.nd, dev.nc)):
        assert np.allclose(W.sum(axis=1), 1.0, atol=1e-14)
        assert np.all(W >= 0)
        S = dev.supersample
        for u in range(W.shape[0]):
            x = ((u + 0.5) / S) * n_ctl / n_px - 0.5
            far = np.abs(np.arange(n_ctl) - x) > dev.filter_r
            # controls farther than r only receive weight through edge replication
            inner = far & (np.arange(n_ctl) > 0) & (np.arange(n_ctl) < n_ctl - 1)
            assert np.all(W[u, inner] == 0)


def test_filter_gaussian_weights_interior():
    """Away from the edges the weights are the normalised Gaussian taps."""
    S, n, r = 4, 20, 3.0
    W = chain.filter_matrix(S * n, n, n, S, r)
    u = 41                       # x = (41.5/4) - 0.5 = 9.875
    x = (u + 0.5) / S - 0.5
    taps = np.arange(7, 13)
    g = np.exp(-(x - taps) ** 2 / (2 * (r / 2) ** 2))
    assert np.allclose(W[u, taps], g / g.sum(), atol=1e-15)
    assert W[u].sum() == pytest.approx(1.0)


def test_half_controls_give_uniform_average_material(dev, ops):
    """C = 1/2 everywhere (the paper's gray start) gives rho = 1/2 exactly."""
    C = np.full((dev.nc, dev.mc), 0.5)
    phi, t, rho = chain.project(dev, C, 8.0, ops)
    assert np.max(np.abs(phi)) < 1e-15
    sv, su = chain.design_slices(dev)
    assert np.max(np.abs(rho[sv, su] - 0.5)) < 1e-15


def test_projection_limits(dev, ops):
    rng = np.random.default_rng(0)
    C = rng.uniform(0, 1, (dev.nc, dev.mc))
    phi, t, rho = chain.project(dev, C, 1e4, ops)
    sv, su = chain.design_slices(dev)
    r = rho[sv, su]
    far = np.abs(phi) > 1e-2
    assert np.all((r[far] < 1e-12) | (r[far] > 1 - 1e-12))     # binary as beta grows
    assert np.all((r >= 0) & (r <= 1))


def test_box_means_straight_edge_fill_fractions(dev, ops):
    """A vertical edge at x_e: each component's <rho> is the exact fraction of
    its window (one cell wide, centred on that E component) left of x_e."""
    S = dev.supersample
    U, V = S * (dev.md + 4), S * (dev.nd + 4)
    xu = (dev.i0 - 2.5) + (np.arange(U) + 0.5) / S
    for x_e in (dev.i0 + 1.25, dev.i0 + 3.0, dev.i0 + 4.5):
        rho = np.broadcast_to((xu < x_e).astype(float), (V, U))
        for c, centre_shift in ((0, 0.5), (1, 0.0), (2, 0.0)):
            R = ops.By[c] @ rho @ ops.Bx[c].T
            m = np.arange(1, dev.md + 3)
            centre = dev.i0 - 2 + m + centre_shift
            expect = np.clip(x_e - (centre - 0.5), 0.0, 1.0)
            assert np.allclose(R[3, m], expect, atol=1e-14)


def test_sobel_gives_gradient_of_linear_fields(dev, ops):
    n, m = ops.My.shape[0], ops.Mx.shape[0]
    a, b = 0.37, -1.1
    R = a * np.arange(m)[None, :] + b * np.arange(n)[:, None]
    Gx = ops.My @ R @ ops.Dx.T / 8.0
    Gy = ops.Dy @ R @ ops.Mx.T / 8.0
    assert np.allclose(Gx[1:-1, 1:-1], a, atol=1e-13)
    assert np.allclose(Gy[1:-1, 1:-1], b, atol=1e-13)


def test_eq7_special_cases(dev, ops):
    S = dev.supersample
    U, V = S * (dev.md + 4), S * (dev.nd + 4)
    # uniform canvas: every component is 1/eps
    for val in (0.0, 1.0, 0.3):
        rho = np.full((V, U), val)
        out = chain.smooth_kappa(dev, rho, ops)
        eps = dev.eps_clad + (dev.eps_core - dev.eps_clad) * val
        kx, ky, kzi = out[7], out[8], out[9]
        assert np.allclose(kx, 1 / eps) and np.allclose(ky, 1 / eps) and np.allclose(kzi, 1 / eps)
    # a vertical edge (normal along x) cutting the E_x window: n_x^2 -> 1 and
    # kappa_x = <1/eps> (harmonic); n_y^2 -> 0 so kappa_y = 1/<eps> (arithmetic)
    xu = (dev.i0 - 2.5) + (np.arange(U) + 0.5) / S
    x_e = dev.i0 + 3.25
    rho = np.broadcast_to((xu < x_e).astype(float), (V, U)).copy()
    eps, P, Q, R, Gx, Gy, n2, kx, ky, kzi, kzf = chain.smooth_kappa(dev, rho, ops)
    col = 5 + 0  # E_x at i0+3+1/2 window [i0+3, i0+4): 1/4 filled
    row = 4
    assert n2[0][row, col] == pytest.approx(1.0, abs=1e-4)
    assert kx[row, col] == pytest.approx(P[0][row, col], rel=1e-4)
    assert ky[row, col] == pytest.approx(1 / Q[1][row, col], rel=1e-12)
    fill = R[0][row, col]
    assert fill == pytest.approx(0.25, abs=1e-14)
    harmonic = fill / dev.eps_core + (1 - fill) / dev.eps_clad
    assert kx[row, col] == pytest.approx(harmonic, rel=1e-4)
    # half-filled slab faces: kappa_z = (<1/eps> + 1/eps_clad)/2
    assert np.allclose(kzf, 0.5 * (P[2] + 1 / dev.eps_clad))


def test_extrusion_and_zsum_are_transposes(dev, ops):
    rng = np.random.default_rng(5)
    st = chain.forward(dev, dev.C, dev.beta, ops)
    x0, y0, z0, bx, by, bz = dev.dft_box()
    g3 = rng.standard_normal((3, bz, by, bx))
    # <extrude(maps), g3> over the box == <maps, zsum(g3)>
    maps = [rng.standard_normal(st.kx.shape) for _ in range(4)]
    st2 = chain.ChainState(st.phi, st.t, st.rho, st.eps, st.P, st.Q, st.R, st.Gx, st.Gy, st.n2,
                           maps[0], maps[1], maps[2], maps[3])
    kap = chain.extrude(dev, st2, np.zeros_like(dev.kappa_bg))
    lhs = np.sum(kap[:, z0:z0 + bz, y0:y0 + by, x0:x0 + bx] * g3)
    gx, gy, gzi, gzf = chain.zsum(dev, g3)
    rhs = sum(np.sum(m * g) for m, g in zip(maps, (gx, gy, gzi, gzf)))
    assert lhs == pytest.approx(rhs, rel=1e-13)


@pytest.mark.parametrize("beta", [4.0, 30.0])
def test_vjp_matches_finite_differences(dev, ops, beta):
    rng = np.random.default_rng(6)
    x0, y0, z0, bx, by, bz = dev.dft_box()
    g3 = rng.standard_normal((3, bz, by, bx))
    C = rng.uniform(0.3, 0.7, (dev.nc, dev.mc))

    def F(Cv):
        kap, _ = chain.kappa(dev, Cv, beta, ops)
        return np.sum(kap[:, z0:z0 + bz, y0:y0 + by, x0:x0 + bx] * g3)

    st = chain.forward(dev, C, beta, ops)
    gC = chain.vjp(dev, st, beta, *chain.zsum(dev, g3), ops)
    h = 1e-6
    for (b, a) in [(0, 0), (2, 3), (dev.nc - 1, dev.mc - 1), (3, 0), (1, 5)]:
        Cp, Cm = C.copy(), C.copy()
        Cp[b, a] += h
        Cm[b, a] -= h
        fd = (F(Cp) - F(Cm)) / (2 * h)
        assert gC[b, a] == pytest.approx(fd, rel=2e-6, abs=1e-9 * np.abs(gC).max())


def test_vjp_finite_at_high_beta(dev, ops):
    rng = np.random.default_rng(8)
    st = chain.forward(dev, dev.C, 1e3, ops)
    x0, y0, z0, bx, by, bz = dev.dft_box()
    g = chain.vjp(dev, st, 1e3, *chain.zsum(dev, rng.standard_normal((3, bz, by, bx))), ops)
    assert np.all(np.isfinite(g))
