"""Pins of the oracle's morphological filters (paper Sec. 3, Eqs. 4-6): the
disc kernel against the lattice-point counts of a circle, the normalised
kernel's fixed points, the hard-morphology limits of the soft operations
(SciPy's grey and binary morphology with the same disc), the transposed
Jacobian against finite differences, and the whole chain with filters."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import chain
from workloads import configs


def morph_dev(ops="edde", d=1.5, alpha=20.0, **kw):
    args = dict(md=10, nd=9, mc=7, nc=6, filter_r=1.5)
    args.update(kw)
    dev = configs.micro(**args)
    dev.morph_ops, dev.morph_d, dev.morph_alpha = ops, d, alpha
    return dev


def disc(taps):
    n = max(max(abs(a), abs(b)) for a, b in taps)
    fp = np.zeros((2 * n + 1, 2 * n + 1), bool)
    for dy, dx in taps:
        fp[dy + n, dx + n] = True
    return fp


def canvas_with_design(dev, design, margin_value):
    S = dev.supersample
    c = np.full((S * (dev.nd + 4), S * (dev.md + 4)), float(margin_value))
    sv, su = chain.design_slices(dev)
    c[sv, su] = design
    return c


def test_disc_tap_counts_are_lattice_points_in_a_circle():
    # integer points with x^2 + y^2 <= r^2 (r = d S / 2): 1, 5, 13, 29, 49, 81
    for r, n in ((0, 1), (1, 5), (2, 13), (3, 29), (4, 49), (5, 81)):
        assert len(chain.disc_taps(2.0 * r, 1)) == n
    # sqrt(2): the four diagonal neighbours join
    assert len(chain.disc_taps(2.0 * np.sqrt(2.0) + 1e-12, 1)) == 9
    t = chain.disc_taps(3.0, 4)
    assert set(t) == {(-a, -b) for a, b in t}          # symmetric
    assert (6, 0) in t and (0, -6) in t and (5, 4) not in t and (4, 4) in t


@pytest.mark.parametrize("op", ["d", "e"])
def test_constant_density_is_a_fixed_point(op):
    dev = morph_dev(op)
    ops = chain.make_ops(dev)
    S = dev.supersample
    for c0 in (0.0, 0.3, 1.0):
        canvas = np.full((S * (dev.nd + 4), S * (dev.md + 4)), c0)
        out, _ = chain.morph_stage(dev, canvas, op, dev.morph_alpha, ops.K)
        assert np.allclose(out, c0, atol=1e-13)


@pytest.mark.parametrize("op", ["d", "e"])
def test_large_sharpness_tends_to_grey_morphology(op):
    # soft dilation lies in [max - log(n)/a, max] over the disc (nearest-edge
    # extension beyond the canvas); erosion in [min, min + log(n)/a]
    dev = morph_dev(op, d=2.0, alpha=200.0)
    ops = chain.make_ops(dev)
    taps = chain.disc_taps(dev.morph_d, dev.supersample)
    rng = np.random.default_rng(21)
    canvas = rng.uniform(size=(dev.supersample * (dev.nd + 4), dev.supersample * (dev.md + 4)))
    out, _ = chain.morph_stage(dev, canvas, op, dev.morph_alpha, ops.K)
    fp = disc(taps)
    hard = (ndimage.grey_dilation if op == "d" else ndimage.grey_erosion)(canvas, footprint=fp,
                                                                          mode="nearest")
    sv, su = chain.design_slices(dev)
    slack = np.log(len(taps)) / dev.morph_alpha
    y, h = out[sv, su], hard[sv, su]
    if op == "d":
        assert np.all(y <= h + 1e-12) and np.all(y >= h - slack)
    else:
        assert np.all(y >= h - 1e-12) and np.all(y <= h + slack)
    # the margin is never written
    m = np.ones_like(canvas, bool)
    m[sv, su] = False
    assert np.array_equal(out[m], canvas[m])


def test_opening_and_closing_match_binary_morphology():
    # a 2 px square (smaller than the 3 px disc) vanishes under opening; a
    # 7 px square survives with rounded corners; a 1-sub-pixel slit in a
    # solid block closes
    dev = morph_dev("ed", d=3.0, alpha=400.0, nx=40, ny=40, md=16, nd=16)
    ops = chain.make_ops(dev)
    S = dev.supersample
    taps = chain.disc_taps(dev.morph_d, S)
    fp = disc(taps)
    img = np.zeros((S * dev.nd, S * dev.md))
    img[8:16, 8:16] = 1.0              # 2 x 2 design pixels
    img[28:56, 28:56] = 1.0            # 7 x 7
    c = canvas_with_design(dev, img, 0.0)
    for op in "ed":
        c, _ = chain.morph_stage(dev, c, op, dev.morph_alpha, ops.K)
    sv, su = chain.design_slices(dev)
    ref = ndimage.binary_opening(canvas_with_design(dev, img, 0.0) > 0.5, structure=fp)
    assert np.array_equal(c[sv, su] > 0.5, ref[sv, su])
    assert not np.any(c[sv, su][8:16, 8:16] > 0.5) and c[sv, su][42, 42] > 0.9

    img = np.zeros((S * dev.nd, S * dev.md))
    img[12:52, 12:52] = 1.0
    img[12:52, 31] = 0.0               # slit one sub-pixel wide
    c = canvas_with_design(dev, img, 0.0)
    for op in "de":
        c, _ = chain.morph_stage(dev, c, op, dev.morph_alpha, ops.K)
    ref = ndimage.binary_closing(canvas_with_design(dev, img, 0.0) > 0.5, structure=fp)
    assert np.array_equal(c[sv, su] > 0.5, ref[sv, su])
    assert c[sv, su][30, 31] > 0.9


@pytest.mark.parametrize("op", ["d", "e"])
def test_stage_vjp_matches_finite_differences(op):
    dev = morph_dev(op, d=1.5, alpha=20.0)
    ops = chain.make_ops(dev)
    rng = np.random.default_rng(22)
    S = dev.supersample
    canvas = rng.uniform(size=(S * (dev.nd + 4), S * (dev.md + 4)))
    sv, su = chain.design_slices(dev)
    w = rng.standard_normal(canvas[sv, su].shape)
    out, sums = chain.morph_stage(dev, canvas, op, dev.morph_alpha, ops.K)
    g = chain.morph_stage_vjp(dev, canvas, op, dev.morph_alpha, ops.K, sums, w)
    def F(c):
        return np.sum(chain.morph_stage(dev, c, op, dev.morph_alpha, ops.K)[0][sv, su] * w)

    h = 1e-6
    # single sub-pixels (cancellation in F(+h) - F(-h) leaves ~1e-7 absolute)
    for (v, u) in [(0, 0), (5, 7), (S * dev.nd - 1, S * dev.md - 1), (17, 3), (20, 30)]:
        cp, cm = canvas.copy(), canvas.copy()
        cp[sv, su][v, u] += h
        cm[sv, su][v, u] -= h
        assert g[v, u] == pytest.approx((F(cp) - F(cm)) / (2 * h), rel=1e-5, abs=2e-7)
    # a random direction over the whole design area
    dirn = rng.standard_normal(w.shape)
    cp, cm = canvas.copy(), canvas.copy()
    cp[sv, su] += h * dirn
    cm[sv, su] -= h * dirn
    assert np.sum(g * dirn) == pytest.approx((F(cp) - F(cm)) / (2 * h), rel=1e-7)


@pytest.mark.parametrize("seq", ["edde", "d", "de"])
def test_chain_vjp_with_filters_matches_finite_differences(seq):
    dev = morph_dev(seq, d=1.5, alpha=20.0)
    ops = chain.make_ops(dev)
    beta = 4.0
    rng = np.random.default_rng(23)
    x0, y0, z0, bx, by, bz = dev.dft_box()
    g3 = rng.standard_normal((3, bz, by, bx))
    C = rng.uniform(0.2, 0.8, (dev.nc, dev.mc))

    def F(Cv):
        kap, _ = chain.kappa(dev, Cv, beta, ops)
        return np.sum(kap[:, z0:z0 + bz, y0:y0 + by, x0:x0 + bx] * g3)

    st = chain.forward(dev, C, beta, ops)
    assert len(st.stages) == len(seq)
    gC = chain.vjp(dev, st, beta, *chain.zsum(dev, g3), ops)
    h = 1e-6
    for (b, a) in [(0, 0), (2, 3), (dev.nc - 1, dev.mc - 1), (3, 0), (1, 5)]:
        Cp, Cm = C.copy(), C.copy()
        Cp[b, a] += h
        Cm[b, a] -= h
        fd = (F(Cp) - F(Cm)) / (2 * h)
        assert gC[b, a] == pytest.approx(fd, rel=5e-6, abs=1e-9 * np.abs(gC).max())


def test_filters_change_the_design_and_binarise_through_eq6():
    dev = morph_dev("edde", d=1.5, alpha=20.0)
    plain = morph_dev("", d=1.5)
    C = np.random.default_rng(24).uniform(size=(dev.nc, dev.mc))
    st = chain.forward(dev, C, 8.0)
    st0 = chain.forward(plain, C, 8.0)
    sv, su = chain.design_slices(dev)
    assert not np.allclose(st.rho[sv, su], st0.rho[sv, su])
    assert np.allclose(st.rho[sv, su], 0.5 * (1 + st.t2))
    # outside the design area the canvas is the background either way
    m = np.ones_like(st.rho, bool)
    m[sv, su] = False
    assert np.array_equal(st.rho[m], st0.rho[m])
