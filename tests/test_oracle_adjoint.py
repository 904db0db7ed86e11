"""Pins of the oracle's adjoint gradient (paper Eq. (1), Appendix A) against
brute-force central finite differences of the forward map, and of the modal
coefficient's normalisation."""
import numpy as np
import pytest

from oracle import adjoint, chain, ports
from workloads import configs

pytestmark = pytest.mark.usefixtures("oracle_built")


def test_alpha_of_the_mode_itself_is_one():
    dev = configs.tiny()
    for m in dev.ports + dev.sources:
        w = ports.monitor_weights(m.e, m.h)
        assert abs(ports.alpha(w, m.e) - 1.0) < 1e-14


def test_adjoint_source_is_minus_conjugate_forward_source():
    rng = np.random.default_rng(1)
    e = rng.standard_normal((2, 5, 7)) + 1j * rng.standard_normal((2, 5, 7))
    h = rng.standard_normal((2, 5, 7)) + 1j * rng.standard_normal((2, 5, 7))
    w = ports.monitor_weights(e, h)
    J = ports.source_current(h)
    N = ports.norm_N(e, h)
    assert np.allclose(w, -np.conj(J) / (2 * N), atol=1e-15)
    # J = n x h: J_t1 = -h_t2, J_t2 = h_t1
    assert np.allclose(J[0], -h[1]) and np.allclose(J[1], h[0])


def _fd(dev, C, idx, h, objective, n_steps):
    Cp, Cm = C.copy(), C.copy()
    Cp[idx] += h
    Cm[idx] -= h
    Fp = objective(adjoint.forward_adjoint(dev, Cp, n_steps=n_steps).alpha)
    Fm = objective(adjoint.forward_adjoint(dev, Cm, n_steps=n_steps).alpha)
    return (Fp - Fm) / (2 * h)


# 4000 steps leave a steady-state residual below 2e-6 on the micro devices
# (1500 steps: 8e-6 and 1.2e-5), and the gradient then agrees with central
# differences to about 2e-4 of its largest entry.  The tolerance, 5e-4 of the
# largest entry, resolves the factor of Eq. (1): with theta = w dt / 2 =
# 0.0785 on these devices, a gradient built with theta in place of
# sin(theta) (or -i w dt in place of -2 i sin(theta)) is off by
# 1 - sin(theta) / theta = 1.03e-3 of each entry, which the entries near the
# largest one expose.
STEPS = 4000
TOL = 5e-4


def test_gradient_abs2_matches_finite_differences():
    """Every one of the micro device's 30 controls."""
    dev = configs.micro(n_steps=STEPS)
    res = adjoint.forward_adjoint(dev)
    assert res.fwd[0][0].resid < 2e-6 and res.adj[0][0].resid < 2e-6
    F, coef = adjoint.objective_abs2(res.alpha)
    g = adjoint.grad_C(dev, res, coef)
    obj = lambda a: float(np.sum(np.abs(a) ** 2))  # noqa: E731
    fd = np.zeros_like(g)
    for idx in np.ndindex(g.shape):
        fd[idx] = _fd(dev, dev.C, idx, 1e-4, obj, None)
    gmax = np.abs(fd).max()
    assert np.abs(g - fd).max() < TOL * gmax, np.abs(g - fd).max() / gmax
    assert np.linalg.norm(g - fd) < TOL * np.linalg.norm(fd)


def test_gradient_wrt_kappa_matches_finite_differences():
    """The FDTD part alone: perturb kappa at single E sites inside the box,
    the site of the largest gradient entry among them."""
    dev = configs.micro(n_steps=STEPS)
    kap0, st = chain.kappa(dev)
    res = adjoint.forward_adjoint(dev)
    _, coef = adjoint.objective_abs2(res.alpha)
    gk = adjoint.grad_kappa(dev, res, coef)
    x0, y0, z0, bx, by, bz = dev.dft_box()
    gmax = np.abs(gk).max()
    top = tuple(int(v) for v in np.unravel_index(np.argmax(np.abs(gk)), gk.shape))
    h = 1e-5
    for (c, k, j, i) in [top, (0, 2, 3, 4), (1, 2, 5, 2), (2, 1, 4, 6)]:
        kp, km = kap0.copy(), kap0.copy()
        kp[c, z0 + k, y0 + j, x0 + i] += h
        km[c, z0 + k, y0 + j, x0 + i] -= h
        Fp = np.sum(np.abs(adjoint.forward_adjoint(dev, kap=kp).alpha) ** 2)
        Fm = np.sum(np.abs(adjoint.forward_adjoint(dev, kap=km).alpha) ** 2)
        fd = (Fp - Fm) / (2 * h)
        assert abs(gk[c, k, j, i] - fd) < TOL * gmax, ((c, k, j, i), gk[c, k, j, i], fd)


def test_gradient_eq9_two_ports_two_wavelengths():
    """F = sum_k (T_k - |alpha_k|^2)^2 with coef = 2 conj(alpha)(|alpha|^2 - T),
    at the control of the largest gradient entry and one other."""
    dev = configs.micro(n_steps=STEPS, ny=30, wavelengths=[0.8e-6, 0.85e-6])
    # a second output port
    from workloads import devices
    dev2 = devices.soi_device("micro2", dev.nx, dev.ny, dev.nz, dev.dx, dev.npml[0],
                              md=dev.md, nd=dev.nd, slab_layers=3, mc=dev.mc, nc=dev.nc,
                              filter_r=dev.filter_r, beta=dev.beta,
                              wavelengths=dev.wavelengths, n_steps=STEPS, seed=dev.seed,
                              mode_w=(3.0, 1.5), ramp_periods=3.0, strip_width=240e-9,
                              src_inset=3, out_offsets=(-0.12e-6, 0.12e-6))
    T = np.array([[[0.3, 0.2], [0.1, 0.4]]])

    def F(a):
        return float(np.sum((T - np.abs(a) ** 2) ** 2))

    res = adjoint.forward_adjoint(dev2)
    a = res.alpha
    coef = 2 * np.conj(a) * (np.abs(a) ** 2 - T)
    g = adjoint.grad_C(dev2, res, coef)
    gmax = np.abs(g).max()
    top = tuple(int(v) for v in np.unravel_index(np.argmax(np.abs(g)), g.shape))
    for idx in [top, (1, 4)]:
        fd = _fd(dev2, dev2.C, idx, 1e-4, F, None)
        assert abs(g[idx] - fd) < TOL * gmax, (idx, g[idx], fd)
