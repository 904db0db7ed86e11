"""Pins of the oracle's optimizer loop (paper Sec. 4): the Eq. (9) coefficient
against finite differences, Adam's closed forms, the Eq. (14) schedule's end
points, the Eq. (15) controller's fixed point, the grey count."""
import math

import numpy as np
import pytest

from oracle import optimize as O


def test_eq9_coefficient_is_the_wirtinger_derivative():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(1, 2, 2)) + 1j * rng.normal(size=(1, 2, 2))
    T = np.array([[[1.0, 0.0], [0.0, 1.0]]])
    F, coef = O.objective_eq9(a, T)
    assert F == pytest.approx(np.sum((T - np.abs(a) ** 2) ** 2))
    h = 1e-7
    for idx in np.ndindex(a.shape):
        for direction, part in ((1.0, "re"), (1j, "im")):
            ap, am = a.copy(), a.copy()
            ap[idx] += h * direction
            am[idx] -= h * direction
            d = (O.objective_eq9(ap, T)[0] - O.objective_eq9(am, T)[0]) / (2 * h)
            # dF/dx = 2 Re(coef), dF/dy = -2 Im(coef) for coef = dF/dalpha
            ref = 2 * coef[idx].real if part == "re" else -2 * coef[idx].imag
            assert d == pytest.approx(ref, rel=1e-6, abs=1e-9)


def test_eq9_untargeted_entries_do_not_count():
    a = np.array([0.5 + 0.5j, 2.0])
    F, coef = O.objective_eq9(a, np.array([np.nan, 1.0]))
    assert F == pytest.approx(9.0)
    assert coef[0] == 0


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(4)
    G = rng.normal(size=50)
    C0 = rng.uniform(size=50)
    M = np.zeros(50)
    V = np.zeros(50)
    C1, M, V = O.adam_step(C0, G, M, V, 1, lr=1e-3, eps=1e-8)
    # bias correction makes the first step -lr G / (|G| + eps)
    assert np.allclose(C1 - C0, -1e-3 * G / (np.abs(G) + 1e-8), rtol=1e-12, atol=0)
    # a constant gradient keeps Mhat = G and Vhat = G^2 exactly
    C2, M, V = O.adam_step(C1, G, M, V, 2, lr=1e-3, eps=1e-8)
    assert np.allclose(C2 - C1, C1 - C0, rtol=1e-9, atol=1e-15)


def test_adam_minimises_a_quadratic():
    target = np.array([0.3, -0.2, 0.9])
    C = np.zeros(3)
    M = np.zeros(3)
    V = np.zeros(3)
    for i in range(1, 3001):
        C, M, V = O.adam_step(C, 2 * (C - target), M, V, i, lr=1e-2)
    assert np.abs(C - target).max() < 1e-3


def test_beta_schedule_end_points_and_growth():
    b = [O.beta_schedule(i, 100, 10.0, 300.0) for i in range(101)]
    assert b[0] == pytest.approx(10.0)
    assert b[100] == pytest.approx(300.0)
    assert all(y > x for x, y in zip(b, b[1:]))
    # the growth is quadratic in i/N at the start
    assert (b[1] - b[0]) == pytest.approx(290.0 * (math.exp(1e-4) - 1) / (math.e - 1))


def test_beta_control_reaches_the_target_unbinarity():
    # a design whose grey fraction obeys 1/u - 1 = c beta: the controller's t
    # tends to c and beta_max to the beta at which u = u0
    c = 0.37
    ctl = O.BetaControl(u0=0.01, gamma=0.9)
    beta = 10.0
    for _ in range(400):
        u = 1.0 / (1.0 + c * beta)
        ctl.update(u, beta)
        beta = 0.5 * (beta + ctl.beta_max)
    assert ctl.t == pytest.approx(c, rel=1e-9)
    assert 1.0 / (1.0 + c * ctl.beta_max) == pytest.approx(0.01, rel=1e-9)


def test_unbinarity_counts_open_interval():
    r = np.array([0.0, 0.01, 0.0101, 0.5, 0.9899, 0.99, 1.0, 0.3])
    assert O.unbinarity(r) == pytest.approx(4 / 8)


@pytest.mark.usefixtures("oracle_built")
def test_oracle_optimizer_iteration_on_micro_demux():
    from workloads import configs
    dev = configs.micro_demux(n_steps=500)
    T = np.full((1, 2, 2), np.nan)
    T[0, 0, 0] = 1.0
    T[0, 1, 1] = 1.0
    h = O.optimize(dev, T, n_iter=2)
    assert all(np.isfinite(h.F)) and len(h.F) == 2
    assert 0 < h.u[0] <= 1
    assert h.beta[0] == 10.0 and h.beta[1] > 10.0 - 1e-12
    # Adam moves each control by at most about lr per step
    assert np.abs(h.C[0] - dev.C).max() <= 1e-3 * (1 + 1e-6)
