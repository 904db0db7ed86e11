"""Pins of the oracle's pulse-excitation route (paper Sec. 2: frequency-domain
fields from Fourier transforms of transients): the sampled pulse's spectrum
against the Gaussian's continuous Fourier transform, the phasors and alpha of
every wavelength against the time-harmonic steady state of the same device,
the residual as a truncation check, and the gradient against finite
differences."""
import math

import numpy as np
import pytest

from oracle import adjoint, fdtd
from workloads import configs


def default_pulse(dev, n_steps, k=1.5, m=4.5):
    w = [dev.omega_dt(lam) for lam in dev.wavelengths]
    w0 = 0.5 * (min(w) + max(w))
    sig = k / (0.5 * (max(w) - min(w)))
    return adjoint.Pulse(w0, sig, m * sig, n_steps, tail=n_steps // 8)


def test_pulse_spectrum_is_the_gaussian_transform():
    # Poisson summation: for sigma >> 1 step the DTFT of the samples equals
    # the continuous transform sigma sqrt(2 pi) exp(-(w - w0)^2 sigma^2 / 2)
    # exp(i (w - w0) t0) up to exponentially small terms
    w0, sig, t0, n = 0.15, 60.0, 400.0, 800
    s = fdtd.pulse_samples(n, w0, sig, t0)
    for w in (0.15, 0.16, 0.13, 0.19):
        S = fdtd.pulse_spectrum(s, w)
        ref = sig * math.sqrt(2 * math.pi) * np.exp(-0.5 * ((w - w0) * sig) ** 2) * \
            np.exp(1j * (w - w0) * t0)
        assert abs(S - ref) <= 1e-9 * sig


@pytest.mark.usefixtures("oracle_built")
def test_pulse_phasors_equal_the_time_harmonic_ones():
    dev = configs.micro_demux(n_steps=2600)
    P = default_pulse(dev, 2600)
    rp = adjoint.forward_adjoint_pulse(dev, P)
    rh = adjoint.forward_adjoint(configs.micro_demux(n_steps=4000))
    for f in range(dev.n_freq):
        assert rp.fwd[0][f].resid < 1e-6            # the field has died away
        for a, b in ((rp.fwd[0][f].box, rh.fwd[0][f].box),
                     (rp.adj[1][f].box, rh.adj[1][f].box)):
            assert np.linalg.norm(a - b) / np.linalg.norm(b) < 2e-5
    assert np.abs(rp.alpha - rh.alpha).max() < 2e-5 * np.abs(rh.alpha).max()


@pytest.mark.usefixtures("oracle_built")
def test_truncated_pulse_run_shows_in_the_residual():
    dev = configs.micro_demux(n_steps=1600)
    P = default_pulse(dev, 1600)
    rp = adjoint.forward_adjoint_pulse(dev, P)
    rh = adjoint.forward_adjoint(configs.micro_demux(n_steps=4000))
    err = np.linalg.norm(rp.fwd[0][0].box - rh.fwd[0][0].box) / np.linalg.norm(rh.fwd[0][0].box)
    assert rp.fwd[0][0].resid > 1e-2 and err > 1e-4


@pytest.mark.usefixtures("oracle_built")
def test_pulse_gradient_matches_finite_differences():
    dev = configs.micro_demux(n_steps=2600)
    dev.C = np.random.default_rng(31).uniform(0.3, 0.7, dev.C.shape)
    P = default_pulse(dev, 2600)
    T = np.array([[[1.0, 0.0], [0.0, 1.0]]])

    def F(C):
        a = adjoint.forward_adjoint_pulse(dev, P, C=C).alpha
        return float(np.sum((T - np.abs(a) ** 2) ** 2))

    res = adjoint.forward_adjoint_pulse(dev, P)
    coef = 2.0 * (np.abs(res.alpha) ** 2 - T) * np.conj(res.alpha)
    g = adjoint.grad_C(dev, res, coef)
    h = 1e-4
    for (b, a) in [(0, 0), (2, 2), (4, 1)]:
        Cp, Cm = dev.C.copy(), dev.C.copy()
        Cp[b, a] += h
        Cm[b, a] -= h
        fd = (F(Cp) - F(Cm)) / (2 * h)
        assert g[b, a] == pytest.approx(fd, rel=2e-4, abs=2e-5 * np.abs(g).max())
