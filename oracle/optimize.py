"""Optimizer loop of the paper's Sec. 4 in FP64.  TEST INFRASTRUCTURE ONLY.

* Objective, Eq. (9): F = sum_k (T_k - |alpha_k|^2)^2 over the modal
  transmissions of interest; its holomorphic Wirtinger derivative
  dF/dalpha_k = 2 (|alpha_k|^2 - T_k) conj(alpha_k) is the coefficient the
  adjoint gradient takes.
* Adam, Eqs. (10)-(11): moving averages M, V of the gradient and its square,
  bias-corrected by 1 - b^i, step -eta Mhat / (sqrt(Vhat) + eps).
* Projection strength, Eqs. (14)-(15): beta_i = beta_min + (beta_max -
  beta_min) (exp((i/N)^2) - 1) / (e - 1), with beta_max re-estimated each
  iteration from the unbinarity u through moving averages (decay gamma):
  t <- gamma t + (1 - gamma) (1/u - 1) / beta and beta_max <- gamma beta_max
  + (1 - gamma) (1/u0 - 1) / t.
* Unbinarity u: the fraction of grey design sub-pixels.

Readings where the paper is silent: a sub-pixel is grey when 0.01 < rho <
0.99 (rho after projection, design area of the high-resolution canvas);
the moving averages t and beta_max start at their first targets (the first
update has no history to average with); while every sub-pixel is grey
(u = 1, e.g. the uniform start C = 1/2) there is no estimate and beta stays
at beta_min; eps = 1e-8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import adjoint, chain


def objective_eq9(alpha: np.ndarray, T: np.ndarray):
    """(F, dF/dalpha) for Eq. (9); entries with T = nan are not targeted."""
    a = np.asarray(alpha, np.complex128)
    T = np.asarray(T, np.float64)
    use = ~np.isnan(T)
    d = np.where(use, np.abs(a) ** 2 - np.nan_to_num(T), 0.0)
    return float(np.sum(d ** 2)), 2.0 * d * np.conj(a)


def adam_step(C, G, M, V, i, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Step i (from 1) of Adam: returns (C, M, V)."""
    M = b1 * M + (1.0 - b1) * G
    V = b2 * V + (1.0 - b2) * G * G
    mh = M / (1.0 - b1 ** i)
    vh = V / (1.0 - b2 ** i)
    return C - lr * mh / (np.sqrt(vh) + eps), M, V


def beta_schedule(i: int, n_iter: int, beta_min: float, beta_max: float) -> float:
    """Eq. (14)."""
    return beta_min + (beta_max - beta_min) * (math.exp((i / n_iter) ** 2) - 1.0) / (math.e - 1.0)


@dataclass
class BetaControl:
    """Eq. (15): moving averages t and beta_max."""
    beta_min: float = 10.0
    gamma: float = 0.95
    u0: float = 0.01
    t: float = float("nan")
    beta_max: float = float("nan")

    def update(self, u: float, beta: float):
        if u >= 1.0:
            return        # an all-grey design says nothing about the beta it needs
        t_new = (1.0 / u - 1.0) / beta
        self.t = t_new if math.isnan(self.t) else self.gamma * self.t + (1.0 - self.gamma) * t_new
        bm_new = (1.0 / self.u0 - 1.0) / self.t
        self.beta_max = (bm_new if math.isnan(self.beta_max)
                         else self.gamma * self.beta_max + (1.0 - self.gamma) * bm_new)


def unbinarity(rho_design: np.ndarray, lo: float = 0.01, hi: float = 0.99) -> float:
    r = np.asarray(rho_design)
    return float(np.count_nonzero((r > lo) & (r < hi))) / r.size


def design_rho(dev, st: chain.ChainState) -> np.ndarray:
    """Projected density on the design area of the canvas."""
    S = dev.supersample
    return st.rho[2 * S:2 * S + S * dev.nd, 2 * S:2 * S + S * dev.md]


@dataclass
class History:
    F: List[float] = field(default_factory=list)
    beta: List[float] = field(default_factory=list)
    u: List[float] = field(default_factory=list)
    beta_max: List[float] = field(default_factory=list)
    C: List[np.ndarray] = field(default_factory=list)


def optimize(dev, T, n_iter: int, iters_total: int = None, lr: float = 1e-3, b1: float = 0.9,
             b2: float = 0.999, eps: float = 1e-8, beta_min: float = 10.0, gamma: float = 0.95,
             u0: float = 0.01, lo: float = 0.01, hi: float = 0.99) -> History:
    """n_iter iterations of: beta from Eq. (14) -> forward + adjoint runs ->
    Eq. (9) and its gradient -> Adam on C -> u -> Eq. (15).  The schedule
    length N is iters_total (default n_iter)."""
    N = iters_total or n_iter
    C = np.asarray(dev.C, np.float64).copy()
    M = np.zeros_like(C)
    V = np.zeros_like(C)
    ctl = BetaControl(beta_min=beta_min, gamma=gamma, u0=u0)
    h = History()
    for i in range(n_iter):
        beta = beta_min if math.isnan(ctl.beta_max) else beta_schedule(i, N, beta_min, ctl.beta_max)
        res = adjoint.forward_adjoint(dev, C, beta)
        F, coef = objective_eq9(res.alpha, T)
        G = adjoint.grad_C(dev, res, coef)
        u = unbinarity(design_rho(dev, res.state), lo, hi)
        h.F.append(F)
        h.beta.append(beta)
        h.u.append(u)
        C, M, V = adam_step(C, G, M, V, i + 1, lr, b1, b2, eps)
        ctl.update(u, beta)
        h.beta_max.append(ctl.beta_max)
        h.C.append(C.copy())
    return h
