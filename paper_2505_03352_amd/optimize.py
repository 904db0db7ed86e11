"""The optimizer loop of the paper's Sec. 4 on the GPU.

Each iteration: the projection strength from Eq. (14), the design set on the
plan, forward and adjoint runs of every right-hand side, the Eq. (9)
objective F = sum_k (T_k - |alpha_k|^2)^2 and its coefficient
dF/dalpha = 2 (|alpha|^2 - T) conj(alpha), the gradient dF/dC, one Adam step
on the controls (Eqs. (10)-(11), a library kernel), the unbinarity u (the
grey fraction of the design, a library reduction) and the Eq. (15) update of
beta_max.

Readings where the paper is silent: grey means 0.01 < rho < 0.99; t and
beta_max start at their first estimates; while the whole design is grey
(u = 1) there is no estimate and beta stays at beta_min; eps = 1e-8.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from ._abi import YO_BOTH
from .plan import Plan, adam_step


def beta_schedule(i: int, n_iter: int, beta_min: float, beta_max: float) -> float:
    """Eq. (14): exponential-in-(i/N)^2 growth from beta_min to beta_max."""
    return beta_min + (beta_max - beta_min) * (math.exp((i / n_iter) ** 2) - 1.0) / (math.e - 1.0)


@dataclass
class BetaControl:
    """Eq. (15): moving averages (decay gamma) of t = (1/u - 1)/beta and of
    the beta_max that would bring the grey fraction to u0."""
    beta_min: float = 10.0
    gamma: float = 0.95
    u0: float = 0.01
    t: float = float("nan")
    beta_max: float = float("nan")

    def beta(self, i: int, n_iter: int) -> float:
        if math.isnan(self.beta_max):
            return self.beta_min
        return beta_schedule(i, n_iter, self.beta_min, self.beta_max)

    def update(self, u: float, beta: float):
        if u >= 1.0:
            return
        tn = (1.0 / u - 1.0) / beta
        self.t = tn if math.isnan(self.t) else self.gamma * self.t + (1.0 - self.gamma) * tn
        bn = (1.0 / self.u0 - 1.0) / self.t
        self.beta_max = bn if math.isnan(self.beta_max) else (
            self.gamma * self.beta_max + (1.0 - self.gamma) * bn)


def eq9(alpha: torch.Tensor, T: torch.Tensor):
    """(F, dF/dalpha) of Eq. (9) on the device; entries of T that are nan are
    not targeted."""
    use = ~torch.isnan(T)
    d = torch.where(use, alpha.abs() ** 2 - torch.nan_to_num(T), torch.zeros_like(T))
    return (d * d).sum(), (2.0 * d) * alpha.conj()


@dataclass
class History:
    F: List[float] = field(default_factory=list)
    beta: List[float] = field(default_factory=list)
    u: List[float] = field(default_factory=list)
    beta_max: List[float] = field(default_factory=list)
    seconds: List[float] = field(default_factory=list)


def optimize(plan: Plan, C0, T, n_iter: int, iters_total: Optional[int] = None, lr: float = 1e-3,
             b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, beta_min: float = 10.0,
             gamma: float = 0.95, u0: float = 0.01, lo: float = 0.01, hi: float = 0.99,
             chunk: int = 100, use_graph: bool = True, stream=None):
    """Run n_iter iterations on `plan` from controls C0 with targets T
    ([sources][ports][wavelengths], nan = not targeted).  Returns (C, history)
    with C the final controls (device tensor)."""
    dev = plan.device
    N = iters_total or n_iter
    C = torch.as_tensor(np.asarray(C0), dtype=torch.float32, device=dev).contiguous().clone()
    M = torch.zeros_like(C)
    V = torch.zeros_like(C)
    Tt = torch.as_tensor(np.asarray(T), dtype=torch.float32, device=dev)
    ctl = BetaControl(beta_min=beta_min, gamma=gamma, u0=u0)
    h = History()
    for i in range(n_iter):
        t0 = time.perf_counter()
        beta = ctl.beta(i, N)
        plan.set_design(C, beta, stream)
        plan.run(YO_BOTH, chunk=chunk, use_graph=use_graph, stream=stream)
        alpha = plan.alpha(stream)
        F, coef = eq9(alpha, Tt)
        G = plan.gradient(coef, stream)
        u = plan.unbinarity(lo, hi, stream)
        adam_step(C, G, M, V, i + 1, lr, b1, b2, eps, stream)
        Fv, uv = float(F), float(u[0])          # one host synchronisation per iteration
        ctl.update(uv, beta)
        h.F.append(Fv)
        h.beta.append(beta)
        h.u.append(uv)
        h.beta_max.append(ctl.beta_max)
        h.seconds.append(time.perf_counter() - t0)
    return C, h
