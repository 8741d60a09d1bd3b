"""Balakrishnan sinc-quadrature shift schedule (oracle, FP64).

Paper passages followed:

* eq. balakrishnan_integral: L^{-beta} = sin(pi beta)/pi int_0^inf
  s^{-beta} (L + s I)^{-1} ds.
* eq. coefficients: y_l = l k, c_const = pi / (2 k sin(pi beta)),
  c_I = c_const exp(-2 beta y_l), c_L = c_I exp(2 y_l), and
  L^{-beta} ~ sum_{l=-K^-}^{K^+} (c_I I + c_L L)^{-1}.
* "Strong error" subsection: the default step k = -1/(beta ln h) and the
  limits K^- = ceil(pi^2 / (4 k^2 beta)), K^+ = ceil(pi^2 / (4 k^2 (1-beta))).

Reading: the sum runs over l = -K^- .. K^+ in increasing order.
"""

from __future__ import annotations

import math

import numpy as np


def paper_step(beta: float, h: float) -> float:
    """k = -1/(beta ln h)."""
    return -1.0 / (beta * math.log(h))


def limits(beta: float, k: float) -> tuple[int, int]:
    """(K^-, K^+) by the paper's rule."""
    km = math.ceil(math.pi ** 2 / (4.0 * k * k * beta))
    kp = math.ceil(math.pi ** 2 / (4.0 * k * k * (1.0 - beta)))
    return int(km), int(kp)


def shifts(beta: float, k: float, k_minus: int | None = None, k_plus: int | None = None):
    """Return (l, c_I, c_L) arrays for l = -K^- .. K^+ (increasing)."""
    if not (0.0 < beta < 1.0):
        raise ValueError("beta must lie in (0, 1)")
    if not (k > 0.0 and math.isfinite(k)):
        raise ValueError("quadrature step must be positive")
    km, kp = limits(beta, k)
    if k_minus is not None and k_minus >= 0:
        km = int(k_minus)
    if k_plus is not None and k_plus >= 0:
        kp = int(k_plus)
    l = np.arange(-km, kp + 1, dtype=np.int64)
    c_const = math.pi / (2.0 * k * math.sin(math.pi * beta))
    y = l.astype(np.float64) * k
    c_I = c_const * np.exp(-2.0 * beta * y)
    c_L = c_I * np.exp(2.0 * y)
    return l, c_I, c_L


def q_k(lam, beta: float, k: float, k_minus: int | None = None, k_plus: int | None = None):
    """Scalar quadrature applied to an eigenvalue: sum_l 1/(c_I + c_L lam).
    This is what the discrete method applies to each generalised eigenvector,
    and it tends to lam^{-beta} as k -> 0."""
    _, c_I, c_L = shifts(beta, k, k_minus, k_plus)
    lam = np.asarray(lam, dtype=np.float64)
    out = np.zeros_like(lam)
    for ci, cl in zip(c_I, c_L):
        out = out + 1.0 / (ci + cl * lam)
    return out
