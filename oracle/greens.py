"""Closed-form 2D homogeneous response to a point pressure source (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

For constant kappa and rho, a point constitutive-defect source w(t) at the
origin, (1/kappa) dp/dt + div v = w(t) delta(x), gives the scalar wave
equation p_tt - c^2 Lap p = kappa w'(t) delta(x) (eliminate v from the
acoustic system of the Operators section).  With the 2D causal Green's
function G(r, t) = H(ct - r) / (2 pi c sqrt(c^2 t^2 - r^2)),

    p(r, t) = kappa (w' * G)(r, t).

The substitution tau = (r/c) cosh(u) removes the square-root singularity:
G(r, tau) dtau = du / (2 pi c^2), so

    p(r, t) = (rho / (2 pi)) int_0^{acosh(ct/r)} w'(t - (r/c) cosh u) du

(using kappa / c^2 = rho), a smooth integrand evaluated here by composite
Gauss-Legendre quadrature.  It assumes w vanishes for t <= 0.
"""
from __future__ import annotations

import math

import numpy as np


def point_source_pressure(r: float, t: np.ndarray, c: float, rho: float,
                          wdot, nodes: int = 64, panels: int = 64) -> np.ndarray:
    """p(r, t) for the source derivative ``wdot`` (callable on arrays)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    for i, ti in enumerate(t):
        if c * ti <= r:
            continue
        U = math.acosh(c * ti / r)
        edges = np.linspace(0.0, U, panels + 1)
        acc = 0.0
        for a, b in zip(edges[:-1], edges[1:]):
            u = 0.5 * (b - a) * xg + 0.5 * (b + a)
            acc += 0.5 * (b - a) * np.sum(wg * wdot(ti - (r / c) * np.cosh(u)))
        out[i] = rho / (2.0 * math.pi) * acc
    return out
