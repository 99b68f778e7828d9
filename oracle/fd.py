"""Staggered finite-difference operators with zero extension (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

The paper's simulator is a staggered-grid scheme of order 2 in time and 2k
in space (Numerical Examples, "Synthetic models and simulation").  Pressure
lives on integer nodes, particle velocity on half nodes.  The operators below
omit the 1/h factor; callers multiply by it.

Conventions (index j along the axis the operator acts on):

* ``dplus(p)[j]  = sum_m c_m (p[j+m] - p[j+1-m])``: node field -> half node
  j+1/2 (stored at index j);
* ``dminus(v)[j] = sum_m c_m (v[j+m-1] - v[j-m])``: half-node field -> node j.

Values outside the array are zero (a rigid box), so each operator is a plain
matrix on the stored samples.  Their transposes are written out term by term
from the definition (``*_T`` functions) rather than derived from an identity,
so that the identity D- = -(D+)^T can be checked, not assumed.
"""
from __future__ import annotations

import numpy as np


def stencil(order: int) -> tuple:
    """Staggered first-derivative coefficients c_1..c_k, k = order/2.

    They are the unique weights for which sum_m c_m ((m-1/2)^q - (1/2-m)^q)
    equals the derivative of x^q at 0 for q = 1..2k-1 (odd q; even q vanish
    by symmetry): solved here from that moment system, not tabulated."""
    if order % 2 or order < 2:
        raise ValueError("order must be even and >= 2")
    k = order // 2
    # unknowns c_m; equations: sum_m c_m * 2 (m - 1/2)^(2q-1) = delta_{q,1}
    A = np.array([[2.0 * (m - 0.5) ** (2 * q - 1) for m in range(1, k + 1)]
                  for q in range(1, k + 1)])
    rhs = np.zeros(k)
    rhs[0] = 1.0
    return tuple(np.linalg.solve(A, rhs))


def _add_shifted(out, u, coef, off, axis):
    """out[j] += coef * u[j + off] along ``axis``, with u taken as zero
    outside its index range."""
    n = u.shape[axis]
    lo, hi = max(0, -off), min(n, n - off)
    if lo >= hi:
        return
    dst = [slice(None)] * u.ndim
    src = [slice(None)] * u.ndim
    dst[axis] = slice(lo, hi)
    src[axis] = slice(lo + off, hi + off)
    out[tuple(dst)] += coef * u[tuple(src)]


def _shift_sum(u, c, axis, offsets_pos, offsets_neg):
    """sum_m c_m (u[j + offsets_pos[m]] - u[j + offsets_neg[m]]) with zeros
    outside the array, along ``axis``."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros_like(u)
    for cm, op, on in zip(c, offsets_pos, offsets_neg):
        _add_shifted(out, u, cm, op, axis)
        _add_shifted(out, u, -cm, on, axis)
    return out


def dplus(p, c, axis):
    k = len(c)
    return _shift_sum(p, c, axis, [m for m in range(1, k + 1)],
                      [1 - m for m in range(1, k + 1)])


def dminus(v, c, axis):
    k = len(c)
    return _shift_sum(v, c, axis, [m - 1 for m in range(1, k + 1)],
                      [-m for m in range(1, k + 1)])


def _scatter_sum(u, c, axis, offsets_pos, offsets_neg):
    """Transpose of _shift_sum: each forward term out[j] += c u_in[j+o]
    becomes out_T[j+o] += c u[j], i.e. out_T[i] += c u[i-o]."""
    return _shift_sum(u, c, axis, [-o for o in offsets_pos],
                      [-o for o in offsets_neg])


def dplus_T(u, c, axis):
    k = len(c)
    return _scatter_sum(u, c, axis, [m for m in range(1, k + 1)],
                        [1 - m for m in range(1, k + 1)])


def dminus_T(u, c, axis):
    k = len(c)
    return _scatter_sum(u, c, axis, [m - 1 for m in range(1, k + 1)],
                        [-m for m in range(1, k + 1)])
