"""Padded grid, absorbing-layer profiles and line geometry (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

Readings of the paper (Numerical Examples, "Synthetic models and
simulation": staggered scheme, PML-type absorbing layer on all sides, linear
interpolation for sampling and its adjoint for injection; the paper gives no
layer parameters):

* the absorbing layer of L cells is added outside the stated physical grid;
  the model is extended into it by copying the nearest physical value;
* density may vary (the operators of the paper carry both kappa and rho):
  rho is given at the pressure nodes and each velocity update uses, at its
  own half node, the mean of the density at its two nodes (the mean density
  of the cell between them, which the momentum equation integrated over
  that cell needs when a jump lies between the nodes); a half node beyond
  the last node takes that node's value;
* it is a split-field PML with profile sigma(d) = sigma_max (d / (L h))^2,
  d the distance into the layer, sigma_max = 3 c_max ln(1/R) / (2 L h);
* a field subject to damping sigma advances as
  u' = a u + b dt (rhs), a = (1 - sigma dt/2)/(1 + sigma dt/2),
  b = 1/(1 + sigma dt/2) (trapezoidal treatment of the damping term);
* a line at depth z is sampled by linear interpolation between the two
  grid rows that bracket it (on p nodes or on v_z half nodes), lateral
  positions lie on grid columns.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Line:
    """Rows (with interpolation weights) and columns of a sampled line on a
    padded grid.  ``gather`` is linear interpolation, ``spread`` its
    transpose."""

    rows: tuple  # ((row, weight), ...)
    cols: np.ndarray  # int column indices, one per trace

    def gather(self, field: np.ndarray) -> np.ndarray:
        out = np.zeros(len(self.cols))
        for r, w in self.rows:
            out += w * field[r, self.cols]
        return out

    def spread(self, values: np.ndarray, shape) -> np.ndarray:
        out = np.zeros(shape)
        self.spread_add(values, out)
        return out

    def spread_add(self, values: np.ndarray, out: np.ndarray, scale=1.0) -> None:
        """out += scale * spread(values), in place."""
        for r, w in self.rows:
            out[r, self.cols] += scale * w * values


class Grid:
    """A padded computational grid: physical nz x nx nodes plus L cells of
    absorbing layer on each side."""

    def __init__(self, kappa_phys: np.ndarray, rho, h: float, dt: float,
                 npml: int, pml_R: float, order: int):
        """rho: a constant density or an array [nz][nx] at the physical
        nodes."""
        kappa_phys = np.asarray(kappa_phys, dtype=np.float64)
        self.nz, self.nx = kappa_phys.shape
        self.h, self.dt = float(h), float(dt)
        self.L = int(npml)
        self.order = int(order)
        L = self.L
        self.NZ, self.NX = self.nz + 2 * L, self.nx + 2 * L
        # edge replication of the model into the layer
        self.kappa = np.pad(kappa_phys, L, mode="edge")
        if np.ndim(rho) == 0:
            self.rho = float(rho)
            self.variable_rho = False
            cmax = float(np.sqrt(kappa_phys.max() / self.rho))
        else:
            rho_phys = np.asarray(rho, dtype=np.float64)
            if rho_phys.shape != kappa_phys.shape:
                raise ValueError("rho must be a scalar or an array shaped like kappa")
            self.variable_rho = True
            self.rho = r = np.pad(rho_phys, L, mode="edge")
            # density at (i, j+1/2) and (i+1/2, j): mean of the two nodes;
            # the velocity updates use its reciprocal (the buoyancy)
            rnx = np.concatenate([r[:, 1:], r[:, -1:]], axis=1)
            rnz = np.concatenate([r[1:, :], r[-1:, :]], axis=0)
            self.bx = 1.0 / (0.5 * (r + rnx))
            self.bz = 1.0 / (0.5 * (r + rnz))
            cmax = float(np.sqrt((kappa_phys / rho_phys).max()))
        self.cmax = cmax
        if L > 0:
            smax = 3.0 * cmax * math.log(1.0 / pml_R) / (2.0 * L * h)
        else:
            smax = 0.0

        def sigma(pos, n_phys):
            # pos: coordinate in cell units on the padded axis; physical
            # nodes occupy [L, L + n_phys - 1]
            d = np.maximum(np.maximum(L - pos, pos - (L + n_phys - 1)), 0.0)
            if L == 0:
                return np.zeros_like(pos)
            return smax * (d / L) ** 2

        def ab(s):
            q = 0.5 * s * dt
            return (1.0 - q) / (1.0 + q), 1.0 / (1.0 + q)

        jn = np.arange(self.NX, dtype=np.float64)
        iN = np.arange(self.NZ, dtype=np.float64)
        self.ax_n, self.bx_n = ab(sigma(jn, self.nx))        # p, x-split
        self.ax_h, self.bx_h = ab(sigma(jn + 0.5, self.nx))  # v_x at j+1/2
        self.az_n, self.bz_n = ab(sigma(iN, self.nz))        # p, z-split
        self.az_h, self.bz_h = ab(sigma(iN + 0.5, self.nz))  # v_z at i+1/2
        self.sigma_max = smax

    # -- lines -------------------------------------------------------------
    def _cols(self, x0: float, n: int) -> np.ndarray:
        j0 = x0 / self.h
        if abs(j0 - round(j0)) > 1e-9:
            raise ValueError("line positions must lie on grid columns")
        cols = self.L + int(round(j0)) + np.arange(n)
        if cols.min() < self.L or cols.max() > self.L + self.nx - 1:
            raise ValueError("line extends outside the physical grid")
        return cols

    def _rows(self, u: float, lo: int, hi: int):
        i0 = int(math.floor(u + 1e-12))
        w1 = u - i0
        if abs(w1) < 1e-12:
            w1 = 0.0
        rows = ((i0, 1.0 - w1),) if w1 == 0.0 else ((i0, 1.0 - w1), (i0 + 1, w1))
        for r, _ in rows:
            if r < lo or r > hi:
                raise ValueError("line lies outside the physical grid")
        return rows

    def p_line(self, z: float, x0: float, n: int) -> Line:
        """Line on pressure nodes at physical depth z (metres)."""
        u = self.L + z / self.h
        return Line(self._rows(u, self.L, self.L + self.nz - 1), self._cols(x0, n))

    def vz_line(self, z: float, x0: float, n: int) -> Line:
        """Line on v_z half nodes (row i holds depth (i - L + 1/2) h)."""
        u = self.L + z / self.h - 0.5
        return Line(self._rows(u, self.L, self.L + self.nz - 2), self._cols(x0, n))
