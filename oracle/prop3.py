"""Three-dimensional acoustic time stepping and its exact transpose (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

The 3D form of the surface-source problem (Operators section: the acoustic
system, with the source a density on the surface z = z_s; Generalizations
among the paper's closing remarks name 3D as the natural extension).  The
continuous system is that of ``prop`` with a third coordinate y:
(1/kappa) dp/dt = -div v + h_s delta(z - z_s), rho dv/dt = -grad p +
f_s e_z delta(z - z_s), zero initial state, h_s and f_s now functions of
(x, y, t) on the plane z = z_s.

Discrete reading, the 2D one of ``prop`` and ``grid`` extended by one axis
(arrays indexed [z][y][x], x fastest; constant density):

* p on integer nodes, split into p_x + p_y + p_z; v_x, v_y, v_z on the half
  nodes of their own axis; leapfrog, p at t_n, v at t_{n+1/2};
* step n -> n+1:
    v_a <- a v_a - b (dt/rho) D_a^+ p              (a = x, y)
    v_z <- a v_z - b (dt/rho) (D_z^+ p - E_f f[n])
    p_a <- a p_a - b dt kappa D_a^- v_a            (a = x, y)
    p_z <- a p_z - b dt kappa (D_z^- v_z - E_h h[n])
  with each axis's absorbing-layer factors a, b at the field's own
  position (the 2D profile and trapezoidal damping, applied per axis), and
  P[n] = R_p p^{n+1}, V[n] = R_vz v_z^{n+1/2} recorded after the step;
* a plane at depth z is sampled by linear interpolation between the two
  bracketing grid planes; its traces sit on grid columns (x) and rows (y),
  trace index iy * nx_traces + ix; E_h, E_f are the transposes of that
  sampling, the 1/h of the z-delta folded into the coefficients as in 2D.

The transpose runs the transposed sub-updates in reverse order, as in
``prop``.  A y-invariant model and source reduce the central y-slice to the
2D scheme exactly while the y-edges are outside its dependency cone, which
the CPU tests use as a pin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fd


@dataclass
class Plane:
    """Depth rows (with interpolation weights) and the lateral grid indices
    of a sampled plane; ``gather`` is linear interpolation in z, ``spread``
    its transpose."""

    rows: tuple       # ((z index, weight), ...)
    ys: np.ndarray    # y indices of the trace rows
    xs: np.ndarray    # x indices of the trace columns

    @property
    def n(self) -> int:
        return len(self.ys) * len(self.xs)

    def gather(self, field: np.ndarray) -> np.ndarray:
        out = np.zeros((len(self.ys), len(self.xs)))
        for r, w in self.rows:
            out += w * field[r][np.ix_(self.ys, self.xs)]
        return out.ravel()

    def spread_add(self, values: np.ndarray, out: np.ndarray, scale=1.0) -> None:
        v = np.asarray(values, dtype=np.float64).reshape(len(self.ys), len(self.xs))
        for r, w in self.rows:
            out[r][np.ix_(self.ys, self.xs)] += scale * w * v


class Grid3:
    """Physical nz x ny x nx nodes plus L cells of absorbing layer on every
    side, the model extended into the layer by edge replication."""

    def __init__(self, kappa_phys: np.ndarray, rho: float, h: float, dt: float,
                 npml: int, pml_R: float, order: int):
        kappa_phys = np.asarray(kappa_phys, dtype=np.float64)
        if kappa_phys.ndim != 3:
            raise ValueError("kappa must be [nz][ny][nx]")
        self.nz, self.ny, self.nx = kappa_phys.shape
        self.h, self.dt, self.L, self.order = float(h), float(dt), int(npml), int(order)
        L = self.L
        self.NZ, self.NY, self.NX = self.nz + 2 * L, self.ny + 2 * L, self.nx + 2 * L
        self.kappa = np.pad(kappa_phys, L, mode="edge")
        self.rho = float(rho)
        self.cmax = float(np.sqrt(kappa_phys.max() / self.rho))
        smax = 3.0 * self.cmax * math.log(1.0 / pml_R) / (2.0 * L * h) if L > 0 else 0.0

        def sigma(pos, n_phys):
            d = np.maximum(np.maximum(L - pos, pos - (L + n_phys - 1)), 0.0)
            return smax * (d / L) ** 2 if L > 0 else np.zeros_like(pos)

        def ab(s):
            q = 0.5 * s * dt
            return (1.0 - q) / (1.0 + q), 1.0 / (1.0 + q)

        # per axis: factors at nodes (p split) and at half nodes (velocity)
        self.fac = {}
        for ax, N, n in (("z", self.NZ, self.nz), ("y", self.NY, self.ny), ("x", self.NX, self.nx)):
            pos = np.arange(N, dtype=np.float64)
            self.fac[ax] = (ab(sigma(pos, n)), ab(sigma(pos + 0.5, n)))

    def _idx(self, x0: float, n: int, n_phys: int) -> np.ndarray:
        j0 = x0 / self.h
        if abs(j0 - round(j0)) > 1e-9:
            raise ValueError("trace positions must lie on grid nodes")
        idx = self.L + int(round(j0)) + np.arange(n)
        if idx.min() < self.L or idx.max() > self.L + n_phys - 1:
            raise ValueError("plane extends outside the physical grid")
        return idx

    def _rows(self, u: float, lo: int, hi: int):
        i0 = int(math.floor(u + 1e-12))
        w1 = u - i0
        if abs(w1) < 1e-12:
            w1 = 0.0
        rows = ((i0, 1.0 - w1),) if w1 == 0.0 else ((i0, 1.0 - w1), (i0 + 1, w1))
        for r, _ in rows:
            if r < lo or r > hi:
                raise ValueError("plane lies outside the physical grid")
        return rows

    def p_plane(self, z: float, x0: float, nx: int, y0: float, ny: int) -> Plane:
        """Plane on pressure nodes at physical depth z (metres)."""
        u = self.L + z / self.h
        return Plane(self._rows(u, self.L, self.L + self.nz - 1),
                     self._idx(y0, ny, self.ny), self._idx(x0, nx, self.nx))

    def vz_plane(self, z: float, x0: float, nx: int, y0: float, ny: int) -> Plane:
        """Plane on v_z half nodes (z index i holds depth (i - L + 1/2) h)."""
        u = self.L + z / self.h - 0.5
        return Plane(self._rows(u, self.L, self.L + self.nz - 2),
                     self._idx(y0, ny, self.ny), self._idx(x0, nx, self.nx))


_AXIS = {"z": 0, "y": 1, "x": 2}


def _bcast(v, ax):
    shape = [1, 1, 1]
    shape[_AXIS[ax]] = -1
    return v.reshape(shape)


def _setup(g: Grid3):
    c = fd.stencil(g.order)
    Cb = g.dt / (g.rho * g.h)        # (dt/rho) (1/h)
    Ck = g.dt * g.kappa / g.h        # dt kappa (1/h)
    node = {ax: tuple(_bcast(v, ax) for v in g.fac[ax][0]) for ax in "zyx"}
    half = {ax: tuple(_bcast(v, ax) for v in g.fac[ax][1]) for ax in "zyx"}
    return c, Cb, Ck, node, half


def forward3(g: Grid3, nt: int, h_src=None, f_src=None, rec_p=None, rec_v=None,
             energy: bool = False):
    """Run nt steps from rest.

    h_src: (Plane on p nodes, traces [nt][n]) constitutive-defect source.
    f_src: (Plane on v_z nodes, traces [nt][n]) normal-load source.
    rec_p / rec_v: Planes where p^{n+1} / v_z^{n+1/2} are recorded.
    energy: also return, per step, 1/2 sum rho v^{n-1/2} v^{n+1/2} +
    1/2 sum (p^n)^2 / kappa (conserved without absorption once the sources
    stop).
    Returns (P [nt][n_p] or None, V [nt][n_v] or None[, energy list])."""
    c, Cb, Ck, node, half = _setup(g)
    shp = (g.NZ, g.NY, g.NX)
    v = {ax: np.zeros(shp) for ax in "zyx"}
    ps = {ax: np.zeros(shp) for ax in "zyx"}
    P = np.zeros((nt, rec_p.n)) if rec_p is not None else None
    V = np.zeros((nt, rec_v.n)) if rec_v is not None else None
    E = []
    for n in range(nt):
        p = ps["x"] + ps["y"] + ps["z"]
        old = dict(v)
        for ax in "xyz":
            grad = fd.dplus(p, c, axis=_AXIS[ax])
            if ax == "z" and f_src is not None:
                f_src[0].spread_add(f_src[1][n], grad, -1.0)
            a, b = half[ax]
            v[ax] = a * v[ax] - b * Cb * grad
        if energy:
            E.append(0.5 * g.rho * sum(np.sum(old[ax] * v[ax]) for ax in "zyx")
                     + 0.5 * np.sum(p * p / g.kappa))
        for ax in "xyz":
            div = fd.dminus(v[ax], c, axis=_AXIS[ax])
            if ax == "z" and h_src is not None:
                h_src[0].spread_add(h_src[1][n], div, -1.0)
            a, b = node[ax]
            ps[ax] = a * ps[ax] - b * Ck * div
        if P is not None:
            P[n] = rec_p.gather(ps["x"] + ps["y"] + ps["z"])
        if V is not None:
            V[n] = rec_v.gather(v["z"])
    if energy:
        return P, V, E
    return P, V


def adjoint3(g: Grid3, nt: int, h_plane: Plane = None, f_plane: Plane = None,
             rec_p=None, rec_v=None):
    """Exact transpose of :func:`forward3` as a map from the source traces
    (h, f) to the recorded traces (P, V).

    rec_p / rec_v: (Plane, traces [nt][n]) adjoint inputs in the P / V slots.
    Returns (hbar [nt][n_h] or None, fbar [nt][n_f] or None)."""
    c, Cb, Ck, node, half = _setup(g)
    shp = (g.NZ, g.NY, g.NX)
    vb = {ax: np.zeros(shp) for ax in "zyx"}
    pb = {ax: np.zeros(shp) for ax in "zyx"}
    hb = np.zeros((nt, h_plane.n)) if h_plane is not None else None
    fb = np.zeros((nt, f_plane.n)) if f_plane is not None else None
    for n in range(nt - 1, -1, -1):
        # recording: P[n] = R_p (p_x + p_y + p_z), V[n] = R_vz v_z
        if rec_p is not None:
            for ax in "zyx":
                rec_p[0].spread_add(rec_p[1][n], pb[ax])
        if rec_v is not None:
            rec_v[0].spread_add(rec_v[1][n], vb["z"])
        # pressure updates: p_a' = a p_a - b Ck (D_a^- v_a [- E_h h])
        if hb is not None:
            hb[n] = h_plane.gather(node["z"][1] * Ck * pb["z"])
        for ax in "zyx":
            a, b = node[ax]
            vb[ax] = vb[ax] - fd.dminus_T(b * Ck * pb[ax], c, axis=_AXIS[ax])
            pb[ax] = a * pb[ax]
        # velocity updates: v_a' = a v_a - b Cb (D_a^+ p [- E_f f]), p the
        # sum of the three parts
        if fb is not None:
            fb[n] = f_plane.gather(half["z"][1] * Cb * vb["z"])
        t = -sum(fd.dplus_T(half[ax][1] * Cb * vb[ax], c, axis=_AXIS[ax]) for ax in "zyx")
        for ax in "zyx":
            pb[ax] = pb[ax] + t
            vb[ax] = half[ax][0] * vb[ax]
    return hb, fb
