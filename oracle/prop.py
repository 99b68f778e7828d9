"""Time stepping of the acoustic system and its exact transpose (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

Continuous system (Operators section, the acoustic wave operator and the
causal surface-source problem): (1/kappa) dp/dt = -div v + h_s delta(z-z_s),
rho dv/dt = -grad p + f_s e_z delta(z-z_s), zero initial state.

Discrete reading (leapfrog, p at t_n = n dt, v at t_{n+1/2}); step n -> n+1:

  v_x <- a v_x - b (dt/rho) D_x^+ p
  v_z <- a v_z - b (dt/rho) (D_z^+ p - E_f f[n])
  p_x <- a p_x - b dt kappa D_x^- v_x
  p_z <- a p_z - b dt kappa (D_z^- v_z - E_h h[n])
  p    = p_x + p_z

with a, b the absorbing-layer factors at each field's own position, E_h and
E_f the transposes of linear interpolation onto p and v_z nodes divided by h
(a line density of the delta function), and traces recorded after the step:
P[n] = R_p p^{n+1}, V[n] = R_vz v_z^{n+1/2}.

The adjoint is the transpose of the whole time loop under the Euclidean
inner product on trace arrays, obtained by transposing each sub-update and
running them in reverse order (the discrete counterpart of the adjoint-state
identity of the Operators section and Appendix A).  No forward states are
stored: the map is linear in the sources.
"""
from __future__ import annotations

import numpy as np

from . import fd
from .grid import Grid, Line


def _coefs(g: Grid):
    """Stencil, velocity coefficients (dt/rho) (1/h) for v_x and v_z (one
    scalar for constant density; arrays of the buoyancy at each velocity's
    own half node otherwise), Ck and the layer factors."""
    c = fd.stencil(g.order)
    if not getattr(g, "variable_rho", False):
        Cbx = Cbz = g.dt / (g.rho * g.h)     # (dt/rho) * (1/h)
    else:
        Cbx = g.dt * g.bx / g.h               # dt b_x * (1/h)
        Cbz = g.dt * g.bz / g.h
    Ck = g.dt * g.kappa / g.h        # dt kappa * (1/h)
    ax_n, bx_n = g.ax_n[None, :], g.bx_n[None, :]
    ax_h, bx_h = g.ax_h[None, :], g.bx_h[None, :]
    az_n, bz_n = g.az_n[:, None], g.bz_n[:, None]
    az_h, bz_h = g.az_h[:, None], g.bz_h[:, None]
    return c, (Cbx, Cbz), Ck, (ax_n, bx_n, ax_h, bx_h, az_n, bz_n, az_h, bz_h)


def forward(g: Grid, nt: int, h_src=None, f_src=None, rec_p=None, rec_v=None,
            energy: bool = False, div_out: list = None):
    """Run nt steps from rest.

    h_src: (Line on p nodes, traces [nt][n]) constitutive-defect source.
    f_src: (Line on v_z nodes, traces [nt][n]) normal-load source.
    rec_p / rec_v: Lines where p^{n+1} / v_z^{n+1/2} are recorded.
    div_out: if a list, receives for every step n the array that the
    pressure update multiplies by Ck, D^- v^{n+1/2} - E_h h^n (the layer's
    split parts summed).
    Returns (P [nt][n_p] or None, V [nt][n_v] or None[, energy list])."""
    c, (Cbx, Cbz), Ck, (ax_n, bx_n, ax_h, bx_h, az_n, bz_n, az_h, bz_h) = _coefs(g)
    shp = (g.NZ, g.NX)
    vx, vz, px, pz = (np.zeros(shp) for _ in range(4))
    # density at the velocity nodes, for the energy: rho_x = 1/b_x
    rho_x = 1.0 / g.bx if getattr(g, "variable_rho", False) else g.rho
    rho_z = 1.0 / g.bz if getattr(g, "variable_rho", False) else g.rho
    P = np.zeros((nt, len(rec_p.cols))) if rec_p is not None else None
    V = np.zeros((nt, len(rec_v.cols))) if rec_v is not None else None
    E = []
    for n in range(nt):
        p = px + pz
        vx_old, vz_old = vx, vz
        vx = ax_h * vx - bx_h * Cbx * fd.dplus(p, c, axis=1)
        gz = fd.dplus(p, c, axis=0)
        if f_src is not None:
            f_src[0].spread_add(f_src[1][n], gz, -1.0)   # D_z^+ p - E_f f (h folded)
        vz = az_h * vz - bz_h * Cbz * gz
        if energy:
            # E^{n-1/2}... recorded as 1/2 sum rho v^{n-1/2} v^{n+1/2}
            # + 1/2 sum p^n p^n / kappa (conserved for sigma = 0), rho at
            # each velocity's own node
            E.append(0.5 * np.sum(rho_x * vx_old * vx + rho_z * vz_old * vz)
                     + 0.5 * np.sum(p * p / g.kappa))
        px = ax_n * px - bx_n * Ck * fd.dminus(vx, c, axis=1)
        dz = fd.dminus(vz, c, axis=0)
        if h_src is not None:
            h_src[0].spread_add(h_src[1][n], dz, -1.0)   # D_z^- v_z - E_h h
        pz = az_n * pz - bz_n * Ck * dz
        if div_out is not None:
            div_out.append(fd.dminus(vx, c, axis=1) + dz)
        if P is not None:
            P[n] = rec_p.gather(px + pz)
        if V is not None:
            V[n] = rec_v.gather(vz)
    if energy:
        return P, V, E
    return P, V


def adjoint(g: Grid, nt: int, h_line: Line = None, f_line: Line = None,
            rec_p=None, rec_v=None, on_p=None):
    """Exact transpose of :func:`forward` as a map from the source traces
    (h, f) to the recorded traces (P, V).

    rec_p / rec_v: (Line, traces [nt][n]) adjoint inputs in the P / V slots.
    on_p: if given, called as on_p(n, pxb, pzb) with the adjoint variables
    of p_x^{n+1} and p_z^{n+1} (the recording of step n included), before
    the transposed pressure update of step n.
    Returns (hbar [nt][n_h] or None, fbar [nt][n_f] or None)."""
    c, (Cbx, Cbz), Ck, (ax_n, bx_n, ax_h, bx_h, az_n, bz_n, az_h, bz_h) = _coefs(g)
    shp = (g.NZ, g.NX)
    vxb, vzb, pxb, pzb = (np.zeros(shp) for _ in range(4))
    hb = np.zeros((nt, len(h_line.cols))) if h_line is not None else None
    fb = np.zeros((nt, len(f_line.cols))) if f_line is not None else None
    for n in range(nt - 1, -1, -1):
        # recording P[n] = R_p (p_x + p_z), V[n] = R_vz v_z
        if rec_p is not None:
            rec_p[0].spread_add(rec_p[1][n], pxb)
            rec_p[0].spread_add(rec_p[1][n], pzb)
        if rec_v is not None:
            rec_v[0].spread_add(rec_v[1][n], vzb)
        if on_p is not None:
            on_p(n, pxb, pzb)
        # p_z update: pz' = az_n pz - bz_n Ck D_z^- vz + bz_n Ck E_h h
        if hb is not None:
            hb[n] = h_line.gather(bz_n * Ck * pzb)
        vxb = vxb - fd.dminus_T(bx_n * Ck * pxb, c, axis=1)
        vzb = vzb - fd.dminus_T(bz_n * Ck * pzb, c, axis=0)
        pxb = ax_n * pxb
        pzb = az_n * pzb
        # v_z update: vz' = az_h vz - bz_h Cb D_z^+ p + bz_h Cb E_f f
        if fb is not None:
            fb[n] = f_line.gather(bz_h * Cbz * vzb)
        t = -(fd.dplus_T(bx_h * Cbx * vxb, c, axis=1)
              + fd.dplus_T(bz_h * Cbz * vzb, c, axis=0))
        pxb = pxb + t
        pzb = pzb + t
        vxb = ax_h * vxb
        vzb = az_h * vzb
    return hb, fb
