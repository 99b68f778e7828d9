"""The 3D surface-source subproblem operators (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

The 2D operators of ``ops`` with a source plane instead of a line
(Introduction: the penalised problem esisp; Accelerated Iterative
Inversion: the preconditioner defprecond; Computing and Symmetrizing
Lambda: the thin-slab composition winvcomp), on the 3D stepping of
``prop3``:

* F h: pressure source on the plane z = z_s, pressure traces on z = z_r;
* A: multiplication by the lateral distance from the physical point,
  sqrt((x - x_s)^2 + (y - y_s)^2), on the source plane;
* W^-1 = s X^T J X on the thin slab around z_s: X a normal-load source on
  z_s recorded as pressure and normal velocity on the datum plane slab_dz
  cells away, J the exchange of the two records, s = 4 sign(slab_dz);
* M^-1 = D W^-1 D, D = (1 + alpha_hat^2 A^2)^(-1/2);
* N = F^T F + alpha^2 A^2, and Algorithm 1 on N h = F^T d with
  alpha = alpha_rel ||F^T d|| / ||d||, as in 2D (``ops.pcg``).
"""
from __future__ import annotations

import math

import numpy as np

from .ops import pcg
from .prop3 import Grid3, adjoint3, forward3


class Model3:
    """The full-grid and thin-slab discretisations of one 3D problem
    (``inputs.Problem3`` with slab_dz, x_s, y_s)."""

    def __init__(self, prob, kappa, rho: float):
        self.prob = prob
        kappa = np.asarray(kappa, dtype=np.float64)
        if kappa.shape != (prob.nz, prob.ny, prob.nx):
            raise ValueError("kappa must be [nz][ny][nx]")
        g = Grid3(kappa, rho, prob.h, prob.dt, prob.npml, prob.pml_R, prob.order)
        self.full = g
        self.h_plane = g.p_plane(prob.z_src, prob.x_src0, prob.nsx, prob.y_src0, prob.nsy)
        self.r_plane = g.p_plane(prob.z_rec, prob.x_rec0, prob.nrx, prob.y_rec0, prob.nry)
        # the thin slab around z_s: physical planes from min(i, i + dz) - k
        # to max(i, i + dz) + k (i the plane at or above z_s, one more below
        # when z_s falls between planes, k = order/2), the model planes
        # copied from the full model (clamped at its top and bottom), plus
        # the absorbing layer, as in 2D
        k = prob.order // 2
        dz = int(prob.slab_dz)
        if dz == 0:
            raise ValueError("slab datum offset must be nonzero")
        i_s = int(math.floor(prob.z_src / prob.h + 1e-12))
        i_lo = min(i_s, i_s + dz) - k
        i_hi = max(i_s, i_s + dz) + k + (1 if prob.z_src / prob.h - i_s > 1e-12 else 0)
        rows = np.clip(np.arange(i_lo, i_hi + 1), 0, prob.nz - 1)
        gs = Grid3(kappa[rows], rho, prob.h, prob.dt, prob.npml, prob.pml_R, prob.order)
        self.slab = gs
        zl = prob.z_src - i_lo * prob.h
        zd = zl + dz * prob.h
        lat = (prob.x_src0, prob.nsx, prob.y_src0, prob.nsy)
        self.f_plane = gs.vz_plane(zl, *lat)
        self.d_p = gs.p_plane(zd, *lat)
        self.d_v = gs.vz_plane(zd, *lat)

    def fwd(self, h):
        """d = F h, h [nt][ns] -> d [nt][nr] (ns = nsx nsy, nr = nrx nry)."""
        P, _ = forward3(self.full, self.prob.nt, h_src=(self.h_plane, h), rec_p=self.r_plane)
        return P

    def adj(self, r):
        """g = F^T r, r [nt][nr] -> g [nt][ns]."""
        hb, _ = adjoint3(self.full, self.prob.nt, h_plane=self.h_plane,
                         rec_p=(self.r_plane, r))
        return hb

    def slab_fwd(self, f):
        """X f = (P, V): normal load f on z_s, datum pressure and v_z."""
        return forward3(self.slab, self.prob.nt, f_src=(self.f_plane, f), rec_p=self.d_p,
                        rec_v=self.d_v)

    def slab_adj(self, a, b):
        """X^T (a, b): a in the datum-pressure slot, b in the datum-v_z slot,
        read from the normal-load slot."""
        _, fb = adjoint3(self.slab, self.prob.nt, f_plane=self.f_plane,
                         rec_p=(self.d_p, a), rec_v=(self.d_v, b))
        return fb

    def winv(self, g):
        """s X^T J X g, J (P, V) = (V, P), s = 4 sign(slab_dz)."""
        P, V = self.slab_fwd(g)
        return 4.0 * math.copysign(1.0, self.prob.slab_dz) * self.slab_adj(V, P)


def lateral_distance3(prob) -> np.ndarray:
    """Distance of each source-plane trace (x_src0 + a h, y_src0 + b h),
    index b nsx + a, from the physical point (x_s, y_s)."""
    x = prob.x_src0 + prob.h * np.arange(prob.nsx)
    y = prob.y_src0 + prob.h * np.arange(prob.nsy)
    return np.sqrt((x[None, :] - prob.x_s) ** 2 + (y[:, None] - prob.y_s) ** 2).ravel()


def penalty3(prob, x):
    """(A x)[n][t] = dist_t x[n][t]."""
    return lateral_distance3(prob)[None, :] * x


def dscale3(prob, alpha_hat: float) -> np.ndarray:
    """Diagonal of D = (1 + alpha_hat^2 dist^2)^(-1/2)."""
    a = lateral_distance3(prob)
    return 1.0 / np.sqrt(1.0 + (alpha_hat * a) ** 2)


def precond3(model: Model3, alpha_hat: float, r):
    """M^-1 r = D W^-1 (D r)."""
    d = dscale3(model.prob, alpha_hat)[None, :]
    return d * model.winv(d * r)


def normal3(model: Model3, alpha: float, p):
    """N p = F^T F p + alpha^2 A^T A p; also returns F p."""
    Fp = model.fwd(p)
    Ap = penalty3(model.prob, p)
    return model.adj(Fp) + alpha * alpha * penalty3(model.prob, Ap), Fp


def pcg_solve3(model: Model3, d, alpha_rel: float, K: int, use_precond: bool = True):
    """b = F^T d, alpha = alpha_rel ||b|| / ||d||, K iterations of
    Algorithm 1 on N h = b with M^-1 = D W^-1 D (alpha_hat = alpha_rel) or
    M = I.  Returns (h_K, history, alpha) as ``ops.pcg_solve``."""
    b = model.adj(d)
    alpha = alpha_rel * math.sqrt(float(np.sum(b * b))) / math.sqrt(float(np.sum(d * d)))
    if use_precond:
        def apply_Minv(r):
            return precond3(model, alpha_rel, r)
    else:
        def apply_Minv(r):
            return r.copy()
    h, hist = pcg(lambda p: normal3(model, alpha, p), apply_Minv, b, K, d_misfit=d)
    return h, hist, alpha
