"""The surface-source subproblem operators and PCG (oracle).

TEST INFRASTRUCTURE ONLY -- see the package header.

* F   = S^+_{z_s,z_r}: pressure source on the line z = z_s to pressure trace
        on z = z_r (Operators section, definition of S as the (0,0) block of
        the vector modelling operator).
* F^T: its exact discrete transpose (adjoint-state identity of the Operators
        section; Appendix A).
* A:   multiplication by the lateral distance |x - x_s| to the physical
        source (Introduction, the penalty operator).
* M^-1 = D W^-1 D with D = (I + a^2 A^T A)^(-1/2) (Accelerated Iterative
        Inversion, the preconditioner) and W^-1 the symmetrised
        pressure-to-source operator computed on a thin slab by one forward
        and one adjoint simulation with the pressure/velocity exchange in
        between (Computing and Symmetrizing Lambda, the W_m^-1 formula and
        the thin-slab datum of the lamnear approximation).
* N   = F^T F + alpha^2 A^T A, the Euclidean normal operator of the penalised
        least-squares problem (Operators section, the esisp problem).
* pcg: Algorithm 1 (standard preconditioned CG, h_0 = 0).
* N_w = F^T W_d F + alpha^2 A^T W_m A with b = F^T W_d d, the normal
        equations in the weighted norms (Accelerated Iterative Inversion,
        the normpart system), W_d the receiver-surface counterpart of W^-1
        and W_m the symmetrised inverse pressure-to-source operator (the
        wcomp formula), both on thin slabs.
* the four blocks of the vector modelling operator (pressure source or
        normal load on z_s to pressure or normal velocity on z_r), F and
        V among them;
* V   = normal load on z_s to normal velocity on z_r (the vdef operator),
        its transpose, the time-reversal inverse 4 V^T of F (Time Reversal,
        the approxinv relations), and Lambda~ with its transpose on either
        thin slab (the lamtilde and lamtransp formulas).

Readings where the paper is silent or inconsistent are listed with the
design notes; the ones that change results here are: the Euclidean normal
equations, alpha = alpha_rel ||F^T d|| / ||d|| with alpha_rel itself inside
D, and the slab scale s = 4 sign(dz) (the paper's -4 on its own datum side);
for the weighted system, W_m on the source-side slab with scale sign(dz)
(positive, and inverse to W^-1 on plane waves) and alpha taken per unit
length in both the penalty and D.
"""
from __future__ import annotations

import math

import numpy as np

from . import fd
from .grid import Grid
from .prop import adjoint, forward


class Model:
    """The full-grid and thin-slab discretisations of one problem."""

    def __init__(self, prob, kappa, rho, engine: str = "numpy"):
        """engine: "numpy" (oracle.prop) or "c" (oracle.cengine, the same
        time stepping as plain C loops, for the full-length runs)."""
        self.prob = prob
        if engine == "numpy":
            self._forward, self._adjoint = forward, adjoint
        elif engine == "c":
            from . import cengine
            self._forward, self._adjoint = cengine.forward, cengine.adjoint
        else:
            raise ValueError(f"unknown oracle engine {engine!r}")
        # constant density, or an array [nz][nx] at the pressure nodes
        self.rho = float(rho) if np.ndim(rho) == 0 else np.asarray(rho, dtype=np.float64)
        kappa = np.asarray(kappa, dtype=np.float64)
        if kappa.shape != (prob.nz, prob.nx):
            raise ValueError("kappa must be [nz][nx]")
        self.kappa = kappa
        self.full = Grid(kappa, rho, prob.h, prob.dt, prob.npml, prob.pml_R,
                         prob.order)
        g = self.full
        self.h_line = g.p_line(prob.z_src, prob.x_src0, prob.ns)
        self.r_line = g.p_line(prob.z_rec, prob.x_rec0, prob.nr)
        self._slab = None
        self._rslab = None

    # -- thin slabs ----------------------------------------------------------
    def _thin_slab(self, z, x0, n, dz):
        """A thin slab around the line at depth z: physical rows from
        min(i, i + dz) - k to max(i, i + dz) + k (i the row at or above z,
        one more row below when z falls between rows, k = order/2), full
        width, model rows copied from the full model (clamped at its top and
        bottom), plus the absorbing layer.  Returns (grid, v_z line at z,
        datum p line at z + dz h, datum v_z line, p line at z); every line
        has n samples from x0."""
        prob = self.prob
        k = prob.order // 2
        dz = int(dz)
        if dz == 0:
            raise ValueError("slab datum offset must be nonzero")
        i_s = int(math.floor(z / prob.h + 1e-12))
        i_lo = min(i_s, i_s + dz) - k
        i_hi = max(i_s, i_s + dz) + k + (1 if z / prob.h - i_s > 1e-12 else 0)
        rows = np.clip(np.arange(i_lo, i_hi + 1), 0, prob.nz - 1)
        rho = self.rho if np.ndim(self.rho) == 0 else self.rho[rows, :]
        g = Grid(self.kappa[rows, :], rho, prob.h, prob.dt, prob.npml, prob.pml_R,
                 prob.order)
        zl = z - i_lo * prob.h
        zd = zl + dz * prob.h
        return (g, g.vz_line(zl, x0, n), g.p_line(zd, x0, n), g.vz_line(zd, x0, n),
                g.p_line(zl, x0, n))

    def slab(self):
        """Source-side slab (datum slab_dz cells from z_s): (grid, source
        line on v_z nodes at z_s, datum line on p nodes, datum line on v_z
        nodes)."""
        if self._slab is None:
            p = self.prob
            self._slab = self._thin_slab(p.z_src, p.x_src0, p.ns, p.slab_dz)
        return self._slab[:4]

    def rslab(self):
        """Receiver-side slab (datum rslab_dz cells from z_r), the same four
        items for the receiver positions."""
        if self._rslab is None:
            p = self.prob
            self._rslab = self._thin_slab(p.z_rec, p.x_rec0, p.nr, p.rslab_dz)
        return self._rslab[:4]

    # -- F and F^T -----------------------------------------------------------
    def fwd(self, h):
        """d = F h, h [nt][ns] -> d [nt][nr]."""
        P, _ = self._forward(self.full, self.prob.nt, h_src=(self.h_line, h),
                       rec_p=self.r_line)
        return P

    def adj(self, r):
        """g = F^T r, r [nt][nr] -> g [nt][ns]."""
        hb, _ = self._adjoint(self.full, self.prob.nt, h_line=self.h_line,
                        rec_p=(self.r_line, r))
        return hb

    # -- V and the time-reversal inverse ---------------------------------------
    def _v_lines(self):
        p, g = self.prob, self.full
        return g.vz_line(p.z_src, p.x_src0, p.ns), g.vz_line(p.z_rec, p.x_rec0, p.nr)

    def fwd_v(self, f):
        """y = V f (the vdef operator): normal load f [nt][ns] on z_s, normal
        velocity traces [nt][nr] recorded on z_r."""
        fl, rl = self._v_lines()
        _, V = self._forward(self.full, self.prob.nt, f_src=(fl, f), rec_v=rl)
        return V

    def adj_v(self, r):
        """g = V^T r: r [nt][nr] enters the normal-velocity trace slot on
        z_r; g [nt][ns] is read from the normal-load slot on z_s."""
        fl, rl = self._v_lines()
        _, fb = self._adjoint(self.full, self.prob.nt, f_line=fl, rec_v=(rl, r))
        return fb

    def block(self, src: int, rec: int, x, transpose: bool = False):
        """A block of the vector modelling operator (Operators section: the
        source vector (h, f) on z = z_s to the traces (P_r p, P_r v_z) on
        z = z_r): src 0 a pressure source, 1 a normal load on the source
        line; rec 0 pressure, 1 normal velocity on the receiver line.
        Block (0, 0) is F, block (1, 1) is V.  With transpose, the exact
        transpose (x then holds receiver traces)."""
        p, g = self.prob, self.full
        s_line = self.h_line if src == 0 else g.vz_line(p.z_src, p.x_src0, p.ns)
        r_line = self.r_line if rec == 0 else g.vz_line(p.z_rec, p.x_rec0, p.nr)
        if not transpose:
            P, V = self._forward(g, p.nt, h_src=(s_line, x) if src == 0 else None,
                           f_src=(s_line, x) if src == 1 else None,
                           rec_p=r_line if rec == 0 else None,
                           rec_v=r_line if rec == 1 else None)
            return P if rec == 0 else V
        hb, fb = self._adjoint(g, p.nt, h_line=s_line if src == 0 else None,
                         f_line=s_line if src == 1 else None,
                         rec_p=(r_line, x) if rec == 0 else None,
                         rec_v=(r_line, x) if rec == 1 else None)
        return hb if src == 0 else fb

    def tr_inverse(self, d):
        """The time-reversal approximate inverse of F (the approxinv
        relations, V^T F ~ I/4): h = 4 V^T d.  (The normal velocity radiated
        by a normal load has the same sign on both sides of the load, so no
        sign depends on whether the receivers lie above or below.)"""
        return 4.0 * self.adj_v(d)

    def lam(self, x, side: str = "s", transpose: bool = False):
        """Lambda~ of the lamtilde formula on a thin slab (side "s": the
        source-side slab; "r": the receiver-side one), or its transpose
        (lamtransp): 2 s X^T (0, P) or 2 s X^T (V, 0) with (P, V) = X x and
        s the slab's scale, so that half their sum is that slab's
        symmetrised operator (W^-1 or W_d)."""
        if side == "s":
            g, f_line, d_p, d_v = self.slab()
            dz = self.prob.slab_dz
        else:
            g, f_line, d_p, d_v = self.rslab()
            dz = self.prob.rslab_dz
        nt = self.prob.nt
        P, V = self._forward(g, nt, f_src=(f_line, x), rec_p=d_p, rec_v=d_v)
        if transpose:
            _, fb = self._adjoint(g, nt, f_line=f_line, rec_p=(d_p, V))
        else:
            _, fb = self._adjoint(g, nt, f_line=f_line, rec_v=(d_v, P))
        return 8.0 * math.copysign(1.0, dz) * fb

    # -- thin-slab vector operator X = Pi-projected S on the slab -------------
    def slab_fwd(self, f):
        """X f = (P, V): normal-load source f on z_s, pressure and normal
        velocity recorded on the datum."""
        g, f_line, d_p, d_v = self.slab()
        return self._forward(g, self.prob.nt, f_src=(f_line, f), rec_p=d_p, rec_v=d_v)

    def slab_adj(self, a, b):
        """X^T (a, b): a enters the pressure-trace slot, b the v_z slot; the
        result is read from the normal-load source slot."""
        g, f_line, d_p, d_v = self.slab()
        _, fb = self._adjoint(g, self.prob.nt, f_line=f_line, rec_p=(d_p, a),
                        rec_v=(d_v, b))
        return fb

    def slab_scale(self) -> float:
        return 4.0 * math.copysign(1.0, self.prob.slab_dz)

    def winv(self, g):
        """Symmetrised thin-slab pressure-to-source operator:
        s X^T J X g with J (P, V) = (V, P)."""
        P, V = self.slab_fwd(g)
        return self.slab_scale() * self.slab_adj(V, P)

    # -- weights of the weighted normal equations -----------------------------
    def wd(self, r):
        """Data-space weight W_d~ = s_r X_r^T J X_r r: the symmetrised
        pressure-to-source operator of the receiver surface, computed like
        W^-1 on the receiver-side slab (normal load on z_r, datum rslab_dz
        cells away), s_r = 4 sign(rslab_dz).  r [nt][nr] -> [nt][nr]."""
        g, f_line, d_p, d_v = self.rslab()
        nt = self.prob.nt
        P, V = self._forward(g, nt, f_src=(f_line, r), rec_p=d_p, rec_v=d_v)
        _, fb = self._adjoint(g, nt, f_line=f_line, rec_p=(d_p, V), rec_v=(d_v, P))
        return 4.0 * math.copysign(1.0, self.prob.rslab_dz) * fb

    def wm(self, x):
        """Model-space weight W_m~, the symmetrised source-to-pressure
        operator: the source-side slab driven by a pressure source on z_s
        instead of a normal load, with the same exchange J of datum
        pressure and velocity, read back from the pressure-source slot;
        scaled by sign(slab_dz) so that it is positive and inverse to W^-1
        on laterally uniform input.  x [nt][ns] -> [nt][ns]."""
        self.slab()
        g, _, d_p, d_v, p_line = self._slab
        nt = self.prob.nt
        P, V = self._forward(g, nt, h_src=(p_line, x), rec_p=d_p, rec_v=d_v)
        hb, _ = self._adjoint(g, nt, h_line=p_line, rec_p=(d_p, V), rec_v=(d_v, P))
        return math.copysign(1.0, self.prob.slab_dz) * hb


# ----------------------------------------------------------------------------
# penalty and diagonal scalings

def lateral_distance(prob, shot: int = 0) -> np.ndarray:
    """|x_k - x_s| for the source-line samples x_k = x_src0 + k h."""
    x = prob.x_src0 + prob.h * np.arange(prob.ns)
    return np.abs(x - prob.xs[shot])


def penalty(prob, x, shot: int = 0):
    """(A x)[n][k] = |x_k - x_s| x[n][k]."""
    return lateral_distance(prob, shot)[None, :] * x


def dscale(prob, alpha_hat: float, shot: int = 0) -> np.ndarray:
    """Diagonal of D = (1 + alpha_hat^2 |x_k - x_s|^2)^(-1/2)."""
    a = lateral_distance(prob, shot)
    return 1.0 / np.sqrt(1.0 + (alpha_hat * a) ** 2)


def precond(model: Model, alpha_hat: float, r, shot: int = 0):
    """M^-1 r = D W^-1 (D r)."""
    d = dscale(model.prob, alpha_hat, shot)[None, :]
    return d * model.winv(d * r)


def normal(model: Model, alpha: float, p, shot: int = 0):
    """N p = F^T F p + alpha^2 A^T A p; also returns F p."""
    Fp = model.fwd(p)
    Ap = penalty(model.prob, p, shot)
    return model.adj(Fp) + alpha * alpha * penalty(model.prob, Ap, shot), Fp


def dot(x, y) -> float:
    return float(np.sum(np.asarray(x, dtype=np.float64) * np.asarray(y, dtype=np.float64)))


def pcg(apply_N, apply_Minv, b, K: int, d_misfit=None):
    """Algorithm 1 (standard PCG), fixed K iterations, h_0 = 0.

    apply_N(p) -> (N p, F p or None); apply_Minv(r) -> M^-1 r.
    Returns (h_K, history) where history[k] = (||r_k||, ||g_k||, <g_k, r_k>,
    ||F h_k - d||) for k = 0..K; the misfit column is NaN unless d_misfit
    (the data d) is given, in which case F h_k - d is updated alongside h
    from the F p_k produced by apply_N."""
    h = np.zeros_like(b)
    r = b.copy()
    g = apply_Minv(r)
    p = g.copy()
    q, Fp = apply_N(p)
    gr = dot(g, r)
    e = -np.asarray(d_misfit, dtype=np.float64) if d_misfit is not None else None
    hist = [(math.sqrt(dot(r, r)), math.sqrt(dot(g, g)), gr,
             math.sqrt(dot(e, e)) if e is not None else math.nan)]
    for k in range(K):
        a = gr / dot(p, q)
        h = h + a * p
        r = r - a * q
        if e is not None:
            e = e + a * Fp
        g = apply_Minv(r)
        gr_new = dot(g, r)
        beta = gr_new / gr
        p = g + beta * p
        gr = gr_new
        hist.append((math.sqrt(dot(r, r)), math.sqrt(dot(g, g)), gr,
                     math.sqrt(dot(e, e)) if e is not None else math.nan))
        if k < K - 1:
            q, Fp = apply_N(p)
    return h, np.array(hist)


def pcg_solve(model: Model, d, alpha_rel: float, K: int, use_precond: bool = True,
              shot: int = 0):
    """The surface-source subproblem solve for one shot: b = F^T d,
    alpha = alpha_rel ||b|| / ||d||, K iterations of Algorithm 1 on
    N h = b with M^-1 = D W^-1 D (alpha_hat = alpha_rel) or M = I."""
    b = model.adj(d)
    alpha = alpha_rel * math.sqrt(dot(b, b)) / math.sqrt(dot(d, d))

    def apply_N(p):
        return normal(model, alpha, p, shot)

    if use_precond:
        def apply_Minv(r):
            return precond(model, alpha_rel, r, shot)
    else:
        def apply_Minv(r):
            return r.copy()
    h, hist = pcg(apply_N, apply_Minv, b, K, d_misfit=d)
    return h, hist, alpha


# ----------------------------------------------------------------------------
# the weighted normal equations (Accelerated Iterative Inversion: the
# normpart system with S* = S^T W_d and A* = A^T W_m; the weights replaced by
# their thin-slab approximations of Computing and Symmetrizing Lambda)

def normal_w(model: Model, alpha: float, p, shot: int = 0):
    """N_w p = F^T W_d~ F p + alpha^2 A^T W_m~ A p; also returns F p.  The
    model-space term is left out when alpha is zero."""
    prob = model.prob
    Fp = model.fwd(p)
    q = model.adj(model.wd(Fp))
    if alpha != 0.0:
        q = q + alpha * alpha * penalty(prob, model.wm(penalty(prob, p, shot)), shot)
    return q, Fp


def pcg_solve_w(model: Model, d, alpha: float, K: int, use_precond: bool = True,
                shot: int = 0):
    """The weighted subproblem solve for one shot: b = F^T W_d~ d, K
    iterations of Algorithm 1 on N_w h = b with M^-1 = D W^-1 D, where the
    same alpha (per unit length, the weighted norms making F nearly unitary)
    sets both the penalty and D; M = I when use_precond is false."""
    b = model.adj(model.wd(d))

    def apply_N(p):
        return normal_w(model, alpha, p, shot)

    if use_precond:
        def apply_Minv(r):
            return precond(model, alpha, r, shot)
    else:
        def apply_Minv(r):
            return r.copy()
    h, hist = pcg(apply_N, apply_Minv, b, K, d_misfit=d)
    return h, hist


# ----------------------------------------------------------------------------
# the gradient of the data misfit with respect to the bulk modulus (the
# derivative that the variable-projection outer problem needs: at the
# subproblem's minimiser the reduced objective's gradient is the partial
# gradient at fixed h, Introduction and Conclusion)

def misfit_gradient(model: Model, h, d):
    """g = dJ/dkappa of J = 1/2 ||F h - d||^2 at fixed h, for every physical
    cell, by the adjoint state of the discrete scheme: kappa enters the
    pressure update through Ck = dt kappa / h, so
        g = -(dt / h) sum_n pbar^{n+1} (D^- v^{n+1/2} - E_h h^n)
    with pbar the adjoint pressure (F^T of the residual).  The absorbing
    layer's coefficients (its copies of the edge values and its damping
    profile) are held fixed, so on the physical grid, where the layer's
    split parts carry equal adjoints, this is the whole derivative.
    Returns (g [nz][nx], J)."""
    prob, g = model.prob, model.full
    divs = []
    P, _ = forward(g, prob.nt, h_src=(model.h_line, h), rec_p=model.r_line, div_out=divs)
    res = P - d
    acc = np.zeros_like(divs[0])

    def on_p(n, pxb, pzb):
        acc[...] += pzb * divs[n]

    adjoint(g, prob.nt, h_line=model.h_line, rec_p=(model.r_line, res), on_p=on_p)
    L = prob.npml
    grad = -(prob.dt / prob.h) * acc[L:L + prob.nz, L:L + prob.nx]
    return grad, 0.5 * float(np.sum(res * res))



# ----------------------------------------------------------------------------
# the subproblem with the normal load as the unknown (Operators section: the
# source vector's second component f_s, observed through the normal
# velocity, V = Pi_1 S Pi_1^T of the vdef definition)

def normal_v(model: Model, alpha: float, p, shot: int = 0):
    """N_v p = V^T V p + alpha^2 A^T A p; also returns V p."""
    Vp = model.fwd_v(p)
    Ap = penalty(model.prob, p, shot)
    return model.adj_v(Vp) + alpha * alpha * penalty(model.prob, Ap, shot), Vp


def pcg_solve_v(model: Model, d, alpha_rel: float, K: int, shot: int = 0):
    """min_f ||V f - d||^2 + alpha^2 ||A f||^2 for normal-velocity data d
    [nt][nr]: b = V^T d, alpha = alpha_rel ||b|| / ||d||, K iterations of
    Algorithm 1 with M = I (the paper derives no preconditioner for this
    form)."""
    b = model.adj_v(d)
    alpha = alpha_rel * math.sqrt(dot(b, b)) / math.sqrt(dot(d, d))
    h, hist = pcg(lambda p: normal_v(model, alpha, p, shot), lambda r: r.copy(), b, K,
                  d_misfit=d)
    return h, hist, alpha
