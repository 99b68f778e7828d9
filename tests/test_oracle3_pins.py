"""Pins of the 3D FP64 oracle (``oracle.prop3``) against facts that do not
come from its own code: the 2D oracle (itself pinned) on a y-invariant
problem inside the discrete dependency cone, the dot-product test,
discrete energy conservation in a rigid box and the closed-form 3D
point-source response."""
import math

import numpy as np
import pytest

import inputs
from oracle.grid import Grid
from oracle.prop import forward, adjoint
from oracle.prop3 import Grid3, forward3, adjoint3

RHO = 1000.0


def layered_kappa2(nz, nx, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1800.0, 2200.0, size=(nz, nx))
    return RHO * c * c


# ---------------------------------------------------------------------------
# The 3D scheme restricted to fields that do not depend on y is the 2D
# scheme: D_y of a y-constant field vanishes exactly, so v_y and p_y stay
# zero and every other update is the 2D one, term for term.  With zero
# extension and the absorbing layer at the y-ends, y-invariance holds on
# the rows farther than the dependency cone (2k cells per step) from the
# rows where the source or the layer breaks it.

@pytest.mark.parametrize("order", [4, 8])
def test_y_invariant_problem_reduces_to_2d(order):
    K = order // 2
    nz, nx, L, nt, h, dt = 14, 18, 4, 10, 10.0, 1e-3
    ny = 2 * (2 * K * nt + K + 2) + 1        # physical rows; the centre is outside every cone
    kap2 = layered_kappa2(nz, nx, 21)
    kap3 = np.repeat(kap2[:, None, :], ny, axis=1)
    g2 = Grid(kap2, RHO, h, dt, L, 1e-3, order)
    g3 = Grid3(kap3, RHO, h, dt, L, 1e-3, order)
    rng = np.random.default_rng(5)
    ns, nr = 10, 12
    w = rng.standard_normal((nt, ns))
    src2 = g2.p_line(35.0, 2 * h, ns)
    rec2 = g2.p_line(95.0, h, nr)
    P2, _ = forward(g2, nt, h_src=(src2, w), rec_p=rec2)
    # the source on every physical y row, traces repeated along y
    src3 = g3.p_plane(35.0, 2 * h, ns, 0.0, ny)
    yc = (ny - 1) // 2
    rec3 = g3.p_plane(95.0, h, nr, yc * h, 1)
    w3 = np.repeat(w[:, None, :], ny, axis=1).reshape(nt, ny * ns)
    P3, _ = forward3(g3, nt, h_src=(src3, w3), rec_p=rec3)
    assert np.abs(P2).max() > 0
    assert np.array_equal(P3, P2)
    # the transposed sweep: receivers on every row, source traces of the
    # centre row; equal up to the order of one three-term sum
    r = rng.standard_normal((nt, nr))
    hb2, _ = adjoint(g2, nt, h_line=src2, rec_p=(rec2, r))
    rec3all = g3.p_plane(95.0, h, nr, 0.0, ny)
    src3c = g3.p_plane(35.0, 2 * h, ns, yc * h, 1)
    r3 = np.repeat(r[:, None, :], ny, axis=1).reshape(nt, ny * nr)
    hb3, _ = adjoint3(g3, nt, h_plane=src3c, rec_p=(rec3all, r3))
    assert np.abs(hb3 - hb2).max() <= 1e-13 * np.abs(hb2).max()


# ---------------------------------------------------------------------------
# The transposed sweep is the transpose: <F x, y> = <x, F^T y> for the
# whole 2 x 2 block (pressure and normal-load sources; pressure and v_z
# recordings), absorbing layer on every side, off-node planes.

@pytest.mark.parametrize("order", [4, 8])
def test_dot_product(order):
    nz, ny, nx, L, nt, h = 12, 10, 14, 3, 16, 10.0
    rng = np.random.default_rng(7)
    c = rng.uniform(1800.0, 2200.0, size=(nz, ny, nx))
    g = Grid3(RHO * c * c, RHO, h, 1e-3, L, 1e-3, order)
    hs = g.p_plane(33.0, 2 * h, 5, h, 4)
    fs = g.vz_plane(37.0, 3 * h, 4, 2 * h, 3)
    rp = g.p_plane(81.0, h, 6, 0.0, 5)
    rv = g.vz_plane(77.0, 2 * h, 5, h, 6)
    x_h = rng.standard_normal((nt, hs.n))
    x_f = rng.standard_normal((nt, fs.n))
    y_p = rng.standard_normal((nt, rp.n))
    y_v = rng.standard_normal((nt, rv.n))
    P, V = forward3(g, nt, h_src=(hs, x_h), f_src=(fs, x_f), rec_p=rp, rec_v=rv)
    hb, fb = adjoint3(g, nt, h_plane=hs, f_plane=fs, rec_p=(rp, y_p), rec_v=(rv, y_v))
    lhs = np.sum(P * y_p) + np.sum(V * y_v)
    rhs = np.sum(x_h * hb) + np.sum(x_f * fb)
    assert abs(lhs) > 0
    assert abs(lhs - rhs) <= 1e-13 * (np.linalg.norm(P) * np.linalg.norm(y_p)
                                      + np.linalg.norm(V) * np.linalg.norm(y_v))


# ---------------------------------------------------------------------------
# Discrete energy 1/2 sum rho v^{n-1/2} v^{n+1/2} + 1/2 sum p^2/kappa is
# conserved by the leapfrog scheme in a rigid box once the source stops.

@pytest.mark.parametrize("order", [4, 8])
def test_energy_conserved_without_absorption(order):
    n, nt, h = 16, 90, 10.0
    rng = np.random.default_rng(9)
    c = rng.uniform(1800.0, 2200.0, size=(n, n, n))
    g = Grid3(RHO * c * c, RHO, h, 1e-3, 0, 1e-3, order)
    src = g.p_plane(75.0, 7 * h, 1, 8 * h, 1)
    w = np.zeros((nt, 1))
    w[:15, 0] = rng.standard_normal(15)
    _, _, E = forward3(g, nt, h_src=(src, w), energy=True)
    E = np.array(E[16:])
    assert E.max() > 0
    assert (E.max() - E.min()) / E.max() < 1e-13


# ---------------------------------------------------------------------------
# Closed form: for constant kappa and rho a point constitutive-defect source
# w(t) delta(x) gives p_tt - c^2 Lap p = kappa w'(t) delta(x), whose causal
# solution is p(r, t) = rho w'(t - r/c) / (4 pi r).  A single trace of value
# w / h^2 is that point source on the grid (the z-delta's 1/h is in the
# coefficients).  Order 8, about 17 cells per dominant wavelength.

def test_point_source_amplitude():
    c, h, f, r, W, order = 2000.0, 10.0, 12.0, 150.0, 400.0, 8
    dt = 0.4 * h / c
    n = int(round(2 * W / h)) + 1
    kap = np.full((n, n, n), RHO * c * c)
    g = Grid3(kap, RHO, h, dt, 0, 1e-3, order)
    nt = int(math.ceil((1.5 / f + r / c + 2.0 / f) / dt))
    w = inputs.ricker((np.arange(nt) + 0.5) * dt, f)
    src = g.p_plane(W, W, 1, W, 1)
    rec = g.p_plane(W + r, W, 1, W, 1)
    P, _ = forward3(g, nt, h_src=(src, (w / h ** 2)[:, None]), rec_p=rec)
    t = (np.arange(nt) + 1) * dt
    s = t - r / c
    ref = RHO * np.where(s > 0, inputs.ricker_deriv(s, f), 0.0) / (4 * math.pi * r)
    err = np.abs(P[:, 0] - ref).max() / np.abs(ref).max()
    assert err < 3e-2, err
