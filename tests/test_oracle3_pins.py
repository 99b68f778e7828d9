"""Pins of the 3D FP64 oracle (``oracle.prop3``, ``oracle.ops3``) against
facts that do not come from its own code: the 2D oracle (itself pinned) on
y-invariant problems inside the discrete dependency cone (propagation and
the thin-slab W^-1), the dot-product test, discrete energy conservation in
a rigid box, the closed-form 3D point-source response, the symmetry of
W^-1, a dense solve, and the Krylov minimisation property of the
preconditioned iterates."""
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


# ---------------------------------------------------------------------------
# the 3D subproblem operators (oracle.ops3)

import oracle  # noqa: E402
from oracle.ops3 import (Model3, lateral_distance3, normal3, pcg_solve3,  # noqa: E402
                         precond3)


@pytest.mark.parametrize("order,dz", [(4, 3), (8, -2)])
def test_y_invariant_thin_slab_reduces_to_2d(order, dz):
    # the thin-slab W^-1 of a y-invariant model and load: its centre row is
    # the 2D W^-1 (itself pinned by the plane-wave scale and symmetry)
    K = order // 2
    nz, nx, L, nt, h = 16, 18, 4, 10, 10.0
    ny = 2 * (2 * K * nt + K + 2) + 1
    kap2 = layered_kappa2(nz, nx, 23)
    kap3 = np.repeat(kap2[:, None, :], ny, axis=1)
    ns = 12
    p2 = inputs.Problem(nz=nz, nx=nx, h=h, dt=1e-3, nt=nt, order=order, npml=L, z_src=65.0,
                        x_src0=3 * h, ns=ns, z_rec=120.0, x_rec0=h, nr=10, slab_dz=dz,
                        xs=(80.0,))
    p3 = inputs.Problem3(nz=nz, ny=ny, nx=nx, h=h, dt=1e-3, nt=nt, order=order, npml=L,
                         z_src=65.0, x_src0=3 * h, y_src0=0.0, nsx=ns, nsy=ny, z_rec=120.0,
                         x_rec0=h, nrx=10, nry=1, slab_dz=dz, x_s=80.0)
    m2 = oracle.Model(p2, kap2, RHO)
    m3 = Model3(p3, kap3, RHO)
    g = np.random.default_rng(8).standard_normal((nt, ns))
    w2 = m2.winv(g)
    w3 = m3.winv(np.repeat(g[:, None, :], ny, axis=1).reshape(nt, -1))
    yc = (ny - 1) // 2
    w3c = w3.reshape(nt, ny, ns)[:, yc, :]
    assert np.abs(w2).max() > 0
    assert np.abs(w3c - w2).max() <= 1e-13 * np.abs(w2).max()


def _small3(order=4, nt=6, nsx=2, nsy=2, dz=3, L=3):
    p = inputs.Problem3(nz=10, ny=9, nx=11, h=10.0, dt=1e-3, nt=nt, order=order, npml=L,
                        z_src=25.0, x_src0=40.0, y_src0=30.0, nsx=nsx, nsy=nsy, z_rec=75.0,
                        x_rec0=10.0, y_rec0=10.0, nrx=8, nry=6, slab_dz=dz, x_s=45.0,
                        y_s=35.0)
    vel = inputs.layered_velocity3(p.nz, p.ny, p.nx, p.h, np.random.default_rng(4))
    return p, Model3(p, RHO * vel * vel, RHO)


def test_thin_slab_operator_symmetric_and_distance():
    p, m = _small3(order=8, nsx=3, nsy=2, dz=-2)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((p.nt, p.ns))
    y = rng.standard_normal((p.nt, p.ns))
    a, b = np.sum(m.winv(x) * y), np.sum(x * m.winv(y))
    assert abs(a) > 0 and abs(a - b) <= 1e-12 * abs(a)
    # distance of trace (a, b) from (x_s, y_s), written out
    dist = lateral_distance3(p)
    assert dist[1 * p.nsx + 2] == pytest.approx(math.hypot(40.0 + 20.0 - 45.0,
                                                           30.0 + 10.0 - 35.0))


def _dense(apply, n, shape):
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(np.asarray(apply(e.reshape(shape))).ravel())
    return np.array(cols).T


def test_pcg_without_preconditioner_reaches_dense_solution():
    p, m = _small3()
    rng = np.random.default_rng(6)
    d = rng.standard_normal((p.nt, p.nr))
    b = m.adj(d)
    alpha = 0.3 * math.sqrt(np.sum(b * b)) / math.sqrt(np.sum(d * d))
    shp = (p.nt, p.ns)
    N = _dense(lambda x: normal3(m, alpha, x)[0], p.nt * p.ns, shp)
    assert np.abs(N - N.T).max() <= 1e-12 * np.abs(N).max()
    hstar = np.linalg.solve(N, b.ravel())
    h, hist, a = pcg_solve3(m, d, 0.3, 30, use_precond=False)   # 24 unknowns
    assert a == pytest.approx(alpha)
    assert np.linalg.norm(h.ravel() - hstar) <= 1e-8 * np.linalg.norm(hstar)


def test_preconditioned_iterates_are_krylov_minimisers():
    # Algorithm 1 with M^-1: iterate k is the N-norm minimiser of the error
    # over K_k(M^-1 N, M^-1 b) (Galerkin on that span), whatever the sign of
    # M^-1 on it
    p, m = _small3(order=8, dz=2)
    rng = np.random.default_rng(12)
    d = rng.standard_normal((p.nt, p.nr))
    b = m.adj(d)
    alpha = 0.5 * math.sqrt(np.sum(b * b)) / math.sqrt(np.sum(d * d))
    shp = (p.nt, p.ns)
    n = p.nt * p.ns
    N = _dense(lambda x: normal3(m, alpha, x)[0], n, shp)
    Minv = _dense(lambda x: precond3(m, 0.5, x), n, shp)
    for k in (1, 2, 3):
        q = Minv @ b.ravel()
        Q = [q / np.linalg.norm(q)]
        for _ in range(k - 1):
            w = Minv @ (N @ Q[-1])
            for _ in range(2):
                for u in Q:
                    w = w - (u @ w) * u
            Q.append(w / np.linalg.norm(w))
        Q = np.array(Q).T
        ref = Q @ np.linalg.solve(Q.T @ N @ Q, Q.T @ b.ravel())
        h, _, _ = pcg_solve3(m, d, 0.5, k)
        assert np.linalg.norm(h.ravel() - ref) <= 1e-9 * np.linalg.norm(ref), k
