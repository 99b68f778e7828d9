"""Pins of the FP64 oracle against facts that do not come from its own code.

Each test names the passage of the paper (or the mathematical fact) it
relies on.  Together they are meant to catch a plausible slip anywhere in
the oracle: a dropped term or factor, a wrong sign, index or time level, a
transposed operand.
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from oracle import fd, greens
from oracle.grid import Grid
from oracle.prop import adjoint, forward

RHO = 1000.0


def tiny_problem(order=4, nz=12, nx=16, L=4, nt=24, h=10.0, dt=1e-3,
                 z_src=35.0, z_rec=80.0, ns=8, nr=10, slab_dz=3, xs=(52.0,), rslab_dz=2):
    return inputs.Problem(nz=nz, nx=nx, h=h, dt=dt, nt=nt, order=order, npml=L,
                          z_src=z_src, x_src0=2 * h, ns=ns, z_rec=z_rec,
                          x_rec0=h, nr=nr, slab_dz=slab_dz, xs=xs, rslab_dz=rslab_dz)


def tiny_kappa(prob, seed=0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1800.0, 2200.0, size=(prob.nz, prob.nx))
    return RHO * c * c


def dense(apply, n_in, shape_in):
    cols = []
    for i in range(n_in):
        e = np.zeros(n_in)
        e[i] = 1.0
        cols.append(np.asarray(apply(e.reshape(shape_in))).ravel())
    return np.array(cols).T


# ---------------------------------------------------------------------------
# stencils (Numerical Examples: staggered scheme, order 2k in space)

@pytest.mark.parametrize("order,expected", [
    (2, (1.0,)),
    (4, (9 / 8, -1 / 24)),
    (8, (1225 / 1024, -245 / 3072, 49 / 5120, -5 / 7168)),
])
def test_stencil_matches_textbook_values(order, expected):
    # the classical staggered Taylor coefficients (Fornberg 1988)
    c = fd.stencil(order)
    assert np.allclose(c, expected, rtol=1e-14, atol=0)
    assert abs(sum((2 * m - 1) * cm for m, cm in enumerate(c, 1)) - 1) < 1e-14


@pytest.mark.parametrize("order", [4, 8])
def test_stencil_polynomial_exactness(order):
    # D+ of x^q sampled on nodes equals q x^(q-1) at half nodes for
    # q <= order (interior points); D- likewise from half nodes to nodes.
    c = fd.stencil(order)
    k = order // 2
    x = np.arange(40, dtype=np.float64) * 0.1 - 2.0
    for q in range(0, order + 1):
        p = x ** q
        dp = fd.dplus(p, c, axis=0) / 0.1
        xh = x + 0.05
        exact = q * xh ** (q - 1) if q > 0 else 0 * xh
        assert np.allclose(dp[k:-k], exact[k:-k], rtol=1e-9, atol=1e-9), q
        v = xh ** q
        dv = fd.dminus(v, c, axis=0) / 0.1
        exact = q * x ** (q - 1) if q > 0 else 0 * x
        assert np.allclose(dv[k:-k], exact[k:-k], rtol=1e-9, atol=1e-9), q


@pytest.mark.parametrize("order", [2, 4, 8])
def test_difference_operators_transpose(order):
    # D- = -(D+)^T exactly with zero extension, and the *_T functions are
    # the dense transposes.
    c = fd.stencil(order)
    n = 13
    Dp = dense(lambda e: fd.dplus(e, c, 0), n, (n,))
    Dm = dense(lambda e: fd.dminus(e, c, 0), n, (n,))
    DpT = dense(lambda e: fd.dplus_T(e, c, 0), n, (n,))
    DmT = dense(lambda e: fd.dminus_T(e, c, 0), n, (n,))
    assert np.array_equal(Dm, -Dp.T)
    assert np.array_equal(DpT, Dp.T)
    assert np.array_equal(DmT, Dm.T)
    # along axis 1 of a 2D array as well
    u = np.random.default_rng(1).standard_normal((5, 11))
    w = np.random.default_rng(2).standard_normal((5, 11))
    assert abs(np.sum(fd.dplus(u, c, 1) * w) + np.sum(u * fd.dminus(w, c, 1))) < 1e-12


# ---------------------------------------------------------------------------
# sampling and injection (linear interpolation and its adjoint)

@pytest.mark.parametrize("z", [30.0, 35.0, 47.5, 80.0])
def test_line_interpolation_exact_on_linear_fields(z):
    prob = tiny_problem()
    g = Grid(tiny_kappa(prob), RHO, prob.h, prob.dt, prob.npml, prob.pml_R, 4)
    I = np.arange(g.NZ)[:, None] * np.ones((1, g.NX))
    # p node row i is at depth (i - L) h, v_z row i at (i - L + 1/2) h
    fp = 3.0 + 0.7 * (I - g.L) * g.h
    fv = 3.0 + 0.7 * (I - g.L + 0.5) * g.h
    lp = g.p_line(z, 20.0, 5)
    lv = g.vz_line(z, 20.0, 5)
    assert np.allclose(lp.gather(fp), 3.0 + 0.7 * z, rtol=1e-14)
    assert np.allclose(lv.gather(fv), 3.0 + 0.7 * z, rtol=1e-14)
    assert abs(sum(w for _, w in lp.rows) - 1) < 1e-15
    # spread is the transpose of gather
    a = np.random.default_rng(0).standard_normal(5)
    F = np.random.default_rng(1).standard_normal((g.NZ, g.NX))
    assert abs(np.sum(lp.spread(a, F.shape) * F) - np.sum(a * lp.gather(F))) < 1e-12


def test_pml_profile_values():
    prob = tiny_problem(L=6)
    g = Grid(tiny_kappa(prob), RHO, prob.h, prob.dt, prob.npml, prob.pml_R, 4)
    L, nx = g.L, g.nx
    # no damping on physical nodes and on half nodes between them
    assert np.all(g.ax_n[L:L + nx] == 1) and np.all(g.bx_n[L:L + nx] == 1)
    assert np.all(g.ax_h[L:L + nx - 1] == 1)
    # outermost node: sigma = sigma_max; a, b from the trapezoidal rule
    q = 0.5 * g.sigma_max * prob.dt
    assert abs(g.ax_n[0] - (1 - q) / (1 + q)) < 1e-15
    assert abs(g.bx_n[0] - 1 / (1 + q)) < 1e-15
    # half node at depth 1/2 cell into the layer: sigma_max (1/(2L))^2
    q = 0.5 * g.sigma_max * (0.5 / L) ** 2 * prob.dt
    assert abs(g.ax_h[L - 1] - (1 - q) / (1 + q)) < 1e-15
    assert abs(g.ax_h[L + nx - 1] - (1 - q) / (1 + q)) < 1e-15
    cmax = math.sqrt(tiny_kappa(prob).max() / RHO)
    assert abs(g.sigma_max - 3 * cmax * math.log(1e3) / (2 * L * prob.h)) < 1e-9


def test_pml_absorbs():
    # A pulse started in the middle of the box: with the absorbing layer the
    # energy left after the wave has crossed the layer is a small fraction of
    # the same run with a rigid box and no layer.
    kap = inputs.homogeneous_kappa(40, 40, 2000.0)
    nt = 600
    w = inputs.ricker((np.arange(nt) + 0.5) * 1e-3, 25.0)
    res = {}
    for L in (0, 20):
        g = Grid(kap, RHO, 10.0, 1e-3, L, 1e-3, 4)
        line = g.p_line(200.0, 200.0, 1)
        _, _, E = forward(g, nt, h_src=(line, (w / 10.0)[:, None]), energy=True)
        res[L] = E
    peak = max(res[0])
    assert res[0][-1] > 0.5 * peak          # rigid box keeps its energy
    assert res[20][-1] < 1e-4 * peak        # layer takes it out


# ---------------------------------------------------------------------------
# P1/P2: adjoint (Operators section, adjoint identity; Appendix A; the
# paper's own pseudorandom dot-product test in Numerical Examples)

@pytest.mark.parametrize("order", [4, 8])
def test_dot_product_full_and_slab(order):
    prob = tiny_problem(order=order, nz=20, nx=24, L=6, nt=60, ns=18, nr=20,
                        z_src=55.0, z_rec=140.0, slab_dz=-4)
    m = oracle.Model(prob, tiny_kappa(prob, 3), RHO)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((prob.nt, prob.ns))
    y = rng.standard_normal((prob.nt, prob.nr))
    Fx = m.fwd(x)
    Fty = m.adj(y)
    err = abs(np.sum(Fx * y) - np.sum(x * Fty)) / (np.linalg.norm(Fx) * np.linalg.norm(y))
    assert err < 1e-14
    P, V = m.slab_fwd(x)
    a = rng.standard_normal(P.shape)
    b = rng.standard_normal(V.shape)
    Xt = m.slab_adj(a, b)
    lhs = np.sum(P * a) + np.sum(V * b)
    err = abs(lhs - np.sum(x * Xt)) / (math.hypot(np.linalg.norm(P), np.linalg.norm(V))
                                       * math.hypot(np.linalg.norm(a), np.linalg.norm(b)))
    assert err < 1e-14


def test_dense_transpose_brute_force():
    prob = tiny_problem()
    m = oracle.Model(prob, tiny_kappa(prob, 5), RHO)
    nin, nout = prob.nt * prob.ns, prob.nt * prob.nr
    F = dense(m.fwd, nin, (prob.nt, prob.ns))
    Ft = dense(m.adj, nout, (prob.nt, prob.nr))
    scale = np.abs(F).max()
    assert np.abs(F.T - Ft).max() <= 1e-14 * scale
    # causality: output sample n depends only on inputs up to n
    Fb = F.reshape(prob.nt, prob.nr, prob.nt, prob.ns)
    for n in range(prob.nt):
        assert np.all(Fb[n, :, n + 1:, :] == 0)


# ---------------------------------------------------------------------------
# P3: discrete energy (the acoustic energy of the Pressure-to-Source
# section; Appendix A's energy argument), rigid box, no absorbing layer

@pytest.mark.parametrize("order", [4, 8])
def test_energy_conserved_without_absorption(order):
    prob = tiny_problem(order=order, nz=30, nx=34, L=0, nt=200, ns=1, z_src=145.0,
                        xs=(0.0,))
    kap = tiny_kappa(prob, 11)
    g = Grid(kap, RHO, prob.h, prob.dt, 0, prob.pml_R, order)
    src = np.zeros((prob.nt, 1))
    src[:20, 0] = np.random.default_rng(3).standard_normal(20)
    line = g.p_line(145.0, 150.0, 1)
    _, _, E = forward(g, prob.nt, h_src=(line, src), energy=True)
    E = np.array(E[21:])
    assert E.max() > 0
    assert (E.max() - E.min()) / E.max() < 1e-13


# ---------------------------------------------------------------------------
# P4: reciprocity (the time-reversal / transpose relations of the Operators
# section applied to a point-to-point pressure response), rigid box

def test_reciprocity_point_sources():
    prob = tiny_problem(nz=26, nx=30, L=0, nt=120)
    kap = tiny_kappa(prob, 13)
    g = Grid(kap, RHO, prob.h, prob.dt, 0, prob.pml_R, 4)
    a = g.p_line(60.0, 70.0, 1)
    b = g.p_line(190.0, 220.0, 1)
    w = np.random.default_rng(4).standard_normal((prob.nt, 1))
    Pab, _ = forward(g, prob.nt, h_src=(a, w), rec_p=b)
    Pba, _ = forward(g, prob.nt, h_src=(b, w), rec_p=a)
    assert np.abs(Pab).max() > 0
    assert np.abs(Pab - Pba).max() <= 1e-13 * np.abs(Pab).max()


# ---------------------------------------------------------------------------
# P5: closed-form 2D Green's function, second-order convergence at fixed
# Courant number (scheme of order 2 in time)

def _green_error(h, order=8, courant=0.4, c=2000.0, f=10.0, r=300.0, W=800.0):
    dt = courant * h / c
    n = int(round(2 * W / h)) + 1
    kap = inputs.homogeneous_kappa(n, n, c)
    g = Grid(kap, RHO, h, dt, 0, 1e-3, order)
    tmax = 1.5 / f + r / c + 2.0 / f
    nt = int(math.ceil(tmax / dt))
    w = inputs.ricker((np.arange(nt) + 0.5) * dt, f)
    src = g.p_line(W, W, 1)            # node at the centre
    rec = g.p_line(W + r, W, 1)        # r below it
    P, _ = forward(g, nt, h_src=(src, (w / h)[:, None]), rec_p=rec)
    t = (np.arange(nt) + 1) * dt
    ref = greens.point_source_pressure(r, t, c, RHO,
                                       lambda s: np.where(s > 0, inputs.ricker_deriv(s, f), 0.0))
    return np.abs(P[:, 0] - ref).max() / np.abs(ref).max()


@pytest.mark.slow
def test_greens_function_second_order():
    e = [_green_error(h) for h in (20.0, 10.0, 5.0)]
    orders = [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]
    assert e[2] < 5e-3, e
    for o in orders:
        assert 1.8 <= o <= 2.2, (e, orders)


def test_greens_function_amplitude_coarse():
    # a single cheap resolution: right scale, sign and arrival time
    assert _green_error(10.0) < 3e-2


# ---------------------------------------------------------------------------
# P6: 1D special case -- a laterally uniform line source makes plane waves:
# p = (rho c / 2) h(t - tau) below a pressure source (jump of v_z equals h,
# Pressure-to-Source section), and the thin-slab operator s X^T J X acts as
# 2/(rho c) on laterally uniform input for either datum side.

def _plane_setup(slab_dz=5, order=4):
    c, h = 2000.0, 10.0
    prob = inputs.Problem(nz=60, nx=201, h=h, dt=1e-3, nt=400, order=order,
                          npml=20, z_src=200.0, x_src0=0.0, ns=201,
                          z_rec=300.0, x_rec0=0.0, nr=201, slab_dz=slab_dz,
                          xs=(1000.0,))
    return prob, oracle.Model(prob, inputs.homogeneous_kappa(60, 201, c), RHO), c


def test_plane_wave_amplitude_pressure_source():
    prob, m, c = _plane_setup()
    f = 10.0
    w = inputs.ricker((np.arange(prob.nt) + 0.5) * prob.dt, f)
    d = m.fwd(np.repeat(w[:, None], prob.ns, axis=1))
    tau = (prob.z_rec - prob.z_src) / c
    expect = 0.5 * RHO * c * inputs.ricker((np.arange(prob.nt) + 1) * prob.dt - tau, f)
    got = d[:, prob.nr // 2]
    assert np.abs(got - expect).max() < 1e-2 * np.abs(expect).max()


def _slab_plane_error(h, dz, order=4, f=10.0, c=2000.0):
    nz, nx = int(600 / h), int(2000 / h) + 1
    dt = 0.2 * h / c
    nt = int(0.4 / dt)
    prob = inputs.Problem(nz=nz, nx=nx, h=h, dt=dt, nt=nt, order=order, npml=20,
                          z_src=200.0, x_src0=0.0, ns=nx, z_rec=300.0, x_rec0=0.0,
                          nr=nx, slab_dz=dz, xs=(1000.0,))
    m = oracle.Model(prob, inputs.homogeneous_kappa(nz, nx, c), RHO)
    w = inputs.ricker((np.arange(nt) + 0.5) * dt, f)
    out = m.winv(np.repeat(w[:, None], nx, axis=1))[:, nx // 2]
    expect = 2.0 / (RHO * c) * w
    return np.abs(out - expect).max() / np.abs(expect).max()


@pytest.mark.parametrize("dz", [5, -5])
def test_plane_wave_slab_operator_scale(dz):
    # The half-row injection of the normal load and the interpolated v_z
    # sampling each average a plane wave over one cell, so the discrete
    # operator approaches 2/(rho c) at second order in h (about 5% low at
    # 20 points per wavelength, 1.4% at 40).  Both datum sides give the
    # same positive scale with s = 4 sign(dz).
    e10 = _slab_plane_error(10.0, dz)
    e5 = _slab_plane_error(5.0, dz)
    assert e5 < 0.02
    assert math.log2(e10 / e5) > 1.7


# ---------------------------------------------------------------------------
# P7: symmetry of the preconditioner by construction (the W_m^-1 formula of
# Computing and Symmetrizing Lambda); spectrum reported, not asserted

def test_preconditioner_symmetric():
    prob = tiny_problem(nz=14, nx=20, L=5, nt=30, ns=16, slab_dz=3, z_src=50.0)
    m = oracle.Model(prob, tiny_kappa(prob, 17), RHO)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((prob.nt, prob.ns))
    y = rng.standard_normal((prob.nt, prob.ns))
    Wx, Wy = m.winv(x), m.winv(y)
    err = abs(np.sum(x * Wy) - np.sum(Wx * y)) / (np.linalg.norm(Wx) * np.linalg.norm(y))
    assert err < 1e-13
    Mx = oracle.precond(m, 1e-3, x)
    My = oracle.precond(m, 1e-3, y)
    assert abs(np.sum(x * My) - np.sum(Mx * y)) <= 1e-13 * np.linalg.norm(Mx) * np.linalg.norm(y)


# ---------------------------------------------------------------------------
# P8/P9: Algorithm 1 against dense linear algebra

def _dense_system(alpha_scale=0.05):
    prob = tiny_problem(nt=20, ns=8, nr=10, xs=(47.0,))  # x_s between nodes
    m = oracle.Model(prob, tiny_kappa(prob, 21), RHO)
    n = prob.nt * prob.ns
    F = dense(m.fwd, n, (prob.nt, prob.ns))
    A = np.tile(oracle.ops.lateral_distance(prob), prob.nt)
    smax = np.linalg.norm(F, 2)
    alpha = alpha_scale * smax / A.max()
    N = F.T @ F + alpha ** 2 * np.diag(A * A)
    d = np.random.default_rng(5).standard_normal(prob.nt * prob.nr)
    b = F.T @ d
    return prob, m, F, N, b, alpha


def test_pcg_converges_to_dense_solution():
    prob, m, F, N, b, alpha = _dense_system(alpha_scale=0.3)
    assert np.abs(N - N.T).max() <= 1e-13 * np.abs(N).max()
    Lc = np.linalg.cholesky(N)
    hstar = np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))
    shp = (prob.nt, prob.ns)

    def apply_N(p):
        return (N @ p.ravel()).reshape(shp), None

    h, hist = oracle.pcg(apply_N, lambda r: r.copy(), b.reshape(shp), 400)
    assert np.linalg.norm(h.ravel() - hstar) <= 1e-9 * np.linalg.norm(hstar)
    # and through the operators themselves (not the dense matrix)
    hop, _ = oracle.pcg(lambda p: oracle.normal(m, alpha, p), lambda r: r.copy(),
                        b.reshape(shp), 400)
    assert np.linalg.norm(hop.ravel() - hstar) <= 1e-9 * np.linalg.norm(hstar)


def _krylov_minimiser(N, Minv, b, k):
    # argmin ||h - h*||_N over K_k(Minv N, Minv b) = Galerkin solution on the
    # span (Golub & Van Loan, Matrix Computations, CG as a projection
    # method).  The span is built by Arnoldi with two Gram-Schmidt passes,
    # which keeps the basis well conditioned when Minv is nearly singular.
    q = Minv @ b
    Q = [q / np.linalg.norm(q)]
    for _ in range(k - 1):
        w = Minv @ (N @ Q[-1])
        for _ in range(2):
            for u in Q:
                w = w - (u @ w) * u
        Q.append(w / np.linalg.norm(w))
    Q = np.array(Q).T
    y = np.linalg.solve(Q.T @ N @ Q, Q.T @ b)
    return Q @ y


def test_pcg_iterates_are_krylov_minimisers():
    prob, m, F, N, b, alpha = _dense_system(alpha_scale=0.3)
    shp = (prob.nt, prob.ns)
    n = prob.nt * prob.ns
    Minv = dense(lambda r: oracle.precond(m, 1e-3, r), n, shp)
    assert np.abs(Minv - Minv.T).max() <= 1e-12 * np.abs(Minv).max()
    ev = np.linalg.eigvalsh(0.5 * (Minv + Minv.T))
    print(f"slab M^-1 spectrum: min {ev.min():.3e} max {ev.max():.3e} "
          f"negative fraction {np.mean(ev < 0):.3f}")

    def apply_N(p):
        return (N @ p.ravel()).reshape(shp), None

    # (beyond k ~ 6 this nearly singular, indefinite M^-1 amplifies rounding
    # by ~50x per iteration, so the comparison stops at k = 5)
    for scale in (1.0, -1.0, 10.0):
        for k in (1, 2, 3, 5):
            hk, _ = oracle.pcg(apply_N, lambda r: scale * (Minv @ r.ravel()).reshape(shp),
                               b.reshape(shp), k)
            ref = _krylov_minimiser(N, Minv, b, k)
            assert np.linalg.norm(hk.ravel() - ref) <= 1e-9 * np.linalg.norm(ref), (scale, k)
    # plain CG is PCG with M = I
    for k in (1, 3, 5):
        hk, _ = oracle.pcg(apply_N, lambda r: r.copy(), b.reshape(shp), k)
        ref = _krylov_minimiser(N, np.eye(n), b, k)
        assert np.linalg.norm(hk.ravel() - ref) <= 1e-9 * np.linalg.norm(ref)


def test_pcg_solve_misfit_history():
    # the misfit column tracked by the recurrence e_{k+1} = e_k + a_k F p_k
    # equals ||F h_k - d|| recomputed from scratch
    prob = tiny_problem(nt=20, xs=(47.0,))
    m = oracle.Model(prob, tiny_kappa(prob, 23), RHO)
    d = np.random.default_rng(6).standard_normal((prob.nt, prob.nr))
    for K in (1, 3):
        h, hist, alpha = oracle.pcg_solve(m, d, 1e-3, K)
        assert abs(hist[-1, 3] - np.linalg.norm(m.fwd(h) - d)) <= 1e-12 * np.linalg.norm(d)
        b = m.adj(d)
        assert abs(alpha - 1e-3 * np.linalg.norm(b) / np.linalg.norm(d)) < 1e-18
        assert abs(hist[0, 0] - np.linalg.norm(b)) <= 1e-12 * np.linalg.norm(b)


# ---------------------------------------------------------------------------
# P10: penalty and diagonal scaling (Introduction, the penalty operator;
# Accelerated Iterative Inversion, the preconditioner's outer factors)

def test_penalty_and_dscale_closed_form():
    prob = tiny_problem(xs=(47.0,))
    x = np.random.default_rng(8).standard_normal((prob.nt, prob.ns))
    Ax = oracle.penalty(prob, x)
    D = oracle.dscale(prob, 0.01)
    for n in range(prob.nt):
        for k in range(prob.ns):
            xk = prob.x_src0 + k * prob.h
            assert Ax[n, k] == abs(xk - 47.0) * x[n, k]
    for k in range(prob.ns):
        xk = prob.x_src0 + k * prob.h
        assert abs(D[k] - (1 + (0.01 * (xk - 47.0)) ** 2) ** -0.5) < 1e-15


# ---------------------------------------------------------------------------
# P11: the weighted normal equations (Accelerated Iterative Inversion: the
# normpart system, S* = S^T W_d, A* = A^T W_m; Computing and Symmetrizing
# Lambda: W_m^-1 by the winvcomp formula, "a similar definition" for W_d, and
# W_m by the wcomp formula, all on thin slabs)

def _two_layer(h, dz=5, rdz=-5, c1=2000.0, c2=2500.0, order=4):
    # source line at 150 m in c1, receiver line at 400 m in c2 (interface at
    # 250 m), the receiver line 50 m short of either edge
    nz, nx = int(600 / h), int(2000 / h) + 1
    dt = 0.2 * h / c2
    vel = np.full((nz, nx), c1)
    vel[int(250 / h):, :] = c2
    prob = inputs.Problem(nz=nz, nx=nx, h=h, dt=dt, nt=int(0.5 / dt), order=order,
                          npml=20, z_src=150.0, x_src0=0.0, ns=nx, z_rec=400.0,
                          x_rec0=50.0, nr=nx - int(100 / h), slab_dz=dz, xs=(1000.0,),
                          rslab_dz=rdz)
    return prob, oracle.Model(prob, inputs.kappa_from_velocity(vel, RHO), RHO)


def _weight_plane_errors(h, dz, rdz, f=10.0, c1=2000.0, c2=2500.0):
    prob, m = _two_layer(h, dz, rdz, c1, c2)
    w = inputs.ricker((np.arange(prob.nt) + 0.5) * prob.dt, f)
    jr = int(round((1000.0 - prob.x_rec0) / prob.h))
    wd = m.wd(np.repeat(w[:, None], prob.nr, axis=1))[:, jr]
    wm = m.wm(np.repeat(w[:, None], prob.ns, axis=1))[:, prob.ns // 2]
    ed = np.abs(wd - 2.0 / (RHO * c2) * w).max() / (2.0 / (RHO * c2) * np.abs(w).max())
    em = np.abs(wm - 0.5 * RHO * c1 * w).max() / (0.5 * RHO * c1 * np.abs(w).max())
    return ed, em


@pytest.mark.parametrize("dz,rdz", [(5, -5), (-5, 5)])
def test_plane_wave_weights(dz, rdz):
    # On laterally uniform input a downgoing plane wave has p = rho c v_z, so
    # the pressure-to-source operator of a surface is 2/(rho c) at that
    # surface and its inverse rho c/2.  W_d must take the impedance at the
    # receiver depth, W_m the one at the source depth (the model has a
    # different velocity at each), at second order in h, for either datum side.
    ed10, em10 = _weight_plane_errors(10.0, dz, rdz)
    ed5, em5 = _weight_plane_errors(5.0, dz, rdz)
    assert ed5 < 0.01 and em5 < 0.01
    assert math.log2(ed10 / ed5) > 1.7
    assert math.log2(em10 / em5) > 1.7


@pytest.mark.slow
def test_weighted_composition_is_energy_transmission():
    # Approximate unitarity (the wunitary relation): W_m^-1 F^T W_d F ~ I.  For
    # a plane wave crossing one interface between the source and receiver
    # surfaces it is exactly the energy transmission coefficient
    # 4 Z1 Z2 / (Z1 + Z2)^2 (F scales by Z1 Z2 / (Z1 + Z2), the weights by
    # 2 / Z2 and 2 / Z1), approached at second order in h.
    c1, c2, f = 2000.0, 2500.0, 10.0
    Z1, Z2 = RHO * c1, RHO * c2
    T = 4.0 * Z1 * Z2 / (Z1 + Z2) ** 2
    errs = []
    for h in (10.0, 5.0):
        prob, m = _two_layer(h, 5, -5, c1, c2)
        w = inputs.ricker((np.arange(prob.nt) + 0.5) * prob.dt, f)
        x = np.repeat(w[:, None], prob.ns, axis=1)
        y = m.winv(m.adj(m.wd(m.fwd(x))))[:, prob.ns // 2]
        errs.append(np.abs(y - T * w).max() / (T * np.abs(w).max()))
    assert errs[1] < 0.03
    assert math.log2(errs[0] / errs[1]) > 1.7


def test_weights_symmetric():
    # both weights are symmetric by construction (the exchange J is symmetric
    # and the adjoint sweep is the exact transpose)
    prob = tiny_problem(nz=16, nx=20, L=5, nt=30, ns=16, nr=14, slab_dz=3, rslab_dz=-2,
                        z_src=50.0, z_rec=120.0)
    m = oracle.Model(prob, tiny_kappa(prob, 31), RHO)
    rng = np.random.default_rng(12)
    for op, n in ((m.wd, prob.nr), (m.wm, prob.ns)):
        x = rng.standard_normal((prob.nt, n))
        y = rng.standard_normal((prob.nt, n))
        Wx, Wy = op(x), op(y)
        assert Wx.shape == x.shape
        err = abs(np.sum(x * Wy) - np.sum(Wx * y)) / (np.linalg.norm(Wx) * np.linalg.norm(y))
        assert err < 1e-13


def _weighted_system():
    prob = tiny_problem(nt=20, ns=8, nr=10, xs=(47.0,), rslab_dz=-2)
    m = oracle.Model(prob, tiny_kappa(prob, 29), RHO)
    d = np.random.default_rng(15).standard_normal((prob.nt, prob.nr))
    # an alpha that makes the two terms of N_w comparable on this grid, whose
    # short record lets little of F reach the receivers
    alpha = 2e-4
    return prob, m, d, alpha


def test_weighted_normal_is_gradient_of_weighted_objective():
    # N_w h - b_w is the gradient of
    #   J(h) = 1/2 <F h - d, W_d (F h - d)> + alpha^2/2 <A h, W_m A h>
    # (the einv objective in the weighted norms), checked by central
    # differences, which are exact for a quadratic up to rounding.
    prob, m, d, alpha = _weighted_system()

    def J(h):
        e = m.fwd(h) - d
        Ah = oracle.penalty(prob, h)
        return 0.5 * np.sum(e * m.wd(e)) + 0.5 * alpha ** 2 * np.sum(Ah * m.wm(Ah))

    rng = np.random.default_rng(16)
    b = m.adj(m.wd(d))
    for h in (np.zeros((prob.nt, prob.ns)), rng.standard_normal((prob.nt, prob.ns))):
        Nh, Fh = oracle.normal_w(m, alpha, h)
        assert np.array_equal(Fh, m.fwd(h))
        for _ in range(2):
            u = rng.standard_normal(h.shape)
            fd_dir = 0.5 * (J(h + u) - J(h - u))
            an_dir = np.sum((Nh - b) * u)
            assert abs(fd_dir - an_dir) <= 1e-9 * (abs(fd_dir) + abs(J(h)) + abs(J(u)))
    # both terms matter at this alpha
    h = rng.standard_normal((prob.nt, prob.ns))
    q0, _ = oracle.normal_w(m, 0.0, h)
    q1, _ = oracle.normal_w(m, alpha, h)
    assert 0.1 < np.linalg.norm(q1 - q0) / np.linalg.norm(q0) < 10.0


def test_weighted_pcg_iterates_are_krylov_projections():
    # pcg_solve_w runs Algorithm 1 on N_w h = F^T W_d d with M^-1 = D W^-1 D
    # at alpha_hat = alpha: its iterates are the Galerkin solutions on the
    # Krylov spaces of the dense operators (plain CG with M = I likewise)
    prob, m, d, alpha = _weighted_system()
    shp = (prob.nt, prob.ns)
    n = prob.nt * prob.ns
    Nw = dense(lambda p: oracle.normal_w(m, alpha, p)[0], n, shp)
    assert np.abs(Nw - Nw.T).max() <= 1e-12 * np.abs(Nw).max()
    Minv = dense(lambda r: oracle.precond(m, alpha, r), n, shp)
    b = m.adj(m.wd(d)).ravel()
    for k in (1, 2, 3):
        hk, hist = oracle.pcg_solve_w(m, d, alpha, k)
        ref = _krylov_minimiser(Nw, Minv, b, k)
        assert np.linalg.norm(hk.ravel() - ref) <= 1e-9 * np.linalg.norm(ref), k
        assert abs(hist[-1, 3] - np.linalg.norm(m.fwd(hk) - d)) <= 1e-12 * np.linalg.norm(d)
        hk, _ = oracle.pcg_solve_w(m, d, alpha, k, use_precond=False)
        ref = _krylov_minimiser(Nw, np.eye(n), b, k)
        assert np.linalg.norm(hk.ravel() - ref) <= 1e-9 * np.linalg.norm(ref), k


# ---------------------------------------------------------------------------
# P12: V, the time-reversal inverse and Lambda~ (Time Reversal: the
# approxinv relations; Unitarity: the sv relation; Computing and
# Symmetrizing Lambda: lamtilde, lamtransp, winvcomp)

def test_v_and_lambda_transposes():
    prob = tiny_problem(nz=16, nx=20, L=5, nt=30, ns=16, nr=14, slab_dz=3, rslab_dz=-2,
                        z_src=50.0, z_rec=120.0)
    m = oracle.Model(prob, tiny_kappa(prob, 41), RHO)
    rng = np.random.default_rng(42)
    f = rng.standard_normal((prob.nt, prob.ns))
    r = rng.standard_normal((prob.nt, prob.nr))
    Vf, Vtr = m.fwd_v(f), m.adj_v(r)
    assert abs(np.sum(Vf * r) - np.sum(f * Vtr)) <= 1e-13 * np.linalg.norm(Vf) * np.linalg.norm(r)
    for side, n in (("s", prob.ns), ("r", prob.nr)):
        x = rng.standard_normal((prob.nt, n))
        y = rng.standard_normal((prob.nt, n))
        Lx, LTy = m.lam(x, side), m.lam(y, side, transpose=True)
        assert abs(np.sum(Lx * y) - np.sum(x * LTy)) <= 1e-13 * np.linalg.norm(Lx) * np.linalg.norm(y)
        # winvcomp: half the sum of Lambda~ and its transpose is the
        # symmetrised operator computed with the datum exchange
        sym = 0.5 * (m.lam(x, side) + m.lam(x, side, transpose=True))
        ref = m.winv(x) if side == "s" else m.wd(x)
        assert np.linalg.norm(sym - ref) <= 1e-13 * np.linalg.norm(ref)
        # and Lambda~ itself is not symmetric on this grid
        assert np.linalg.norm(Lx - m.lam(x, side, transpose=True)) > 1e-3 * np.linalg.norm(Lx)


def _v_plane_errors(h, down, f=10.0, c1=2000.0, c2=2500.0):
    # source line in c1, receivers in c2, the interface between them;
    # down: receivers below the sources, else above (layers mirrored)
    nz, nx = int(600 / h), int(2000 / h) + 1
    dt = 0.2 * h / c2
    vel = np.full((nz, nx), c1)
    if down:
        vel[int(250 / h):, :] = c2
        zs, zr = 150.0, 400.0
    else:
        vel[:int(350 / h), :] = c2
        zs, zr = 450.0, 200.0
    prob = inputs.Problem(nz=nz, nx=nx, h=h, dt=dt, nt=int(0.5 / dt), order=4, npml=20,
                          z_src=zs, x_src0=0.0, ns=nx, z_rec=zr, x_rec0=50.0,
                          nr=nx - int(100 / h), slab_dz=5, xs=(1000.0,), rslab_dz=-5)
    m = oracle.Model(prob, inputs.kappa_from_velocity(vel, RHO), RHO)
    w = inputs.ricker((np.arange(prob.nt) + 0.5) * prob.dt, f)
    x = np.repeat(w[:, None], prob.ns, axis=1)
    jr, jc = int(round((1000.0 - prob.x_rec0) / h)), prob.ns // 2
    Z1, Z2 = RHO * c1, RHO * c2
    Vx = m.fwd_v(x)[:, jr]
    Fx = m.fwd(x)
    # peak values: the traces' timing conventions differ by fractions of a
    # step (pressure at whole steps, velocity at half steps), so whole-trace
    # differences would converge at first order only

    def peak(y):
        return y[np.argmax(np.abs(y))]

    # V on a plane wave: the transmitted normal velocity f / (Z1 + Z2), of the
    # same sign whichever way the wave travels (v_z is even across a normal
    # load)
    ev = peak(Vx) * (Z1 + Z2) / peak(w) - 1.0
    # 4 V^T F: the energy transmission coefficient (approxinv, exact in 1D)
    T = 4 * Z1 * Z2 / (Z1 + Z2) ** 2
    et = peak(m.tr_inverse(Fx)[:, jc]) / (T * peak(w)) - 1.0
    # sv: 1/4 Lambda_r F Lambda_s = V
    es = peak(0.25 * m.lam(m.fwd(m.lam(x, "s")), "r")[:, jr]) / peak(Vx) - 1.0
    return abs(ev), abs(et), abs(es)


@pytest.mark.slow
@pytest.mark.parametrize("down", [True, False])
def test_plane_wave_v_time_reversal_and_sv(down):
    e10 = _v_plane_errors(10.0, down)
    e5 = _v_plane_errors(5.0, down)
    print(f"down={down}: V / 4V^T F / sv errors h=10 {e10}, h=5 {e5}")
    for a, b in zip(e10, e5):
        assert b < 0.025
        assert math.log2(a / b) > 1.5


def test_modelling_operator_blocks():
    # the four blocks: (0,0) is F and (1,1) is V; every block's transpose
    # passes the dot test
    prob = tiny_problem(nz=16, nx=20, L=5, nt=30, ns=16, nr=14, z_src=50.0, z_rec=120.0)
    m = oracle.Model(prob, tiny_kappa(prob, 43), RHO)
    rng = np.random.default_rng(44)
    x = rng.standard_normal((prob.nt, prob.ns))
    y = rng.standard_normal((prob.nt, prob.nr))
    assert np.array_equal(m.block(0, 0, x), m.fwd(x))
    assert np.array_equal(m.block(1, 1, x), m.fwd_v(x))
    for src in (0, 1):
        for rec in (0, 1):
            Bx = m.block(src, rec, x)
            BTy = m.block(src, rec, y, transpose=True)
            assert abs(np.sum(Bx * y) - np.sum(x * BTy)) <= 1e-13 * np.linalg.norm(Bx) * np.linalg.norm(y)


@pytest.mark.parametrize("down", [True, False])
def test_plane_wave_off_diagonal_blocks(down):
    # A pressure source radiates pressure Z1 h / 2 to both sides and normal
    # velocity of the sign of the direction of travel; a normal load the
    # reverse (the jump conditions of the Pressure-to-Source section).
    # Through the interface: pressure source -> v_z = s Z1 / (Z1 + Z2),
    # normal load -> p = s Z2 / (Z1 + Z2), s = +1 for receivers below, -1
    # above, at second order in h.
    errs = []
    for h in (10.0, 5.0):
        c1, c2, f = 2000.0, 2500.0, 10.0
        nz, nx = int(600 / h), int(2000 / h) + 1
        dt = 0.2 * h / c2
        vel = np.full((nz, nx), c1)
        if down:
            vel[int(250 / h):, :] = c2
            zs, zr = 150.0, 400.0
        else:
            vel[:int(350 / h), :] = c2
            zs, zr = 450.0, 200.0
        prob = inputs.Problem(nz=nz, nx=nx, h=h, dt=dt, nt=int(0.5 / dt), order=4, npml=20,
                              z_src=zs, x_src0=0.0, ns=nx, z_rec=zr, x_rec0=50.0,
                              nr=nx - int(100 / h), slab_dz=5, xs=(1000.0,))
        m = oracle.Model(prob, inputs.kappa_from_velocity(vel, RHO), RHO)
        w = inputs.ricker((np.arange(prob.nt) + 0.5) * prob.dt, f)
        x = np.repeat(w[:, None], prob.ns, axis=1)
        jr = int(round((1000.0 - prob.x_rec0) / h))
        Z1, Z2 = RHO * c1, RHO * c2
        sgn = 1.0 if down else -1.0

        def peak(y):
            return y[np.argmax(np.abs(y))]

        hv = peak(m.block(0, 1, x)[:, jr]) / (sgn * Z1 / (Z1 + Z2) * peak(w)) - 1.0
        fp = peak(m.block(1, 0, x)[:, jr]) / (sgn * Z2 / (Z1 + Z2) * peak(w)) - 1.0
        errs.append((abs(hv), abs(fp)))
    for a, b in zip(errs[0], errs[1]):
        assert b < 0.02
        assert math.log2(a / b) > 1.5


# ---------------------------------------------------------------------------
# P13: the misfit gradient in kappa (adjoint state of the discrete scheme)

@pytest.mark.parametrize("order", [4, 8])
def test_misfit_gradient_central_differences(order):
    # <g, dk> against (J(k + e dk) - J(k - e dk)) / 2e, for dk on physical
    # cells off the grid's edges (the absorbing layer copies only edge
    # values) and off the fastest cell (whose value sets the layer's
    # damping); the central difference of this smooth J is exact to O(e^2)
    prob = tiny_problem(order=order, nz=16, nx=20, L=5, nt=40, ns=14, nr=16, z_src=50.0,
                        z_rec=120.0)
    kap = tiny_kappa(prob, 51)
    m = oracle.Model(prob, kap, RHO)
    rng = np.random.default_rng(52)
    h = rng.standard_normal((prob.nt, prob.ns))
    d = rng.standard_normal((prob.nt, prob.nr)) * np.abs(m.fwd(h)).max()
    g, J0 = oracle.misfit_gradient(m, h, d)
    assert g.shape == kap.shape
    assert abs(J0 - 0.5 * np.sum((m.fwd(h) - d) ** 2)) <= 1e-12 * J0

    def J(k):
        mm = oracle.Model(prob, k, RHO)
        return 0.5 * np.sum((mm.fwd(h) - d) ** 2)

    for trial in range(2):
        dk = np.zeros_like(kap)
        dk[1:-1, 1:-1] = rng.standard_normal((prob.nz - 2, prob.nx - 2))
        dk[np.unravel_index(np.argmax(kap), kap.shape)] = 0.0
        eps = 1e-5 * kap.mean() / np.abs(dk).max()
        fdiff = (J(kap + eps * dk) - J(kap - eps * dk)) / (2 * eps)
        an = float(np.sum(g * dk))
        assert abs(fdiff - an) <= 1e-6 * abs(an), (fdiff, an)
    # a single interior cell, both ways round
    dk = np.zeros_like(kap)
    dk[8, 9] = 1.0
    eps = 1e-5 * kap[8, 9]
    fdiff = (J(kap + eps * dk) - J(kap - eps * dk)) / (2 * eps)
    assert abs(fdiff - g[8, 9]) <= 1e-5 * abs(g).max()


def test_reduced_objective_gradient_is_partial_gradient():
    # variable projection: with h*(kappa) the exact minimiser of
    # 1/2 ||F h - d||^2 + alpha^2/2 ||A h||^2, the reduced objective's
    # derivative in kappa is the misfit gradient at fixed h = h*
    # (the penalty does not depend on kappa); checked by central
    # differences of the reduced objective, each side solved densely
    prob = tiny_problem(nz=12, nx=16, L=4, nt=16, ns=6, nr=10, xs=(47.0,))
    kap = tiny_kappa(prob, 61)
    d = np.random.default_rng(62).standard_normal((prob.nt, prob.nr))
    Adiag = np.tile(oracle.ops.lateral_distance(prob), prob.nt)
    n = prob.nt * prob.ns

    def solve(k):
        m = oracle.Model(prob, k, RHO)
        F = dense(m.fwd, n, (prob.nt, prob.ns))
        alpha = 0.2 * np.linalg.norm(F, 2) / Adiag.max()
        N = F.T @ F + alpha ** 2 * np.diag(Adiag ** 2)
        hs = np.linalg.solve(N, F.T @ d.ravel())
        r = F @ hs - d.ravel()
        return m, hs.reshape(prob.nt, prob.ns), 0.5 * r @ r + 0.5 * alpha ** 2 * np.sum((Adiag * hs) ** 2), alpha

    m, hs, J0, alpha = solve(kap)
    g, _ = oracle.misfit_gradient(m, hs, d)
    rng = np.random.default_rng(63)
    dk = np.zeros_like(kap)
    dk[1:-1, 1:-1] = rng.standard_normal((prob.nz - 2, prob.nx - 2))
    dk[np.unravel_index(np.argmax(kap), kap.shape)] = 0.0
    eps = 1e-5 * kap.mean() / np.abs(dk).max()

    def Jr(k):
        # alpha held at its value for kappa (it is a fixed weight of the problem)
        mm = oracle.Model(prob, k, RHO)
        F = dense(mm.fwd, n, (prob.nt, prob.ns))
        N = F.T @ F + alpha ** 2 * np.diag(Adiag ** 2)
        hk = np.linalg.solve(N, F.T @ d.ravel())
        r = F @ hk - d.ravel()
        return 0.5 * r @ r + 0.5 * alpha ** 2 * np.sum((Adiag * hk) ** 2)

    fdiff = (Jr(kap + eps * dk) - Jr(kap - eps * dk)) / (2 * eps)
    an = float(np.sum(g * dk))
    assert abs(fdiff - an) <= 1e-5 * abs(an), (fdiff, an)


def test_normal_load_subproblem_converges_to_dense_solution():
    # the normal-load form: N_v = V^T V + alpha^2 A^T A assembled densely
    # from V is SPD; Algorithm 1 with M = I reaches its Cholesky solution,
    # and alpha follows the relative rule with b = V^T d
    prob = tiny_problem(nt=20, ns=8, nr=10, xs=(47.0,))
    m = oracle.Model(prob, tiny_kappa(prob, 71), RHO)
    n = prob.nt * prob.ns
    Vd = dense(m.fwd_v, n, (prob.nt, prob.ns))
    d = np.random.default_rng(72).standard_normal((prob.nt, prob.nr))
    b = Vd.T @ d.ravel()
    alpha = 1e-2 * np.linalg.norm(b) / np.linalg.norm(d)
    A = np.tile(oracle.ops.lateral_distance(prob), prob.nt)
    N = Vd.T @ Vd + alpha ** 2 * np.diag(A * A)
    Lc = np.linalg.cholesky(N)
    hstar = np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))
    h, hist, al = oracle.pcg_solve_v(m, d, 1e-2, 400)
    assert abs(al - alpha) <= 1e-15 * alpha
    assert np.linalg.norm(h.ravel() - hstar) <= 1e-8 * np.linalg.norm(hstar)
    assert abs(hist[-1, 3] - np.linalg.norm(m.fwd_v(h) - d)) <= 1e-10 * np.linalg.norm(d)


# ---------------------------------------------------------------------------
# Variable density (the operators of the Operators section carry kappa and
# rho): rho at the pressure nodes, buoyancy at the velocity half nodes as the
# mean of 1/rho at the two nodes.

def _rho_field(prob, seed=3):
    rng = np.random.default_rng(seed)
    return rng.uniform(800.0, 2600.0, size=(prob.nz, prob.nx))


@pytest.mark.parametrize("order", [4, 8])
def test_variable_density_dot_products(order):
    prob = tiny_problem(order=order, nz=14, nx=18, L=4, nt=40)
    m = oracle.Model(prob, tiny_kappa(prob), _rho_field(prob))
    rng = np.random.default_rng(order)
    x = rng.standard_normal((prob.nt, prob.ns))
    y = rng.standard_normal((prob.nt, prob.nr))
    Fx, Fty = m.fwd(x), m.adj(y)
    assert abs(np.sum(Fx * y) - np.sum(x * Fty)) <= 1e-13 * np.linalg.norm(Fx) * np.linalg.norm(y)
    a = rng.standard_normal((prob.nt, prob.ns))
    b = rng.standard_normal((prob.nt, prob.ns))
    P, V = m.slab_fwd(x)
    lhs = np.sum(P * a) + np.sum(V * b)
    rhs = np.sum(x * m.slab_adj(a, b))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(P * P) + np.sum(V * V)) * np.sqrt(
        np.sum(a * a) + np.sum(b * b))


def test_variable_density_energy_conserved():
    # no absorbing layer, the source off after its first samples: the
    # discrete energy with rho at each velocity's own node is constant
    prob = tiny_problem(order=8, nz=20, nx=24, L=0, nt=160, z_src=95.0, z_rec=150.0,
                        ns=10, nr=12)
    rho = _rho_field(prob, 5)
    g = Grid(tiny_kappa(prob), rho, prob.h, prob.dt, 0, prob.pml_R, prob.order)
    src = np.zeros((prob.nt, prob.ns))
    src[:6] = np.random.default_rng(2).standard_normal((6, prob.ns))
    _, _, E = forward(g, prob.nt, h_src=(g.p_line(prob.z_src, prob.x_src0, prob.ns), src),
                      energy=True)
    E = np.array(E[8:])
    assert np.max(np.abs(E - E[0])) <= 1e-13 * abs(E[0])


def test_constant_density_array_equals_scalar():
    prob = tiny_problem(order=8)
    kap = tiny_kappa(prob)
    ms = oracle.Model(prob, kap, RHO)
    ma = oracle.Model(prob, kap, np.full((prob.nz, prob.nx), RHO))
    x = np.random.default_rng(4).standard_normal((prob.nt, prob.ns))
    for a, b in ((ma.fwd(x), ms.fwd(x)), (ma.winv(x), ms.winv(x))):
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def _density_jump_error(h, below):
    # a laterally uniform pressure source at 200 m in c = 2000 m/s, density
    # 1000 on the nodes above 400 m and 2500 from 400 m down (impedances Z1,
    # Z2 = 2.5 Z1), so that the continuum interface lies midway between the
    # last node of one density and the first of the other, z_i = 400 - h/2:
    # receivers at 100 m see the direct wave (rho1 c / 2) w(t - tau_d) and
    # its reflection R times it, R = (Z2 - Z1) / (Z2 + Z1); receivers at
    # 500 m the transmitted wave T (rho1 c / 2) w(t - tau_t), T = 2 Z2 /
    # (Z1 + Z2) (pressure, normal incidence)
    c, f, rho1, rho2 = 2000.0, 10.0, 1000.0, 2500.0
    nz, nx = int(700 / h), int(2000 / h) + 1
    dt = 0.25 * h / c
    nt = int(0.42 / dt)
    z_rec = 500.0 if below else 100.0
    prob = inputs.Problem(nz=nz, nx=nx, h=h, dt=dt, nt=nt, order=8, npml=20,
                          z_src=200.0, x_src0=0.0, ns=nx, z_rec=z_rec, x_rec0=0.0, nr=nx,
                          slab_dz=5, xs=(1000.0,))
    zi = int(round(400.0 / h))
    rho = np.full((nz, nx), rho1)
    rho[zi:, :] = rho2
    kappa = rho * c * c
    m = oracle.Model(prob, kappa, rho)
    w = inputs.ricker((np.arange(nt) + 0.5) * dt, f)
    d = m.fwd(np.repeat(w[:, None], nx, axis=1))[:, nx // 2]
    t = (np.arange(nt) + 1) * dt
    Z1, Z2 = rho1 * c, rho2 * c
    amp = 0.5 * rho1 * c
    z_int = (zi - 0.5) * h
    if below:
        expect = (2 * Z2 / (Z1 + Z2)) * amp * inputs.ricker(t - (z_rec - 200.0) / c, f)
    else:
        R = (Z2 - Z1) / (Z2 + Z1)
        expect = amp * (inputs.ricker(t - (200.0 - z_rec) / c, f)
                        + R * inputs.ricker(t - (2 * z_int - 200.0 - z_rec) / c, f))
    return np.abs(d - expect).max() / np.abs(expect).max()


@pytest.mark.slow
@pytest.mark.parametrize("below", [False, True])
def test_plane_wave_density_jump(below):
    # reflection and transmission at a density-only impedance jump (same
    # velocity on both sides), at second order as the grid is refined (the
    # mean of the two node densities at a velocity half node; the mean of
    # their reciprocals converges at first order only)
    e10 = _density_jump_error(10.0, below)
    e5 = _density_jump_error(5.0, below)
    assert e5 < 5e-3, (e10, e5)
    assert math.log2(e10 / e5) > 1.6, (e10, e5)
