"""Pins of the oracle's C engine (oracle/cprop.c), which runs the oracle's
time stepping as plain C loops for the full-length golden runs.

It must compute what the NumPy time stepping computes (that one is pinned
by the physics and transposition tests of test_oracle_pins.py): equal to
rounding on every operator built on forward / adjoint runs, for both
stencil orders, both slab datum signs and lines on and between rows.  It is
also pinned directly by the dot-product test (its adjoint is the transpose
of its forward run), so a slip in either direction fails on its own.
"""
import numpy as np
import pytest

import inputs
import oracle

RHO = 1000.0


def problem(order, slab_dz, z_src, z_rec):
    return inputs.Problem(nz=21, nx=29, h=10.0, dt=1e-3, nt=50, order=order, npml=5,
                          z_src=z_src, x_src0=20.0, ns=19, z_rec=z_rec, x_rec0=0.0, nr=29,
                          slab_dz=slab_dz, xs=(113.0,), rslab_dz=-2)


def models(prob, seed):
    rng = np.random.default_rng(seed)
    kappa = RHO * rng.uniform(1800.0, 2400.0, size=(prob.nz, prob.nx)) ** 2
    return oracle.Model(prob, kappa, RHO), oracle.Model(prob, kappa, RHO, engine="c")


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("order,slab_dz,z_src,z_rec", [
    (4, 3, 45.0, 150.0), (8, -3, 47.5, 152.5), (8, 4, 150.0, 40.0)])
def test_c_engine_equals_numpy_engine(order, slab_dz, z_src, z_rec):
    prob = problem(order, slab_dz, z_src, z_rec)
    mn, mc = models(prob, order + slab_dz)
    rng = np.random.default_rng(3)
    h = rng.standard_normal((prob.nt, prob.ns))
    r = rng.standard_normal((prob.nt, prob.nr))
    pairs = [
        (mc.fwd(h), mn.fwd(h)), (mc.adj(r), mn.adj(r)),
        (mc.fwd_v(h), mn.fwd_v(h)), (mc.adj_v(r), mn.adj_v(r)),
        (mc.winv(h), mn.winv(h)), (mc.wd(r), mn.wd(r)), (mc.wm(h), mn.wm(h)),
        (mc.lam(h), mn.lam(h)), (mc.lam(h, transpose=True), mn.lam(h, transpose=True)),
        (mc.slab_adj(h, 2 * h), mn.slab_adj(h, 2 * h)),
    ]
    for src in (0, 1):
        for rec in (0, 1):
            pairs.append((mc.block(src, rec, h), mn.block(src, rec, h)))
            pairs.append((mc.block(src, rec, r, transpose=True),
                          mn.block(src, rec, r, transpose=True)))
    errs = [rel(a, b) for a, b in pairs]
    assert max(errs) <= 1e-14, errs


@pytest.mark.parametrize("order", [4, 8])
def test_c_engine_dot_product(order):
    # <F x, y> = <x, F^T y> and the same for the slab operator X, computed
    # by the C engine alone
    prob = problem(order, 3, 45.0, 150.0)
    _, mc = models(prob, 11)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((prob.nt, prob.ns))
    y = rng.standard_normal((prob.nt, prob.nr))
    Fx, Fty = mc.fwd(x), mc.adj(y)
    assert abs(np.sum(Fx * y) - np.sum(x * Fty)) <= 1e-13 * np.linalg.norm(Fx) * np.linalg.norm(y)
    a = rng.standard_normal((prob.nt, prob.ns))
    b = rng.standard_normal((prob.nt, prob.ns))
    P, V = mc.slab_fwd(x)
    lhs = np.sum(P * a) + np.sum(V * b)
    rhs = np.sum(x * mc.slab_adj(a, b))
    assert abs(lhs - rhs) <= 1e-13 * np.sqrt(np.sum(P * P) + np.sum(V * V)) * np.sqrt(
        np.sum(a * a) + np.sum(b * b))


def test_c_engine_pcg_equals_numpy_engine():
    prob = problem(8, 3, 45.0, 150.0)
    mn, mc = models(prob, 7)
    d = mn.fwd(inputs.spike_gather(prob, inputs.source_wavelet(prob, 25.0)))
    hn, histn, an = oracle.pcg_solve(mn, d, 1e-3, 4)
    hc, histc, ac = oracle.pcg_solve(mc, d, 1e-3, 4)
    assert rel(hc, hn) <= 1e-13
    assert np.allclose(histc, histn, rtol=1e-13, atol=0)
    assert abs(ac - an) <= 1e-14 * an
