"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: FP64 wavefields 1e-12 relative L2 per propagation (the
rounding of two independent FP64 evaluations of the same linear map); FP32
1e-5 per propagation and 1e-4 on the CG solution (the stated targets).
"""
import math

import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402

RHO = 1000.0
TOL = {"f64": 1e-12, "f32": 1e-5}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def dev(x, fd):
    return torch.tensor(np.ascontiguousarray(x),
                        dtype=torch.float64 if fd == "f64" else torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def small_problem(order=8, nshots=2, **kw):
    # 3 tiles across x with a ragged tail, off-grid source and receiver depths
    base = dict(nz=37, nx=150, h=10.0, dt=1e-3, nt=200, order=order, npml=10,
                z_src=45.0, x_src0=30.0, ns=100, z_rec=203.0, x_rec0=0.0, nr=150,
                slab_dz=5, xs=tuple(300.0 + 417.0 * s for s in range(nshots)))
    base.update(kw)
    return inputs.Problem(**base)


def small_kappa(prob, seed=1):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1800.0, 2400.0, size=(prob.nz, prob.nx))
    return RHO * c * c


@pytest.fixture(scope="module")
def setups():
    cache = {}

    def get(order, fd, nshots=2, **kw):
        key = (order, fd, nshots, tuple(sorted(kw.items())))
        if key not in cache:
            prob = small_problem(order, nshots, **kw)
            kap = small_kappa(prob)
            cache[key] = (prob, kap, oracle.Model(prob, kap, RHO),
                          ssx.Context(prob, kap, RHO, field_dtype=fd))
        return cache[key]
    yield get
    for v in cache.values():
        v[3].close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("order", [4, 8])
def test_fwd_adj_parity(setups, fd, order):
    prob, kap, m, ctx = setups(order, fd)
    print(f"case fwd/adj order={order} dtype={fd}", flush=True)
    rng = np.random.default_rng(order)
    h = rng.standard_normal((2, prob.nt, prob.ns))
    r = rng.standard_normal((2, prob.nt, prob.nr))
    d = host(ctx.fwd(dev(h, fd), ctx.empty_r()))
    g = host(ctx.adj(dev(r, fd), ctx.empty_s()))
    for s in range(2):
        assert rel(d[s], m.fwd(h[s])) < TOL[fd]
        assert rel(g[s], m.adj(r[s])) < TOL[fd]


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("order,dz", [(4, 5), (8, -5), (8, 3)])
def test_slab_parity(setups, fd, order, dz):
    prob, kap, m, ctx = setups(order, fd, slab_dz=dz)
    print(f"case slab order={order} dz={dz} dtype={fd}", flush=True)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((2, prob.nt, prob.ns))
    a = rng.standard_normal((2, prob.nt, prob.ns))
    b = rng.standard_normal((2, prob.nt, prob.ns))
    P, V = ctx.slab_fwd(dev(f, fd), ctx.empty_s(), ctx.empty_s())
    P, V = host(P), host(V)
    fb = host(ctx.slab_adj(dev(a, fd), dev(b, fd), ctx.empty_s()))
    for s in range(2):
        Pr, Vr = m.slab_fwd(f[s])
        assert rel(P[s], Pr) < TOL[fd]
        assert rel(V[s], Vr) < TOL[fd]
        assert rel(fb[s], m.slab_adj(a[s], b[s])) < TOL[fd]


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_penalty_precond_normal_parity(setups, fd):
    prob, kap, m, ctx = setups(8, fd)
    print(f"case penalty/precond/normal dtype={fd}", flush=True)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, prob.nt, prob.ns))
    xt = dev(x, fd)
    tol = 1e-15 if fd == "f64" else 1e-7
    for op, fn in ((ssx.PEN_A, lambda v, s: oracle.penalty(prob, v, s)),
                   (ssx.PEN_ATA, lambda v, s: oracle.penalty(prob, oracle.penalty(prob, v, s), s)),
                   (ssx.PEN_DHALF, lambda v, s: oracle.dscale(prob, 2e-3, s)[None, :] * v)):
        y = host(ctx.penalty(op, 2e-3, xt, ctx.empty_s()))
        for s in range(2):
            assert rel(y[s], fn(x[s], s)) < tol, op
    g = host(ctx.precond(1e-3, xt, ctx.empty_s()))
    for s in range(2):
        assert rel(g[s], oracle.precond(m, 1e-3, x[s], s)) < TOL[fd]
    Fp = ctx.empty_r()
    q = host(ctx.normal(0.37, xt, ctx.empty_s(), Fp))
    Fp = host(Fp)
    for s in range(2):
        qr, Fpr = oracle.normal(m, 0.37, x[s], s)
        assert rel(q[s], qr) < TOL[fd]
        assert rel(Fp[s], Fpr) < TOL[fd]


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_gpu_dot_product_tests(setups, fd):
    # the paper's adjoint test, run entirely on the device
    prob, kap, m, ctx = setups(8, fd)
    print(f"case gpu dot test dtype={fd}", flush=True)
    rng = np.random.default_rng(5)
    x = dev(rng.standard_normal((2, prob.nt, prob.ns)), fd)
    y = dev(rng.standard_normal((2, prob.nt, prob.nr)), fd)
    Fx = ctx.fwd(x, ctx.empty_r())
    Fty = ctx.adj(y, ctx.empty_s())
    lhs, rhs = ctx.dot(Fx, y), ctx.dot(x, Fty)
    nrm = np.sqrt(ctx.dot(Fx, Fx) * ctx.dot(y, y))
    tol = 1e-13 if fd == "f64" else 2e-6
    assert np.all(np.abs(lhs - rhs) <= tol * nrm), (lhs, rhs)
    # FP64 reduction itself against numpy
    ref = [float(np.dot(host(Fx)[s].ravel(), host(y)[s].ravel())) for s in range(2)]
    assert np.allclose(lhs, ref, rtol=1e-12)


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("use_precond", [True, False])
def test_pcg_parity_small(setups, fd, use_precond):
    prob, kap, m, ctx = setups(8, fd)
    print(f"case pcg small dtype={fd} precond={use_precond}", flush=True)
    rng = np.random.default_rng(6)
    d = rng.standard_normal((2, prob.nt, prob.nr))
    K = 5
    h, hist, it, st = ctx.pcg_solve(dev(d, fd), 1e-3, K, use_precond=use_precond)
    h = host(h)
    assert it == K and st == 0
    tol = 1e-10 if fd == "f64" else 1e-4
    for s in range(2):
        hr, histr, _ = oracle.pcg_solve(m, d[s], 1e-3, K, use_precond=use_precond, shot=s)
        assert rel(h[s], hr) < tol
        assert np.allclose(hist[s], histr, rtol=10 * tol, atol=0)


def test_pcg_zero_data_is_converged(setups):
    prob, kap, m, ctx = setups(8, "f64")
    d = torch.zeros((2, prob.nt, prob.nr), dtype=torch.float64, device="cuda")
    h, hist, it, st = ctx.pcg_solve(d, 1e-3, 3)
    assert st == 0
    assert float(torch.abs(h).max()) == 0.0


@pytest.fixture(scope="module")
def c1_reference():
    wl = inputs.workload(1)
    prob = wl.prob
    m = oracle.Model(prob, wl.kappa, wl.rho)
    w = inputs.source_wavelet(prob, wl.freq)
    d = m.fwd(inputs.spike_gather(prob, w))
    h, hist, alpha = oracle.pcg_solve(m, d, wl.alpha_rel, wl.K)
    return wl, d, h, hist


def test_pcg_parity_c1_fp64(c1_reference):
    # the full small configuration: 101 x 201 lens model, 2-4, 1000 steps,
    # 10 preconditioned iterations, FP64
    wl, d, h_ref, hist_ref = c1_reference
    print("case pcg c1 f64", flush=True)
    ctx = ssx.Context(wl.prob, wl.kappa, wl.rho, field_dtype="f64")
    h, hist, it, st = ctx.pcg_solve(dev(d[None], "f64"), wl.alpha_rel, wl.K)
    assert st == 0 and it == wl.K
    assert rel(host(h)[0], h_ref) < 1e-9
    assert np.allclose(hist[0], hist_ref, rtol=1e-9)
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("order", [4, 8])
def test_parity_with_interior_tiles(fd, order):
    # a grid with interior tiles (no per-cell tests) beside frame and line
    # tiles, lines deep inside and part width: F, F^T, X, X^T
    prob = small_problem(order, 1, nz=100, nx=300, nt=150, z_src=603.0, x_src0=450.0,
                         ns=150, z_rec=455.0, x_rec0=1000.0, nr=170, xs=(1700.0,))
    print(f"case interior parity order={order} dtype={fd}", flush=True)
    kap = small_kappa(prob, seed=2)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(11)
    h = rng.standard_normal((1, prob.nt, prob.ns))
    r = rng.standard_normal((1, prob.nt, prob.nr))
    d = host(ctx.fwd(dev(h, fd), ctx.empty_r()))
    g = host(ctx.adj(dev(r, fd), ctx.empty_s()))
    P, V = ctx.slab_fwd(dev(h, fd), ctx.empty_s(), ctx.empty_s())
    f = host(ctx.slab_adj(dev(h, fd), dev(r[:, :, :prob.ns], fd), ctx.empty_s()))
    Pr, Vr = m.slab_fwd(h[0])
    assert rel(d[0], m.fwd(h[0])) < TOL[fd]
    assert rel(g[0], m.adj(r[0])) < TOL[fd]
    assert rel(host(P)[0], Pr) < TOL[fd] and rel(host(V)[0], Vr) < TOL[fd]
    assert rel(f[0], m.slab_adj(h[0], r[0, :, :prob.ns])) < TOL[fd]
    ctx.close()


def bench_context(wl, fd):
    """A context in the launch configuration bench.py times (autotuned)."""
    from paper_2203_16573_amd import autotune
    ctx = ssx.Context(wl.prob, wl.kappa, wl.rho, field_dtype=fd)
    choice = autotune.choose(wl.prob, wl.kappa, wl.rho, field_dtype=fd)
    autotune.apply(ctx, choice)
    print(f"  launch shape {ctx.launch_shape()} choice "
          f"{ {k: v for k, v in choice.items() if k != 'us'} }", flush=True)
    return ctx


def truncated_parity(wl, fd, N, shots, tol, seed):
    # F and the slab X are causal and time-invariant: the first N output
    # samples equal an N-step oracle run on the first N inputs; F^T and X^T
    # likewise for the last N samples.
    prob = wl.prob
    S = prob.nshots
    rng = np.random.default_rng(seed)
    h = np.zeros((S, prob.nt, prob.ns))
    h[:, :N] = rng.standard_normal((S, N, prob.ns))
    r = np.zeros((S, prob.nt, prob.nr))
    r[:, -N:] = rng.standard_normal((S, N, prob.nr))
    a = np.zeros((S, prob.nt, prob.ns))
    a[:, -N:] = rng.standard_normal((S, N, prob.ns))
    b = np.zeros((S, prob.nt, prob.ns))
    b[:, -N:] = rng.standard_normal((S, N, prob.ns))
    vf = "f64" if fd == "f64" else "f32"
    ctx = bench_context(wl, fd)
    d = host(ctx.fwd(dev(h, vf), ctx.empty_r()))
    g = host(ctx.adj(dev(r, vf), ctx.empty_s()))
    P, V = ctx.slab_fwd(dev(h, vf), ctx.empty_s(), ctx.empty_s())
    P, V = host(P), host(V)
    f = host(ctx.slab_adj(dev(a, vf), dev(b, vf), ctx.empty_s()))
    ctx.close()
    errs = []
    for s in shots:
        m = oracle.Model(prob.replace(nt=N, xs=(prob.xs[s],)), wl.kappa, wl.rho)
        Pr, Vr = m.slab_fwd(h[s, :N])
        errs += [rel(d[s, :N], m.fwd(h[s, :N])), rel(g[s, -N:], m.adj(r[s, -N:])),
                 rel(P[s, :N], Pr), rel(V[s, :N], Vr),
                 rel(f[s, -N:], m.slab_adj(a[s, -N:], b[s, -N:]))]
    print(f"  relative errors {['%.2e' % e for e in errs]}", flush=True)
    assert max(errs) < tol, errs


def test_c2_full_size_truncated_parity():
    # 801 x 1601 at 5 m, 2-8, FP32, nt = 4000, bench's launch configuration
    print("case c2 truncated parity", flush=True)
    truncated_parity(inputs.workload(2), "f32", 40, (0,), 1e-5, 7)


@pytest.mark.parametrize("fd,tol", [("f16", 1e-2), ("bf16", 5e-2)])
def test_c4_full_size_truncated_parity(fd, tol):
    # the c2 grid with 16-bit wavefield storage (FP32 arithmetic)
    print(f"case c4 truncated parity {fd}", flush=True)
    truncated_parity(inputs.workload(4), fd, 40, (0,), tol, 17)


def test_c2_full_size_dot_product():
    # full 4000-step propagations at the benchmark size, FP32 fields with
    # FP64 reductions
    wl = inputs.workload(2)
    prob = wl.prob
    print("case c2 dot test", flush=True)
    ctx = ssx.Context(prob, wl.kappa, wl.rho, field_dtype="f32")
    rng = np.random.default_rng(8)
    x = dev(rng.standard_normal((1, prob.nt, prob.ns)), "f32")
    y = dev(rng.standard_normal((1, prob.nt, prob.nr)), "f32")
    Fx = ctx.fwd(x, ctx.empty_r())
    Fty = ctx.adj(y, ctx.empty_s())
    lhs, rhs = ctx.dot(Fx, y)[0], ctx.dot(x, Fty)[0]
    nrm = math.sqrt(ctx.dot(Fx, Fx)[0] * ctx.dot(y, y)[0])
    ctx.close()
    assert abs(lhs - rhs) <= 1e-5 * nrm, (lhs, rhs, nrm)
