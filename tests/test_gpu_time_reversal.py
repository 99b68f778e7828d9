"""Parity of V, its transpose, the time-reversal inverse 4 V^T and Lambda~
(with its transpose, on either thin slab) on the HIP path with the FP64
oracle.  Tolerances: 1e-12 (FP64) and 1e-5 (FP32) relative L2 per
operator."""
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


def problem(order=8, nshots=2, **kw):
    # 3 tiles across x with a ragged tail; off-grid depths; part-width lines
    base = dict(nz=37, nx=150, h=10.0, dt=1e-3, nt=200, order=order, npml=10,
                z_src=45.0, x_src0=30.0, ns=100, z_rec=203.0, x_rec0=10.0, nr=130,
                slab_dz=5, rslab_dz=-4, xs=tuple(300.0 + 417.0 * s for s in range(nshots)))
    base.update(kw)
    return inputs.Problem(**base)


def kappa(prob, seed=1):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1800.0, 2400.0, size=(prob.nz, prob.nx))
    return RHO * c * c


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("order,zs,zr", [(4, 45.0, 203.0), (8, 250.0, 37.5)])
def test_v_parity(fd, order, zs, zr):
    prob = problem(order, z_src=zs, z_rec=zr)
    print(f"case V order={order} zs={zs} zr={zr} dtype={fd}", flush=True)
    kap = kappa(prob, order)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(order)
    f = rng.standard_normal((2, prob.nt, prob.ns))
    r = rng.standard_normal((2, prob.nt, prob.nr))
    y = host(ctx.fwd_v(dev(f, fd), ctx.empty_r()))
    g = host(ctx.adj_v(dev(r, fd), ctx.empty_s()))
    h = host(ctx.tr_inverse(dev(r, fd), ctx.empty_s()))
    for s in range(2):
        assert rel(y[s], m.fwd_v(f[s])) < TOL[fd]
        gr = m.adj_v(r[s])
        assert rel(g[s], gr) < TOL[fd]
        assert rel(h[s], 4.0 * gr) < TOL[fd]
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("side", [0, 1])
def test_lambda_parity(fd, side):
    prob = problem(8)
    print(f"case lambda side={side} dtype={fd}", flush=True)
    kap = kappa(prob, 3)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    n = prob.ns if side == 0 else prob.nr
    rng = np.random.default_rng(10 + side)
    x = rng.standard_normal((2, prob.nt, n))
    out = dev(np.zeros((2, prob.nt, n)), fd)
    for transpose in (False, True):
        y = host(ctx.lam(side, transpose, dev(x, fd), out))
        for s in range(2):
            assert rel(y[s], m.lam(x[s], "s" if side == 0 else "r", transpose)) < TOL[fd]
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_v_with_interior_tiles_and_tile_loop(fd):
    # lines deep inside a grid with interior tiles: the tile-loop lists must
    # count the normal-velocity rows of both lines as line rows
    prob = problem(8, 1, nz=100, nx=300, nt=150, z_src=603.0, x_src0=450.0, ns=150,
                   z_rec=455.0, x_rec0=1000.0, nr=170, xs=(1700.0,))
    print(f"case V interior tiles dtype={fd}", flush=True)
    kap = kappa(prob, 2)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(12)
    f = rng.standard_normal((1, prob.nt, prob.ns))
    r = rng.standard_normal((1, prob.nt, prob.nr))
    ref_y, ref_g = m.fwd_v(f[0]), m.adj_v(r[0])
    results = []
    for loop in (0, 1):
        ctx.set_option(ssx.OPT_TILE_LOOP, loop)
        y = ctx.fwd_v(dev(f, fd), ctx.empty_r())
        g = ctx.adj_v(dev(r, fd), ctx.empty_s())
        results.append((y.cpu(), g.cpu()))
        assert rel(host(y)[0], ref_y) < TOL[fd]
        assert rel(host(g)[0], ref_g) < TOL[fd]
    assert torch.equal(results[0][0], results[1][0]) and torch.equal(results[0][1], results[1][1])
    ctx.close()


def test_v_needs_velocity_rows():
    # a receiver line on the last physical row has no normal-velocity row
    # pair below it: V is refused, the other operators work
    prob = problem(8, 1, z_rec=360.0, xs=(500.0,))
    ctx = ssx.Context(prob, kappa(prob), RHO, field_dtype="f32")
    x = ctx.empty_s().zero_()
    r = ctx.empty_r().zero_()
    for call in (lambda: ctx.fwd_v(x, ctx.empty_r()), lambda: ctx.adj_v(r, ctx.empty_s()),
                 lambda: ctx.tr_inverse(r, ctx.empty_s())):
        with pytest.raises(ssx.SSXError) as e:
            call()
        assert e.value.status == 1
    ctx.fwd(x, ctx.empty_r())
    ctx.close()


def test_v_transpose_at_production_size():
    # at the 801 x 1601 size, 4000 steps, in the launch configuration the
    # benchmark times: <V f, r> = <f, V^T r>
    from test_gpu_parity import bench_context
    wl = inputs.workload(2)
    print("case V dot test c2 f32", flush=True)
    ctx = bench_context(wl, "f32")
    prob = wl.prob
    rng = np.random.default_rng(31)
    f = dev(rng.standard_normal((1, prob.nt, prob.ns)), "f32")
    r = dev(rng.standard_normal((1, prob.nt, prob.nr)), "f32")
    Vf = ctx.fwd_v(f, ctx.empty_r())
    Vtr = ctx.adj_v(r, ctx.empty_s())
    lhs, rhs = ctx.dot(Vf, r)[0], ctx.dot(f, Vtr)[0]
    nrm = np.sqrt(ctx.dot(Vf, Vf)[0] * ctx.dot(r, r)[0])
    print(f"  transpose defect {abs(lhs - rhs) / nrm:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * nrm
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_modelling_operator_blocks_parity(fd):
    prob = problem(8, z_src=45.0, z_rec=203.0)
    print(f"case blocks dtype={fd}", flush=True)
    kap = kappa(prob, 6)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(14)
    x = rng.standard_normal((2, prob.nt, prob.ns))
    r = rng.standard_normal((2, prob.nt, prob.nr))
    for src in (0, 1):
        for rec in (0, 1):
            y = host(ctx.block(src, rec, False, dev(x, fd), ctx.empty_r()))
            g = host(ctx.block(src, rec, True, dev(r, fd), ctx.empty_s()))
            for s in range(2):
                assert rel(y[s], m.block(src, rec, x[s])) < TOL[fd], (src, rec)
                assert rel(g[s], m.block(src, rec, r[s], transpose=True)) < TOL[fd], (src, rec)
    ctx.close()


@pytest.mark.parametrize("fd,tol", [("f16", 2e-2), ("bf16", 1e-1)])
def test_blocks_and_lambda_half_precision_storage_error(fd, tol):
    # 16-bit wavefield storage with FP32 arithmetic (per-grid field scales):
    # error against the FP64 oracle, stated and bounded like the other
    # propagations
    prob = problem(8)
    print(f"case blocks/lambda storage dtype={fd}", flush=True)
    kap = kappa(prob, 7)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(15)
    x = rng.standard_normal((2, prob.nt, prob.ns)) * 1e3   # arbitrary scale
    errs = []
    for src, rec in ((1, 1), (0, 1), (1, 0)):
        y = host(ctx.block(src, rec, False, dev(x, "f32"), ctx.empty_r()))
        errs += [rel(y[s], m.block(src, rec, x[s])) for s in range(2)]
    y = host(ctx.lam(0, False, dev(x, "f32"), ctx.empty_s()))
    errs += [rel(y[s], m.lam(x[s], "s")) for s in range(2)]
    print(f"{fd} storage: relative L2 errors {errs}")
    assert max(errs) < tol
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_pcg_solve_v_parity(fd):
    # the normal load as the unknown: Algorithm 1 with M = I on N_v
    prob = problem(8)
    print(f"case pcg_v dtype={fd}", flush=True)
    kap = kappa(prob, 8)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(16)
    d = rng.standard_normal((2, prob.nt, prob.nr))
    K = 5
    f, hist, it, st = ctx.pcg_solve_v(dev(d, fd), 1e-3, K)
    assert it == K and st == 0
    f = host(f)
    tol = 1e-10 if fd == "f64" else 1e-4
    for s in range(2):
        fr, histr, _ = oracle.pcg_solve_v(m, d[s], 1e-3, K, shot=s)
        assert rel(f[s], fr) < tol
        assert np.allclose(hist[s], histr, rtol=10 * tol, atol=0)
    ctx.close()
    # refused without normal-velocity rows at the receiver depth
    prob = problem(8, 1, z_rec=360.0, xs=(500.0,))
    ctx = ssx.Context(prob, kappa(prob), RHO, field_dtype="f32")
    with pytest.raises(ssx.SSXError):
        ctx.pcg_solve_v(ctx.empty_r().zero_(), 1e-3, 2)
    ctx.close()
