"""Parity of the weighted normal equations on the HIP path with the FP64
oracle: the data-space weight W_d (receiver-side slab), the model-space
weight W_m (source-side slab driven by a pressure source), the weighted
normal operator N_w and Algorithm 1 on N_w h = F^T W_d d.

Tolerances as for the unweighted operators: 1e-12 (FP64) and 1e-5 (FP32)
relative L2 per operator of two slab simulations, 1e-10 / 1e-4 on the
PCG iterate; 16-bit storage with FP32 arithmetic bounded like the other
propagations (2e-2 FP16, 1e-1 BF16).
"""
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
    # 3 tiles across x with a ragged tail; off-grid source and receiver
    # depths, part-width lines at different offsets
    base = dict(nz=37, nx=150, h=10.0, dt=1e-3, nt=200, order=order, npml=10,
                z_src=45.0, x_src0=30.0, ns=100, z_rec=203.0, x_rec0=10.0, nr=130,
                slab_dz=5, rslab_dz=4, xs=tuple(300.0 + 417.0 * s for s in range(nshots)))
    base.update(kw)
    return inputs.Problem(**base)


def kappa(prob, seed=1):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1800.0, 2400.0, size=(prob.nz, prob.nx))
    return RHO * c * c


@pytest.fixture(scope="module")
def setups():
    cache = {}

    def get(order, fd, **kw):
        key = (order, fd, tuple(sorted(kw.items())))
        if key not in cache:
            prob = problem(order, **kw)
            kap = kappa(prob)
            cache[key] = (prob, oracle.Model(prob, kap, RHO),
                          ssx.Context(prob, kap, RHO, field_dtype=fd))
        return cache[key]
    yield get
    for v in cache.values():
        v[2].close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("order,dz,rdz", [(4, 5, -4), (8, -5, 3), (8, 3, 6)])
def test_weights_parity(setups, fd, order, dz, rdz):
    prob, m, ctx = setups(order, fd, slab_dz=dz, rslab_dz=rdz)
    print(f"case weights order={order} dz={dz} rdz={rdz} dtype={fd}", flush=True)
    rng = np.random.default_rng(order + dz)
    r = rng.standard_normal((2, prob.nt, prob.nr))
    x = rng.standard_normal((2, prob.nt, prob.ns))
    yd = host(ctx.weight_d(dev(r, fd), ctx.empty_r()))
    ym = host(ctx.weight_m(dev(x, fd), ctx.empty_s()))
    for s in range(2):
        assert rel(yd[s], m.wd(r[s])) < TOL[fd]
        assert rel(ym[s], m.wm(x[s])) < TOL[fd]


@pytest.mark.parametrize("spl", [4, 8])
def test_weights_parity_multistep_slab(spl):
    # both slabs through the kernel that holds a strip's whole slab height in
    # LDS and advances it several steps per launch
    prob = problem(8, 1, xs=(700.0,))
    print(f"case weights multistep slab spl={spl}", flush=True)
    kap = kappa(prob, 3)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype="f32")
    ctx.set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, spl)
    rng = np.random.default_rng(spl)
    r = rng.standard_normal((1, prob.nt, prob.nr))
    x = rng.standard_normal((1, prob.nt, prob.ns))
    yd = host(ctx.weight_d(dev(r, "f32"), ctx.empty_r()))
    ym = host(ctx.weight_m(dev(x, "f32"), ctx.empty_s()))
    assert rel(yd[0], m.wd(r[0])) < TOL["f32"]
    assert rel(ym[0], m.wm(x[0])) < TOL["f32"]
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("alpha", [0.0, 1e-3])
def test_normal_w_parity(setups, fd, alpha):
    prob, m, ctx = setups(8, fd)
    print(f"case normal_w alpha={alpha} dtype={fd}", flush=True)
    rng = np.random.default_rng(7)
    p = rng.standard_normal((2, prob.nt, prob.ns))
    Fp = ctx.empty_r()
    q = host(ctx.normal_w(alpha, dev(p, fd), ctx.empty_s(), Fp))
    Fp = host(Fp)
    for s in range(2):
        qr, Fpr = oracle.normal_w(m, alpha, p[s], s)
        assert rel(q[s], qr) < TOL[fd]
        assert rel(Fp[s], Fpr) < TOL[fd]


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("use_precond,alpha", [(True, 1e-3), (True, 0.0), (False, 1e-3)])
def test_pcg_w_parity(setups, fd, use_precond, alpha):
    prob, m, ctx = setups(8, fd)
    print(f"case pcg_w dtype={fd} precond={use_precond} alpha={alpha}", flush=True)
    rng = np.random.default_rng(8)
    d = rng.standard_normal((2, prob.nt, prob.nr))
    K = 5
    h, hist, it, st = ctx.pcg_solve_w(dev(d, fd), alpha, K, use_precond=use_precond)
    h = host(h)
    assert it == K and st == 0
    tol = 1e-10 if fd == "f64" else 1e-4
    for s in range(2):
        hr, histr = oracle.pcg_solve_w(m, d[s], alpha, K, use_precond=use_precond, shot=s)
        assert rel(h[s], hr) < tol
        assert np.allclose(hist[s], histr, rtol=10 * tol, atol=0)


def test_weighted_replays_are_identical(setups):
    # the captured graphs of the four new propagations replay exactly
    prob, m, ctx = setups(8, "f32")
    rng = np.random.default_rng(9)
    d = dev(rng.standard_normal((2, prob.nt, prob.nr)), "f32")
    a, _, _, _ = ctx.pcg_solve_w(d, 1e-3, 3)
    a = a.clone()
    ctx.fwd(ctx.empty_s().zero_(), ctx.empty_r())  # other work in between
    b, _, _, _ = ctx.pcg_solve_w(d, 1e-3, 3)
    ctx.set_graphs(False)
    c, _, _, _ = ctx.pcg_solve_w(d, 1e-3, 3)
    ctx.set_graphs(True)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


@pytest.mark.parametrize("fd,tol", [("f16", 2e-2), ("bf16", 1e-1)])
def test_weights_half_precision_storage_error(fd, tol):
    prob = problem(8)
    print(f"case weights storage dtype={fd}", flush=True)
    kap = kappa(prob, 5)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(13)
    r = rng.standard_normal((2, prob.nt, prob.nr)) * 1e4   # arbitrary scales
    x = rng.standard_normal((2, prob.nt, prob.ns)) * 1e-4
    yd = host(ctx.weight_d(dev(r, "f32"), ctx.empty_r()))
    ym = host(ctx.weight_m(dev(x, "f32"), ctx.empty_s()))
    q = host(ctx.normal_w(1e-3, dev(x, "f32"), ctx.empty_s()))
    errs = []
    for s in range(2):
        errs += [rel(yd[s], m.wd(r[s])), rel(ym[s], m.wm(x[s])),
                 rel(q[s], oracle.normal_w(m, 1e-3, x[s], s)[0])]
    print(f"{fd} storage: relative L2 errors W_d/W_m/N_w {errs}")
    assert max(errs) < tol
    ctx.close()


def test_weighted_entry_points_need_the_receiver_slab():
    prob = problem(8, 1, rslab_dz=0, xs=(500.0,))
    ctx = ssx.Context(prob, kappa(prob), RHO, field_dtype="f32")
    x = ctx.empty_s().zero_()
    r = ctx.empty_r().zero_()
    for call in (lambda: ctx.weight_d(r, ctx.empty_r()),
                 lambda: ctx.weight_m(x, ctx.empty_s()),
                 lambda: ctx.normal_w(1e-3, x, ctx.empty_s()),
                 lambda: ctx.pcg_solve_w(r, 1e-3, 2)):
        with pytest.raises(ssx.SSXError) as e:
            call()
        assert e.value.status == 1 and "receiver-side slab" in str(e.value)
    # the unweighted path is unaffected
    ctx.pcg_solve(r, 1e-3, 2)
    ctx.close()


def test_crosswell_geometry_parity():
    # the paper's crosswell example at 100 m cells (the oracle's size): data
    # from the point source in the lens model, CG and weighted PCG in the
    # homogeneous model, FP64 against the oracle
    prob = inputs.crosswell_problem(h=100.0, dt=20e-3, nt=200, order=8, npml=10)
    print("case crosswell 41x81 f64", flush=True)
    lens = inputs.crosswell_kappa(prob.nz, prob.nx, prob.h, lens=True)
    hom = inputs.crosswell_kappa(prob.nz, prob.nx, prob.h, lens=False)
    pp = inputs.crosswell_point_problem(prob)
    w = inputs.bandpass_wavelet((np.arange(prob.nt) + 0.5) * prob.dt)
    d_ref = oracle.Model(pp, lens, RHO).fwd((w / prob.h)[:, None])
    pctx = ssx.Context(pp, lens, RHO, field_dtype="f64")
    d = pctx.fwd(dev((w / prob.h)[None, :, None], "f64"), pctx.empty_r())
    assert rel(host(d)[0], d_ref) < 1e-12
    pctx.close()
    m = oracle.Model(prob, hom, RHO)
    ctx = ssx.Context(prob, hom, RHO, field_dtype="f64")
    K = 4
    for alpha in (0.0, 1e-3):
        h, hist, _, st = ctx.pcg_solve_w(d, alpha, K)
        hr, histr = oracle.pcg_solve_w(m, d_ref, alpha, K)
        assert st == 0 and rel(host(h)[0], hr) < 1e-10
        assert np.allclose(hist[0], histr, rtol=1e-9, atol=0)
        h, hist, _, st = ctx.pcg_solve(d, alpha, K, use_precond=False)
        hr, histr, _ = oracle.pcg_solve(m, d_ref, alpha, K, use_precond=False)
        assert st == 0 and rel(host(h)[0], hr) < 1e-10
    ctx.close()


def test_weights_symmetric_at_production_size():
    # at the 801 x 1601 size, 4000 steps, in the launch configuration the
    # benchmark times: W_d and W_m are symmetric (a property that holds at any
    # size; small sizes are compared with the oracle element by element)
    from test_gpu_parity import bench_context
    wl = inputs.workload(2)
    wl.prob = wl.prob.replace(rslab_dz=-5)
    print("case weights symmetric c2 f32", flush=True)
    ctx = bench_context(wl, "f32")
    prob = wl.prob
    rng = np.random.default_rng(21)
    for op, n in ((ctx.weight_d, prob.nr), (ctx.weight_m, prob.ns)):
        x = dev(rng.standard_normal((1, prob.nt, n)), "f32")
        y = dev(rng.standard_normal((1, prob.nt, n)), "f32")
        out = torch.empty_like(x)
        Wx = op(x, out).clone()
        Wy = op(y, out).clone()
        lhs, rhs = ctx.dot(x, Wy)[0], ctx.dot(Wx, y)[0]
        nrm = np.sqrt(ctx.dot(Wx, Wx)[0] * ctx.dot(y, y)[0])
        print(f"  symmetry defect {abs(lhs - rhs) / nrm:.2e}")
        assert abs(lhs - rhs) <= 1e-5 * nrm
    ctx.close()


@pytest.mark.parametrize("fd", ["f32", "f16"])
def test_overlap_is_bitwise_neutral(setups, fd):
    # the model-space term on the second stream gives the same bits as the
    # same work on the context's stream (16-bit fields: each grid keeps its
    # own field scales)
    if fd == "f16":
        prob = problem(8)
        kap = kappa(prob)
        ctx = ssx.Context(prob, kap, RHO, field_dtype="f16")
    else:
        prob, m, ctx = setups(8, fd)
    print(f"case overlap dtype={fd}", flush=True)
    rng = np.random.default_rng(17)
    d = dev(rng.standard_normal((2, prob.nt, prob.nr)), "f32")
    p = dev(rng.standard_normal((2, prob.nt, prob.ns)), "f32")
    out = {}
    for ov in (1, 0):
        ctx.set_option(ssx.OPT_OVERLAP, ov)
        q = ctx.normal_w(1e-3, p, ctx.empty_s()).clone()
        h, hist, _, _ = ctx.pcg_solve_w(d, 1e-3, 4)
        torch.cuda.synchronize()
        out[ov] = (q.cpu(), h.clone().cpu(), hist)
    ctx.set_option(ssx.OPT_OVERLAP, 1)
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])
    if fd == "f16":
        ctx.close()
