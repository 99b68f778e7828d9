"""Variable density (ssx_create_density) on the HIP path against the FP64
oracle, and its kernel variants against each other.

The operators of the paper carry both kappa and rho; here rho is an array
at the pressure nodes, each velocity update using the mean density of its
two nodes (the oracle's grid module; its pins fix the reflection and
transmission of a density-only jump at second order).  Tolerances as the
constant-density parity tests: FP64 1e-12 per propagation, FP32 1e-5; PCG
1e-10 (FP64) and 1e-4 (FP32).  The multi-step kernel takes the density array on 64-column
strips and agrees bitwise with the split kernels.
"""
import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402
from paper_2203_16573_amd.autotune import multi_shapes, tallest_slab  # noqa: E402

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
    # three tiles across x with a ragged tail, interior tiles below the lines
    base = dict(nz=90, nx=150, h=10.0, dt=1e-3, nt=160, order=order, npml=10,
                z_src=45.0, x_src0=30.0, ns=100, z_rec=203.0, x_rec0=0.0, nr=150,
                slab_dz=5, xs=tuple(300.0 + 417.0 * s for s in range(nshots)))
    base.update(kw)
    return inputs.Problem(**base)


def model(prob, seed=1):
    # a layered density with a smooth lateral variation, velocities 1.8-2.4 km/s
    rng = np.random.default_rng(seed)
    c = rng.uniform(1800.0, 2400.0, size=(prob.nz, prob.nx))
    z = np.arange(prob.nz)[:, None]
    x = np.arange(prob.nx)[None, :]
    rho = 1000.0 + 800.0 * (z > prob.nz // 2) + 300.0 * np.sin(x / 17.0) * np.cos(z / 11.0)
    rho = rho + 50.0 * rng.standard_normal((prob.nz, prob.nx))
    return rho * c * c, rho


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("order", [4, 8])
def test_density_parity(fd, order):
    prob = problem(order)
    kappa, rho = model(prob)
    print(f"case density parity {fd} order {order}", flush=True)
    ctx = ssx.Context(prob, kappa, rho, field_dtype=fd)
    rng = np.random.default_rng(2)
    S = prob.nshots
    h = rng.standard_normal((S, prob.nt, prob.ns))
    r = rng.standard_normal((S, prob.nt, prob.nr))
    d = host(ctx.fwd(dev(h, fd), ctx.empty_r()))
    g = host(ctx.adj(dev(r, fd), ctx.empty_s()))
    P, V = ctx.slab_fwd(dev(h, fd), ctx.empty_s(), ctx.empty_s())
    P, V = host(P), host(V)
    f = host(ctx.slab_adj(dev(h, fd), dev(r[:, :, :prob.ns], fd), ctx.empty_s()))
    Mr = host(ctx.precond(1e-3, dev(h, fd), ctx.empty_s()))
    ctx.close()
    for s in range(S):
        m = oracle.Model(prob.replace(xs=(prob.xs[s],)), kappa, rho)
        Pr, Vr = m.slab_fwd(h[s])
        errs = [rel(d[s], m.fwd(h[s])), rel(g[s], m.adj(r[s])), rel(P[s], Pr), rel(V[s], Vr),
                rel(f[s], m.slab_adj(h[s], r[s, :, :prob.ns])),
                rel(Mr[s], oracle.precond(m, 1e-3, h[s]))]
        print(f"  shot {s}: {['%.2e' % e for e in errs]}", flush=True)
        assert max(errs) < TOL[fd], errs


@pytest.mark.parametrize("fd,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_density_pcg_parity(fd, tol):
    prob = problem(8, nshots=1, nt=140)
    kappa, rho = model(prob, 3)
    m = oracle.Model(prob, kappa, rho)
    wav = inputs.source_wavelet(prob, 25.0)
    d = m.fwd(inputs.spike_gather(prob, wav, 0))
    print(f"case density PCG {fd}", flush=True)
    ctx = ssx.Context(prob, kappa, rho, field_dtype=fd)
    hs, hist, it, _ = ctx.pcg_solve(dev(d[None], fd), 1e-3, 6)
    ctx.close()
    h_ref, hist_ref, _ = oracle.pcg_solve(m, d, 1e-3, 6)
    e = rel(host(hs)[0], h_ref)
    eh = rel(np.asarray(hist)[0, :, 0], hist_ref[:, 0])
    print(f"  h {e:.2e}, ||r_k|| {eh:.2e}", flush=True)
    assert e < tol and eh < tol


@pytest.mark.parametrize("fd", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("order", [4, 8])
def test_density_fused_equals_split_bitwise(fd, order):
    prob = problem(order, nt=121)
    kappa, rho = model(prob, 4)
    print(f"case density fused-vs-split {fd} order {order}", flush=True)
    ctx = ssx.Context(prob, kappa, rho, field_dtype=fd)
    ctx.set_graphs(False)
    dt = torch.float64 if fd == "f64" else torch.float32
    gen = torch.Generator(device="cpu").manual_seed(5)
    h = torch.randn((prob.nshots, prob.nt, prob.ns), generator=gen, dtype=torch.float64)
    r = torch.randn((prob.nshots, prob.nt, prob.nr), generator=gen, dtype=torch.float64)
    h, r = h.to(dt).cuda(), r.to(dt).cuda()

    def run():
        out = [ctx.fwd(h, ctx.empty_r()), ctx.adj(r, ctx.empty_s()),
               *ctx.slab_fwd(h, ctx.empty_s(), ctx.empty_s())]
        torch.cuda.synchronize()
        return [t.cpu().numpy().copy() for t in out]

    ctx.set_option(ssx.OPT_STEP_KERNEL, 0)
    split = run()
    ctx.set_option(ssx.OPT_STEP_KERNEL, 1)
    for tz in [8, 16] + ([32] if fd != "f64" else []):
        ctx.set_option(ssx.OPT_TILE_Z, tz)
        fused = run()
        for a, b in zip(split, fused):
            assert np.array_equal(a, b), (fd, tz)
    # several steps per launch on 64-column strips, on the full grid (row
    # windows) and on the slab; the odd record leaves a one-step remainder
    NZ = prob.nz + 2 * prob.npml
    for opt_spl, opt_strip, rows in (
            (ssx.OPT_STEPS_PER_LAUNCH, ssx.OPT_STRIP, NZ),
            (ssx.OPT_STEPS_PER_LAUNCH_SLAB, ssx.OPT_SLAB_STRIP, tallest_slab(prob))):
        shapes = multi_shapes(order, fd, rows, variable_density=True)
        assert shapes and all(strip == 64 for _, strip in shapes)
        for spl, strip in shapes:
            print(f"  multi-step spl={spl} strip={strip} rows={rows}", flush=True)
            ctx.set_option(opt_strip, 0)
            ctx.set_option(opt_spl, spl)
            ctx.set_option(opt_strip, strip)
            for a, b in zip(split, run()):
                assert np.array_equal(a, b), (fd, order, spl, strip, rows)
        ctx.set_option(opt_strip, 0)
        ctx.set_option(opt_spl, 1)
    # a density array: one tile per workgroup, 64-column strips
    with pytest.raises(ssx.SSXError):
        ctx.set_option(ssx.OPT_TILE_LOOP, 1)
    ctx.set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, 2)
    with pytest.raises(ssx.SSXError):
        ctx.set_option(ssx.OPT_SLAB_STRIP, 128)
    ctx.close()


def test_constant_density_array_matches_scalar():
    prob = problem(8, nshots=1)
    kappa, _ = model(prob)
    rho = np.full((prob.nz, prob.nx), 1000.0)
    x = dev(np.random.default_rng(6).standard_normal((1, prob.nt, prob.ns)), "f64")
    out = []
    for r in (1000.0, rho):
        ctx = ssx.Context(prob, kappa, r, field_dtype="f64")
        out.append(host(ctx.fwd(x, ctx.empty_r())))
        ctx.close()
    assert rel(out[1], out[0]) < 1e-13


def test_density_misfit_gradient():
    # the gradient in kappa at fixed density against the oracle's
    prob = problem(8, nshots=1, nt=120)
    kappa, rho = model(prob, 7)
    m = oracle.Model(prob, kappa, rho)
    rng = np.random.default_rng(8)
    h = rng.standard_normal((prob.nt, prob.ns))
    d = rng.standard_normal((prob.nt, prob.nr))
    g_ref, J_ref = oracle.misfit_gradient(m, h, d)
    print("case density gradient", flush=True)
    ctx = ssx.Context(prob, kappa, rho, field_dtype="f64")
    g, J = ctx.misfit_gradient(dev(h[None], "f64"), dev(d[None], "f64"))
    ctx.close()
    e = rel(host(g)[0], g_ref)
    print(f"  gradient {e:.2e}, J {abs(J[0] / J_ref - 1):.2e}", flush=True)
    assert e < 1e-10 and abs(J[0] / J_ref - 1) < 1e-12


def test_density_rejects_bad_values():
    prob = problem(8, nshots=1)
    kappa, rho = model(prob)
    for bad in (np.where(np.arange(rho.size).reshape(rho.shape) == 5, -1.0, rho),
                np.where(np.arange(rho.size).reshape(rho.shape) == 7, np.nan, rho)):
        with pytest.raises(ssx.SSXError):
            ssx.Context(prob, kappa, bad, field_dtype="f32")
