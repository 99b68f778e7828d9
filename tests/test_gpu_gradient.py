"""Parity of the misfit gradient in kappa (adjoint state of the discrete
scheme) on the HIP path with the FP64 oracle, and a full-size check of it
against central differences of the misfit.

Tolerances: 1e-10 relative L2 with FP64 fields (two FP64 evaluations of the
same sums, accumulated over every step), 1e-4 with FP32 fields."""
import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402

RHO = 1000.0


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
    base = dict(nz=37, nx=150, h=10.0, dt=1e-3, nt=160, order=order, npml=10,
                z_src=45.0, x_src0=30.0, ns=100, z_rec=203.0, x_rec0=10.0, nr=130,
                slab_dz=5, xs=tuple(300.0 + 417.0 * s for s in range(nshots)))
    base.update(kw)
    return inputs.Problem(**base)


def kappa(prob, seed=1):
    rng = np.random.default_rng(seed)
    c = rng.uniform(1800.0, 2400.0, size=(prob.nz, prob.nx))
    return RHO * c * c


@pytest.mark.parametrize("fd", ["f64", "f32"])
@pytest.mark.parametrize("order", [4, 8])
def test_gradient_parity(fd, order):
    prob = problem(order)
    print(f"case gradient order={order} dtype={fd}", flush=True)
    kap = kappa(prob, order)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(20 + order)
    h = rng.standard_normal((2, prob.nt, prob.ns))
    d = rng.standard_normal((2, prob.nt, prob.nr)) * np.abs(m.fwd(h[0])).max()
    g, J = ctx.misfit_gradient(dev(h, fd), dev(d, fd))
    g = host(g)
    tol = 1e-10 if fd == "f64" else 1e-4
    for s in range(2):
        gr, Jr = oracle.misfit_gradient(m, h[s], d[s])
        assert rel(g[s], gr) < tol
        assert abs(J[s] - Jr) <= tol * Jr
    ctx.close()


def test_gradient_independent_of_launch_options():
    # one step per launch in every form of the step kernel: the same bits
    prob = problem(8, 3, nz=60, nx=200, xs=(300.0, 900.0, 1500.0))
    print("case gradient options f32", flush=True)
    kap = kappa(prob, 5)
    ctx = ssx.Context(prob, kap, RHO, field_dtype="f32")
    rng = np.random.default_rng(25)
    h = dev(rng.standard_normal((3, prob.nt, prob.ns)), "f32")
    d = dev(rng.standard_normal((3, prob.nt, prob.nr)), "f32")
    ref, Jref = ctx.misfit_gradient(h, d)
    ref = ref.clone()
    # a replay of the captured graph, then each option in turn (eager
    # launches, other step kernels and launch shapes)
    # (the fused forward step stores the history itself at every tile
    # height, with and without the tile loop; the split kernels store it
    # with a kernel of its own)
    for opt, val in ((None, None), (ssx.OPT_GRAPHS, 0), (ssx.OPT_GRAPHS, 1), (ssx.OPT_TILE_LOOP, 1),
                     (ssx.OPT_TILE_Z, 8), (ssx.OPT_TILE_Z, 32), (ssx.OPT_TILE_LOOP, 0),
                     (ssx.OPT_TILE_Z, 16), (ssx.OPT_SHOT_GROUP, 2),
                     (ssx.OPT_STEP_KERNEL, 0)):
        if opt is not None:
            ctx.set_option(opt, val)
        g, J = ctx.misfit_gradient(h, d)
        torch.cuda.synchronize()
        assert torch.equal(g, ref), (opt, val)
        assert np.array_equal(J, Jref)
    ctx.close()


def test_gradient_needs_wide_fields():
    prob = problem(8, 1, xs=(500.0,))
    ctx = ssx.Context(prob, kappa(prob), RHO, field_dtype="f16")
    with pytest.raises(ssx.SSXError) as e:
        ctx.misfit_gradient(ctx.empty_s().zero_(), ctx.empty_r().zero_())
    assert e.value.status == 1
    ctx.close()


def test_gradient_central_differences_at_production_size():
    # 801 x 1601, 4000 steps, FP64 fields: <g, dk> against the central
    # difference of the misfit, dk on interior physical cells (off the edges
    # that the absorbing layer copies and off the fastest cell)
    wl = inputs.workload(2)
    prob = wl.prob
    print("case gradient central differences c2 f64", flush=True)
    rng = np.random.default_rng(33)
    kap = wl.kappa
    ctx = ssx.Context(prob, kap, wl.rho, field_dtype="f64")
    w = inputs.source_wavelet(prob, wl.freq)
    htrue = inputs.spike_gather(prob, w)[None]
    d = ctx.fwd(dev(htrue, "f64"), ctx.empty_r()).clone()
    # a source estimate that does not fit: the spike moved by 40 cells
    h = np.roll(htrue, 40, axis=2)
    g, J0 = ctx.misfit_gradient(dev(h, "f64"), d)
    g = host(g)[0]
    ctx.close()
    dk = np.zeros_like(kap)
    dk[1:-1, 1:-1] = rng.standard_normal((prob.nz - 2, prob.nx - 2))
    dk[np.unravel_index(np.argmax(kap), kap.shape)] = 0.0
    eps = 1e-6 * kap.mean() / np.abs(dk).max()

    def J(k):
        c = ssx.Context(prob, k, wl.rho, field_dtype="f64")
        e = c.fwd(dev(h, "f64"), c.empty_r()) - d
        val = 0.5 * float(torch.sum(e * e))
        c.close()
        return val

    fdiff = (J(kap + eps * dk) - J(kap - eps * dk)) / (2 * eps)
    an = float(np.sum(g * dk))
    print(f"  <g, dk> {an:.10e}  central difference {fdiff:.10e}")
    assert abs(fdiff - an) <= 1e-5 * abs(an)


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_gradient_edge_geometry(fd):
    # no absorbing layer (the stencils reach into the zero ghost cells), odd
    # sizes, a single shot, one step and a record of several
    for nt in (1, 37):
        prob = problem(8, 1, nz=23, nx=131, nt=nt, npml=0, z_src=107.5, x_src0=10.0, ns=117,
                       z_rec=33.3, x_rec0=0.0, nr=131, slab_dz=-4, xs=(500.0,))
        print(f"case gradient edge nt={nt} dtype={fd}", flush=True)
        kap = kappa(prob, 9)
        m = oracle.Model(prob, kap, RHO)
        ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
        rng = np.random.default_rng(nt)
        h = rng.standard_normal((1, prob.nt, prob.ns))
        d = rng.standard_normal((1, prob.nt, prob.nr))
        g, J = ctx.misfit_gradient(dev(h, fd), dev(d, fd))
        gr, Jr = oracle.misfit_gradient(m, h[0], d[0])
        tol = 1e-10 if fd == "f64" else 1e-4
        if np.linalg.norm(gr) > 0:
            assert rel(host(g)[0], gr) < tol
        else:
            assert np.abs(host(g)[0]).max() == 0.0
        assert abs(J[0] - Jr) <= tol * Jr
        ctx.close()
