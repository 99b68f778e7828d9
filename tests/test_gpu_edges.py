"""Edge cases of the HIP path against the oracle, and error paths of the
C ABI that need a device."""
import ctypes

import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402

RHO = 1000.0


def kappa(nz, nx, seed=0):
    c = np.random.default_rng(seed).uniform(1900.0, 2300.0, size=(nz, nx))
    return RHO * c * c


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300)


CASES = [
    # one trace each side, single step
    dict(nz=12, nx=14, nt=1, order=4, npml=3, z_src=45.0, x_src0=60.0, ns=1, z_rec=20.0,
         x_rec0=70.0, nr=1, slab_dz=2),
    # two steps, order 8, lines on the first and last physical rows
    dict(nz=20, nx=70, nt=2, order=8, npml=5, z_src=0.0, x_src0=0.0, ns=70, z_rec=190.0,
         x_rec0=0.0, nr=70, slab_dz=3),
    # odd sizes everywhere, off-grid depths, negative datum, no absorbing layer
    dict(nz=23, nx=131, nt=37, order=8, npml=0, z_src=107.5, x_src0=10.0, ns=117, z_rec=33.3,
         x_rec0=0.0, nr=131, slab_dz=-4),
    # exactly one 64-column tile plus one column
    dict(nz=17, nx=45, nt=25, order=4, npml=10, z_src=55.0, x_src0=0.0, ns=45, z_rec=125.0,
         x_rec0=0.0, nr=45, slab_dz=5),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_edge_geometries(case, fd):
    kw = dict(CASES[case])
    prob = inputs.Problem(h=10.0, dt=1e-3, xs=(kw["x_src0"] + 3.0, kw["x_src0"] + 7.0), **kw)
    print(f"case edge {case} dtype={fd}", flush=True)
    kap = kappa(prob.nz, prob.nx, case)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    vdt = torch.float64 if fd == "f64" else torch.float32
    rng = np.random.default_rng(case)
    h = rng.standard_normal((2, prob.nt, prob.ns))
    r = rng.standard_normal((2, prob.nt, prob.nr))
    d = ctx.fwd(torch.tensor(h, dtype=vdt, device="cuda"), ctx.empty_r()).double().cpu().numpy()
    g = ctx.adj(torch.tensor(r, dtype=vdt, device="cuda"), ctx.empty_s()).double().cpu().numpy()
    w = ctx.precond(1e-3, torch.tensor(h, dtype=vdt, device="cuda"), ctx.empty_s()).double().cpu().numpy()
    tol = 1e-12 if fd == "f64" else 1e-5
    for s in range(2):
        assert rel(d[s], m.fwd(h[s])) < tol
        assert rel(g[s], m.adj(r[s])) < tol
        assert rel(w[s], oracle.precond(m, 1e-3, h[s], s)) < tol
    # the tile-loop launch (tile lists built for these geometries) gives the
    # same bits at every tile height
    for tz in (8, 16) + ((32,) if fd != "f64" else ()):
        ctx.set_option(ssx.OPT_TILE_Z, tz)
        ctx.set_option(ssx.OPT_TILE_LOOP, 0)
        d0 = ctx.fwd(torch.tensor(h, dtype=vdt, device="cuda"), ctx.empty_r()).cpu()
        g0 = ctx.adj(torch.tensor(r, dtype=vdt, device="cuda"), ctx.empty_s()).cpu()
        for loop in (1, 8):
            ctx.set_option(ssx.OPT_TILE_LOOP, loop)
            d1 = ctx.fwd(torch.tensor(h, dtype=vdt, device="cuda"), ctx.empty_r()).cpu()
            g1 = ctx.adj(torch.tensor(r, dtype=vdt, device="cuda"), ctx.empty_s()).cpu()
            assert torch.equal(d0, d1) and torch.equal(g0, g1), (case, fd, tz, loop)
    ctx.close()


def test_error_paths():
    prob = inputs.Problem(nz=20, nx=40, h=10.0, dt=1e-3, nt=30, order=4, npml=5, z_src=50.0,
                          x_src0=0.0, ns=40, z_rec=20.0, x_rec0=0.0, nr=40, slab_dz=3,
                          xs=(100.0,))
    ctx = ssx.Context(prob, kappa(20, 40), RHO, field_dtype="f64")
    L = ssx.lib()
    h = ctx.empty_s()
    d = ctx.empty_r()
    assert L.ssx_fwd(ctx._ctx, None, ctypes.c_void_p(d.data_ptr())) == 1
    assert L.ssx_penalty(ctx._ctx, 7, 0.0, ctypes.c_void_p(h.data_ptr()),
                         ctypes.c_void_p(h.data_ptr())) == 1
    assert L.ssx_pcg_solve(ctx._ctx, ctypes.c_void_p(d.data_ptr()), 1e-3, 100000, 0.0, 1,
                           ctypes.c_void_p(h.data_ptr()), None, None) == 1
    assert "maxit" in L.ssx_last_error().decode()
    # workspace smaller than the footprint
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(ssx.SSXError) as e:
        ssx.Context(prob, kappa(20, 40), RHO, field_dtype="f64", workspace=ws)
    assert e.value.status == 3
    # non-finite data: PCG reports it instead of returning silently
    d.fill_(float("nan"))
    _, _, it, st = ctx.pcg_solve(d, 1e-3, 3, raise_on_breakdown=False)
    assert st == 6
    # the context is still usable afterwards
    d.fill_(0.0)
    _, _, it, st = ctx.pcg_solve(d, 1e-3, 3)
    assert st == 0
    ctx.close()


def test_workspace_context_matches_library_allocation():
    prob = inputs.Problem(nz=30, nx=90, h=10.0, dt=1e-3, nt=60, order=8, npml=8, z_src=40.0,
                          x_src0=0.0, ns=90, z_rec=20.0, x_rec0=0.0, nr=90, slab_dz=5,
                          xs=(200.0, 650.0))
    kap = kappa(30, 90, 3)
    ws = torch.empty(ssx.footprint(prob, "f32"), dtype=torch.uint8, device="cuda")
    a = ssx.Context(prob, kap, RHO, field_dtype="f32", workspace=ws)
    b = ssx.Context(prob, kap, RHO, field_dtype="f32")
    d = torch.randn((2, prob.nt, prob.nr), device="cuda")
    ha, _, _, _ = a.pcg_solve(d, 1e-3, 3)
    hb, _, _, _ = b.pcg_solve(d, 1e-3, 3)
    assert torch.equal(ha, hb)
    a.close()
    b.close()


def test_rtol_stops_early():
    prob = inputs.Problem(nz=30, nx=90, h=10.0, dt=1e-3, nt=60, order=8, npml=8, z_src=40.0,
                          x_src0=0.0, ns=90, z_rec=20.0, x_rec0=0.0, nr=90, slab_dz=5,
                          xs=(200.0,))
    ctx = ssx.Context(prob, kappa(30, 90, 4), RHO, field_dtype="f64")
    d = torch.randn((1, prob.nt, prob.nr), dtype=torch.float64, device="cuda")
    _, hist, it, st = ctx.pcg_solve(d, 1e-3, 50, rtol=0.5, use_precond=False)
    assert it < 50
    assert hist[0, it, 0] <= 0.5 * hist[0, 0, 0]
    assert hist[0, it - 1, 0] > 0.5 * hist[0, 0, 0] or it == 1
    ctx.close()


def test_graph_cache_eviction_keeps_results():
    # more distinct propagations than the graph cache holds: evicted graphs
    # are destroyed and re-captured, every result stays the same
    prob = inputs.Problem(nz=20, nx=40, h=10.0, dt=1e-3, nt=30, order=4, npml=5, z_src=50.0,
                          x_src0=0.0, ns=40, z_rec=20.0, x_rec0=0.0, nr=40, slab_dz=3,
                          xs=(100.0,))
    print("case graph cache eviction", flush=True)
    ctx = ssx.Context(prob, kappa(20, 40, 8), RHO, field_dtype="f64")
    h = torch.tensor(np.random.default_rng(3).standard_normal((1, prob.nt, prob.ns)),
                     device="cuda")
    outs = [ctx.empty_r() for _ in range(40)]
    for o in outs:
        ctx.fwd(h, o)
    ref = outs[0].clone()
    for o in outs[::-1]:
        ctx.fwd(h, o)
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o, ref)
    ctx.close()
