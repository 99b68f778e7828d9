"""Execution variants of the HIP path must not change results: the fused
one-step launch equals the split velocity/pressure launches bitwise (every
field type), tile heights agree bitwise, the multi-step kernel (several
steps per launch on strips and row windows with recomputed halos) agrees
bitwise on the full grid and on the slab, and captured-graph replays equal
eager launches on every replay."""
import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402
from paper_2203_16573_amd.autotune import multi_shapes, tallest_slab  # noqa: E402

RHO = 1000.0


GEOMS = {
    # every tile touches the absorbing frame or a line
    "small": dict(nz=37, nx=150, z_src=45.0, x_src0=30.0, ns=100, z_rec=203.0, x_rec0=0.0,
                  nr=150),
    # interior tiles (no per-cell tests) beside frame and line tiles
    "wide": dict(nz=100, nx=300, z_src=45.0, x_src0=30.0, ns=200, z_rec=203.0, x_rec0=0.0,
                 nr=300),
    # lines deep inside, part width: interior tiles above, between and below
    "deep": dict(nz=130, nx=300, z_src=603.0, x_src0=450.0, ns=150, z_rec=455.0,
                 x_rec0=1000.0, nr=170),
    # pressure lines whose two interpolation rows (31/32 and 27/28 of the
    # padded grid) lie on either side of the boundary between the owned rows
    # of two windows of the multi-step kernel (32 rows owned per window at
    # order 4 and 4 steps, 8 at 8 steps; 28 at order 8 and 2 steps)
    "straddle": dict(nz=100, nx=200, z_src=215.0, x_src0=100.0, ns=120, z_rec=175.0,
                     x_rec0=0.0, nr=200),
}


def problem(order, geom="small", **kw):
    base = dict(h=10.0, dt=1e-3, nt=120, order=order, npml=10, slab_dz=5, xs=(300.0, 717.0))
    base.update(GEOMS[geom])
    base.update(kw)
    return inputs.Problem(**base)


def kappa(prob, seed=1):
    c = np.random.default_rng(seed).uniform(1800.0, 2400.0, size=(prob.nz, prob.nx))
    return RHO * c * c


def check_multistep(ctx, prob, fd, order, ref):
    """Every (steps per launch, strip width) of the multi-step kernel on the
    full grid, then on the slab, against ref bitwise."""
    NZ = prob.nz + 2 * prob.npml
    for opt_spl, opt_strip, rows, where in (
            (ssx.OPT_STEPS_PER_LAUNCH, ssx.OPT_STRIP, NZ, "full"),
            (ssx.OPT_STEPS_PER_LAUNCH_SLAB, ssx.OPT_SLAB_STRIP, tallest_slab(prob), "slab")):
        shapes = multi_shapes(order, fd, rows)
        assert shapes, (where, rows)
        for spl, strip in shapes:
            print(f"  multi-step {where} spl={spl} strip={strip}", flush=True)
            ctx.set_option(opt_strip, 0)
            ctx.set_option(opt_spl, spl)
            ctx.set_option(opt_strip, strip)
            got = run_all(ctx, prob, fd)
            for i, (a, b) in enumerate(zip(ref, got)):
                assert np.array_equal(a, b), (fd, order, where, spl, strip, i)
        ctx.set_option(opt_strip, 0)
        ctx.set_option(opt_spl, 1)


def run_all(ctx, prob, fd, seed=0):
    dt = torch.float64 if fd == "f64" else torch.float32
    g = torch.Generator(device="cpu").manual_seed(seed)
    S = len(prob.xs)
    h = torch.randn((S, prob.nt, prob.ns), generator=g, dtype=torch.float64).to(dt).cuda()
    r = torch.randn((S, prob.nt, prob.nr), generator=g, dtype=torch.float64).to(dt).cuda()
    d = ctx.fwd(h, ctx.empty_r())
    gg = ctx.adj(r, ctx.empty_s())
    P, V = ctx.slab_fwd(h, ctx.empty_s(), ctx.empty_s())
    f = ctx.slab_adj(h, r[:, :, :prob.ns].contiguous(), ctx.empty_s())
    torch.cuda.synchronize()
    return [t.cpu().numpy().copy() for t in (d, gg, P, V, f)]


@pytest.mark.parametrize("geom", ["small", "wide", "deep"])
@pytest.mark.parametrize("fd", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("order,nt", [(4, 120), (8, 121)])
def test_fused_equals_split_bitwise(fd, order, nt, geom):
    # one-step fused kernel at every tile height against the split
    # reference; an odd record length exercises the multi-step slab
    # kernel's one-step remainder
    prob = problem(order, geom, nt=nt)
    print(f"case fused-vs-split order={order} nt={nt} dtype={fd} geom={geom}", flush=True)
    ctx = ssx.Context(prob, kappa(prob), RHO, field_dtype=fd)
    ctx.set_graphs(False)
    ctx.set_option(ssx.OPT_STEP_KERNEL, 0)
    split = run_all(ctx, prob, fd)
    ctx.set_option(ssx.OPT_STEP_KERNEL, 1)
    tiles = [8, 16] + ([32] if fd != "f64" else [])
    for tz in tiles:
        ctx.set_option(ssx.OPT_TILE_Z, tz)
        fused = run_all(ctx, prob, fd)
        for a, b in zip(split, fused):
            assert np.array_equal(a, b), (fd, order, tz)
        # workgroups looping over the interior tiles with the next tile's
        # loads in flight (8 looping workgroups: several tiles each)
        for loop in (1, 8):
            ctx.set_option(ssx.OPT_TILE_LOOP, loop)
            looped = run_all(ctx, prob, fd)
            for a, b in zip(split, looped):
                assert np.array_equal(a, b), (fd, order, tz, "tile loop", loop)
        ctx.set_option(ssx.OPT_TILE_LOOP, 0)
    # regions held in LDS over several steps, on the full grid (row windows
    # where it is taller than one region) and on the slab; the odd record
    # leaves a one-step remainder
    check_multistep(ctx, prob, fd, order, split)
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32", "f16"])
@pytest.mark.parametrize("order", [4, 8])
def test_multistep_windows_lines_across_boundaries(fd, order):
    # lines whose interpolation rows lie in two windows' owned rows: each
    # window injects what falls in its region, the window owning the first
    # row samples
    prob = problem(order, "straddle", nt=123)
    print(f"case multi-step straddle order={order} dtype={fd}", flush=True)
    ctx = ssx.Context(prob, kappa(prob, 2), RHO, field_dtype=fd)
    ctx.set_graphs(False)
    ctx.set_option(ssx.OPT_STEP_KERNEL, 0)
    split = run_all(ctx, prob, fd)
    ctx.set_option(ssx.OPT_STEP_KERNEL, 1)
    check_multistep(ctx, prob, fd, order, split)
    ctx.close()


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_graph_replays_equal_eager(fd):
    prob = problem(8)
    print(f"case graph replay dtype={fd}", flush=True)
    ctx = ssx.Context(prob, kappa(prob), RHO, field_dtype=fd)
    ctx.set_graphs(False)
    eager = run_all(ctx, prob, fd, seed=3)
    ctx.set_graphs(True)
    dt = torch.float64 if fd == "f64" else torch.float32
    g = torch.Generator(device="cpu").manual_seed(3)
    h = torch.randn((2, prob.nt, prob.ns), generator=g, dtype=torch.float64).to(dt).cuda()
    d = ctx.empty_r()
    for rep in range(4):
        d.fill_(float(rep))          # eager work between replays
        x = torch.ones(1000, device="cuda").sum()
        torch.cuda.synchronize()
        ctx.fwd(h, d)
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy(), eager[0]), rep
        del x
    for rep in range(2):
        got = run_all(ctx, prob, fd, seed=3)
        for a, b in zip(eager, got):
            assert np.array_equal(a, b), rep
    ctx.close()


def test_options_rejected():
    prob = problem(8)
    ctx = ssx.Context(prob, kappa(prob), RHO, field_dtype="f64")
    # (order 8, F64 fields, 57 rows: windows of 2 steps only, 64-column
    # strips only)
    for opt, val in ((ssx.OPT_TILE_Z, 32), (ssx.OPT_TILE_Z, 12), (ssx.OPT_STEP_KERNEL, 2),
                     (ssx.OPT_STEPS_PER_LAUNCH, 3), (ssx.OPT_STEPS_PER_LAUNCH, 4),
                     (ssx.OPT_STEPS_PER_LAUNCH, 8), (ssx.OPT_STEPS_PER_LAUNCH_SLAB, 8),
                     (ssx.OPT_TILE_LOOP, 2), (ssx.OPT_TILE_LOOP, 7), (ssx.OPT_TILE_LOOP, -1),
                     (ssx.OPT_SLAB_STRIP, 96), (ssx.OPT_STRIP, 96), (ssx.OPT_SHOT_GROUP, -1),
                     (99, 1)):
        with pytest.raises(ssx.SSXError):
            ctx.set_option(opt, val)
    # steps per launch and strip width are checked together, and a rejected
    # value leaves the previous one in place
    ctx.set_option(ssx.OPT_STEPS_PER_LAUNCH, 2)
    with pytest.raises(ssx.SSXError):
        ctx.set_option(ssx.OPT_STRIP, 128)
    assert ctx.launch_shape()[1] == 2
    ctx.set_option(ssx.OPT_STEPS_PER_LAUNCH, 1)
    ctx.set_option(ssx.OPT_STRIP, 128)     # allowed while one step per launch
    with pytest.raises(ssx.SSXError):
        ctx.set_option(ssx.OPT_STEPS_PER_LAUNCH, 2)
    ctx.set_option(ssx.OPT_STRIP, 0)
    # the tile-loop setting is reported in the launch shape (a cap of 8 or
    # more is kept as given)
    for val in (0, 1, 8, 100):
        ctx.set_option(ssx.OPT_TILE_LOOP, val)
        assert ctx.launch_shape()[3] == val
    ctx.close()


@pytest.mark.parametrize("fd,tol", [("f16", 2e-2), ("bf16", 1e-1)])
def test_half_precision_storage_error(fd, tol):
    # 16-bit wavefield storage with FP32 arithmetic: error against the FP64
    # oracle per propagation, stated and bounded
    import oracle
    prob = problem(8)
    kap = kappa(prob)
    m = oracle.Model(prob, kap, RHO)
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)
    rng = np.random.default_rng(11)
    h = rng.standard_normal((2, prob.nt, prob.ns)) * 1e-3   # arbitrary scale
    r = rng.standard_normal((2, prob.nt, prob.nr)) * 1e5
    d = ctx.fwd(torch.tensor(h, dtype=torch.float32, device="cuda"), ctx.empty_r())
    g = ctx.adj(torch.tensor(r, dtype=torch.float32, device="cuda"), ctx.empty_s())
    w = ctx.precond(1e-3, torch.tensor(h, dtype=torch.float32, device="cuda"), ctx.empty_s())
    torch.cuda.synchronize()
    errs = []
    for s in range(2):
        for got, ref in ((d[s], m.fwd(h[s])), (g[s], m.adj(r[s])),
                         (w[s], oracle.precond(m, 1e-3, h[s], s))):
            got = got.double().cpu().numpy()
            errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print(f"{fd} storage: relative L2 errors fwd/adj/precond {errs}")
    assert max(errs) < tol
    ctx.close()


def test_autotune_choice_applies_and_keeps_results():
    # the tuner's choice is a valid option set, and results under it equal
    # the defaults bitwise
    from paper_2203_16573_amd import autotune
    prob = problem(8, "wide", nt=40, xs=(300.0, 717.0, 1500.0))
    print("case autotune wide f32", flush=True)
    kap = kappa(prob)
    choice = autotune.choose(prob, kap, RHO, field_dtype="f32", cache_path=None, nt_tune=20)
    for key in ("step_kernel", "steps_per_launch", "tile_z", "tile_loop", "strip", "shot_group",
                "steps_per_launch_slab", "tile_z_slab", "slab_strip", "shot_group_slab"):
        assert key in choice, key
    assert 1 <= choice["shot_group"] <= 3
    ctx = ssx.Context(prob, kap, RHO, field_dtype="f32")
    ref = run_all(ctx, prob, "f32")
    autotune.apply(ctx, choice)
    tz, spl, grp, loop = ctx.launch_shape()
    if choice["step_kernel"] == 1:
        assert (tz, spl) == (choice["tile_z"], choice["steps_per_launch"])
        assert loop == (choice["tile_loop"] if spl == 1 else 0)
    assert grp == choice["shot_group"]
    assert ctx.cells_per_launch() == (prob.nz + 20) * (prob.nx + 20) * grp
    for a, b in zip(ref, run_all(ctx, prob, "f32")):
        assert np.array_equal(a, b)
    ctx.close()
