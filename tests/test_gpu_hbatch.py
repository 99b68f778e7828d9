"""Heterogeneous batch (ssx_batch_*): contexts of different grid sizes,
records, shot counts, lines and models solved together, every propagation
stage merged into one launch per time step.  Each member's iterate and
residual history must equal, bitwise, those of its own ssx_pcg_solve (whose
parity with the FP64 oracle the other GPU tests establish)."""
import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402

RHO = 1000.0

MEMBERS = [
    # (nz, nx, nt, shots, z_src, z_rec, density array)
    (37, 150, 120, 2, 45.0, 203.0, False),
    (100, 300, 90, 1, 45.0, 203.0, False),
    (130, 300, 131, 3, 603.0, 455.0, False),
    (100, 200, 100, 1, 215.0, 175.0, True),
    (60, 120, 77, 2, 105.0, 305.0, False),
    (45, 90, 64, 1, 205.0, 85.0, True),
    (80, 160, 110, 2, 125.0, 305.0, False),
]


def member(i, order, fd, nt_scale=1.0):
    nz, nx, nt, shots, zs, zr, vrho = MEMBERS[i]
    h = 10.0
    width = (nx - 1) * h
    prob = inputs.Problem(nz=nz, nx=nx, h=h, dt=1e-3, nt=max(8, int(nt * nt_scale)), order=order,
                          npml=10, z_src=zs, x_src0=0.0, ns=nx, z_rec=zr, x_rec0=0.0, nr=nx,
                          slab_dz=5, xs=inputs.shot_positions(shots, width))
    rng = np.random.default_rng(100 + i)
    c = rng.uniform(1800.0, 2400.0, size=(nz, nx))
    if vrho:
        rho = 1500.0 + 500.0 * rng.uniform(size=(nz, nx))
    else:
        rho = RHO
    kappa = rho * c * c
    ctx = ssx.Context(prob, kappa, rho, field_dtype=fd)
    wav = inputs.source_wavelet(prob, 15.0)
    h_true = np.stack([inputs.spike_gather(prob, wav, s) for s in range(shots)])
    dt = torch.float64 if fd == "f64" else torch.float32
    d = ctx.fwd(torch.tensor(h_true, dtype=dt, device="cuda"), ctx.empty_r())
    torch.cuda.synchronize()
    return ctx, d


def arrays(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().copy()


@pytest.mark.parametrize("fd,order,count", [("f32", 8, 7), ("f64", 4, 4), ("f16", 8, 3)])
def test_batch_equals_own_solves_bitwise(fd, order, count):
    # 7 members: two launches per time step while six or seven records run
    print(f"case hbatch {fd} order {order} members {count}", flush=True)
    ms = [member(i, order, fd) for i in range(count)]
    ctxs = [c for c, _ in ms]
    ds = [d for _, d in ms]
    alphas = [1e-3 * (1 + i % 3) for i in range(count)]
    K = 5
    b = ssx.Batch(ctxs)
    hs, hists, its, sts = b.pcg_solve(ds, alphas, K)
    assert sts == [0] * count
    b.close()
    for i, (ctx, d) in enumerate(ms):
        h1, hist1, it1, _ = ctx.pcg_solve(d, alphas[i], K)
        assert its[i] == it1 == K
        assert np.array_equal(arrays(hs[i]), arrays(h1)), i
        assert np.array_equal(hists[i], hist1), i
        ctx.close()


def test_batch_members_stop_at_their_own_iteration():
    # a residual target each member reaches at its own iteration: members
    # leave the lockstep one by one, with the results of their own solves
    fd, order = "f32", 4
    print("case hbatch rtol", flush=True)
    ms = [member(i, order, fd) for i in (0, 1, 3, 4)]
    ctxs = [c for c, _ in ms]
    ds = [d for _, d in ms]
    b = ssx.Batch(ctxs)
    hs, hists, its, _ = b.pcg_solve(ds, 0.0, 12, rtol=0.3)
    b.close()
    for i, (ctx, d) in enumerate(ms):
        h1, hist1, it1, _ = ctx.pcg_solve(d, 0.0, 12, rtol=0.3)
        assert its[i] == it1, (i, its, it1)
        assert np.array_equal(arrays(hs[i]), arrays(h1)), i
        assert np.array_equal(hists[i], hist1), i
        ctx.close()
    print(f"  iterations {its}", flush=True)


def test_batch_with_tuned_members_and_graph_replays():
    # members with other launch options (multi-step slab kernel, tile loop)
    # and a second batch solve replaying the captured merged propagations
    fd, order = "f32", 8
    print("case hbatch tuned members", flush=True)
    ms = [member(i, order, fd) for i in (0, 2, 4)]
    ctxs = [c for c, _ in ms]
    ds = [d for _, d in ms]
    ctxs[0].set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, 4)
    ctxs[1].set_option(ssx.OPT_TILE_LOOP, 1)
    ctxs[2].set_option(ssx.OPT_STEP_KERNEL, 0)
    ref = []
    for ctx, d in ms:
        h1, hist1, _, _ = ctx.pcg_solve(d, 1e-3, 4)
        ref.append((arrays(h1), hist1))
    b = ssx.Batch(ctxs)
    for rep in range(2):
        hs, hists, its, _ = b.pcg_solve(ds, 1e-3, 4)
        for i in range(3):
            assert np.array_equal(arrays(hs[i]), ref[i][0]), (rep, i)
            assert np.array_equal(hists[i], ref[i][1]), (rep, i)
    b.close()
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("fd,order", [("f32", 8), ("f64", 4), ("f16", 4)])
def test_batch_members_with_multistep_options_bitwise(fd, order):
    # members whose own options take several steps per launch (on the slab,
    # the full grid or both; 2, 4 or 8 steps on 64- or 128-column strips;
    # density arrays; a full grid taller than one window) beside a member
    # stepping once per launch: in the batch every member steps once per
    # merged launch, and its result must still equal its own solve's, bit
    # for bit; the second solve replays the captured merged propagations
    print(f"case hbatch multistep {fd} order {order}", flush=True)
    ms = [member(i, order, fd) for i in range(6)]
    ctxs = [c for c, _ in ms]
    ds = [d for _, d in ms]
    # order 8: four steps leave no owned rows in a window, so the full grids
    # (taller than one window) take two, and their batch steps one per launch
    full = 4 if order == 4 else 2
    ctxs[0].set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, 4)
    ctxs[1].set_option(ssx.OPT_STEPS_PER_LAUNCH, full)
    ctxs[1].set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, 4)
    ctxs[3].set_option(ssx.OPT_STEPS_PER_LAUNCH, full)
    ctxs[3].set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, 2)
    ctxs[4].set_option(ssx.OPT_STEPS_PER_LAUNCH_SLAB, 8 if order == 4 else 2)
    ctxs[4].set_option(ssx.OPT_SLAB_STRIP, 64)
    ctxs[5].set_option(ssx.OPT_STEPS_PER_LAUNCH, 2)
    alphas = [1e-3 * (1 + i % 2) for i in range(6)]
    ref = []
    for i, (ctx, d) in enumerate(ms):
        h1, hist1, _, _ = ctx.pcg_solve(d, alphas[i], 4)
        ref.append((arrays(h1), hist1))
    b = ssx.Batch(ctxs)
    for rep in range(2):
        hs, hists, its, sts = b.pcg_solve(ds, alphas, 4)
        assert sts == [0] * 6
        for i in range(6):
            assert np.array_equal(arrays(hs[i]), ref[i][0]), (rep, i)
            assert np.array_equal(hists[i], ref[i][1]), (rep, i)
    b.close()
    for c in ctxs:
        c.close()


def test_batch_rejects_mixed_contexts():
    a, _ = member(0, 8, "f32")
    c4, _ = member(1, 4, "f32")
    d64, _ = member(2, 8, "f64")
    for bad in ([a, c4], [a, d64], [a, a], []):
        with pytest.raises(ssx.SSXError):
            ssx.Batch(bad)
    for c in (a, c4, d64):
        c.close()
