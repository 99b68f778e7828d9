"""Batched shots (several subproblems in one launch per time step) against
the same subproblems run one at a time, and the batched configuration at
full size against the oracle."""
import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402

RHO = 1000.0


def problem(xs, **kw):
    base = dict(nz=41, nx=130, h=10.0, dt=1e-3, nt=150, order=8, npml=12,
                z_src=20.0, x_src0=0.0, ns=130, z_rec=10.0, x_rec0=0.0, nr=130,
                slab_dz=5, xs=tuple(xs))
    base.update(kw)
    return inputs.Problem(**base)


@pytest.mark.parametrize("fd", ["f64", "f32", "f16"])
def test_batched_equals_looped_bitwise(fd):
    xs = (105.0, 431.0, 777.0, 1212.0)
    prob = problem(xs)
    print(f"case batched-vs-looped dtype={fd}", flush=True)
    kap = inputs.kappa_from_velocity(
        inputs.layered_velocity(prob.nz, prob.nx, prob.h, np.random.default_rng(3)))
    vdt = torch.float64 if fd == "f64" else torch.float32
    rng = np.random.default_rng(4)
    d = torch.tensor(rng.standard_normal((len(xs), prob.nt, prob.nr)), dtype=vdt, device="cuda")
    h = torch.tensor(rng.standard_normal((len(xs), prob.nt, prob.ns)), dtype=vdt, device="cuda")
    batch = ssx.Context(prob, kap, RHO, field_dtype=fd)
    outs_b = [batch.fwd(h, batch.empty_r()), batch.adj(d, batch.empty_s()),
              batch.precond(1e-3, h, batch.empty_s())]
    hb, histb, _, _ = batch.pcg_solve(d, 1e-3, 4)
    torch.cuda.synchronize()
    for s, x in enumerate(xs):
        one = ssx.Context(prob.replace(xs=(x,)), kap, RHO, field_dtype=fd)
        hs, ds = h[s:s + 1].contiguous(), d[s:s + 1].contiguous()
        outs_1 = [one.fwd(hs, one.empty_r()), one.adj(ds, one.empty_s()),
                  one.precond(1e-3, hs, one.empty_s())]
        h1, hist1, _, _ = one.pcg_solve(ds, 1e-3, 4)
        torch.cuda.synchronize()
        for ob, o1 in zip(outs_b, outs_1):
            assert torch.equal(ob[s], o1[0]), s
        assert torch.equal(hb[s], h1[0])
        assert np.array_equal(histb[s], hist1[0])
        one.close()
    batch.close()


@pytest.mark.parametrize("fd", ["f32", "f16"])
def test_shot_groups_bitwise(fd):
    # five shots advanced one at a time, in balanced groups (3 + 2 and
    # 2 + 2 + 1), all at once and in the default grouping, with the full grid
    # and the slab grouped differently, with and without graphs: every output
    # bitwise equal
    xs = (105.0, 431.0, 777.0, 1010.0, 1212.0)
    prob = problem(xs)
    print(f"case shot groups dtype={fd}", flush=True)
    kap = inputs.kappa_from_velocity(
        inputs.layered_velocity(prob.nz, prob.nx, prob.h, np.random.default_rng(3)))
    rng = np.random.default_rng(5)
    d = torch.tensor(rng.standard_normal((len(xs), prob.nt, prob.nr)), dtype=torch.float32,
                     device="cuda")
    h = torch.tensor(rng.standard_normal((len(xs), prob.nt, prob.ns)), dtype=torch.float32,
                     device="cuda")
    ctx = ssx.Context(prob, kap, RHO, field_dtype=fd)

    def run():
        out = [ctx.fwd(h, ctx.empty_r()), ctx.adj(d, ctx.empty_s()),
               ctx.precond(1e-3, h, ctx.empty_s())]
        hk, hist, _, _ = ctx.pcg_solve(d, 1e-3, 3)
        torch.cuda.synchronize()
        return [t.cpu() for t in out] + [hk.cpu(), torch.tensor(hist)]

    ctx.set_option(ssx.OPT_SHOT_GROUP, len(xs))
    ref = run()
    for graphs in (True, False):
        ctx.set_graphs(graphs)
        for full, slab in ((1, 1), (3, 3), (2, 5), (5, 2), (0, 0)):
            ctx.set_option(ssx.OPT_SHOT_GROUP, full)
            ctx.set_option(ssx.OPT_SHOT_GROUP_SLAB, slab)
            for i, (a, b) in enumerate(zip(ref, run())):
                assert torch.equal(a, b), (fd, graphs, full, slab, i)
    with pytest.raises(ssx.SSXError):
        ctx.set_option(ssx.OPT_SHOT_GROUP, -1)
    ctx.close()


def test_c3_full_size_truncated_parity():
    # 64 shots on the 401 x 801 layered model (nt = 2000) in bench's launch
    # configuration (autotuned shot groups, tiles, slab kernel): first / last
    # N samples of F, F^T, X, X^T for two shots in different groups against
    # the oracle
    from test_gpu_parity import truncated_parity
    print("case c3 truncated parity", flush=True)
    truncated_parity(inputs.workload(3), "f32", 30, (0, 63), 1e-5, 9)
