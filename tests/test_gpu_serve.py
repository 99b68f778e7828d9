"""Serving: requests of different sizes admitted as memory and slots free
up, overlapping on the device; every result equals the same request solved
alone, and the mixed-precision solutions stay close to the FP64 oracle."""
import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402
from paper_2203_16573_amd import serve  # noqa: E402

RHO = 1000.0
SHAPES = ((31, 61, 20.0), (41, 81, 15.0), (25, 101, 20.0))


def make_requests(n=6, K=3, fd="f16"):
    reqs = []
    for i in range(n):
        nz, nx, h = SHAPES[i % len(SHAPES)]
        nshots = 1 + (i % 3)
        nt = 120 + 20 * (i % 4)
        rng = np.random.default_rng(100 + i)
        vel = inputs.layered_velocity(nz, nx, h, rng, zrange=(2 * h, (nz - 2) * h),
                                      min_gap=2 * h)
        dt = 0.25 * h / vel.max() * 2.0
        prob = inputs.Problem(nz=nz, nx=nx, h=h, dt=dt, nt=nt, order=8, npml=10,
                              z_src=4 * h, x_src0=0.0, ns=nx, z_rec=2 * h, x_rec0=0.0,
                              nr=nx, slab_dz=5,
                              xs=tuple((k + 0.5) * (nx - 1) * h / nshots for k in range(nshots)))
        kap = inputs.kappa_from_velocity(vel)
        # data of a Ricker point source at each shot's x_s (d = F h_true)
        gen = ssx.Context(prob, kap, RHO, field_dtype="f32")
        wav = inputs.source_wavelet(prob, 0.5 / (4 * dt * 5))
        ht = np.stack([inputs.spike_gather(prob, wav, s) for s in range(nshots)])
        d = gen.fwd(torch.tensor(ht, dtype=torch.float32, device="cuda"), gen.empty_r())
        torch.cuda.synchronize()
        gen.close()
        reqs.append(serve.Request(i, prob, kap, RHO, d, K=K, field_dtype=fd,
                                  arrival=0.004 * i))
    torch.cuda.synchronize()
    return reqs


@pytest.mark.parametrize("graphs", [False, True])
def test_mix_equals_alone(graphs):
    # each request's result is the same served alone and in an overlapping
    # mix, with plain launches and with per-request captured graphs
    print(f"case serving mix vs alone graphs={graphs}", flush=True)
    reqs = make_requests()
    mixed = serve.Server(budget_bytes=8 << 30, slots=3, graphs=graphs).run(reqs, realtime=True)
    assert [r.rid for r in mixed] == list(range(len(reqs)))
    # overlap actually happened: some request was admitted before another finished
    spans = sorted((r.t_admit, r.t_done) for r in mixed)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for req, res in zip(reqs, mixed):
        alone = serve.Server(budget_bytes=8 << 30, slots=1).run([req], realtime=False)[0]
        assert alone.status == res.status and alone.iters == res.iters
        assert torch.equal(alone.h, res.h), req.rid
        assert np.array_equal(alone.hist, res.hist)


@pytest.mark.parametrize("graphs", [False, True])
def test_batched_serving_equals_alone(graphs):
    # slots taking up to three queued requests at once as one heterogeneous
    # batch (propagations merged): every result equals the request served
    # alone
    print(f"case serving batched graphs={graphs}", flush=True)
    reqs = make_requests(n=7)
    res = serve.Server(budget_bytes=8 << 30, slots=2, graphs=graphs, batch=3).run(
        reqs, realtime=False)
    assert [r.rid for r in res] == list(range(len(reqs)))
    # some requests shared a solve: admitted and completed together
    spans = [(r.t_admit, r.t_done) for r in res]
    assert len(set(spans)) < len(spans), spans
    for req, r in zip(reqs, res):
        alone = serve.Server(budget_bytes=8 << 30, slots=1).run([req], realtime=False)[0]
        assert alone.status == r.status and alone.iters == r.iters
        assert torch.equal(alone.h, r.h), req.rid
        assert np.array_equal(alone.hist, r.hist)


def test_budget_limits_residency():
    # a budget of the largest request's footprint: at every admission the
    # requests then resident (admitted, not yet done) fit the budget, and
    # the largest one cannot share it, so some request waits for memory
    print("case serving budget", flush=True)
    reqs = make_requests(n=4)
    size = {r.rid: serve.request_bytes(r) for r in reqs}
    budget = max(size.values())
    res = serve.Server(budget_bytes=budget, slots=4).run(reqs, realtime=False)
    assert len(res) == len(reqs)
    for r in res:
        resident = [q for q in res if q.t_admit <= r.t_admit < q.t_done]
        assert r in resident
        assert sum(size[q.rid] for q in resident) <= budget, (r.rid, [q.rid for q in resident])
    waited = [r for r in res if r.t_admit > min(q.t_done for q in res if q is not r) - 1e-9]
    assert waited, [(r.rid, r.t_admit, r.t_done) for r in res]


@pytest.mark.parametrize("fd,tol", [("f16", 3e-2), ("bf16", 1e-1), ("f32", 1e-4)])
def test_served_solution_against_oracle(fd, tol):
    import oracle
    print(f"case serving vs oracle {fd}", flush=True)
    req = make_requests(n=1, K=3, fd=fd)[0]
    res = serve.Server(budget_bytes=8 << 30, slots=1).run([req], realtime=False)[0]
    m = oracle.Model(req.prob, req.kappa, RHO)
    d = req.d.double().cpu().numpy()
    h_ref, hist_ref, _ = oracle.pcg_solve(m, d[0], req.alpha_rel, req.K)
    h = res.h.double().cpu().numpy()[0]
    err = np.linalg.norm(h - h_ref) / np.linalg.norm(h_ref)
    herr = np.abs(res.hist[0][:, 0] - hist_ref[:, 0]) / hist_ref[:, 0]
    print(f"{fd}: solution rel err {err:.3e}; per-iteration ||r|| rel err {herr}")
    assert err < tol


def test_seeded_stream_requests_against_oracle():
    # the first three requests of the seeded serving stream (its grids, shot
    # counts and layered models), truncated to 40 steps and 3 iterations,
    # served together with FP16 storage; shot 0 of each against the FP64
    # oracle (its C engine, equal to the NumPy stepping)
    import oracle
    stream = inputs.serving_requests(3)
    reqs = []
    for i, (t, wl) in enumerate(stream):
        prob = wl.prob.replace(nt=40)
        print(f"case seeded request {i}: {prob.nz}x{prob.nx}, {prob.nshots} shots", flush=True)
        gen = ssx.Context(prob, wl.kappa, wl.rho, field_dtype="f32")
        wav = inputs.source_wavelet(prob, 0.5 / (4 * prob.dt * 5))
        ht = np.stack([inputs.spike_gather(prob, wav, s) for s in range(prob.nshots)])
        d = gen.fwd(torch.tensor(ht, dtype=torch.float32, device="cuda"), gen.empty_r())
        torch.cuda.synchronize()
        gen.close()
        reqs.append(serve.Request(i, prob, wl.kappa, wl.rho, d, alpha_rel=wl.alpha_rel, K=3,
                                  field_dtype="f16", arrival=0.0))
    res = serve.Server(budget_bytes=64 << 30, slots=3).run(reqs, realtime=False)
    for req, r in zip(reqs, res):
        p1 = req.prob.replace(xs=(req.prob.xs[0],))
        m = oracle.Model(p1, req.kappa, req.rho, engine="c")
        d0 = req.d[0].double().cpu().numpy()
        h_ref, _, _ = oracle.pcg_solve(m, d0, req.alpha_rel, req.K)
        h = r.h[0].double().cpu().numpy()
        err = np.linalg.norm(h - h_ref) / np.linalg.norm(h_ref)
        print(f"  request {req.rid}: FP16 solution rel err {err:.2e}", flush=True)
        assert err < 3e-2
