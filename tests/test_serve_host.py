"""Host-side checks of the serving runtime (no GPU work)."""
import numpy as np
import pytest

import inputs
from paper_2203_16573_amd import serve


def test_request_bytes_and_rejection():
    prob = inputs.Problem(nz=31, nx=61, h=20.0, dt=2e-3, nt=100, order=8, npml=10,
                          z_src=80.0, x_src0=0.0, ns=61, z_rec=40.0, x_rec0=0.0, nr=61,
                          slab_dz=5, xs=(300.0, 900.0))
    req = serve.Request(0, prob, np.full((31, 61), 4e9), 1000.0, d=None, field_dtype="f16")
    nb = serve.request_bytes(req)
    assert nb > 2 * 100 * 61 * 4
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=nb - 1).run([req])


def test_summary_percentiles():
    class H:
        shape = (2,)
    res = [serve.Result(i, H(), None, 1, 0, 0.0, 0.0, float(i + 1)) for i in range(100)]
    s = serve.summarize(res, wall=10.0)
    assert s["solves"] == 200 and s["requests"] == 100
    assert abs(s["latency_p50_s"] - 50.5) < 1e-9
    assert s["latency_p99_s"] > 99



def _req(rid, nz, nx, nt, shots, order=8, fd="f16", K=20):
    prob = inputs.Problem(nz=nz, nx=nx, h=20.0, dt=2e-3, nt=nt, order=order, npml=10,
                          z_src=80.0, x_src0=0.0, ns=nx, z_rec=40.0, x_rec0=0.0, nr=nx,
                          slab_dz=5, xs=tuple(100.0 * (k + 1) for k in range(shots)))
    return serve.Request(rid, prob, np.full((nz, nx), 4e9), 1000.0, d=None, field_dtype=fd, K=K)


def test_batch_grouping_rule():
    # the head, then later compatible requests in queue order: same order,
    # field type and K, small enough, records within the ratio, within the
    # free memory, at most `batch` in all
    from collections import deque
    reqs = [_req(0, 31, 61, 100, 1), _req(1, 31, 61, 120, 2), _req(2, 31, 61, 100, 1, order=4),
            _req(3, 31, 61, 100, 1, fd="f32"), _req(4, 31, 61, 400, 1), _req(5, 91, 181, 110, 1),
            _req(6, 31, 61, 140, 1, K=10), _req(7, 31, 61, 90, 1), _req(8, 31, 61, 100, 1)]
    sizes = {r.rid: 100 for r in reqs}
    q = deque(reqs)
    group, nb = serve.take_group(q, sizes, free=10_000, batch=4, batch_cells=20_000,
                                 batch_nt_ratio=1.5)
    # 2: other order; 3: other field type; 4: record 4x longer; 5: 111 x 201
    # cells above the limit; 6: other K
    assert [r.rid for r in group] == [0, 1, 7, 8] and nb == 400
    assert [r.rid for r in q] == [2, 3, 4, 5, 6]
    # free memory bounds the group; batch = 1 takes the head alone
    q = deque(reqs)
    group, nb = serve.take_group(q, sizes, free=250, batch=4, batch_cells=20_000,
                                 batch_nt_ratio=1.5)
    assert [r.rid for r in group] == [0, 1] and nb == 200
    q = deque(reqs)
    group, _ = serve.take_group(q, sizes, free=10_000, batch=1, batch_cells=20_000,
                                batch_nt_ratio=1.5)
    assert [r.rid for r in group] == [0] and len(q) == len(reqs) - 1
    # a head above the size limit runs alone
    q = deque([reqs[5]] + reqs[:2])
    group, _ = serve.take_group(q, sizes, free=10_000, batch=4, batch_cells=20_000,
                                batch_nt_ratio=1.5)
    assert [r.rid for r in group] == [5]
