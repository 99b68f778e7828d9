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

