"""ssx_dot_static, the entry point that allocates no device memory: its
output equals ssx_dot's (the same kernels and reduction order, bitwise) on
two calls in a row, the second with a smaller input, in FP64 and FP32."""
import ctypes

import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402


def context(nshots, nt, ns, fd):
    prob = inputs.Problem(nz=20, nx=ns, h=10.0, dt=1e-3, nt=nt, order=4, npml=4,
                          z_src=50.0, x_src0=0.0, ns=ns, z_rec=20.0, x_rec0=0.0, nr=ns,
                          slab_dz=3, xs=tuple(100.0 + 37.0 * s for s in range(nshots)))
    rng = np.random.default_rng(0)
    kappa = 1000.0 * rng.uniform(1800.0, 2200.0, size=(prob.nz, prob.nx)) ** 2
    return ssx.Context(prob, kappa, 1000.0, field_dtype=fd)


@pytest.mark.parametrize("fd", ["f64", "f32"])
def test_dot_static_equals_dot(fd):
    L = ssx.lib()
    dt = torch.float64 if fd == "f64" else torch.float32
    stream = torch.cuda.current_stream()
    # first call: 5 shots of 700 x 333, then a smaller one: 2 shots of 40 x 61
    for nshots, nt, ns, seed in ((5, 700, 333, 1), (2, 40, 61, 2)):
        print(f"case ssx_dot_static {fd} nshots {nshots} n {nt * ns}", flush=True)
        ctx = context(nshots, nt, ns, fd)
        g = torch.Generator(device="cuda").manual_seed(seed)
        x = torch.randn((nshots, nt, ns), dtype=dt, device="cuda", generator=g)
        y = torch.randn((nshots, nt, ns), dtype=dt, device="cuda", generator=g)
        out = torch.full((nshots,), float("nan"), dtype=torch.float64, device="cuda")
        st = L.ssx_dot_static(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                              nt * ns, nshots, 0 if fd == "f64" else 1,
                              ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(stream.cuda_stream))
        assert st == 0, L.ssx_last_error()
        ref = ctx.dot(x, y)   # ssx_dot: the context's own scratch, synchronises
        got = out.cpu().numpy()
        ctx.close()
        assert np.array_equal(got, ref), (got, ref)
        # and against a plain FP64 sum
        exact = (x.double() * y.double()).sum(dim=(1, 2)).cpu().numpy()
        assert np.allclose(got, exact, rtol=1e-12, atol=1e-9 * nt * ns)


def test_dot_static_rejects_sizes_beyond_the_maximum():
    L = ssx.lib()
    x = torch.zeros(65, dtype=torch.float64, device="cuda")
    out = torch.zeros(65, dtype=torch.float64, device="cuda")
    for nshots in (0, ssx.DOT_STATIC_MAX_SHOTS + 1):
        st = L.ssx_dot_static(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 1,
                              nshots, 0, ctypes.c_void_p(out.data_ptr()), None)
        assert st == 1 and b"nshots" in L.ssx_last_error()
    st = L.ssx_dot_static(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 1, 1, 2,
                          ctypes.c_void_p(out.data_ptr()), None)
    assert st == 1
