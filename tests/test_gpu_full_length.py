"""Full-length parity of the benchmark configurations with the FP64 oracle.

The expected values were written once by tests/golden/make_full_length.py,
which calls only the oracle (its C engine) and the seeded input
generators; tests/golden/SHA256SUMS holds their hashes.  Here the HIP path
runs the same seeded inputs in the launch configuration the benchmark times
(autotuned), through the C ABI, and is compared on what the files keep of
each output: the values on every 32nd (801 x 1601) or 16th (401 x 801)
trace for all time samples, and the row and column sums and the norm of the
whole array, which every element enters.

Tolerances: FP64 fields 1e-12 (sums, norm); FP32 fields 1e-5 per 4000-step
propagation and 1e-4 on the K = 30 solution and its residual history (the
stated targets).  The data d of the solves are the FP64 propagation rounded
to FP32 on both sides.  FP16 / BF16 fields (FP32 arithmetic) are held to
the error bounds they are documented with, which miss the 1e-4 target.
"""
import hashlib
import os

import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SEED_X, SEED_Y = 20220401, 20220402


def golden(name):
    sums = {}
    with open(os.path.join(GOLDEN, "SHA256SUMS")) as f:
        for line in f:
            h, n = line.split()
            sums[n] = h
    path = os.path.join(GOLDEN, name)
    with open(path, "rb") as f:
        assert hashlib.sha256(f.read()).hexdigest() == sums[name], f"{name}: hash mismatch"
    return np.load(path)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def errors(z, name, a):
    """Relative errors of a full output array against the kept values."""
    a = np.asarray(a, dtype=np.float64)
    cols = z[f"{name}_cols"]
    return {"sample": rel(a[:, cols], z[f"{name}_sample"]),
            "rowsum": rel(a.sum(axis=1), z[f"{name}_rowsum"]),
            "colsum": rel(a.sum(axis=0), z[f"{name}_colsum"]),
            "norm": abs(np.linalg.norm(a) / float(z[f"{name}_norm"]) - 1.0)}


def check(z, name, a, tol, tol_sample=None):
    e = errors(z, name, a)
    print(f"  {name}: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    ts = tol if tol_sample is None else tol_sample
    assert e["sample"] <= ts and e["rowsum"] <= tol and e["colsum"] <= tol and e["norm"] <= tol, e
    return e


def hist_errors(h, h_ref):
    """Residual history: relative L2 of each column, and the largest
    relative error of ||r_k|| entry by entry."""
    cols = [rel(h[:, j], h_ref[:, j]) for j in range(4)]
    rk = float(np.max(np.abs(h[:, 0] - h_ref[:, 0]) / h_ref[:, 0]))
    return cols, rk


def dev(x, fd):
    return torch.tensor(np.ascontiguousarray(x),
                        dtype=torch.float64 if fd == "f64" else torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def bench_context(wl, fd):
    """A context in the launch configuration bench.py times (autotuned)."""
    from paper_2203_16573_amd import autotune
    ctx = ssx.Context(wl.prob, wl.kappa, wl.rho, field_dtype=fd)
    choice = autotune.choose(wl.prob, wl.kappa, wl.rho, field_dtype=fd)
    autotune.apply(ctx, choice)
    print(f"  {fd} launch shape {ctx.launch_shape()}", flush=True)
    return ctx


def htrue_of(wl):
    wav = inputs.source_wavelet(wl.prob, wl.freq)
    return np.stack([inputs.spike_gather(wl.prob, wav, s) for s in range(wl.prob.nshots)])


@pytest.fixture(scope="module")
def c2():
    z = golden("c2_full_length.npz")
    wl = inputs.workload(2)
    print("case c2 full length: FP64 data", flush=True)
    ctx = ssx.Context(wl.prob, wl.kappa, wl.rho, field_dtype="f64")
    d64 = host(ctx.fwd(dev(htrue_of(wl), "f64"), ctx.empty_r()))
    ctx.close()
    return wl, z, d64


def test_c2_fp64_data_full_length(c2):
    # F h_true over 4000 steps with FP64 fields against the oracle
    _, z, d64 = c2
    check(z, "d", d64[0], 1e-12, tol_sample=1e-7)


def test_c2_fp32_propagations_full_length(c2):
    wl, z, d64 = c2
    prob = wl.prob
    print("case c2 full length: FP32 propagations", flush=True)
    ctx = bench_context(wl, "f32")
    x = inputs.random_traces((prob.nt, prob.ns), SEED_X)[None]
    y = inputs.random_traces((prob.nt, prob.nr), SEED_Y)[None]
    d32 = d64.astype(np.float32)
    errs = [check(z, "d", host(ctx.fwd(dev(htrue_of(wl), "f32"), ctx.empty_r()))[0], 1e-5),
            check(z, "Fx", host(ctx.fwd(dev(x, "f32"), ctx.empty_r()))[0], 1e-5),
            check(z, "FTy", host(ctx.adj(dev(y, "f32"), ctx.empty_s()))[0], 1e-5),
            check(z, "b", host(ctx.adj(dev(d32, "f32"), ctx.empty_s()))[0], 1e-5)]
    ctx.close()
    assert errs


def c2_solve(wl, z, d64, fd):
    ctx = bench_context(wl, fd)
    h, hist, it, _ = ctx.pcg_solve(dev(d64.astype(np.float32), "f32"), wl.alpha_rel, wl.K,
                                   raise_on_breakdown=False)
    h = host(h)[0]
    hist = np.asarray(hist)[0]
    ctx.close()
    assert it == wl.K
    e = errors(z, "h", h)
    cols, rk = hist_errors(hist, z["hist"])
    print(f"  {fd} K = {wl.K}: h " + ", ".join(f"{k} {v:.2e}" for k, v in e.items()) +
          f"; history columns {['%.2e' % c for c in cols]}, max ||r_k|| entry {rk:.2e}",
          flush=True)
    return e, cols, rk


def test_c2_fp32_pcg_full_length(c2):
    wl, z, d64 = c2
    print("case c2 full length: FP32 PCG", flush=True)
    e, cols, rk = c2_solve(wl, z, d64, "f32")
    assert max(e.values()) <= 1e-4, e
    assert max(cols) <= 1e-4 and rk <= 1e-4, (cols, rk)
    assert abs(float(z["alpha"])) > 0


@pytest.mark.parametrize("fd,bound", [("f16", 3e-2), ("bf16", 1.5e-1)])
def test_c4_16bit_pcg_against_oracle(c2, fd, bound):
    # 16-bit wavefield storage (FP32 arithmetic, FP64 dots): the error of the
    # full solve against the oracle is reported and held to its documented
    # bound (it does not meet the 1e-4 target)
    wl, z, d64 = c2
    print(f"case c4 full length: {fd} PCG", flush=True)
    e, cols, rk = c2_solve(wl, z, d64, fd)
    assert e["sample"] <= bound and e["norm"] <= bound, e


def test_c3_full_length(tmp_path):
    z = golden("c3_full_length.npz")
    wl = inputs.workload(3)
    shots = [int(s) for s in z["shots"]]
    print("case c3 full length: FP64 data, 64 shots", flush=True)
    ctx = ssx.Context(wl.prob, wl.kappa, wl.rho, field_dtype="f64")
    d64 = host(ctx.fwd(dev(htrue_of(wl), "f64"), ctx.empty_r()))
    ctx.close()
    for s in shots:
        check(z, f"d{s}", d64[s], 1e-12, tol_sample=1e-7)
    print("case c3 full length: FP32 PCG, 64 shots", flush=True)
    ctx = bench_context(wl, "f32")
    h, hist, it, _ = ctx.pcg_solve(dev(d64.astype(np.float32), "f32"), wl.alpha_rel, wl.K,
                                   raise_on_breakdown=False)
    h = host(h)
    hist = np.asarray(hist)
    ctx.close()
    assert it == wl.K
    for s in shots:
        e = check(z, f"h{s}", h[s], 1e-4)
        cols, rk = hist_errors(hist[s], z[f"hist{s}"])
        print(f"  shot {s} history columns {['%.2e' % c for c in cols]}, "
              f"max ||r_k|| entry {rk:.2e}", flush=True)
        assert max(cols) <= 1e-4 and rk <= 1e-4, (cols, rk)
        assert e
