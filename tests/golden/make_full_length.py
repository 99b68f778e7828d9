"""Writes the full-length expected values of the two headline configurations
from the FP64 oracle alone (run once; the GPU tests read what it writes).

It imports only ``inputs`` (seeded problems, models, wavelets and random
traces) and ``oracle`` (with its C engine, bitwise equal to the NumPy time
stepping), never the HIP library, so no expected value comes from the path
under test.

* 801 x 1601 grid at 5 m, order 8, 4000 steps (the single-subproblem
  production configuration): d = F h_true for the Ricker point source at
  x_s = 4000 m; F x and F^T y for seeded N(0,1) traces x, y (rounded to FP32,
  the GPU's input type, so both sides see identical inputs); b = F^T d32 and
  K = 30 iterations of Algorithm 1 with the thin-slab preconditioner on the
  Euclidean normal equations (alpha_rel = 1e-3), d32 = d rounded to FP32.
* 401 x 801 grid at 10 m, order 8, 2000 steps (the 64-shot batched
  configuration), shots 0 and 40: d = F h_true and K = 20 iterations.

Each output array is kept as (a) the values on every 32nd (c2) or 16th (c3)
trace for all time samples, rounded to FP32, (b) its row sums (over traces,
one per time sample) and column sums (over time, one per trace) in FP64,
which every element enters, and (c) its FP64 norm.  The PCG histories
(||r_k||, ||g_k||, <g_k, r_k>, ||F h_k - d||) and alpha are kept whole.
tests/golden/SHA256SUMS lists the files' hashes.

Usage: python tests/golden/make_full_length.py [c2|c3 ...]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402

SEED_X, SEED_Y = 20220401, 20220402
C3_SHOTS = (0, 40)


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def keep(out: dict, name: str, a: np.ndarray, step: int) -> None:
    a = np.asarray(a, dtype=np.float64)
    cols = np.arange(0, a.shape[1], step)
    out[f"{name}_cols"] = cols.astype(np.int32)
    out[f"{name}_sample"] = a[:, cols].astype(np.float32)
    out[f"{name}_rowsum"] = a.sum(axis=1)
    out[f"{name}_colsum"] = a.sum(axis=0)
    out[f"{name}_norm"] = np.array(np.linalg.norm(a))


def fp32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def make_c2() -> str:
    wl = inputs.workload(2)
    prob = wl.prob
    m = oracle.Model(prob, wl.kappa, wl.rho, engine="c")
    out = {}
    htrue = inputs.spike_gather(prob, inputs.source_wavelet(prob, wl.freq), 0)
    log("c2: d = F h_true")
    d = m.fwd(htrue)
    keep(out, "d", d, 32)
    d32 = fp32(d)
    log("c2: F x")
    x = fp32(inputs.random_traces((prob.nt, prob.ns), SEED_X))
    keep(out, "Fx", m.fwd(x), 32)
    log("c2: F^T y")
    y = fp32(inputs.random_traces((prob.nt, prob.nr), SEED_Y))
    keep(out, "FTy", m.adj(y), 32)
    log("c2: b = F^T d32")
    keep(out, "b", m.adj(d32), 32)
    path = os.path.join(HERE, "c2_full_length.npz")
    np.savez_compressed(path, **out)
    log(f"c2: propagations written; PCG K = {wl.K}")
    h, hist, alpha = oracle.pcg_solve(m, d32, wl.alpha_rel, wl.K)
    keep(out, "h", h, 32)
    out["hist"] = hist
    out["alpha"] = np.array(alpha)
    np.savez_compressed(path, **out)
    log("c2: done")
    return path


def make_c3() -> str:
    wl = inputs.workload(3)
    prob = wl.prob
    out = {"shots": np.array(C3_SHOTS, dtype=np.int32)}
    wav = inputs.source_wavelet(prob, wl.freq)
    for s in C3_SHOTS:
        p1 = prob.replace(xs=(prob.xs[s],))
        m = oracle.Model(p1, wl.kappa, wl.rho, engine="c")
        htrue = inputs.spike_gather(p1, wav, 0)
        log(f"c3 shot {s}: d = F h_true")
        d = m.fwd(htrue)
        keep(out, f"d{s}", d, 16)
        log(f"c3 shot {s}: PCG K = {wl.K}")
        h, hist, alpha = oracle.pcg_solve(m, fp32(d), wl.alpha_rel, wl.K)
        keep(out, f"h{s}", h, 16)
        out[f"hist{s}"] = hist
        out[f"alpha{s}"] = np.array(alpha)
    path = os.path.join(HERE, "c3_full_length.npz")
    np.savez_compressed(path, **out)
    log("c3: done")
    return path


def write_sums() -> None:
    lines = []
    for name in sorted(os.listdir(HERE)):
        if name.endswith(".npz"):
            with open(os.path.join(HERE, name), "rb") as f:
                lines.append(f"{hashlib.sha256(f.read()).hexdigest()}  {name}\n")
    with open(os.path.join(HERE, "SHA256SUMS"), "w") as f:
        f.writelines(lines)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3"]
    for w in which:
        {"c2": make_c2, "c3": make_c3}[w]()
        write_sums()
