"""Host-side checks of the C ABI: the library loads, exports every entry
point declared in include/ssx.h, and validates problems without a GPU."""
import os
import re

import numpy as np
import pytest

import inputs
import paper_2203_16573_amd as ssx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "ssx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ssx3?_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert set(declared_functions()) == set(ssx.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ssx.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_validate_accepts_the_benchmark_configurations():
    for c in (1, 2, 3):
        wl = inputs.workload(c)
        fd = "f64" if wl.dtype == "f64" else "f32"
        ssx.validate(wl.prob, wl.kappa, wl.rho, field_dtype=fd)
        assert ssx.footprint(wl.prob, field_dtype=fd) > 0


@pytest.mark.parametrize("change,status", [
    (dict(dt=6e-3), 2),                 # Courant number above the bound
    (dict(order=6), 1),
    (dict(z_src=-5.0), 1),              # line above the grid
    (dict(z_rec=2010.0), 1),            # line below the grid
    (dict(x_src0=15.0), 1),             # not on a grid column
    (dict(ns=10_000), 1),
    (dict(slab_dz=0), 1),
    (dict(nt=0), 1),
    (dict(npml=-1), 1),
    (dict(nz=5), 1),
])
def test_validate_rejects(change, status):
    wl = inputs.workload(1)
    prob = wl.prob.replace(**change)
    with pytest.raises(ssx.SSXError) as e:
        kap = wl.kappa if prob.nz == wl.prob.nz else None
        ssx.validate(prob, kap, wl.rho, field_dtype="f64")
    assert e.value.status == status


def test_validate_rejects_bad_models_and_dtypes():
    wl = inputs.workload(1)
    bad = wl.kappa.copy()
    bad[3, 4] = np.nan
    with pytest.raises(ssx.SSXError):
        ssx.validate(wl.prob, bad, wl.rho, field_dtype="f64")
    bad[3, 4] = -1.0
    with pytest.raises(ssx.SSXError):
        ssx.validate(wl.prob, bad, wl.rho, field_dtype="f64")
    with pytest.raises(ssx.SSXError):
        ssx.validate(wl.prob, wl.kappa, -1.0, field_dtype="f64")
    P = ssx.make_problem(wl.prob, 1, "f32")
    P.vec_dtype = 0  # F32 fields with F64 vectors is not a supported pair
    import ctypes
    assert ssx.lib().ssx_validate(ctypes.byref(P), None, 1000.0) == 1
    assert ssx.lib().ssx_footprint(ctypes.byref(P)) == 0


def test_footprint_scales_with_shots():
    wl = inputs.workload(3)
    one = ssx.footprint(wl.prob, nshots=1)
    many = ssx.footprint(wl.prob, nshots=64)
    assert 40 * one < many < 70 * one


def test_problem_struct_matches_header(tmp_path):
    # the ctypes mirror of ssx_problem has the header's size and offsets
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    names = [f[0] for f in ssx.ssx_problem._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"ssx.h\"\n"
                   "int main(void) {\n  printf(\"%zu\\n\", sizeof(ssx_problem));\n" +
                   "".join(f"  printf(\"%zu\\n\", offsetof(ssx_problem, {n}));\n" for n in names) +
                   "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert out[0] == ctypes.sizeof(ssx.ssx_problem)
    for n, off in zip(names, out[1:]):
        assert off == getattr(ssx.ssx_problem, n).offset, n


def test_footprint_counts_the_receiver_side_slab():
    wl = inputs.workload(1)
    base = ssx.footprint(wl.prob, field_dtype="f64")
    both = ssx.footprint(wl.prob.replace(rslab_dz=-5), field_dtype="f64")
    # one more slab of fields and coefficients plus three trace vectors
    assert base < both < 1.5 * base
    ssx.validate(wl.prob.replace(rslab_dz=4), wl.kappa, wl.rho, field_dtype="f64")


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


# ---------------------------------------------------------------------------
# the 3D entry points (host-only checks)

def _prob3(**kw):
    base = dict(nz=20, ny=16, nx=24, h=10.0, dt=1e-3, nt=10, order=8, npml=5,
                z_src=35.0, x_src0=20.0, y_src0=10.0, nsx=10, nsy=6,
                z_rec=120.0, x_rec0=0.0, y_rec0=0.0, nrx=24, nry=16)
    base.update(kw)
    return inputs.Problem3(**base)


def test_validate3_accepts_and_sizes():
    prob = _prob3()
    kap = np.full((prob.nz, prob.ny, prob.nx), 1000.0 * 3000.0 ** 2)
    ssx.validate3(prob, kap, 1000.0, field_dtype="f32")
    ssx.validate3(prob, kap, 1000.0, field_dtype="f64")
    n = (prob.nz + 10) * (prob.ny + 10) * (prob.nx + 10)
    f32, f64 = ssx.footprint3(prob, "f32"), ssx.footprint3(prob, "f64")
    # the full grid's seven fields and ck at least, plus the slab and vectors
    assert f32 > 8 * n * 4 and f64 > 8 * n * 8 and f64 < 2 * f32 + 8 * 1024


@pytest.mark.parametrize("change,status", [
    (dict(order=6), 1),
    (dict(nz=8), 1),                    # below order + 1 nodes
    (dict(npml=-1), 1),
    (dict(x_src0=15.0), 1),             # off a grid node
    (dict(nsx=23), 1),                  # past the last column
    (dict(y_rec0=10.0, nry=16), 1),     # past the last row
    (dict(z_src=195.0), 1),             # between the last node and beyond
    (dict(z_rec=-1.0), 1),
    (dict(nt=0), 1),
    (dict(pml_R=1.0), 1),
    (dict(dt=2e-3), 2),                 # c dt / h above 1 / (sqrt 3 sum |c_m|)
    (dict(slab_dz=0), 1),
    (dict(x_s=float("nan")), 1),
])
def test_validate3_rejects(change, status):
    prob = _prob3(**change)
    kap = np.full((prob.nz, prob.ny, prob.nx), 1000.0 * 3000.0 ** 2)
    with pytest.raises(ssx.SSXError) as e:
        ssx.validate3(prob, kap, 1000.0)
    assert e.value.status == status


def test_validate3_rejects_models_and_dtypes():
    prob = _prob3()
    kap = np.full((prob.nz, prob.ny, prob.nx), 1000.0 * 3000.0 ** 2)
    bad = kap.copy()
    bad[3, 4, 5] = -1.0
    with pytest.raises(ssx.SSXError):
        ssx.validate3(prob, bad, 1000.0)
    with pytest.raises(ssx.SSXError):
        ssx.validate3(prob, kap, 0.0)
    P = ssx.make_problem3(prob, "f32")
    P.field_dtype = 2   # F16: not a 3D field type
    assert ssx.lib().ssx3_validate(P, None, 1000.0) == 1
    assert ssx.lib().ssx3_footprint(P) == 0
    with pytest.raises(ValueError):
        ssx.make_problem3(prob, "bf16")
