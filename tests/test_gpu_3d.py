"""3D propagation (ssx3_*) on the GPU against the 3D FP64 oracle: F and
F^T element by element on a grid that spans two x workgroups with a ragged
tail and a ragged y block, a source plane between grid planes, both
stencil orders, FP64 and FP32 fields; and the dot-product identity of the
GPU pair at a larger size."""
import numpy as np
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2203_16573_amd as ssx  # noqa: E402
from oracle.prop3 import Grid3, adjoint3, forward3  # noqa: E402

RHO = 1000.0


def problem(order, nz=14, ny=11, nx=70, L=4, nt=24):
    h = 10.0
    return inputs.Problem3(nz=nz, ny=ny, nx=nx, h=h, dt=1e-3, nt=nt, order=order, npml=L,
                           z_src=35.0, x_src0=3 * h, y_src0=2 * h, nsx=60, nsy=7,
                           z_rec=90.0, x_rec0=h, y_rec0=h, nrx=66, nry=9)


def model(prob, seed=3):
    vel = inputs.layered_velocity3(prob.nz, prob.ny, prob.nx, prob.h,
                                   np.random.default_rng(seed))
    return RHO * vel * vel


def planes(g, prob):
    src = g.p_plane(prob.z_src, prob.x_src0, prob.nsx, prob.y_src0, prob.nsy)
    rec = g.p_plane(prob.z_rec, prob.x_rec0, prob.nrx, prob.y_rec0, prob.nry)
    return src, rec


@pytest.mark.parametrize("order", [4, 8])
@pytest.mark.parametrize("fd,tol", [("f64", 1e-12), ("f32", 2e-5)])
def test_forward_and_transpose_against_oracle(order, fd, tol):
    print(f"case 3d parity order {order} {fd}", flush=True)
    prob = problem(order)
    kap = model(prob)
    rng = np.random.default_rng(11)
    h = rng.standard_normal((prob.nt, prob.nsy, prob.nsx))
    r = rng.standard_normal((prob.nt, prob.nry, prob.nrx))
    g = Grid3(kap, RHO, prob.h, prob.dt, prob.npml, prob.pml_R, order)
    src, rec = planes(g, prob)
    P_ref, _ = forward3(g, prob.nt, h_src=(src, h.reshape(prob.nt, -1)), rec_p=rec)
    hb_ref, _ = adjoint3(g, prob.nt, h_plane=src, rec_p=(rec, r.reshape(prob.nt, -1)))
    ctx = ssx.Context3(prob, kap, RHO, field_dtype=fd)
    dt = ctx.dtype
    d = ctx.fwd(torch.tensor(h, dtype=dt, device="cuda"), ctx.empty_rec())
    gb = ctx.adj(torch.tensor(r, dtype=dt, device="cuda"), ctx.empty_src())
    torch.cuda.synchronize()
    P = d.double().cpu().numpy().reshape(prob.nt, -1)
    hb = gb.double().cpu().numpy().reshape(prob.nt, -1)
    ctx.close()
    assert np.abs(P_ref).max() > 0 and np.abs(hb_ref).max() > 0
    eP = np.abs(P - P_ref).max() / np.abs(P_ref).max()
    eh = np.abs(hb - hb_ref).max() / np.abs(hb_ref).max()
    print(f"  F {eP:.2e}  F^T {eh:.2e}", flush=True)
    assert eP <= tol and eh <= tol, (eP, eh)


@pytest.mark.parametrize("fd,tol", [("f64", 1e-12), ("f32", 1e-4)])
def test_dot_product_on_gpu(fd, tol):
    # <F h, r> = <h, F^T r> with both sides from the GPU pair, at a size of
    # several x and y blocks and z planes in every direction
    print(f"case 3d dot {fd}", flush=True)
    prob = problem(8, nz=60, ny=50, nx=150, L=10, nt=120).replace(
        z_src=200.0, nsx=140, nsy=40, z_rec=405.0, nrx=148, nry=48)
    kap = model(prob, 5)
    ctx = ssx.Context3(prob, kap, RHO, field_dtype=fd)
    gen = torch.Generator(device="cuda").manual_seed(2)
    h = torch.randn((prob.nt, prob.nsy, prob.nsx), dtype=ctx.dtype, device="cuda",
                    generator=gen)
    r = torch.randn((prob.nt, prob.nry, prob.nrx), dtype=ctx.dtype, device="cuda",
                    generator=gen)
    d = ctx.fwd(h, ctx.empty_rec())
    g = ctx.adj(r, ctx.empty_src())
    torch.cuda.synchronize()
    lhs = float((d.double() * r.double()).sum())
    rhs = float((h.double() * g.double()).sum())
    scale = float(d.double().norm() * r.double().norm())
    ctx.close()
    assert scale > 0
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs)


def test_rejects_bad_arguments():
    prob = problem(4, nt=4)
    kap = model(prob)
    ctx = ssx.Context3(prob, kap, RHO, field_dtype="f32")
    with pytest.raises(ValueError):
        ctx.fwd(torch.zeros((prob.nt, prob.nsy, prob.nsx + 1), device="cuda"), ctx.empty_rec())
    with pytest.raises(ValueError):
        ctx.fwd(ctx.empty_src().double(), ctx.empty_rec())
    ctx.close()
    with pytest.raises(ValueError):
        ssx.Context3(prob, kap[:, :, :-1], RHO)


# ---------------------------------------------------------------------------
# the 3D subproblem: penalty, thin-slab M^-1 and Algorithm 1 against the
# 3D oracle (oracle.ops3)

from oracle.ops3 import (Model3, dscale3, lateral_distance3, pcg_solve3,  # noqa: E402
                         precond3)


def problem_s(order, dz):
    return problem(order).replace(slab_dz=dz, x_s=345.0, y_s=45.0)


@pytest.mark.parametrize("order,dz", [(4, 3), (8, -2)])
@pytest.mark.parametrize("fd,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_preconditioner_and_penalty_against_oracle(order, dz, fd, tol):
    print(f"case 3d precond order {order} dz {dz} {fd}", flush=True)
    prob = problem_s(order, dz)
    kap = model(prob)
    m = Model3(prob, kap, RHO)
    rng = np.random.default_rng(17)
    r = rng.standard_normal((prob.nt, prob.ns))
    ref = precond3(m, 2e-3, r)
    ctx = ssx.Context3(prob, kap, RHO, field_dtype=fd)
    rt = torch.tensor(r.reshape(prob.nt, prob.nsy, prob.nsx), dtype=ctx.dtype, device="cuda")
    g = ctx.precond(2e-3, rt, ctx.empty_src())
    a = ctx.penalty(ssx.PEN_A, 0.0, rt, ctx.empty_src())
    dh = ctx.penalty(ssx.PEN_DHALF, 2e-3, rt, ctx.empty_src())
    torch.cuda.synchronize()
    out = g.double().cpu().numpy().reshape(prob.nt, -1)
    ctx_a = a.double().cpu().numpy().reshape(prob.nt, -1)
    ctx_d = dh.double().cpu().numpy().reshape(prob.nt, -1)
    ctx.close()
    e = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"  M^-1 {e:.2e}", flush=True)
    assert e <= tol
    dist = lateral_distance3(prob)[None, :]
    assert np.abs(ctx_a - dist * r).max() <= tol * np.abs(dist * r).max()
    dref = dscale3(prob, 2e-3)[None, :] * r
    assert np.abs(ctx_d - dref).max() <= tol * np.abs(dref).max()


@pytest.mark.parametrize("fd,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_pcg_solve_against_oracle(fd, tol):
    print(f"case 3d pcg {fd}", flush=True)
    prob = problem_s(8, 3)
    kap = model(prob)
    m = Model3(prob, kap, RHO)
    rng = np.random.default_rng(19)
    d = m.fwd(rng.standard_normal((prob.nt, prob.ns)))
    K = 4
    h_ref, hist_ref, _ = pcg_solve3(m, d, 1e-3, K)
    ctx = ssx.Context3(prob, kap, RHO, field_dtype=fd)
    dt = torch.tensor(d.reshape(prob.nt, prob.nry, prob.nrx), dtype=ctx.dtype, device="cuda")
    h, hist, it = ctx.pcg_solve(dt, 1e-3, K)
    torch.cuda.synchronize()
    hh = h.double().cpu().numpy().reshape(prob.nt, -1)
    ctx.close()
    assert it == K
    e = np.linalg.norm(hh - h_ref) / np.linalg.norm(h_ref)
    eh = np.abs(hist - hist_ref).max(axis=0) / np.abs(hist_ref).max(axis=0)
    print(f"  h {e:.2e}, history {eh}", flush=True)
    assert e <= tol
    assert np.all(eh <= tol), eh
