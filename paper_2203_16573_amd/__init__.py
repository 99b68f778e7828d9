"""Python binding of libssx (surface-source subproblem on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libssx.so``.  PyTorch supplies device memory and the stream.
The binding fails loudly when the library is missing; there is no CPU path.

Function names follow the C ABI (include/ssx.h):

    ctx = Context(prob, kappa, rho, xs, field_dtype="f32")
    ctx.fwd(h, d)          d = F h
    ctx.adj(r, g)          g = F^T r
    ctx.slab_fwd(f, P, V)  thin-slab X f = (P, V)
    ctx.slab_adj(a, b, f)  f = X^T (a, b)
    ctx.penalty(op, a, x, y)
    ctx.precond(alpha_hat, r, g)
    ctx.normal(alpha, p, q, Fp=None)
    ctx.pcg_solve(d, alpha_rel, maxit, ...) -> (h, hist, iters, status)
    ctx.weight_d(r, y)     y = W_d r   (receiver-side slab)
    ctx.weight_m(x, y)     y = W_m x   (source-side slab)
    ctx.normal_w(alpha, p, q, Fp=None)
    ctx.pcg_solve_w(d, alpha, maxit, ...) -> (h, hist, iters, status)
    ctx.fwd_v(f, y)        y = V f
    ctx.adj_v(r, g)        g = V^T r
    ctx.tr_inverse(d, h)   h = 4 V^T d (time-reversal inverse of F)
    ctx.lam(side, transpose, x, y)   y = Lambda~ x or its transpose
    ctx.block(src, rec, transpose, x, y)   a block of the modelling operator
    ctx.misfit_gradient(h, d, g) -> J   dJ/dkappa of 1/2 ||F h - d||^2
    ctx.pcg_solve_v(d, alpha_rel, maxit)   the normal load as the unknown

``prob`` is any object with the fields of ``ssx_problem`` (nz, nx, h, dt,
nt, order, npml, pml_R, z_src, x_src0, ns, z_rec, x_rec0, nr, slab_dz and,
optionally, rslab_dz); the number of shots is ``len(xs)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssx.so")

DTYPES = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
PEN_A, PEN_ATA, PEN_DHALF = 0, 1, 2
OPT_GRAPHS, OPT_STEP_KERNEL, OPT_TILE_Z, OPT_TILE_Z_SLAB = 0, 1, 2, 3
OPT_STEPS_PER_LAUNCH, OPT_STEPS_PER_LAUNCH_SLAB = 4, 5
OPT_SHOT_GROUP, OPT_SHOT_GROUP_SLAB, OPT_SLAB_STRIP = 6, 7, 8
OPT_TILE_LOOP = 9
OPT_OVERLAP = 10
OPT_STRIP = 11

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_CFL", 3: "ERR_OOM", 4: "ERR_HIP",
          5: "ERR_BREAKDOWN", 6: "ERR_NONFINITE"}

EXPORTS = ("ssx_validate", "ssx_footprint", "ssx_create", "ssx_destroy", "ssx_fwd",
           "ssx_adj", "ssx_slab_fwd", "ssx_slab_adj", "ssx_penalty", "ssx_precond",
           "ssx_normal", "ssx_dot", "ssx_pcg_solve", "ssx_set_option", "ssx_last_error",
           "ssx_step_kernel_name", "ssx_cells_per_launch", "ssx_launch_shape",
           "ssx_weight_d", "ssx_weight_m", "ssx_normal_w", "ssx_pcg_solve_w",
           "ssx_fwd_v", "ssx_adj_v", "ssx_tr_inverse", "ssx_lambda", "ssx_block",
           "ssx_misfit_gradient", "ssx_pcg_solve_v", "ssx_dot_static", "ssx_create_density",
           "ssx_batch_create", "ssx_batch_pcg_solve", "ssx_batch_destroy",
           "ssx3_validate", "ssx3_footprint", "ssx3_create", "ssx3_fwd", "ssx3_adj",
           "ssx3_penalty", "ssx3_precond", "ssx3_pcg_solve", "ssx3_destroy")

DOT_STATIC_MAX_SHOTS = 64  # SSX_DOT_STATIC_MAX_SHOTS


class SSXError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class ssx_problem(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("h", ctypes.c_double), ("dt", ctypes.c_double),
                ("nt", ctypes.c_int32), ("order", ctypes.c_int32),
                ("npml", ctypes.c_int32), ("pml_R", ctypes.c_double),
                ("z_src", ctypes.c_double), ("x_src0", ctypes.c_double),
                ("ns", ctypes.c_int32), ("z_rec", ctypes.c_double),
                ("x_rec0", ctypes.c_double), ("nr", ctypes.c_int32),
                ("slab_dz", ctypes.c_int32), ("nshots", ctypes.c_int32),
                ("field_dtype", ctypes.c_int32), ("vec_dtype", ctypes.c_int32),
                ("rslab_dz", ctypes.c_int32)]


class ssx3_problem(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("h", ctypes.c_double), ("dt", ctypes.c_double),
                ("nt", ctypes.c_int32), ("order", ctypes.c_int32),
                ("npml", ctypes.c_int32), ("pml_R", ctypes.c_double),
                ("z_src", ctypes.c_double), ("x_src0", ctypes.c_double),
                ("y_src0", ctypes.c_double), ("nsx", ctypes.c_int32), ("nsy", ctypes.c_int32),
                ("z_rec", ctypes.c_double), ("x_rec0", ctypes.c_double),
                ("y_rec0", ctypes.c_double), ("nrx", ctypes.c_int32), ("nry", ctypes.c_int32),
                ("field_dtype", ctypes.c_int32), ("slab_dz", ctypes.c_int32),
                ("x_s", ctypes.c_double), ("y_s", ctypes.c_double)]


_lib = None


def lib():
    """Load libssx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_2203_16573_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, c_int, c_dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        for name in EXPORTS:
            getattr(L, name).restype = c_int
        P = ctypes.POINTER(ssx_problem)
        dp = ctypes.POINTER(ctypes.c_double)
        L.ssx_validate.argtypes = [P, dp, c_dbl]
        L.ssx_footprint.argtypes = [P]
        L.ssx_footprint.restype = ctypes.c_size_t
        L.ssx_create.argtypes = [P, dp, c_dbl, dp, vp, vp, ctypes.c_size_t,
                                 ctypes.POINTER(vp)]
        L.ssx_create_density.argtypes = [P, dp, dp, dp, vp, vp, ctypes.c_size_t,
                                         ctypes.POINTER(vp)]
        L.ssx_destroy.argtypes = [vp]
        L.ssx_destroy.restype = None
        L.ssx_fwd.argtypes = [vp, vp, vp]
        L.ssx_adj.argtypes = [vp, vp, vp]
        L.ssx_slab_fwd.argtypes = [vp, vp, vp, vp]
        L.ssx_slab_adj.argtypes = [vp, vp, vp, vp]
        L.ssx_penalty.argtypes = [vp, c_int, c_dbl, vp, vp]
        L.ssx_precond.argtypes = [vp, c_dbl, vp, vp]
        L.ssx_normal.argtypes = [vp, c_dbl, vp, vp, vp]
        L.ssx_dot.argtypes = [vp, vp, vp, ctypes.c_int64, dp]
        L.ssx_dot_static.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     vp, vp]
        L.ssx_pcg_solve.argtypes = [vp, vp, c_dbl, ctypes.c_int32, c_dbl, ctypes.c_int32,
                                    vp, dp, ctypes.POINTER(ctypes.c_int32)]
        L.ssx_weight_d.argtypes = [vp, vp, vp]
        L.ssx_weight_m.argtypes = [vp, vp, vp]
        L.ssx_normal_w.argtypes = [vp, c_dbl, vp, vp, vp]
        L.ssx_pcg_solve_w.argtypes = L.ssx_pcg_solve.argtypes
        L.ssx_fwd_v.argtypes = [vp, vp, vp]
        L.ssx_adj_v.argtypes = [vp, vp, vp]
        L.ssx_tr_inverse.argtypes = [vp, vp, vp]
        L.ssx_lambda.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp]
        L.ssx_block.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp]
        L.ssx_misfit_gradient.argtypes = [vp, vp, vp, vp, dp]
        L.ssx_pcg_solve_v.argtypes = [vp, vp, c_dbl, ctypes.c_int32, c_dbl, vp, dp,
                                      ctypes.POINTER(ctypes.c_int32)]
        L.ssx_set_option.argtypes = [vp, c_int, c_int]
        L.ssx_last_error.restype = ctypes.c_char_p
        L.ssx_step_kernel_name.argtypes = [vp]
        L.ssx_step_kernel_name.restype = ctypes.c_char_p
        L.ssx_cells_per_launch.argtypes = [vp]
        L.ssx_cells_per_launch.restype = ctypes.c_int64
        L.ssx_launch_shape.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.ssx_launch_shape.restype = ctypes.c_int
        L.ssx_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.ssx_batch_pcg_solve.argtypes = [vp, ctypes.POINTER(vp), dp, ctypes.c_int32, c_dbl,
                                          ctypes.c_int32, ctypes.POINTER(vp),
                                          ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32)]
        L.ssx_batch_destroy.argtypes = [vp]
        L.ssx_batch_destroy.restype = None
        P3 = ctypes.POINTER(ssx3_problem)
        L.ssx3_validate.argtypes = [P3, dp, c_dbl]
        L.ssx3_footprint.argtypes = [P3]
        L.ssx3_footprint.restype = ctypes.c_size_t
        L.ssx3_create.argtypes = [P3, dp, c_dbl, vp, ctypes.POINTER(vp)]
        L.ssx3_fwd.argtypes = [vp, vp, vp]
        L.ssx3_adj.argtypes = [vp, vp, vp]
        L.ssx3_penalty.argtypes = [vp, c_int, c_dbl, vp, vp]
        L.ssx3_precond.argtypes = [vp, c_dbl, vp, vp]
        L.ssx3_pcg_solve.argtypes = [vp, vp, c_dbl, ctypes.c_int32, ctypes.c_int32, vp, dp,
                                     ctypes.POINTER(ctypes.c_int32)]
        L.ssx3_destroy.argtypes = [vp]
        L.ssx3_destroy.restype = None
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise SSXError(status, lib().ssx_last_error().decode())


def make_problem(prob, nshots: int, field_dtype: str = "f32") -> ssx_problem:
    fd = DTYPES[field_dtype]
    vd = 0 if fd == 0 else 1
    return ssx_problem(int(prob.nz), int(prob.nx), float(prob.h), float(prob.dt),
                       int(prob.nt), int(prob.order), int(prob.npml), float(prob.pml_R),
                       float(prob.z_src), float(prob.x_src0), int(prob.ns),
                       float(prob.z_rec), float(prob.x_rec0), int(prob.nr),
                       int(prob.slab_dz), int(nshots), fd, vd,
                       int(getattr(prob, "rslab_dz", 0)))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def validate(prob, kappa=None, rho: float = 1000.0, field_dtype: str = "f32",
             nshots: int | None = None) -> None:
    """Host-only validation; raises SSXError."""
    ns = len(prob.xs) if nshots is None else nshots
    P = make_problem(prob, ns, field_dtype)
    k = None
    if kappa is not None:
        k = np.ascontiguousarray(kappa, dtype=np.float64)
    _check(lib().ssx_validate(ctypes.byref(P), _dptr(k) if k is not None else None, rho))


def footprint(prob, field_dtype: str = "f32", nshots: int | None = None) -> int:
    ns = len(prob.xs) if nshots is None else nshots
    P = make_problem(prob, ns, field_dtype)
    return int(lib().ssx_footprint(ctypes.byref(P)))


def dot_static(x, y, nshots: int, out=None, stream=None):
    """Per-shot FP64 inner products <x, y> of device tensors (nshots vectors
    each, float64 or float32) through ssx_dot_static, the entry point that
    allocates no device memory; out: a float64 device tensor [nshots]
    (allocated here when None).  Stream-ordered, no synchronisation."""
    import torch

    for t, name in ((x, "x"), (y, "y")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous device tensor")
    if x.dtype != y.dtype or x.numel() != y.numel() or x.dtype not in (torch.float64,
                                                                        torch.float32):
        raise ValueError("x and y: same float64 / float32 dtype and size")
    if nshots < 1 or x.numel() % nshots:
        raise ValueError("nshots must divide the vector length")
    if out is None:
        out = torch.empty(nshots, dtype=torch.float64, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    vdt = 0 if x.dtype == torch.float64 else 1
    _check(lib().ssx_dot_static(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                x.numel() // nshots, int(nshots), vdt,
                                ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(st.cuda_stream)))
    return out


class Context:
    """An ssx_ctx bound to a torch device stream (the current stream by default)."""

    def __init__(self, prob, kappa, rho, xs=None, field_dtype: str = "f32",
                 stream=None, workspace=None):
        import torch

        self.prob = prob
        xs = tuple(prob.xs) if xs is None else tuple(xs)
        self.nshots = len(xs)
        self.field_dtype = field_dtype
        self.vdtype = torch.float64 if field_dtype == "f64" else torch.float32
        self._P = make_problem(prob, self.nshots, field_dtype)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        k = np.ascontiguousarray(kappa, dtype=np.float64)
        xsa = np.ascontiguousarray(xs, dtype=np.float64)
        ctx = ctypes.c_void_p()
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
        self._workspace = workspace
        if np.ndim(rho) == 0:
            _check(lib().ssx_create(ctypes.byref(self._P), _dptr(k), float(rho), _dptr(xsa),
                                    ctypes.c_void_p(self.stream.cuda_stream), ws_ptr, ws_bytes,
                                    ctypes.byref(ctx)))
        else:
            # density at every node: [nz][nx]
            r = np.ascontiguousarray(rho, dtype=np.float64)
            if r.shape != k.shape:
                raise ValueError("rho must be a scalar or an array shaped like kappa")
            _check(lib().ssx_create_density(ctypes.byref(self._P), _dptr(k), _dptr(r),
                                            _dptr(xsa),
                                            ctypes.c_void_p(self.stream.cuda_stream), ws_ptr,
                                            ws_bytes, ctypes.byref(ctx)))
        self._ctx = ctx

    # -- helpers --------------------------------------------------------------
    def _vec(self, t, n, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != self.vdtype or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: expected contiguous {self.vdtype} with {n} elements, "
                             f"got {t.dtype} {tuple(t.shape)}")
        return ctypes.c_void_p(t.data_ptr())

    @property
    def n_s(self):
        return self.nshots * self.prob.nt * self.prob.ns

    @property
    def n_r(self):
        return self.nshots * self.prob.nt * self.prob.nr

    def empty_s(self):
        import torch
        return torch.empty((self.nshots, self.prob.nt, self.prob.ns), dtype=self.vdtype,
                           device="cuda")

    def empty_r(self):
        import torch
        return torch.empty((self.nshots, self.prob.nt, self.prob.nr), dtype=self.vdtype,
                           device="cuda")

    # -- operators ------------------------------------------------------------
    def fwd(self, h, d):
        _check(lib().ssx_fwd(self._ctx, self._vec(h, self.n_s, "h"), self._vec(d, self.n_r, "d")))
        return d

    def adj(self, r, g):
        _check(lib().ssx_adj(self._ctx, self._vec(r, self.n_r, "r"), self._vec(g, self.n_s, "g")))
        return g

    def slab_fwd(self, f, P, V):
        _check(lib().ssx_slab_fwd(self._ctx, self._vec(f, self.n_s, "f"),
                                  self._vec(P, self.n_s, "P"), self._vec(V, self.n_s, "V")))
        return P, V

    def slab_adj(self, a, b, f):
        _check(lib().ssx_slab_adj(self._ctx, self._vec(a, self.n_s, "a"),
                                  self._vec(b, self.n_s, "b"), self._vec(f, self.n_s, "f")))
        return f

    def penalty(self, op, a, x, y):
        _check(lib().ssx_penalty(self._ctx, int(op), float(a), self._vec(x, self.n_s, "x"),
                                 self._vec(y, self.n_s, "y")))
        return y

    def precond(self, alpha_hat, r, g):
        _check(lib().ssx_precond(self._ctx, float(alpha_hat), self._vec(r, self.n_s, "r"),
                                 self._vec(g, self.n_s, "g")))
        return g

    def normal(self, alpha, p, q, Fp=None):
        fp = self._vec(Fp, self.n_r, "Fp") if Fp is not None else None
        _check(lib().ssx_normal(self._ctx, float(alpha), self._vec(p, self.n_s, "p"),
                                self._vec(q, self.n_s, "q"), fp))
        return q

    def dot(self, x, y):
        n = x.numel() // self.nshots
        out = np.zeros(self.nshots)
        _check(lib().ssx_dot(self._ctx, self._vec(x, x.numel(), "x"),
                             self._vec(y, x.numel(), "y"), n, _dptr(out)))
        return out

    def _pcg(self, fn, d, alpha, maxit, rtol, use_precond, h, raise_on_breakdown):
        if h is None:
            h = self.empty_s()
        hist = np.zeros((self.nshots, maxit + 1, 4))
        it = ctypes.c_int32(0)
        st = fn(self._ctx, self._vec(d, self.n_r, "d"), float(alpha), int(maxit), float(rtol),
                int(bool(use_precond)), self._vec(h, self.n_s, "h"), _dptr(hist),
                ctypes.byref(it))
        if st != 0 and (raise_on_breakdown or st not in (5, 6)):
            _check(st)
        return h, hist[:, : it.value + 1], it.value, st

    def pcg_solve(self, d, alpha_rel, maxit, rtol=0.0, use_precond=True, h=None,
                  raise_on_breakdown=True):
        """Returns (h, hist [nshots][maxit+1][4], iterations, status)."""
        return self._pcg(lib().ssx_pcg_solve, d, alpha_rel, maxit, rtol, use_precond, h,
                         raise_on_breakdown)

    # -- weighted normal equations (context created with rslab_dz != 0) ------
    def weight_d(self, r, y):
        _check(lib().ssx_weight_d(self._ctx, self._vec(r, self.n_r, "r"),
                                  self._vec(y, self.n_r, "y")))
        return y

    def weight_m(self, x, y):
        _check(lib().ssx_weight_m(self._ctx, self._vec(x, self.n_s, "x"),
                                  self._vec(y, self.n_s, "y")))
        return y

    def normal_w(self, alpha, p, q, Fp=None):
        fp = self._vec(Fp, self.n_r, "Fp") if Fp is not None else None
        _check(lib().ssx_normal_w(self._ctx, float(alpha), self._vec(p, self.n_s, "p"),
                                  self._vec(q, self.n_s, "q"), fp))
        return q

    def pcg_solve_w(self, d, alpha, maxit, rtol=0.0, use_precond=True, h=None,
                    raise_on_breakdown=True):
        """Algorithm 1 on the weighted normal equations, alpha per metre.
        Returns (h, hist [nshots][maxit+1][4], iterations, status)."""
        return self._pcg(lib().ssx_pcg_solve_w, d, alpha, maxit, rtol, use_precond, h,
                         raise_on_breakdown)

    # -- V, time-reversal inverse, Lambda~ --------------------------------------
    def fwd_v(self, f, y):
        _check(lib().ssx_fwd_v(self._ctx, self._vec(f, self.n_s, "f"), self._vec(y, self.n_r, "y")))
        return y

    def adj_v(self, r, g):
        _check(lib().ssx_adj_v(self._ctx, self._vec(r, self.n_r, "r"), self._vec(g, self.n_s, "g")))
        return g

    def tr_inverse(self, d, h):
        _check(lib().ssx_tr_inverse(self._ctx, self._vec(d, self.n_r, "d"),
                                    self._vec(h, self.n_s, "h")))
        return h

    def lam(self, side, transpose, x, y):
        """side 0: source-side slab ([nshots][nt][ns]); 1: receiver-side
        slab ([nshots][nt][nr])."""
        n = self.n_s if int(side) == 0 else self.n_r
        _check(lib().ssx_lambda(self._ctx, int(side), int(bool(transpose)), self._vec(x, n, "x"),
                                self._vec(y, n, "y")))
        return y

    def block(self, src, rec, transpose, x, y):
        """src 0 pressure source / 1 normal load on the source line; rec 0
        pressure / 1 normal velocity on the receiver line."""
        nin, nout = (self.n_s, self.n_r) if not transpose else (self.n_r, self.n_s)
        _check(lib().ssx_block(self._ctx, int(src), int(rec), int(bool(transpose)),
                               self._vec(x, nin, "x"), self._vec(y, nout, "y")))
        return y

    def pcg_solve_v(self, d, alpha_rel, maxit, rtol=0.0, f=None, raise_on_breakdown=True):
        """The normal load as the unknown: d [nshots][nt][nr] normal-velocity
        traces.  Returns (f, hist, iterations, status)."""
        if f is None:
            f = self.empty_s()
        hist = np.zeros((self.nshots, maxit + 1, 4))
        it = ctypes.c_int32(0)
        st = lib().ssx_pcg_solve_v(self._ctx, self._vec(d, self.n_r, "d"), float(alpha_rel),
                                   int(maxit), float(rtol), self._vec(f, self.n_s, "f"),
                                   _dptr(hist), ctypes.byref(it))
        if st != 0 and (raise_on_breakdown or st not in (5, 6)):
            _check(st)
        return f, hist[:, : it.value + 1], it.value, st

    def empty_model(self):
        import torch
        return torch.empty((self.nshots, self.prob.nz, self.prob.nx), dtype=self.vdtype,
                           device="cuda")

    def misfit_gradient(self, h, d, g=None):
        """g [nshots][nz][nx] = dJ/dkappa of J = 1/2 ||F h - d||^2 at fixed h
        (physical cells); returns (g, J [nshots])."""
        if g is None:
            g = self.empty_model()
        J = np.zeros(self.nshots)
        _check(lib().ssx_misfit_gradient(self._ctx, self._vec(h, self.n_s, "h"),
                                         self._vec(d, self.n_r, "d"),
                                         self._vec(g, self.nshots * self.prob.nz * self.prob.nx,
                                                   "g"), _dptr(J)))
        return g, J

    def set_option(self, option: int, value: int):
        _check(lib().ssx_set_option(self._ctx, int(option), int(value)))

    def set_graphs(self, enable: bool):
        self.set_option(OPT_GRAPHS, int(bool(enable)))

    def step_kernel_name(self) -> str:
        return lib().ssx_step_kernel_name(self._ctx).decode()

    def cells_per_launch(self) -> int:
        return int(lib().ssx_cells_per_launch(self._ctx))

    def launch_shape(self) -> tuple:
        """(tile height, steps per launch, shots per launch, tile-loop setting)
        of the full-grid step."""
        shape = (ctypes.c_int32 * 4)()
        _check(lib().ssx_launch_shape(self._ctx, shape))
        return tuple(int(v) for v in shape)

    def tile_z(self) -> int:
        return self.launch_shape()[0]

    def close(self):
        if getattr(self, "_ctx", None):
            lib().ssx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several contexts (any grids, records, shots and models; one stencil
    order, field and vector type and stream) solved together with their
    propagations merged (ssx_batch_*): each member's results are bitwise
    those of its own solve.  Holds the contexts; close it before them."""

    def __init__(self, contexts):
        self.contexts = list(contexts)
        n = len(self.contexts)
        arr = (ctypes.c_void_p * n)(*[c._ctx for c in self.contexts])
        out = ctypes.c_void_p()
        _check(lib().ssx_batch_create(n, arr, ctypes.byref(out)))
        self._b = out

    def pcg_solve(self, ds, alpha_rel, maxit, rtol=0.0, use_precond=True, hs=None,
                  raise_on_breakdown=True):
        """Algorithm 1 for every member: ds[i] member i's data; alpha_rel a
        number or one per member.  Returns (hs, hists, iterations, statuses),
        hists[i] [nshots_i][iterations_i + 1][4]; with raise_on_breakdown
        False, a member's breakdown (status 5 or 6) is reported in statuses
        instead of raised."""
        cs = self.contexts
        n = len(cs)
        if len(ds) != n:
            raise ValueError(f"expected {n} data arrays, got {len(ds)}")
        alphas = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha_rel, dtype=np.float64),
                                                      (n,)))
        if hs is None:
            hs = [c.empty_s() for c in cs]
        hists = [np.zeros((c.nshots, maxit + 1, 4)) for c in cs]
        vp = ctypes.c_void_p
        dptrs = (vp * n)(*[c._vec(d, c.n_r, "d") for c, d in zip(cs, ds)])
        hptrs = (vp * n)(*[c._vec(h, c.n_s, "h") for c, h in zip(cs, hs)])
        histp = (ctypes.POINTER(ctypes.c_double) * n)(*[_dptr(x) for x in hists])
        its = (ctypes.c_int32 * n)()
        sts = (ctypes.c_int32 * n)()
        st = lib().ssx_batch_pcg_solve(self._b, dptrs, _dptr(alphas), int(maxit), float(rtol),
                                       int(bool(use_precond)), hptrs, histp, its, sts)
        if st != 0 and (raise_on_breakdown or any(x not in (0, 5, 6) for x in sts)):
            _check(st)
        return hs, [x[:, : its[i] + 1] for i, x in enumerate(hists)], list(its), list(sts)

    def close(self):
        if getattr(self, "_b", None):
            lib().ssx_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# three dimensions (ssx3_*)

def make_problem3(prob, field_dtype: str = "f32") -> ssx3_problem:
    if field_dtype not in ("f64", "f32"):
        raise ValueError("3D fields are f64 or f32")
    return ssx3_problem(int(prob.nz), int(prob.ny), int(prob.nx), float(prob.h),
                        float(prob.dt), int(prob.nt), int(prob.order), int(prob.npml),
                        float(prob.pml_R), float(prob.z_src), float(prob.x_src0),
                        float(prob.y_src0), int(prob.nsx), int(prob.nsy), float(prob.z_rec),
                        float(prob.x_rec0), float(prob.y_rec0), int(prob.nrx), int(prob.nry),
                        DTYPES[field_dtype], int(prob.slab_dz), float(prob.x_s),
                        float(prob.y_s))


def validate3(prob, kappa=None, rho: float = 1000.0, field_dtype: str = "f32") -> None:
    """Host-only validation of a 3D problem (and model); raises SSXError."""
    P = make_problem3(prob, field_dtype)
    k = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    _check(lib().ssx3_validate(ctypes.byref(P), _dptr(k) if k is not None else None, rho))


def footprint3(prob, field_dtype: str = "f32") -> int:
    P = make_problem3(prob, field_dtype)
    return int(lib().ssx3_footprint(ctypes.byref(P)))


class Context3:
    """An ssx3_ctx (3D F and F^T) bound to a torch device stream (the current
    stream by default).  Traces: device tensors [nt][nsy][nsx] (source
    plane) and [nt][nry][nrx] (receiver plane) of float64 for f64 fields,
    float32 for f32."""

    def __init__(self, prob, kappa, rho: float, field_dtype: str = "f32", stream=None):
        import torch

        self.prob = prob
        self.field_dtype = field_dtype
        self.dtype = torch.float64 if field_dtype == "f64" else torch.float32
        self._P = make_problem3(prob, field_dtype)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        k = np.ascontiguousarray(kappa, dtype=np.float64)
        if k.shape != (prob.nz, prob.ny, prob.nx):
            raise ValueError("kappa must be [nz][ny][nx]")
        ctx = ctypes.c_void_p()
        _check(lib().ssx3_create(ctypes.byref(self._P), _dptr(k), float(rho),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx

    def _arg(self, t, shape, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a device tensor")
        if t.dtype != self.dtype or not t.is_contiguous() or t.numel() != int(np.prod(shape)):
            raise ValueError(f"{name}: expected contiguous {self.dtype} of shape {shape}")
        return ctypes.c_void_p(t.data_ptr())

    def empty_src(self):
        import torch
        p = self.prob
        return torch.zeros((p.nt, p.nsy, p.nsx), dtype=self.dtype, device="cuda")

    def empty_rec(self):
        import torch
        p = self.prob
        return torch.zeros((p.nt, p.nry, p.nrx), dtype=self.dtype, device="cuda")

    def fwd(self, h, d):
        p = self.prob
        _check(lib().ssx3_fwd(self._ctx, self._arg(h, (p.nt, p.nsy, p.nsx), "h"),
                              self._arg(d, (p.nt, p.nry, p.nrx), "d")))
        return d

    def adj(self, r, g):
        p = self.prob
        _check(lib().ssx3_adj(self._ctx, self._arg(r, (p.nt, p.nry, p.nrx), "r"),
                              self._arg(g, (p.nt, p.nsy, p.nsx), "g")))
        return g

    def penalty(self, op, a, x, y):
        p = self.prob
        shp = (p.nt, p.nsy, p.nsx)
        _check(lib().ssx3_penalty(self._ctx, int(op), float(a), self._arg(x, shp, "x"),
                                  self._arg(y, shp, "y")))
        return y

    def precond(self, alpha_hat, r, g):
        p = self.prob
        shp = (p.nt, p.nsy, p.nsx)
        _check(lib().ssx3_precond(self._ctx, float(alpha_hat), self._arg(r, shp, "r"),
                                  self._arg(g, shp, "g")))
        return g

    def pcg_solve(self, d, alpha_rel, maxit, use_precond=True, h=None):
        """Algorithm 1 on N h = F^T d; returns (h, history [maxit+1][4],
        iterations)."""
        p = self.prob
        if h is None:
            h = self.empty_src()
        hist = np.zeros((maxit + 1, 4), dtype=np.float64)
        it = ctypes.c_int32(0)
        _check(lib().ssx3_pcg_solve(self._ctx, self._arg(d, (p.nt, p.nry, p.nrx), "d"),
                                    float(alpha_rel), int(maxit), int(bool(use_precond)),
                                    self._arg(h, (p.nt, p.nsy, p.nsx), "h"), _dptr(hist),
                                    ctypes.byref(it)))
        return h, hist[: it.value + 1], it.value

    def close(self):
        if getattr(self, "_ctx", None):
            lib().ssx3_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
