"""The oracle's time stepping as plain C loops (oracle engine "c").

TEST INFRASTRUCTURE ONLY -- see the package header.

``forward`` and ``adjoint`` take the same arguments as those of
:mod:`oracle.prop` and return the same arrays; the work is done by
``cprop.c`` (FP64, the same sub-updates in the same order, each stencil sum
accumulated term by term as in the NumPy version, the rows of each
sub-update shared out over OpenMP threads).  It exists because the NumPy
version needs hours for the full-length runs of the 801 x 1601 grid; it is
pinned to the NumPy version (equal to rounding on every operator) and by the
dot-product test in the CPU tests.

The shared library is built by :func:`build` (``gcc -O3 -fopenmp
-ffp-contract=off``) next to the source, on first use if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import fd

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cprop.c")
LIB = os.path.join(HERE, "liboc.so")

_lib = None


class _Line(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int), ("row", ctypes.c_int * 2),
                ("w", ctypes.c_double * 2), ("n", ctypes.c_int),
                ("cols", ctypes.POINTER(ctypes.c_int))]


class _Pml(ctypes.Structure):
    _fields_ = [(name, ctypes.POINTER(ctypes.c_double))
                for name in ("axn", "bxn", "axh", "bxh", "azn", "bzn", "azh", "bzh")]


def build() -> str:
    """Compile cprop.c into liboc.so (always); returns its path."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", SRC,
           "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed building the oracle engine:\n" + res.stderr)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(_Line)
        common = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_double, dp,
                  ctypes.POINTER(_Pml), ctypes.c_int]
        L.oc_forward.argtypes = common + [lp, dp, lp, dp, lp, dp, lp, dp]
        L.oc_forward.restype = ctypes.c_int
        L.oc_adjoint.argtypes = common + [lp, dp, lp, dp, lp, dp, lp, dp]
        L.oc_adjoint.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


class _Ctx:
    """Contiguous FP64 copies of one grid's coefficients, kept alive for a call."""

    def __init__(self, g):
        if getattr(g, "variable_rho", False):
            raise ValueError("the C engine takes constant density only")
        self.keep = []
        self.c = np.ascontiguousarray(fd.stencil(g.order), dtype=np.float64)
        self.Cb = g.dt / (g.rho * g.h)
        self.Ck = np.ascontiguousarray(g.dt * g.kappa / g.h, dtype=np.float64)
        arrs = [np.ascontiguousarray(x, dtype=np.float64)
                for x in (g.ax_n, g.bx_n, g.ax_h, g.bx_h, g.az_n, g.bz_n, g.az_h, g.bz_h)]
        self.keep += arrs
        self.pml = _Pml(*[_dptr(x) for x in arrs])

    def line(self, ln):
        if ln is None:
            return None
        cols = np.ascontiguousarray(ln.cols, dtype=np.int32)
        self.keep.append(cols)
        rows = list(ln.rows)
        r = (ctypes.c_int * 2)(*[rw[0] for rw in rows] + [0] * (2 - len(rows)))
        w = (ctypes.c_double * 2)(*[rw[1] for rw in rows] + [0.0] * (2 - len(rows)))
        s = _Line(len(rows), r, w, len(cols), cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        self.keep.append(s)
        return ctypes.pointer(s)

    def traces(self, a, nt, n):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != (nt, n):
            raise ValueError(f"trace array of shape {a.shape}, expected {(nt, n)}")
        self.keep.append(a)
        return a


def forward(g, nt: int, h_src=None, f_src=None, rec_p=None, rec_v=None):
    """As :func:`oracle.prop.forward` (without the energy and step hooks)."""
    x = _Ctx(g)
    hl = x.line(h_src[0]) if h_src is not None else None
    h = x.traces(h_src[1], nt, len(h_src[0].cols)) if h_src is not None else None
    fl = x.line(f_src[0]) if f_src is not None else None
    f = x.traces(f_src[1], nt, len(f_src[0].cols)) if f_src is not None else None
    P = np.zeros((nt, len(rec_p.cols))) if rec_p is not None else None
    V = np.zeros((nt, len(rec_v.cols))) if rec_v is not None else None
    rc = lib().oc_forward(g.NZ, g.NX, len(x.c), _dptr(x.c), x.Cb, _dptr(x.Ck),
                          ctypes.byref(x.pml), nt, hl, _dptr(h), fl, _dptr(f),
                          x.line(rec_p), _dptr(P), x.line(rec_v), _dptr(V))
    if rc != 0:
        raise MemoryError("oracle engine: out of memory")
    return P, V


def adjoint(g, nt: int, h_line=None, f_line=None, rec_p=None, rec_v=None):
    """As :func:`oracle.prop.adjoint` (without the step hook)."""
    x = _Ctx(g)
    hb = np.zeros((nt, len(h_line.cols))) if h_line is not None else None
    fb = np.zeros((nt, len(f_line.cols))) if f_line is not None else None
    a = x.traces(rec_p[1], nt, len(rec_p[0].cols)) if rec_p is not None else None
    b = x.traces(rec_v[1], nt, len(rec_v[0].cols)) if rec_v is not None else None
    rc = lib().oc_adjoint(g.NZ, g.NX, len(x.c), _dptr(x.c), x.Cb, _dptr(x.Ck),
                          ctypes.byref(x.pml), nt, x.line(h_line), _dptr(hb),
                          x.line(f_line), _dptr(fb),
                          x.line(rec_p[0]) if rec_p is not None else None, _dptr(a),
                          x.line(rec_v[0]) if rec_v is not None else None, _dptr(b))
    if rc != 0:
        raise MemoryError("oracle engine: out of memory")
    return hb, fb
