"""Plain FP64 CPU oracle (test infrastructure only).

Python view of ``oracle/oracle.c``: the slow, obviously-correct reference that the
GPU library is checked against.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package; the product
library never does.  It shares no code with the GPU path.

What it computes (arXiv:1606.03743): the potential and field of constant-density
triangles and rectangles at field points, each element replaced by the point
charges of a Gaussian cubature rule (Sec. 4, Eq. 4.1; rules of App. A and B or a
tensor Gauss-Legendre rule), with recursive subdivision below distance ratio 3
and exact polar integration for points lying on an element.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-std=gnu11", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("tri_rule", ctypes.c_int), ("rect_gl_n", ctypes.c_int),
                ("rect_table_n", ctypes.c_int), ("near_dr", ctypes.c_double),
                ("max_depth", ctypes.c_int), ("dr_rules", ctypes.c_int),
                ("tri_dr", ctypes.c_double * 3), ("rect_dr", ctypes.c_double * 3)]


class _Stats(ctypes.Structure):
    _fields_ = [("near_pairs", ctypes.c_int64), ("leaves", ctypes.c_int64),
                ("cap_hits", ctypes.c_int64), ("on_surface", ctypes.c_int64),
                ("max_depth", ctypes.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.orc_coulomb_constant.restype = ctypes.c_double
        lib.orc_tri_rule.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_rect_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        lib.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        lib.orc_eval.argtypes = [dp, i64, dp, i64, dp, ctypes.POINTER(_Params), dp, i64, dp, dp,
                                 dp, dp, ctypes.POINTER(_Stats), ctypes.c_int]
        lib.orc_eval_gradient.argtypes = [dp, i64, dp, i64, dp, ctypes.POINTER(_Params), dp, i64, dp, dp, dp,
                                          ctypes.POINTER(_Stats), ctypes.c_int]
        lib.orc_collocation.argtypes = [dp, i64, dp, i64, dp, ctypes.c_int, ctypes.POINTER(_Params),
                                        ctypes.POINTER(ctypes.c_int64), i64, dp, dp,
                                        ctypes.POINTER(_Stats), ctypes.c_int]
        lib.orc_element.argtypes = [ctypes.c_int, dp, dp, ctypes.POINTER(_Params), ctypes.c_int, dp,
                                    ctypes.POINTER(_Stats)]
        lib.orc_element_geometry.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape_last=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape_last is not None:
        a = a.reshape(-1, shape_last)
    return a


# distance-ratio limits of the rule levels (triangles 7/12/19 points, rectangles Tables
# B2/B3/B4): the paper's potential limits for triangles scaled by 1.25 for the field,
# rectangle limits from the same field-error criterion
TRI_DR = (100.0, 25.0, 10.0)
RECT_DR = (150.0, 40.0, 15.0)


def params(tri_rule=33, rect_gl_n=7, rect_table_n=0, near_dr=3.0, max_depth=24, dr_rules=False,
           tri_dr=TRI_DR, rect_dr=RECT_DR):
    return _Params(tri_rule, rect_gl_n, rect_table_n, near_dr, max_depth, int(dr_rules),
                   (ctypes.c_double * 3)(*tri_dr), (ctypes.c_double * 3)(*rect_dr))


def coulomb_constant() -> float:
    return _load().orc_coulomb_constant()


def tri_rule(n):
    lam = np.zeros((64, 3)); w = np.zeros(64)
    k = _load().orc_tri_rule(n, _ptr(lam), _ptr(w))
    if k < 0:
        raise ValueError(f"unknown triangle rule {n}")
    return lam[:k].copy(), w[:k].copy()


def rect_rule(gl_n=0, table_n=0):
    xy = np.zeros((256, 2)); w = np.zeros(256)
    k = _load().orc_rect_rule(gl_n, table_n, _ptr(xy), _ptr(w))
    if k < 0:
        raise ValueError(f"unknown rectangle rule gl_n={gl_n} table_n={table_n}")
    return xy[:k].copy(), w[:k].copy()


def gauss_legendre(n):
    x = np.zeros(n); w = np.zeros(n)
    if _load().orc_gauss_legendre(n, _ptr(x), _ptr(w)) < 0:
        raise ValueError(n)
    return x, w


def _stats_dict(st):
    return {f: int(getattr(st, f)) for f, _ in _Stats._fields_}


def evaluate(tri, rect, sigma, pts, prm=None, nthreads=0, with_abs=False):
    """phi[n], E[n,3] (+ abs sums and stats) at points pts[n,3]."""
    lib = _load()
    prm = prm or params()
    tri = _f64(tri if tri is not None else np.zeros((0, 9)), 9)
    rect = _f64(rect if rect is not None else np.zeros((0, 9)), 9)
    sigma = _f64(sigma).ravel()
    pts = _f64(pts, 3)
    n = pts.shape[0]
    if sigma.size != tri.shape[0] + rect.shape[0]:
        raise ValueError("sigma length must equal the element count")
    phi = np.zeros(n); E = np.zeros((n, 3)); aphi = np.zeros(n); aE = np.zeros(n)
    st = _Stats()
    rc = lib.orc_eval(_ptr(tri), tri.shape[0], _ptr(rect), rect.shape[0], _ptr(sigma), ctypes.byref(prm),
                      _ptr(pts), n, _ptr(phi), _ptr(E), _ptr(aphi), _ptr(aE), ctypes.byref(st), nthreads)
    if rc < 0:
        raise ValueError(f"orc_eval failed ({rc})")
    out = {"phi": phi, "E": E, "stats": _stats_dict(st), "threads": rc}
    if with_abs:
        out["abs_phi"] = aphi
        out["abs_E"] = aE
    return out


def gradient(tri, rect, sigma, pts, prm=None, nthreads=0):
    """G[n, 6] = dE_i/dx_j as (xx, yy, zz, xy, xz, yz); abs_G[n] (per-element scale) and
    abs_T[n] (per-term scale: the rounding scale of the sum); stats."""
    lib = _load()
    prm = prm or params()
    tri = _f64(tri if tri is not None else np.zeros((0, 9)), 9)
    rect = _f64(rect if rect is not None else np.zeros((0, 9)), 9)
    sigma = _f64(sigma).ravel()
    pts = _f64(pts, 3)
    n = pts.shape[0]
    if sigma.size != tri.shape[0] + rect.shape[0]:
        raise ValueError("sigma length must equal the element count")
    G = np.zeros((n, 6)); aG = np.zeros(n); aT = np.zeros(n)
    st = _Stats()
    rc = lib.orc_eval_gradient(_ptr(tri), tri.shape[0], _ptr(rect), rect.shape[0], _ptr(sigma),
                               ctypes.byref(prm), _ptr(pts), n, _ptr(G), _ptr(aG), _ptr(aT), ctypes.byref(st),
                               nthreads)
    if rc < 0:
        raise ValueError(f"orc_eval_gradient failed ({rc})")
    return {"G": G, "abs_G": aG, "abs_T": aT, "stats": _stats_dict(st), "threads": rc}


def gradient_matrix(g6):
    """[..., 6] (xx, yy, zz, xy, xz, yz) -> symmetric [..., 3, 3]."""
    g6 = np.asarray(g6)
    m = np.empty(g6.shape[:-1] + (3, 3))
    m[..., 0, 0], m[..., 1, 1], m[..., 2, 2] = g6[..., 0], g6[..., 1], g6[..., 2]
    m[..., 0, 1] = m[..., 1, 0] = g6[..., 3]
    m[..., 0, 2] = m[..., 2, 0] = g6[..., 4]
    m[..., 1, 2] = m[..., 2, 1] = g6[..., 5]
    return m


def collocation(tri, rect, sigma, rows=None, prm=None, nthreads=0):
    """out[n_rhs, n_rows]: potential at element centroids (rows) from densities sigma[n_rhs, n_E];
    abs[n_rhs, n_rows]: K sum_j |sigma_rj phi_j| per right-hand side (error normaliser)."""
    lib = _load()
    prm = prm or params()
    tri = _f64(tri if tri is not None else np.zeros((0, 9)), 9)
    rect = _f64(rect if rect is not None else np.zeros((0, 9)), 9)
    ne = tri.shape[0] + rect.shape[0]
    sigma = _f64(sigma).reshape(-1, ne)
    nrhs = sigma.shape[0]
    rows = np.arange(ne, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((nrhs, rows.size)); aout = np.zeros((nrhs, rows.size))
    st = _Stats()
    rc = lib.orc_collocation(_ptr(tri), tri.shape[0], _ptr(rect), rect.shape[0], _ptr(sigma), nrhs,
                             ctypes.byref(prm), rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             rows.size, _ptr(out), _ptr(aout), ctypes.byref(st), nthreads)
    if rc < 0:
        raise ValueError(f"orc_collocation failed ({rc})")
    return {"out": out, "abs": aout, "stats": _stats_dict(st), "threads": rc}


def element(kind, geom, P, prm=None, mode=1, grad=False):
    """(phi, Ex, Ey, Ez[, gradient xx yy zz xy xz yz]) of one element with unit density and
    no Coulomb constant."""
    lib = _load()
    prm = prm or params()
    g = _f64(geom).ravel(); P = _f64(P).ravel(); out = np.zeros(10 if grad else 4)
    mode = mode | (2 if grad else 0)
    st = _Stats()
    rc = lib.orc_element(kind, _ptr(g), _ptr(P), ctypes.byref(prm), mode, _ptr(out), ctypes.byref(st))
    if rc < 0:
        raise ValueError(f"orc_element failed ({rc})")
    return out, _stats_dict(st)


def element_geometry(kind, geom):
    lib = _load()
    g = _f64(geom).ravel(); c = np.zeros(3); a = np.zeros(1); L = np.zeros(1)
    rc = lib.orc_element_geometry(kind, _ptr(g), _ptr(c), _ptr(a), _ptr(L))
    if rc < 0:
        raise ValueError(f"invalid element ({rc})")
    return c, float(a[0]), float(L[0])
