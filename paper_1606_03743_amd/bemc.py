"""Python binding of the C ABI in ``include/bemc.h`` (argument marshalling only).

Every computation runs in the HIP library ``libbemc.so`` built next to this file; torch
provides device memory and the current HIP stream.  There is no CPU fallback: if the
library is missing or no GPU is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbemc.so")

OK = 0
E_INVALID_ARG = -1
E_DEGENERATE_ELEMENT = -2
E_NOT_RECTANGLE = -3
E_NONFINITE = -4
E_NO_GEOMETRY = -5
E_OUT_OF_MEMORY = -6
E_ADMISSION = -7
E_DEVICE = -8
E_LIMIT = -9
W_ON_SURFACE = 1

FP64 = 0
MIXED = 1
MIXED_REFINE = 2  # solver only
_PREC = {"fp64": FP64, "mixed": MIXED, FP64: FP64, MIXED: MIXED}
_SOLVE_PREC = dict(_PREC, refine=MIXED_REFINE)
_SOLVE_PREC[MIXED_REFINE] = MIXED_REFINE

EXPORTED = ["bemc_last_error", "bemc_create", "bemc_destroy", "bemc_set_rules", "bemc_upload_geometry",
            "bemc_upload_densities", "bemc_eval", "bemc_eval_gradient", "bemc_collocation_matvec", "bemc_query_stats",
            "bemc_server_start", "bemc_server_submit", "bemc_server_poll", "bemc_server_wait",
            "bemc_server_stop", "bemc_coulomb_constant", "bemc_rule_size", "bemc_set_near_capacity",
            "bemc_set_dr_rules", "bemc_solve_densities", "bemc_eval_noalloc"]


class BemcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bemc error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("node_interactions", ctypes.c_int64),
                ("near_pairs", ctypes.c_int64), ("leaves", ctypes.c_int64), ("cap_hits", ctypes.c_int64),
                ("on_surface", ctypes.c_int64), ("max_depth", ctypes.c_int64),
                ("near_capacity", ctypes.c_int64), ("far_ms", ctypes.c_double), ("near_ms", ctypes.c_double),
                ("node_interactions_pair_rule", ctypes.c_int64)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("refinements", ctypes.c_int)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_size_t), ("max_batch_points", ctypes.c_int64),
                ("n_streams", ctypes.c_int), ("precision", ctypes.c_int),
                ("small_query_points", ctypes.c_int64)]


class QueryInfo(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int), ("status", ctypes.c_int), ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("end_s", ctypes.c_double), ("batch_id", ctypes.c_int64),
                ("batch_points", ctypes.c_int64)]


_lib = None


def load_library():
    """Load libbemc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python paper_1606_03743_amd/build.py)")
    # One HIP runtime per process: torch ships its own libamdhip64.so.7.  Importing torch
    # first makes the library's libamdhip64.so.7 dependency bind to that same runtime, so
    # torch's device pointers and streams are valid in the library.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, i64, ci = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int
    lib.bemc_last_error.restype = ctypes.c_char_p
    lib.bemc_create.argtypes = [ci, ctypes.POINTER(vp)]
    lib.bemc_destroy.argtypes = [vp]
    lib.bemc_set_rules.argtypes = [vp, ci, ci, ctypes.c_double, ci]
    lib.bemc_upload_geometry.argtypes = [vp, vp, i64, vp, i64, vp]
    lib.bemc_upload_densities.argtypes = [vp, vp, ci, ci, vp]
    lib.bemc_eval.argtypes = [vp, vp, i64, ci, ci, vp, vp, vp]
    lib.bemc_eval_noalloc.argtypes = [vp, vp, i64, ci, ci, vp, vp, vp]
    lib.bemc_eval_gradient.argtypes = [vp, vp, i64, ci, ci, vp, vp]
    lib.bemc_collocation_matvec.argtypes = [vp, vp, ci, ci, vp, vp]
    lib.bemc_query_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.bemc_set_near_capacity.argtypes = [vp, i64, ci]
    lib.bemc_set_dr_rules.argtypes = [vp, ci, vp, vp]
    lib.bemc_solve_densities.argtypes = [vp, vp, vp, ctypes.c_double, ci, ci, ci, ctypes.POINTER(SolveInfo), vp]
    lib.bemc_server_start.argtypes = [vp, ctypes.POINTER(ServerConfig)]
    lib.bemc_server_submit.argtypes = [vp, vp, i64, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.bemc_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(QueryInfo)]
    lib.bemc_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(QueryInfo)]
    lib.bemc_server_stop.argtypes = [vp]
    lib.bemc_coulomb_constant.restype = ctypes.c_double
    lib.bemc_rule_size.argtypes = [ci]
    for name in EXPORTED:
        lib[name]
    _lib = lib
    return lib


def _check(rc, allow_warning=False):
    if rc == OK or (allow_warning and rc == W_ON_SURFACE):
        return rc
    msg = load_library().bemc_last_error().decode(errors="replace")
    raise BemcError(rc, msg)


def _torch():
    import torch

    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(t, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a float64 CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One electrode geometry with its densities, resident on one GPU."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = ctypes.c_void_p()
        _check(self.lib.bemc_create(device, ctypes.byref(h)))
        self.h = h
        self.n_tri = self.n_rect = 0
        self.n_rhs = 0

    # -- lifetime
    def close(self):
        if getattr(self, "h", None):
            self.lib.bemc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- setup
    def set_rules(self, tri_rule=33, rect_rule=7, near_dr=3.0, max_depth=24):
        """rect_rule > 0: Gauss-Legendre rect_rule x rect_rule; < 0: Table B with -rect_rule points."""
        _check(self.lib.bemc_set_rules(self.h, tri_rule, rect_rule, float(near_dr), max_depth))

    def set_dr_rules(self, enable=True, tri_dr=None, rect_dr=None):
        t = None if tri_dr is None else (ctypes.c_double * 3)(*tri_dr)
        r = None if rect_dr is None else (ctypes.c_double * 3)(*rect_dr)
        _check(self.lib.bemc_set_dr_rules(self.h, int(enable), t, r))

    def upload_geometry(self, tri, rect):
        tri = np.ascontiguousarray(np.zeros((0, 9)) if tri is None else tri, dtype=np.float64).reshape(-1, 9)
        rect = np.ascontiguousarray(np.zeros((0, 9)) if rect is None else rect, dtype=np.float64).reshape(-1, 9)
        _check(self.lib.bemc_upload_geometry(self.h, tri.ctypes.data_as(ctypes.c_void_p), tri.shape[0],
                                             rect.ctypes.data_as(ctypes.c_void_p), rect.shape[0], _stream_ptr()))
        self.n_tri, self.n_rect = tri.shape[0], rect.shape[0]
        self.n_rhs = 0

    @property
    def n_elements(self):
        return self.n_tri + self.n_rect

    def upload_densities(self, sigma):
        torch = _torch()
        if isinstance(sigma, torch.Tensor) and sigma.is_cuda:
            s = sigma.reshape(-1, self.n_elements).contiguous()
            _check(self.lib.bemc_upload_densities(self.h, _dev_f64(s), s.shape[0], 1, _stream_ptr()))
            self.n_rhs = s.shape[0]
        else:
            s = np.ascontiguousarray(sigma, dtype=np.float64).reshape(-1, self.n_elements)
            _check(self.lib.bemc_upload_densities(self.h, s.ctypes.data_as(ctypes.c_void_p), s.shape[0], 0,
                                                  _stream_ptr()))
            self.n_rhs = s.shape[0]

    # -- evaluation
    def eval(self, pts, precision="fp64", rhs=0, with_E=True, phi=None, E=None):
        """pts: float64 CUDA tensor [3, n] (SoA).  Returns (phi [n], E [3, n] or None, status of
        the call).  The evaluation is enqueued on the current stream; stats() waits for it and
        reports points on elements (status W_ON_SURFACE)."""
        torch = _torch()
        n = pts.shape[1]
        _dev_f64(pts, (3, n))
        if phi is None:
            phi = torch.empty(n, dtype=torch.float64, device=pts.device)
        if with_E and E is None:
            E = torch.empty((3, n), dtype=torch.float64, device=pts.device)
        rc = self.lib.bemc_eval(self.h, _dev_f64(pts), n, _PREC[precision], rhs, _dev_f64(phi, (n,)),
                                _dev_f64(E, (3, n)) if with_E else None, _stream_ptr())
        _check(rc, allow_warning=True)
        return phi, (E if with_E else None), rc

    def eval_noalloc(self, pts, phi, E=None, precision="fp64", rhs=0):
        """bemc_eval_noalloc: as eval() into caller-provided phi [n] (and E [3, n]); the library
        allocates nothing (n <= 65536).  Returns the status of the call."""
        n = pts.shape[1]
        rc = self.lib.bemc_eval_noalloc(self.h, _dev_f64(pts, (3, n)), n, _PREC[precision], rhs, _dev_f64(phi, (n,)),
                                        None if E is None else _dev_f64(E, (3, n)), _stream_ptr())
        _check(rc, allow_warning=True)
        return rc

    def eval_gradient(self, pts, precision="fp64", rhs=0, G=None):
        """pts: float64 CUDA tensor [3, n].  Returns (G [6, n] rows xx yy zz xy xz yz, status of
        the call); enqueued like eval()."""
        torch = _torch()
        n = pts.shape[1]
        _dev_f64(pts, (3, n))
        if G is None:
            G = torch.empty((6, n), dtype=torch.float64, device=pts.device)
        rc = self.lib.bemc_eval_gradient(self.h, _dev_f64(pts), n, _PREC[precision], rhs, _dev_f64(G, (6, n)),
                                         _stream_ptr())
        _check(rc, allow_warning=True)
        return G, rc

    def collocation(self, sigma, precision="fp64", out=None):
        """sigma: float64 CUDA tensor [n_rhs, n_E]; returns out [n_rhs, n_E]."""
        torch = _torch()
        s = sigma.reshape(-1, self.n_elements)
        if out is None:
            out = torch.empty_like(s)
        _check(self.lib.bemc_collocation_matvec(self.h, _dev_f64(s), s.shape[0], _PREC[precision],
                                                _dev_f64(out, tuple(s.shape)), _stream_ptr()))
        return out

    def set_near_capacity(self, pairs, grow=False):
        """Near-pair list of `pairs` entries; grow=False: fixed (evaluations never wait on the
        host, an overflow is reported by stats()), grow=True: grows to what evaluations need."""
        _check(self.lib.bemc_set_near_capacity(self.h, int(pairs), int(bool(grow))))

    def solve(self, potential, tol=1e-10, max_iter=500, restart=50, precision="fp64", sigma=None):
        """Densities sigma [n_E] (CUDA float64) whose collocation potentials equal `potential` [n_E]."""
        torch = _torch()
        _dev_f64(potential, (self.n_elements,))
        if sigma is None:
            sigma = torch.empty_like(potential)
        info = SolveInfo()
        _check(self.lib.bemc_solve_densities(self.h, _dev_f64(potential), _dev_f64(sigma, (self.n_elements,)),
                                             float(tol), int(max_iter), int(restart), _SOLVE_PREC[precision],
                                             ctypes.byref(info), _stream_ptr()))
        return sigma, {f: getattr(info, f) for f, _ in SolveInfo._fields_}

    def stats(self):
        """Waits for the last evaluation; its counters and "status" (OK or W_ON_SURFACE).
        Raises for an error of an evaluation since the last report (e.g. an overflowing fixed
        near-pair list)."""
        st = Stats()
        rc = _check(self.lib.bemc_query_stats(self.h, ctypes.byref(st)), allow_warning=True)
        out = {f: getattr(st, f) for f, _ in Stats._fields_}
        out["status"] = rc
        return out

    # -- serving
    def server_start(self, mem_budget_bytes=8 << 30, max_batch_points=1 << 17, n_streams=4, precision="mixed",
                     small_query_points=0):
        cfg = ServerConfig(mem_budget_bytes, max_batch_points, n_streams, _PREC[precision], small_query_points)
        _check(self.lib.bemc_server_start(self.h, ctypes.byref(cfg)))

    def server_submit(self, pts_host, phi_host, E_host=None):
        """pts_host [n, 3] float64 C-contiguous numpy (kept alive by the caller until done)."""
        t = ctypes.c_uint64()
        n = pts_host.shape[0]
        _check(self.lib.bemc_server_submit(self.h, pts_host.ctypes.data_as(ctypes.c_void_p), n,
                                           phi_host.ctypes.data_as(ctypes.c_void_p),
                                           None if E_host is None else E_host.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(t)))
        return t.value

    def server_poll(self, ticket):
        info = QueryInfo()
        _check(self.lib.bemc_server_poll(self.h, ticket, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in QueryInfo._fields_}

    def server_wait(self, ticket, timeout_s=-1.0):
        info = QueryInfo()
        _check(self.lib.bemc_server_wait(self.h, ticket, float(timeout_s), ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in QueryInfo._fields_}

    def server_stop(self):
        _check(self.lib.bemc_server_stop(self.h))


def coulomb_constant():
    return load_library().bemc_coulomb_constant()


def rule_size(n):
    return load_library().bemc_rule_size(n)
