"""CPU oracle for the AMG-PCG solve phase -- TEST INFRASTRUCTURE ONLY.

A ctypes view of ``libpsc_oracle.so`` (plain FP64 C, see psc_oracle.c).
Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product library never does, and this package imports
nothing from it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

OK, NOCONV, ERR_ARG, ERR_NOT_SPD, ERR_NAN, ERR_OOM, ERR_COARSEN = 0, 1, -1, -2, -3, -5, -6
SMOOTH_L1JACOBI, SMOOTH_AINV, SMOOTH_INVK, SMOOTH_CHEB4 = 0, 1, 2, 3
PREC_VCYCLE, PREC_NONE, PREC_L1JACOBI, PREC_JACOBI, PREC_VCYCLE32 = 0, 1, 2, 3, 4

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def _opt(t):
    """ndpointer that also accepts None."""
    class _P(t):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return t.from_param(obj)
    return _P


_oi32 = _opt(_i32p)
_of64 = _opt(_f64p)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.LIB
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build()
    L = C.CDLL(path)
    vp = C.c_void_p
    L.orc_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
    L.orc_spmv.restype = None
    L.orc_edge_key.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_edge_key.restype = C.c_longlong
    L.orc_match.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p]
    L.orc_match.restype = C.c_int
    L.orc_build.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                            C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int,
                            C.c_double, C.POINTER(vp)]
    L.orc_cheb4_apply.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _f64p, _f64p]
    L.orc_cheb4_apply.restype = None
    L.orc_fai_nnz.argtypes = [vp, C.c_int]
    L.orc_fai_nnz.restype = C.c_longlong
    L.orc_fai_get.argtypes = [vp, C.c_int, _i32p, _i32p, _f64p, _f64p]
    L.orc_fai_get.restype = C.c_int
    L.orc_fai_single.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, C.c_double, C.c_int, C.c_int,
                                 C.POINTER(C.c_int)]
    L.orc_fai_single.restype = vp
    L.orc_fai_single_nnz.argtypes = [vp]
    L.orc_fai_single_nnz.restype = C.c_longlong
    L.orc_fai_single_get.argtypes = [vp, _i32p, _i32p, _f64p, _f64p]
    L.orc_fai_single_get.restype = None
    L.orc_fai_single_free.argtypes = [vp]
    L.orc_fai_single_free.restype = None
    L.orc_prol_nnz.argtypes = [vp, C.c_int]
    L.orc_prol_nnz.restype = C.c_longlong
    L.orc_prol_get.argtypes = [vp, C.c_int, _i32p, _i32p, _f64p, C.POINTER(C.c_double)]
    L.orc_prol_get.restype = C.c_int
    L.orc_coarse_sweeps.argtypes = [vp]
    L.orc_coarse_sweeps.restype = C.c_int
    L.orc_build.restype = C.c_int
    L.orc_free.argtypes = [vp]
    L.orc_free.restype = None
    L.orc_nlevels.argtypes = [vp]
    L.orc_nlevels.restype = C.c_int
    L.orc_level_info.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_longlong), C.POINTER(C.c_int)]
    L.orc_level_info.restype = C.c_int
    L.orc_level_get.argtypes = [vp, C.c_int, _oi32, _oi32, _of64, _oi32, _of64, _of64, _of64]
    L.orc_level_get.restype = C.c_int
    L.orc_coarse_factor.argtypes = [vp, _f64p]
    L.orc_coarse_factor.restype = C.c_int
    L.orc_vcycle.argtypes = [vp, _f64p, _f64p]
    L.orc_vcycle.restype = None
    L.orc_vcycle32.argtypes = [vp, _f64p, _f64p]
    L.orc_vcycle32.restype = None
    L.orc_pcg.argtypes = [vp, C.c_int, _f64p, _f64p, C.c_double, C.c_int,
                          C.POINTER(C.c_int), C.POINTER(C.c_double), _of64]
    L.orc_pcg.restype = C.c_int
    L.orc_fcg.argtypes = [vp, C.c_int, _of64, C.c_int, C.c_int, C.c_int, _f64p, _f64p,
                          C.c_double, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double),
                          C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.orc_fcg.restype = C.c_int
    L.orc_net_param_count.argtypes = []
    L.orc_net_param_count.restype = C.c_int
    L.orc_bf16.argtypes = [C.c_double]
    L.orc_bf16.restype = C.c_double
    L.orc_net_forward.argtypes = [_f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _f64p, _f64p, _of64]
    L.orc_net_forward.restype = None
    L.orc_net_loss_grad.argtypes = [_f64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                    _f64p, _f64p, C.c_int, _of64]
    L.orc_net_loss_grad.restype = C.c_double
    L.orc_adam_step.argtypes = [C.c_int, _f64p, _f64p, _f64p, _f64p, C.c_int,
                                C.c_double, C.c_double, C.c_double, C.c_double]
    L.orc_adam_step.restype = None
    L.orc_net_apply.argtypes = [_f64p, C.c_int, C.c_int, C.c_int, _f64p, _f64p]
    L.orc_net_apply.restype = None
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = None
    L.orc_get_threads.argtypes = []
    L.orc_get_threads.restype = C.c_int
    _lib = L
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(t):
    """Host threads of the oracle's row loops (results do not depend on it)."""
    lib().orc_set_threads(int(t))


def get_threads():
    return lib().orc_get_threads()


def spmv(rowptr, col, val, x):
    rowptr, col, val, x = _i32(rowptr), _i32(col), _f64(val), _f64(x)
    y = np.empty(len(rowptr) - 1)
    lib().orc_spmv(len(rowptr) - 1, rowptr, col, val, x, y)
    return y


def fai_factor(rowptr, col, val, kind, tau=0.1, fill1=0, fill2=1):
    """Stand-alone AINV (kind 1) or INVK (kind 2) of an SPD CSR matrix:
    (zr, zi, zv, d) with Z by columns, A^-1 ~ Z diag(d)^-1 Z^T."""
    rowptr, col, val = _i32(rowptr), _i32(col), _f64(val)
    st = C.c_int()
    S = lib().orc_fai_single(len(rowptr) - 1, rowptr, col, val, kind, tau, fill1, fill2, C.byref(st))
    if not S:
        raise RuntimeError(f"oracle factorisation failed with status {st.value}")
    try:
        n = len(rowptr) - 1
        nnz = lib().orc_fai_single_nnz(S)
        zr, zi, zv, d = np.empty(n + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz), np.empty(n)
        lib().orc_fai_single_get(S, zr, zi, zv, d)
    finally:
        lib().orc_fai_single_free(S)
    return zr, zi, zv, d


def cheb4_apply(rowptr, col, val, nu, b):
    """Degree-nu fourth-kind Chebyshev smoother (l1-Jacobi preconditioned) from x = 0."""
    rowptr, col, val, b = _i32(rowptr), _i32(col), _f64(val), _f64(b)
    x = np.empty(len(b))
    lib().orc_cheb4_apply(len(rowptr) - 1, rowptr, col, val, nu, b, x)
    return x


def edge_key(sij, sii, sjj):
    return lib().orc_edge_key(sij, sii, sjj)


def match(rowptr, col, S):
    rowptr, col, S = _i32(rowptr), _i32(col), _f64(S)
    mate = np.empty(len(rowptr) - 1, dtype=np.int32)
    lib().orc_match(len(rowptr) - 1, rowptr, col, S, mate)
    return mate


class Hierarchy:
    """Oracle AMG hierarchy (C.2 of the readings): levels of (A_l, agg, p, w, minv)."""

    def __init__(self, rowptr, col, val, sweeps=2, coarse_max=200, max_levels=30, coarse_sweeps=30,
                 prol=0, nu=1, nu_double=False, aggr=0, theta=0.01, smoother=SMOOTH_L1JACOBI, ainv_tau=0.1,
                 invk_fill=0, invk_inv_fill=1, coarse_pcg=0, coarse_rtol=1e-4):
        self._rowptr, self._col, self._val = _i32(rowptr), _i32(col), _f64(val)
        h = C.c_void_p()
        st = lib().orc_build(len(rowptr) - 1, self._rowptr, self._col, self._val,
                             sweeps, coarse_max, max_levels, coarse_sweeps, prol, nu, int(nu_double), aggr, theta,
                             smoother, ainv_tau, invk_fill, invk_inv_fill, coarse_pcg, coarse_rtol, C.byref(h))
        self.status = st
        if st != OK:
            raise RuntimeError(f"oracle build failed with status {st}")
        self._h = h
        self.n = len(rowptr) - 1

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    @property
    def nlevels(self):
        return lib().orc_nlevels(self._h)

    def prolongator(self, l):
        """(rowptr, col, val, omega) of the prolongator of level l."""
        n = self.level_info(l)[0]
        nnz = lib().orc_prol_nnz(self._h, l)
        if nnz < 0:
            raise ValueError("no prolongator at the coarsest level")
        rp, ci, v = np.empty(n + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz)
        om = C.c_double()
        lib().orc_prol_get(self._h, l, rp, ci, v, C.byref(om))
        return rp, ci, v, om.value

    def fai(self, l):
        """AINV / INVK factor of level l: (zr, zi, zv, d), Z by columns, or None."""
        nnz = lib().orc_fai_nnz(self._h, l)
        if nnz < 0:
            return None
        n = self.level_info(l)[0]
        zr, zi, zv, d = np.empty(n + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz), np.empty(n)
        lib().orc_fai_get(self._h, l, zr, zi, zv, d)
        return zr, zi, zv, d

    @property
    def coarse_sweeps(self):
        """0 when the coarsest level is factored, else the l1-Jacobi sweep count."""
        return lib().orc_coarse_sweeps(self._h)

    def level_info(self, l):
        n, nnz, nc = C.c_int(), C.c_longlong(), C.c_int()
        lib().orc_level_info(self._h, l, C.byref(n), C.byref(nnz), C.byref(nc))
        return n.value, nnz.value, nc.value

    def sizes(self):
        return [self.level_info(l)[0] for l in range(self.nlevels)]

    def nnzs(self):
        return [self.level_info(l)[1] for l in range(self.nlevels)]

    def operator_complexity(self):
        z = self.nnzs()
        return sum(z) / z[0]

    def level(self, l):
        n, nnz, nc = self.level_info(l)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz)
        w = np.empty(n)
        minv = np.empty(n)
        coarsest = l == self.nlevels - 1
        agg = None if coarsest else np.empty(n, np.int32)
        p = None if coarsest else np.empty(n)
        lib().orc_level_get(self._h, l, rp, ci, v, agg, p, w, minv)
        return dict(n=n, nnz=nnz, nc=nc, rowptr=rp, col=ci, val=v, agg=agg, p=p, w=w, minv=minv)

    def coarse_factor(self):
        n = self.sizes()[-1]
        L = np.empty(n * n)
        lib().orc_coarse_factor(self._h, L)
        return L.reshape(n, n)

    def vcycle(self, b):
        b = _f64(b)
        x = np.empty_like(b)
        lib().orc_vcycle(self._h, b, x)
        return x

    def vcycle32(self, b):
        b = _f64(b)
        x = np.empty_like(b)
        lib().orc_vcycle32(self._h, b, x)
        return x

    def pcg(self, b, x0=None, rtol=1e-6, maxit=1000, prec=PREC_VCYCLE, history=False):
        b = _f64(b)
        x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
        it, rr = C.c_int(), C.c_double()
        hist = np.zeros(2 * maxit) if history else None
        st = lib().orc_pcg(self._h, prec, b, x, rtol, maxit, C.byref(it), C.byref(rr), hist)
        out = dict(status=st, x=x, iters=it.value, relres=rr.value)
        if history:
            out["alpha"] = hist[0:2 * it.value:2]
            out["beta"] = hist[1:2 * it.value:2]
        return out

    def fcg(self, b, x0=None, rtol=1e-6, maxit=1000, form=0, params=None, dims=None, alt_jacobi=False):
        """FCG(1); form 0/1: FP64/FP32 V-cycle. params: the learned form's
        network; alt_jacobi: the same schedule with z = M_0^-1 r in place of
        the network (params unused)."""
        b = _f64(b)
        if alt_jacobi:
            form, params = form | 4, None
        x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
        it, rr, fb, ne = C.c_int(), C.c_double(), C.c_int(), C.c_int()
        nx = ny = nz = 0
        if params is not None:
            nz, ny, nx = dims
            params = _f64(params)
        st = lib().orc_fcg(self._h, form, params, nx, ny, nz, b, x, rtol, maxit,
                           C.byref(it), C.byref(rr), C.byref(fb), C.byref(ne))
        return dict(status=st, x=x, iters=it.value, relres=rr.value, fallbacks=fb.value, net_evals=ne.value)


def net_param_count():
    return lib().orc_net_param_count()


def bf16(x):
    return np.vectorize(lib().orc_bf16)(np.asarray(x, dtype=np.float64))


def net_forward(params, inp, round_bf16=True, keep_act=False):
    """inp: (B, D, H, W) float64 -> out (B, D, H, W)."""
    inp = _f64(inp)
    B, D, H, W = inp.shape
    out = np.empty_like(inp)
    act = np.empty(B * 4 * 16 * D * H * W) if keep_act else None
    lib().orc_net_forward(_f64(params), int(round_bf16), B, D, H, W, inp, out, act)
    if keep_act:
        return out, act.reshape(B, 4, 16, D, H, W)
    return out


def net_loss_grad(params, inp, target, margin, round_bf16=True):
    inp, target = _f64(inp), _f64(target)
    B, D, H, W = inp.shape
    g = np.empty(net_param_count())
    loss = lib().orc_net_loss_grad(_f64(params), int(round_bf16), B, D, H, W, inp, target, margin, g)
    return loss, g


def adam_step(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    p, m, v = _f64(p).copy(), _f64(m).copy(), _f64(v).copy()
    lib().orc_adam_step(len(p), p, m, v, _f64(g), t, lr, b1, b2, eps)
    return p, m, v


def net_apply(params, r, dims):
    nz, ny, nx = dims
    r = _f64(r)
    z = np.empty_like(r)
    lib().orc_net_apply(_f64(params), nx, ny, nz, r, z)
    return z
