"""Thin ctypes binding over the C ABI of libpsc.so (include/psc.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels. Device buffers are torch CUDA tensors (their ``data_ptr()``) and
the HIP stream is torch's current stream, so torch serves as the allocator
and stream provider and nothing else. Importing this module raises if the
library has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsc.so")

OK, NOCONV = 0, 1
ERR_ARG, ERR_NOT_SPD, ERR_NAN, ERR_HIP, ERR_OOM, ERR_COARSEN, ERR_STATE, ERR_IO = -1, -2, -3, -4, -5, -6, -7, -8
FP64, FP32 = 0, 1
TUNE_GRID_MAX, TUNE_FUSED_PCG, TUNE_UNROLL4, TUNE_BUFLOAD, TUNE_SPMV2, TUNE_SPLIT, TUNE_DIA, TUNE_TAIL = 1, 2, 3, 4, 5, 6, 7, 8
TUNE_DIA_UNIFORM, TUNE_XCD, TUNE_MIXED_SPLIT, TUNE_FP64_SPLIT, TUNE_DIA_ALIGN = 9, 10, 11, 12, 13
TUNE_CAPPED, TUNE_PAIR_R, TUNE_MIXED_Z32 = 14, 15, 16
AGGR_MATCHING, AGGR_VBM = 0, 1
SMOOTH_L1JACOBI, SMOOTH_AINV, SMOOTH_INVK, SMOOTH_CHEB4 = 0, 1, 2, 3
MAX_LEVELS = 32
NET_NOALLOC_MAX_CELLS = 262144
NET_TUNE_FUSED = 1
TIMING_KERNELS = 8
TIMING_NAMES = ["spmv_dot", "cg_update", "pre_smooth_l0", "restrict_l0", "post_smooth_l0",
                "dir_update", "vcycle", "other_levels"]

_STATUS = {OK: "PSC_OK", NOCONV: "PSC_NOCONV", ERR_ARG: "PSC_ERR_ARG", ERR_NOT_SPD: "PSC_ERR_NOT_SPD",
           ERR_NAN: "PSC_ERR_NAN", ERR_HIP: "PSC_ERR_HIP", ERR_OOM: "PSC_ERR_OOM",
           ERR_COARSEN: "PSC_ERR_COARSEN", ERR_STATE: "PSC_ERR_STATE", ERR_IO: "PSC_ERR_IO"}


class PscError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class AmgOpts(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
                ("build_fp32", C.c_int32), ("use_graph", C.c_int32), ("host_only", C.c_int32),
                ("coarse_sweeps", C.c_int32), ("smoothed_prol", C.c_int32), ("smoother_sweeps", C.c_int32),
                ("vcycle_double", C.c_int32), ("aggregation", C.c_int32), ("setup_device", C.c_int32),
                ("smoother", C.c_int32), ("invk_fill", C.c_int32), ("invk_inv_fill", C.c_int32),
                ("setup_device_products", C.c_int32), ("vbm_theta", C.c_double), ("ainv_tau", C.c_double),
                ("coarse_pcg_iters", C.c_int32), ("capped_min_rows", C.c_int32), ("coarse_rtol", C.c_double)]


class HierStats(C.Structure):
    _fields_ = [("levels", C.c_int32),
                ("rows", C.c_int64 * MAX_LEVELS), ("nnz", C.c_int64 * MAX_LEVELS),
                ("ell_slots", C.c_int64 * MAX_LEVELS),
                ("operator_complexity", C.c_double), ("vcycle_bytes_fp64", C.c_double),
                ("vcycle_bytes_fp32", C.c_double), ("spmv_bytes_fp64", C.c_double),
                ("setup_seconds", C.c_double), ("device_bytes", C.c_int64),
                ("coarse_sweeps", C.c_int32), ("sp_nnz", C.c_int64 * MAX_LEVELS),
                ("dia_slots", C.c_int64 * MAX_LEVELS), ("p_nnz", C.c_int64 * MAX_LEVELS),
                ("omega", C.c_double * MAX_LEVELS), ("smoother_sweeps", C.c_int32), ("smoothed_prol", C.c_int32),
                ("vcycle_double", C.c_int32), ("aggregation", C.c_int32), ("smoother", C.c_int32),
                ("smoother_nnz", C.c_int64 * MAX_LEVELS), ("rebuild_seconds", C.c_double),
                ("coarse_pcg_iters", C.c_int32), ("tail_level", C.c_int32), ("tail_lds_bytes", C.c_int32),
                ("capped_cap", C.c_int32 * MAX_LEVELS), ("capped_slots", C.c_int64 * MAX_LEVELS),
                ("pair_restrict", C.c_int32 * MAX_LEVELS)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_2406_19754_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
    P = C.POINTER
    sig = {
        "psc_last_error": ([], C.c_char_p),
        "psc_amg_opts_default": ([P(AmgOpts)], None),
        "psc_amg_build": ([i32, vp, vp, vp, P(AmgOpts), vp, P(vp)], C.c_int),
        "psc_amg_rebuild": ([vp, vp], C.c_int),
        "psc_pcg_solve": ([vp, vp, vp, f64, i32, P(i32), P(f64)], C.c_int),
        "psc_fcg_solve": ([vp, vp, i32, vp, vp, f64, i32, P(i32), P(f64), P(i32)], C.c_int),
        "psc_hier_info": ([vp, P(HierStats)], C.c_int),
        "psc_hier_export_level": ([vp, i32, vp, vp, vp, vp, vp, vp], C.c_int),
        "psc_hier_export_prolongator": ([vp, i32, vp, vp, vp], C.c_int),
        "psc_hier_export_smoother": ([vp, i32, vp, vp, vp, vp], C.c_int),
        "psc_vcycle_apply": ([vp, i32, vp, vp], C.c_int),
        "psc_spmv": ([vp, i32, i32, vp, vp], C.c_int),
        "psc_timing_enable": ([vp, i32], C.c_int),
        "psc_timing_get": ([vp, vp, vp], C.c_int),
        "psc_tune": ([vp, i32, i32], C.c_int),
        "psc_hier_free": ([vp], None),
        "psc_net_param_count": ([], i32),
        "psc_net_create": ([vp, vp, P(vp)], C.c_int),
        "psc_net_get_params": ([vp, vp], C.c_int),
        "psc_net_set_params": ([vp, vp], C.c_int),
        "psc_net_apply": ([vp, vp, vp, i32, i32, i32], C.c_int),
        "psc_net_set_grid": ([vp, i32, i32, i32], C.c_int),
        "psc_net_tune": ([vp, i32, i32], C.c_int),
        "psc_net_apply_noalloc": ([vp, vp, vp, i32, i32, i32], C.c_int),
        "psc_net_forward_batch": ([vp, vp, vp, i32, i32], C.c_int),
        "psc_net_loss_grad": ([vp, vp, vp, i32, i32, i32, P(f32), vp], C.c_int),
        "psc_pairs_collect": ([vp, vp, i32, i32, i32, f64, i32, i32, i32, vp, i32, vp, vp, i32, P(i32)], C.c_int),
        "psc_net_train": ([vp, vp, vp, i32, i32, i32, vp, i32, i32, f32, f32, f32, f32, vp], C.c_int),
        "psc_net_save": ([vp, C.c_char_p], C.c_int),
        "psc_net_create_l1jacobi": ([vp, vp, P(vp)], C.c_int),
        "psc_net_load": ([C.c_char_p, vp, P(vp)], C.c_int),
        "psc_net_free": ([vp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    return L


_lib = _load()


def lib():
    return _lib


def _check(st, allow_noconv=False):
    if st == OK or (allow_noconv and st == NOCONV):
        return st
    raise PscError(st, _lib.psc_last_error().decode())


def _stream(stream):
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def _dptr(t, dtype=None, numel=None):
    """Device pointer of a contiguous CUDA tensor (or an int address)."""
    if isinstance(t, int):
        return t
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _hptr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


class Hierarchy:
    """AMG hierarchy handle (psc_amg_build)."""

    def __init__(self, rowptr, col, val, sweeps=2, coarse_max=200, max_levels=30,
                 build_fp32=False, use_graph=True, host_only=False, stream=None, coarse_sweeps=30,
                 smoothed_prol=False, smoother_sweeps=1, vcycle_double=False, aggregation=0, vbm_theta=0.01,
                 setup_device=True, smoother=SMOOTH_L1JACOBI, ainv_tau=0.1, invk_fill=0, invk_inv_fill=1,
                 coarse_pcg_iters=0, coarse_rtol=1e-4, setup_device_products=False, capped_min_rows=None):
        import torch
        o = AmgOpts()
        _lib.psc_amg_opts_default(C.byref(o))
        o.sweeps, o.coarse_max, o.max_levels = sweeps, coarse_max, max_levels
        o.coarse_sweeps = coarse_sweeps
        o.smoothed_prol, o.smoother_sweeps = int(smoothed_prol), smoother_sweeps
        o.vcycle_double = int(vcycle_double)
        o.aggregation, o.vbm_theta = aggregation, vbm_theta
        o.setup_device, o.setup_device_products = int(setup_device), int(setup_device_products)
        o.smoother, o.ainv_tau, o.invk_fill, o.invk_inv_fill = smoother, ainv_tau, invk_fill, invk_inv_fill
        o.coarse_pcg_iters, o.coarse_rtol = coarse_pcg_iters, coarse_rtol
        if capped_min_rows is not None:
            o.capped_min_rows = capped_min_rows
        o.build_fp32, o.use_graph, o.host_only = int(build_fp32), int(use_graph), int(host_only)
        rp, prp = _hptr(rowptr, np.int32)
        ci, pci = _hptr(col, np.int32)
        v, pv = _hptr(val, np.float64)
        self.n = len(rp) - 1
        self._h = C.c_void_p()
        self.stream = 0 if host_only else _stream(stream)
        _check(_lib.psc_amg_build(self.n, prp, pci, pv, C.byref(o), C.c_void_p(self.stream), C.byref(self._h)))
        self._torch = torch

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.psc_hier_free(self._h)
            self._h = None

    __del__ = close

    def info(self):
        s = HierStats()
        _check(_lib.psc_hier_info(self._h, C.byref(s)))
        L = s.levels
        return dict(levels=L, rows=list(s.rows[:L]), nnz=list(s.nnz[:L]), ell_slots=list(s.ell_slots[:L]),
                    operator_complexity=s.operator_complexity, vcycle_bytes_fp64=s.vcycle_bytes_fp64,
                    vcycle_bytes_fp32=s.vcycle_bytes_fp32, spmv_bytes_fp64=s.spmv_bytes_fp64,
                    setup_seconds=s.setup_seconds, device_bytes=s.device_bytes,
                    coarse_sweeps=s.coarse_sweeps, sp_nnz=list(s.sp_nnz[:L]), dia_slots=list(s.dia_slots[:L]),
                    p_nnz=list(s.p_nnz[:L]), omega=list(s.omega[:L]), smoother_sweeps=s.smoother_sweeps,
                    smoothed_prol=s.smoothed_prol, vcycle_double=s.vcycle_double, aggregation=s.aggregation,
                    smoother=s.smoother, smoother_nnz=list(s.smoother_nnz[:L]),
                    rebuild_seconds=s.rebuild_seconds, coarse_pcg_iters=s.coarse_pcg_iters,
                    tail_level=s.tail_level, tail_lds_bytes=s.tail_lds_bytes,
                    capped_cap=list(s.capped_cap[:L]), capped_slots=list(s.capped_slots[:L]),
                    pair_restrict=list(s.pair_restrict[:L]))

    def rebuild(self, val):
        """Numeric-only rebuild with new values of A (same pattern as at build)."""
        v, pv = _hptr(val, np.float64)
        _check(_lib.psc_amg_rebuild(self._h, pv))

    def export_level(self, l):
        inf = self.info()
        n, nnz = inf["rows"][l], inf["nnz"][l]
        coarsest = l == inf["levels"] - 1
        agg = None if coarsest else np.empty(n, np.int32)
        p = None if coarsest else np.empty(n)
        minv = np.empty(n)
        rp = np.empty(n + 1, np.int32)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz)
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        _check(_lib.psc_hier_export_level(self._h, l, ptr(agg), ptr(p), ptr(minv), ptr(rp), ptr(ci), ptr(v)))
        return dict(n=n, nnz=nnz, agg=agg, p=p, minv=minv, rowptr=rp, col=ci, val=v)

    def export_prolongator(self, l):
        """(rowptr, col, val) of the prolongator P_l the V-cycle uses."""
        inf = self.info()
        n, nnz = inf["rows"][l], inf["p_nnz"][l]
        rp, ci, v = np.empty(n + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz)
        _check(_lib.psc_hier_export_prolongator(self._h, l, rp.ctypes.data_as(C.c_void_p),
                                                ci.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p)))
        return rp, ci, v

    def export_smoother(self, l):
        """(colptr, row, val, d): the AINV / INVK factor Z_l by columns and its pivots."""
        inf = self.info()
        n, nnz = inf["rows"][l], inf["smoother_nnz"][l]
        zr, zi, zv, d = np.empty(n + 1, np.int64), np.empty(nnz, np.int32), np.empty(nnz), np.empty(n)
        ptr = lambda a: a.ctypes.data_as(C.c_void_p)
        _check(_lib.psc_hier_export_smoother(self._h, l, ptr(zr), ptr(zi), ptr(zv), ptr(d)))
        return zr, zi, zv, d

    def pcg(self, b, x, rtol=1e-6, maxit=1000):
        it, rr = C.c_int32(), C.c_double()
        f64 = self._torch.float64
        st = _lib.psc_pcg_solve(self._h, _dptr(b, f64, self.n), _dptr(x, f64, self.n), rtol, maxit,
                                C.byref(it), C.byref(rr))
        _check(st, allow_noconv=True)
        return dict(status=st, iters=it.value, relres=rr.value)

    def fcg(self, b, x, rtol=1e-6, maxit=1000, prec=FP64, net=None):
        it, rr, fb = C.c_int32(), C.c_double(), C.c_int32()
        f64 = self._torch.float64
        st = _lib.psc_fcg_solve(self._h, None if net is None else net._h, prec,
                                _dptr(b, f64, self.n), _dptr(x, f64, self.n), rtol, maxit,
                                C.byref(it), C.byref(rr), C.byref(fb))
        _check(st, allow_noconv=True)
        return dict(status=st, iters=it.value, relres=rr.value, fallbacks=fb.value)

    def vcycle(self, r, z, prec=FP64):
        f64 = self._torch.float64
        _check(_lib.psc_vcycle_apply(self._h, prec, _dptr(r, f64, self.n), _dptr(z, f64, self.n)))

    def spmv(self, x, y, level=0, prec=FP64):
        _check(_lib.psc_spmv(self._h, level, prec, _dptr(x), _dptr(y)))

    def timing(self, on=True):
        _check(_lib.psc_timing_enable(self._h, int(on)))

    def timing_get(self):
        cnt = np.zeros(TIMING_KERNELS, np.int64)
        ms = np.zeros(TIMING_KERNELS)
        _check(_lib.psc_timing_get(self._h, cnt.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p)))
        return {TIMING_NAMES[k]: (int(cnt[k]), float(ms[k])) for k in range(TIMING_KERNELS)}

    def tune(self, key, value):
        _check(_lib.psc_tune(self._h, key, value))


def net_param_count():
    return int(_lib.psc_net_param_count())


class Net:
    """Learned convolutional preconditioner handle (psc_net_create)."""

    def __init__(self, params, stream=None):
        import torch
        self._torch = torch
        self._h = C.c_void_p()
        if params is None:      # filled by load()
            return
        p, pp = _hptr(params, np.float32)
        if p.size != net_param_count():
            raise ValueError(f"expected {net_param_count()} parameters")
        _check(_lib.psc_net_create(pp, C.c_void_p(_stream(stream)), C.byref(self._h)))

    @classmethod
    def l1jacobi(cls, hier, stream=None):
        """psc_net_create_l1jacobi: the learned schedule's comparison arm,
        z = M_0^-1 r in place of the network."""
        net = cls(None)
        _check(_lib.psc_net_create_l1jacobi(hier._h, C.c_void_p(_stream(stream)), C.byref(net._h)))
        return net

    @classmethod
    def load(cls, path, stream=None):
        """psc_net_load: a new network from a checkpoint written by save()."""
        net = cls(None)
        _check(_lib.psc_net_load(os.fsencode(path), C.c_void_p(_stream(stream)), C.byref(net._h)))
        return net

    def save(self, path):
        """psc_net_save: master weights and Adam state to `path`."""
        _check(_lib.psc_net_save(self._h, os.fsencode(path)))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.psc_net_free(self._h)
            self._h = None

    __del__ = close

    def params(self):
        out = np.empty(net_param_count(), np.float32)
        _check(_lib.psc_net_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, params):
        p, pp = _hptr(params, np.float32)
        _check(_lib.psc_net_set_params(self._h, pp))

    def set_grid(self, dims):
        nz, ny, nx = dims
        _check(_lib.psc_net_set_grid(self._h, nx, ny, nz))

    def tune(self, key, value):
        """psc_net_tune (NET_TUNE_FUSED: fused 3-layer inference kernel or one
        kernel per layer)."""
        _check(_lib.psc_net_tune(self._h, key, value))

    def apply(self, r, z, dims):
        nz, ny, nx = dims
        f64 = self._torch.float64
        _check(_lib.psc_net_apply(self._h, _dptr(r, f64), _dptr(z, f64), nx, ny, nz))

    def apply_noalloc(self, r, z, dims):
        """psc_net_apply_noalloc: the same result without device allocation
        (grids up to NET_NOALLOC_MAX_CELLS cells)."""
        nz, ny, nx = dims
        f64 = self._torch.float64
        _check(_lib.psc_net_apply_noalloc(self._h, _dptr(r, f64), _dptr(z, f64), nx, ny, nz))

    def forward_batch(self, inp, out):
        B, D = inp.shape[0], inp.shape[1]
        f32 = self._torch.float32
        _check(_lib.psc_net_forward_batch(self._h, _dptr(inp, f32), _dptr(out, f32), B, D))

    def loss_grad(self, inp, target, margin):
        B, D = inp.shape[0], inp.shape[1]
        f32 = self._torch.float32
        loss = C.c_float()
        g = np.empty(net_param_count(), np.float32)
        _check(_lib.psc_net_loss_grad(self._h, _dptr(inp, f32), _dptr(target, f32), B, D, margin,
                                      C.byref(loss), g.ctypes.data_as(C.c_void_p)))
        return float(loss.value), g

    def train(self, r_crops, z_crops, order, steps, batch, margin, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8):
        f32 = self._torch.float32
        ncrops, crop = r_crops.shape[0], r_crops.shape[1]
        o, po = _hptr(order, np.int32)
        if o.size < steps * batch or o.min() < 0 or o.max() >= ncrops:
            raise ValueError("order must hold steps*batch crop indices in range")
        losses = np.empty(steps, np.float32)
        _check(_lib.psc_net_train(self._h, _dptr(r_crops, f32), _dptr(z_crops, f32), ncrops, crop, margin,
                                  po, steps, batch, lr, beta1, beta2, eps,
                                  losses.ctypes.data_as(C.c_void_p)))
        return losses


def pairs_collect(h, b, dims, crop, crops_per_iter, origins, r_out, z_out, count=0, rtol=1e-6, maxit=200):
    import torch
    nz, ny, nx = dims
    o, po = _hptr(origins, np.int32)
    cnt = C.c_int32(count)
    _check(_lib.psc_pairs_collect(h._h, _dptr(b, torch.float64), nx, ny, nz, rtol, maxit, crop,
                                  crops_per_iter, po, o.size // 3, _dptr(r_out, torch.float32),
                                  _dptr(z_out, torch.float32), r_out.shape[0], C.byref(cnt)))
    return cnt.value
