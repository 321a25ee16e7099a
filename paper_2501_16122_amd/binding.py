"""Thin ctypes binding of libmapmaker (the C ABI in include/mapmaker.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every computation runs in the library's HIP kernels.
There is no fallback: if the shared library is missing, importing the
functions below raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmapmaker.so")

MM_OK, MM_NOTCONVERGED = 0, 1
MM_EINVAL, MM_ENOSPC, MM_EHIP, MM_EBREAKDOWN = -1, -2, -3, -4
MM_F64, MM_F32 = 0, 1
MM_STOKES_I, MM_STOKES_QU, MM_STOKES_IQU = 1, 2, 3

_c = ctypes
_vp = _c.c_void_p
_i32, _i64, _f64, _sz = _c.c_int32, _c.c_int64, _c.c_double, _c.c_size_t
_pi32 = _c.POINTER(_c.c_int32)
_pi64 = _c.POINTER(_c.c_int64)
_pf64 = _c.POINTER(_c.c_double)
_psz = _c.POINTER(_c.c_size_t)


class SolveOpts(_c.Structure):
    _fields_ = [("tol", _f64), ("max_iter", _i32), ("fixed_iter", _i32), ("check_every", _i32),
                ("mixed", _i32), ("max_outer", _i32), ("inner_tol", _f64), ("timing", _i32),
                ("autotune", _i32), ("op_variant", _i32), ("graph", _i32), ("x0", _vp), ("bj_start", _i32)]


class TuneEntry(_c.Structure):
    _fields_ = [("device", _i32), ("log2_samples", _i32), ("dtype", _i32), ("arith", _i32), ("n_rhs", _i32),
                ("ncomp", _i32), ("lambda_", _i32), ("noise_kind", _i32), ("op_variant", _i32)]


class SolveInfo(_c.Structure):
    _fields_ = [("iters", _i32), ("outer_iters", _i32), ("converged", _i32), ("breakdown", _i32),
                ("rel_resid", _f64), ("true_rel_resid", _f64), ("op_ms", _f64), ("op_launches", _i32),
                ("op_variant", _i32), ("iter_ms_p50", _f64), ("iter_ms_p99", _f64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes); every symbol include/mapmaker.h declares
SIGNATURES = {
    "mm_last_error": (_c.c_char_p, []),
    "mm_abi_version": (_c.c_int, []),
    "mm_pointing_workspace_size": (_c.c_int, [_i64, _i32, _i32, _i32, _psz]),
    "mm_pointing_build": (_c.c_int, [_vp, _vp, _i32, _i64, _pi64, _i32, _pf64, _i32, _i32, _f64, _vp, _sz, _vp,
                                     _c.POINTER(_vp)]),
    "mm_pointing_build_stokes": (_c.c_int, [_vp, _vp, _i32, _i64, _pi64, _i32, _pf64, _i32, _i32, _i32, _f64, _vp,
                                            _sz, _vp, _c.POINTER(_vp)]),
    "mm_pointing_stokes": (_c.c_int, [_vp, _pi32]),
    "mm_pointing_info": (_c.c_int, [_vp, _pi32, _pi64, _pi32, _pi32, _pi32]),
    "mm_pointing_export": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mm_pointing_attach_weights": (_c.c_int, [_vp, _vp, _vp]),
    "mm_pointing_destroy": (_c.c_int, [_vp]),
    "mm_noise_white_workspace_size": (_c.c_int, [_i32, _psz]),
    "mm_noise_white": (_c.c_int, [_pf64, _i32, _vp, _sz, _vp, _c.POINTER(_vp)]),
    "mm_noise_toeplitz_workspace_size": (_c.c_int, [_i32, _i32, _pi64, _i64, _psz]),
    "mm_noise_toeplitz": (_c.c_int, [_pf64, _i32, _i32, _pi64, _pi32, _i64, _vp, _sz, _vp, _c.POINTER(_vp)]),
    "mm_noise_circulant": (_c.c_int, [_pf64, _i32, _i32, _pi64, _pi32, _i64, _vp, _sz, _vp, _c.POINTER(_vp)]),
    "mm_noise_templates_workspace_size": (_c.c_int, [_i32, _i64, _psz]),
    "mm_noise_templates": (_c.c_int, [_pf64, _i32, _pi64, _pi32, _i32, _i64, _vp, _sz, _vp, _c.POINTER(_vp)]),
    "mm_noise_destroy": (_c.c_int, [_vp]),
    "mm_apply_P": (_c.c_int, [_vp, _vp, _vp, _i32, _vp]),
    "mm_apply_PT": (_c.c_int, [_vp, _vp, _vp, _i32, _vp]),
    "mm_apply_Ninv": (_c.c_int, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "mm_apply_A": (_c.c_int, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "mm_apply_A_variant": (_c.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _vp]),
    "mm_rhs": (_c.c_int, [_vp, _vp, _vp, _vp, _i32, _vp]),
    "mm_apply_A_multi": (_c.c_int, [_vp, _vp, _i32, _vp, _vp, _i32, _vp]),
    "mm_apply_M": (_c.c_int, [_vp, _vp, _vp, _vp]),
    "mm_expand_map": (_c.c_int, [_vp, _vp, _vp, _vp]),
    "mm_solve_opts_default": (_c.c_int, [_c.POINTER(SolveOpts)]),
    "mm_solve_workspace_size": (_c.c_int, [_vp, _vp, _c.POINTER(SolveOpts), _psz]),
    "mm_solve": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.POINTER(SolveOpts), _c.POINTER(SolveInfo), _pf64, _i32,
                            _vp, _sz, _vp]),
    "mm_solve_noalloc": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.POINTER(SolveOpts), _c.POINTER(SolveInfo), _vp]),
    "mm_solver_workspace_bound": (_c.c_int, [_i32, _i32, _i32, _c.POINTER(SolveOpts), _psz]),
    "mm_solver_workspace_size": (_c.c_int, [_vp, _vp, _i32, _c.POINTER(SolveOpts), _psz]),
    "mm_solver_create": (_c.c_int, [_vp, _vp, _i32, _vp, _c.POINTER(SolveOpts), _vp, _sz, _vp, _c.POINTER(_vp)]),
    "mm_solver_step": (_c.c_int, [_vp, _i32]),
    "mm_solver_poll": (_c.c_int, [_vp, _pi32, _pi32, _c.POINTER(SolveInfo)]),
    "mm_solver_finish": (_c.c_int, [_vp, _vp, _vp, _c.POINTER(SolveInfo), _pf64, _i32]),
    "mm_solver_snapshot_size": (_c.c_int, [_vp, _psz]),
    "mm_solver_snapshot": (_c.c_int, [_vp, _vp, _sz]),
    "mm_solver_restore": (_c.c_int, [_vp, _vp, _sz]),
    "mm_solver_destroy": (_c.c_int, [_vp]),
    "mm_batch_step": (_c.c_int, [_c.POINTER(_vp), _i32, _i32]),
    "mm_tune_cache_get": (_c.c_int, [_c.POINTER(TuneEntry), _i32, _pi32]),
    "mm_tune_cache_put": (_c.c_int, [_c.POINTER(TuneEntry), _i32]),
}

# A JSON file of the autotuner's choices: read when the library is loaded
# and written when the process exits, if this variable names one.
TUNE_CACHE_ENV = "MM_TUNE_CACHE"

_lib = None


def load(path: str = LIB_PATH):
    """Load libmapmaker.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2501_16122_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    cache = os.environ.get(TUNE_CACHE_ENV)
    if cache:
        import atexit
        if os.path.exists(cache):
            try:
                tune_cache_load(cache)
            except (OSError, ValueError, KeyError, TypeError, MapMakerError) as e:
                # a broken file costs only the cached choices (the tuner times again)
                import warnings
                warnings.warn(f"{TUNE_CACHE_ENV}={cache}: not loaded ({e})")
        atexit.register(tune_cache_save, cache)
    return lib


class MapMakerError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmapmaker error {code}: {msg}")
        self.code = code


def _check(rc, allow=(MM_OK,)):
    if rc in allow:
        return rc
    msg = load().mm_last_error()
    raise MapMakerError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return MM_F64
    if t.dtype == torch.float32:
        return MM_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev_check(t, dtype=None, numel=None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def _arith(a) -> int:
    if a in ("f64", MM_F64, None):
        return MM_F64
    if a in ("f32", MM_F32):
        return MM_F32
    raise ValueError(f"bad arith {a!r}")


STOKES = {"IQU": MM_STOKES_IQU, "QU": MM_STOKES_QU, "I": MM_STOKES_I}


class Pointing:
    """Handle over the precomputed pointing (hits, masks, nc x nc inverse
    blocks) for one map form: ``stokes`` "IQU" (3 values per pixel), "QU" (2)
    or "I" (1; ``psi`` may then be None, with ``tod_dtype`` giving the
    timeline dtype).  ``min_hits`` defaults to nc.

    Borrows ``pix`` and ``psi`` (device tensors) for its lifetime and owns a
    device workspace tensor."""

    def __init__(self, pix, psi, det_offsets, det_weight, n_pix, min_hits=None, cond_max=1e3, stream=None,
                 stokes="IQU", tod_dtype=None):
        torch = _torch()
        lib = load()
        if stokes not in STOKES:
            raise ValueError(f"stokes must be one of {sorted(STOKES)}")
        self.stokes, self.ncomp = stokes, STOKES[stokes]
        if min_hits is None:
            min_hits = self.ncomp
        _dev_check(pix, torch.int32, name="pix")
        n = pix.numel()
        if psi is None:
            if stokes != "I":
                raise ValueError("psi is needed unless stokes='I'")
            if tod_dtype is None:
                raise ValueError("give tod_dtype when psi is None")
            self.tod_dtype = tod_dtype
        else:
            _dev_check(psi, name="psi")
            if psi.numel() != n:
                raise ValueError("pix and psi differ in length")
            self.tod_dtype = psi.dtype
        self.dtype = MM_F64 if self.tod_dtype == torch.float64 else MM_F32
        if self.tod_dtype not in (torch.float64, torch.float32):
            raise TypeError(f"unsupported dtype {self.tod_dtype}")
        offs = np.ascontiguousarray(det_offsets, dtype=np.int64)
        w = np.ascontiguousarray(det_weight, dtype=np.float64)
        n_det = offs.size - 1
        sz = _c.c_size_t()
        _check(lib.mm_pointing_workspace_size(n, n_det, int(n_pix), self.dtype, _c.byref(sz)))
        self.workspace = torch.empty(max(1, sz.value), dtype=torch.uint8, device=pix.device)
        h = _vp()
        _check(lib.mm_pointing_build_stokes(_ptr(pix), _ptr(psi), self.dtype, n, offs.ctypes.data_as(_pi64), n_det,
                                            w.ctypes.data_as(_pf64), int(n_pix), self.ncomp, int(min_hits),
                                            float(cond_max), _ptr(self.workspace), sz.value, _stream(stream),
                                            _c.byref(h)))
        self.handle = h
        self._keep = (pix, psi)
        self.n_samples, self.n_pix, self.n_det = n, int(n_pix), n_det
        nk = _c.c_int32()
        _check(lib.mm_pointing_info(h, _c.byref(nk), None, None, None, None))
        self.n_kept = nk.value
        self.device = pix.device
        self.weights = None

    def export(self, stream=None):
        torch = _torch()
        dev = self.device
        hits = torch.empty(self.n_pix, dtype=torch.int32, device=dev)
        mask = torch.empty(self.n_pix, dtype=torch.uint8, device=dev)
        compact = torch.empty(self.n_pix, dtype=torch.int32, device=dev)
        kept = torch.empty(max(1, self.n_kept), dtype=torch.int32, device=dev)
        nc = self.ncomp
        minv = torch.empty(max(1, nc * nc * self.n_kept), dtype=torch.float64, device=dev)
        _check(load().mm_pointing_export(self.handle, _ptr(hits), _ptr(mask), _ptr(compact), _ptr(kept), _ptr(minv),
                                         _stream(stream)))
        return {"hits": hits, "mask": mask, "compact": compact, "kept": kept[:self.n_kept],
                "minv": minv[:nc * nc * self.n_kept].view(-1, nc, nc)}

    def attach_weights(self, stream=None):
        """Precompute the pointing weight u = tan(psi) of every sample into a
        device tensor the handle keeps; the band-Toeplitz and template
        operators then stream it and rebuild (cos 2psi, sin 2psi) from it.
        The intensity-only form reads no angle: nothing to attach (None)."""
        torch = _torch()
        if self.ncomp == 1:
            self.weights = None
            return None
        self.weights = torch.empty(max(1, self.n_samples), dtype=self.tod_dtype, device=self.device)
        _check(load().mm_pointing_attach_weights(self.handle, _ptr(self.weights), _stream(stream)))
        return self.weights

    def detach_weights(self):
        _check(load().mm_pointing_attach_weights(self.handle, None, None))
        self.weights = None

    def close(self):
        if getattr(self, "handle", None):
            load().mm_pointing_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Noise:
    """N^-1 (or a general weight W): white, band-Toeplitz or circulant per chunk, or
    white with polynomial templates marginalised per interval."""

    def __init__(self, handle, workspace, kind):
        self.handle, self.workspace, self.kind = handle, workspace, kind

    @classmethod
    def white(cls, det_weight, device, stream=None):
        torch = _torch()
        lib = load()
        w = np.ascontiguousarray(det_weight, dtype=np.float64)
        sz = _c.c_size_t()
        _check(lib.mm_noise_white_workspace_size(w.size, _c.byref(sz)))
        ws = torch.empty(sz.value, dtype=torch.uint8, device=device)
        h = _vp()
        _check(lib.mm_noise_white(w.ctypes.data_as(_pf64), w.size, _ptr(ws), sz.value, _stream(stream), _c.byref(h)))
        return cls(h, ws, "white")

    @classmethod
    def toeplitz(cls, coeff, chunk_offsets, device, chunk_filter=None, stream=None, circulant=False):
        """Band-Toeplitz N^-1 per chunk (circulant=True: the same band filter
        on each chunk taken as periodic)."""
        torch = _torch()
        lib = load()
        c = np.ascontiguousarray(np.atleast_2d(coeff), dtype=np.float64)
        offs = np.ascontiguousarray(chunk_offsets, dtype=np.int64)
        n_chunks = offs.size - 1
        filt = None
        if chunk_filter is not None:
            filt = np.ascontiguousarray(chunk_filter, dtype=np.int32)
        sz = _c.c_size_t()
        _check(lib.mm_noise_toeplitz_workspace_size(c.shape[1], c.shape[0], offs.ctypes.data_as(_pi64), n_chunks,
                                                    _c.byref(sz)))
        ws = torch.empty(sz.value, dtype=torch.uint8, device=device)
        h = _vp()
        make = lib.mm_noise_circulant if circulant else lib.mm_noise_toeplitz
        _check(make(c.ctypes.data_as(_pf64), c.shape[1], c.shape[0], offs.ctypes.data_as(_pi64),
                    None if filt is None else filt.ctypes.data_as(_pi32), n_chunks, _ptr(ws), sz.value,
                    _stream(stream), _c.byref(h)))
        return cls(h, ws, "circulant" if circulant else "toeplitz")

    @classmethod
    def circulant(cls, coeff, chunk_offsets, device, chunk_filter=None, stream=None):
        return cls.toeplitz(coeff, chunk_offsets, device, chunk_filter, stream, circulant=True)

    @classmethod
    def templates(cls, det_weight, interval_offsets, order, device, orders=None, stream=None):
        """White weights with polynomial baselines of degree < order (or
        orders[i] per interval) marginalised on each interval; the intervals
        partition the timeline."""
        torch = _torch()
        lib = load()
        w = np.ascontiguousarray(det_weight, dtype=np.float64)
        offs = np.ascontiguousarray(interval_offsets, dtype=np.int64)
        n = offs.size - 1
        o = None if orders is None else np.ascontiguousarray(orders, dtype=np.int32)
        sz = _c.c_size_t()
        _check(lib.mm_noise_templates_workspace_size(w.size, n, _c.byref(sz)))
        ws = torch.empty(max(1, sz.value), dtype=torch.uint8, device=device)
        h = _vp()
        _check(lib.mm_noise_templates(w.ctypes.data_as(_pf64), w.size, offs.ctypes.data_as(_pi64),
                                      None if o is None else o.ctypes.data_as(_pi32), int(order), n, _ptr(ws),
                                      sz.value, _stream(stream), _c.byref(h)))
        return cls(h, ws, "templates")

    def close(self):
        if getattr(self, "handle", None):
            load().mm_noise_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _vec(pt: Pointing, x, name):
    torch = _torch()
    _dev_check(x, torch.float64, pt.ncomp * pt.n_kept, name)


def _tod(pt: Pointing, t, name):
    _dev_check(t, pt.tod_dtype, pt.n_samples, name)


def apply_P(pt: Pointing, x, tod=None, arith="f64", stream=None):
    torch = _torch()
    _vec(pt, x, "x")
    if tod is None:
        tod = torch.empty(pt.n_samples, dtype=pt.tod_dtype, device=pt.device)
    _tod(pt, tod, "tod")
    _check(load().mm_apply_P(pt.handle, _ptr(x), _ptr(tod), _arith(arith), _stream(stream)))
    return tod


def apply_PT(pt: Pointing, tod, q=None, arith="f64", stream=None):
    torch = _torch()
    _tod(pt, tod, "tod")
    if q is None:
        q = torch.empty(pt.ncomp * pt.n_kept, dtype=torch.float64, device=pt.device)
    _vec(pt, q, "q")
    _check(load().mm_apply_PT(pt.handle, _ptr(tod), _ptr(q), _arith(arith), _stream(stream)))
    return q


def apply_Ninv(nz: Noise, pt: Pointing, tod_in, tod_out=None, arith="f64", stream=None):
    torch = _torch()
    _tod(pt, tod_in, "tod_in")
    if tod_out is None:
        tod_out = torch.empty_like(tod_in)
    _tod(pt, tod_out, "tod_out")
    _check(load().mm_apply_Ninv(nz.handle, pt.handle, _ptr(tod_in), _ptr(tod_out), _arith(arith), _stream(stream)))
    return tod_out


def apply_A(pt: Pointing, nz: Noise, x, q=None, arith="f64", stream=None, variant=None):
    """q = P^T N^-1 P x; ``variant`` selects a band-Toeplitz operator variant
    (the bits of the solve option op_variant), None = the default."""
    torch = _torch()
    _vec(pt, x, "x")
    if q is None:
        q = torch.empty(pt.ncomp * pt.n_kept, dtype=torch.float64, device=pt.device)
    _vec(pt, q, "q")
    if variant is None:
        _check(load().mm_apply_A(pt.handle, nz.handle, _ptr(x), _ptr(q), _arith(arith), _stream(stream)))
    else:
        _check(load().mm_apply_A_variant(pt.handle, nz.handle, _ptr(x), _ptr(q), _arith(arith), int(variant),
                                         _stream(stream)))
    return q


def rhs(pt: Pointing, nz: Noise, tod, b=None, arith="f64", stream=None):
    torch = _torch()
    _tod(pt, tod, "tod")
    if b is None:
        b = torch.empty(pt.ncomp * pt.n_kept, dtype=torch.float64, device=pt.device)
    _vec(pt, b, "b")
    _check(load().mm_rhs(pt.handle, nz.handle, _ptr(tod), _ptr(b), _arith(arith), _stream(stream)))
    return b


def apply_A_multi(pt: Pointing, nz: Noise, x, q=None, arith="f64", stream=None):
    """Q = A X for X of shape (n_rhs, nc n_kept) in one launch."""
    torch = _torch()
    n_rhs = x.shape[0]
    _dev_check(x, torch.float64, n_rhs * pt.ncomp * pt.n_kept, "x")
    if q is None:
        q = torch.empty_like(x)
    _dev_check(q, torch.float64, n_rhs * pt.ncomp * pt.n_kept, "q")
    _check(load().mm_apply_A_multi(pt.handle, nz.handle, n_rhs, _ptr(x), _ptr(q), _arith(arith), _stream(stream)))
    return q


def apply_M(pt: Pointing, r, z=None, stream=None):
    torch = _torch()
    _vec(pt, r, "r")
    if z is None:
        z = torch.empty_like(r)
    _vec(pt, z, "z")
    _check(load().mm_apply_M(pt.handle, _ptr(r), _ptr(z), _stream(stream)))
    return z


def expand_map(pt: Pointing, x, out=None, stream=None):
    torch = _torch()
    _vec(pt, x, "x")
    if out is None:
        out = torch.empty(pt.ncomp * pt.n_pix, dtype=torch.float64, device=pt.device)
    _dev_check(out, torch.float64, pt.ncomp * pt.n_pix, "map")
    _check(load().mm_expand_map(pt.handle, _ptr(x), _ptr(out), _stream(stream)))
    return out


def solve_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    _check(load().mm_solve_opts_default(_c.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Solver:
    """Reusable solve workspace for one (pointing, noise) pair."""

    def __init__(self, pt: Pointing, nz: Noise, **opts):
        torch = _torch()
        self.pt, self.nz = pt, nz
        self.opts = solve_opts(**opts)
        sz = _c.c_size_t()
        _check(load().mm_solve_workspace_size(pt.handle, nz.handle, _c.byref(self.opts), _c.byref(sz)))
        self.workspace = torch.empty(max(1, sz.value), dtype=torch.uint8, device=pt.device)
        self.hist_len = max(self.opts.max_iter, self.opts.fixed_iter, self.opts.max_outer) + 1

    def solve(self, tod, map_out=None, x_out=None, stream=None, history=False, x0=None):
        """x0: optional start vector (f64[nc * n_kept] device tensor)."""
        torch = _torch()
        pt = self.pt
        _tod(pt, tod, "tod")
        if x0 is not None:
            _vec(pt, x0, "x0")
        self.opts.x0 = None if x0 is None else x0.data_ptr()
        if map_out is None:
            map_out = torch.empty(pt.ncomp * pt.n_pix, dtype=torch.float64, device=pt.device)
        if x_out is None:
            x_out = torch.empty(max(1, pt.ncomp * pt.n_kept), dtype=torch.float64, device=pt.device)
        info = SolveInfo()
        hist = np.zeros(self.hist_len) if history else None
        rc = load().mm_solve(pt.handle, self.nz.handle, _ptr(tod), _ptr(map_out), _ptr(x_out),
                             _c.byref(self.opts), _c.byref(info),
                             None if hist is None else hist.ctypes.data_as(_pf64),
                             0 if hist is None else hist.size, _ptr(self.workspace), self.workspace.numel(),
                             _stream(stream))
        _check(rc, allow=(MM_OK, MM_NOTCONVERGED))
        out = {"map": map_out, "x": x_out[:pt.ncomp * pt.n_kept], "info": info.as_dict(), "status": rc}
        if hist is not None:
            n = (info.iters + 1) if not self.opts.mixed else info.outer_iters + 1
            out["history"] = hist[:n]
        return out


def batch_step(solvers, k=8):
    """Advance several AsyncSolvers (same stream, dtype and precision mode,
    at most 16 right-hand sides in all) by up to k iterations in shared
    launches; poll and finish each one as usual."""
    arr = (_vp * len(solvers))(*[sv.handle for sv in solvers])
    _check(load().mm_batch_step(arr, len(solvers), int(k)))


_TUNE_KEYS = ("device", "log2_samples", "dtype", "arith", "n_rhs", "ncomp", "lambda", "noise_kind", "op_variant")


def tune_cache_get() -> list:
    """The autotuner's cached choices, one dict per problem class."""
    lib = load()
    n = _c.c_int32()
    _check(lib.mm_tune_cache_get(None, 0, _c.byref(n)))
    arr = (TuneEntry * max(n.value, 1))()
    _check(lib.mm_tune_cache_get(arr, n.value, _c.byref(n)))
    return [{k: getattr(e, "lambda_" if k == "lambda" else k) for k in _TUNE_KEYS} for e in arr[:n.value]]


def tune_cache_put(entries) -> None:
    """Add choices (dicts with the keys of tune_cache_get); a cached class
    takes the new choice."""
    entries = list(entries)
    arr = (TuneEntry * max(len(entries), 1))()
    for e, d in zip(arr, entries):
        for k in _TUNE_KEYS:
            setattr(e, "lambda_" if k == "lambda" else k, int(d[k]))
    _check(load().mm_tune_cache_put(arr, len(entries)))


def tune_cache_save(path: str) -> None:
    """Write the cached choices to a JSON file (atomically replaced)."""
    import json
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump({"keys": list(_TUNE_KEYS), "entries": tune_cache_get()}, f, indent=1)
    os.replace(tmp, path)


def tune_cache_load(path: str) -> None:
    """Add the choices of a JSON file written by tune_cache_save."""
    import json
    with open(path) as f:
        tune_cache_put(json.load(f)["entries"])


class AsyncSolver:
    """A resumable solve of n_rhs timelines (tod: (n_rhs, n_samples), or one
    timeline) sharing ``pt`` and ``nz``; advanced by ``step`` on its own
    stream, polled without blocking, finished by ``finish``."""

    def __init__(self, pt: Pointing, nz: Noise, tod, stream=None, x0=None, **opts):
        torch = _torch()
        lib = load()
        self.pt, self.nz = pt, nz
        self.n_rhs = 1 if tod.dim() == 1 else tod.shape[0]
        _dev_check(tod, pt.tod_dtype, self.n_rhs * pt.n_samples, "tod")
        self.opts = solve_opts(**opts)
        if x0 is not None:  # start vector(s), read on the solver's stream at creation
            _dev_check(x0, torch.float64, self.n_rhs * pt.ncomp * pt.n_kept, "x0")
            self.opts.x0 = x0.data_ptr()
        self._x0 = x0
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        sz = _c.c_size_t()
        _check(lib.mm_solver_workspace_size(pt.handle, nz.handle, self.n_rhs, _c.byref(self.opts), _c.byref(sz)))
        self.workspace_bytes = sz.value
        self.workspace = torch.empty(max(1, sz.value), dtype=torch.uint8, device=pt.device)
        self._tod = tod
        h = _vp()
        _check(lib.mm_solver_create(pt.handle, nz.handle, self.n_rhs, _ptr(tod), _c.byref(self.opts),
                                    _ptr(self.workspace), sz.value, self.stream.cuda_stream, _c.byref(h)))
        self.handle = h
        self.done = False

    def step(self, k=None):
        _check(load().mm_solver_step(self.handle, int(self.opts.check_every if k is None else k)))

    def poll(self, with_info=False):
        """(done, in_flight[, infos]) without blocking."""
        done = _c.c_int32()
        flight = _c.c_int32()
        infos = (SolveInfo * self.n_rhs)() if with_info else None
        _check(load().mm_solver_poll(self.handle, _c.byref(done), _c.byref(flight), infos))
        self.done = bool(done.value)
        if with_info:
            return self.done, bool(flight.value), [i.as_dict() for i in infos]
        return self.done, bool(flight.value)

    def finish(self, history=False):
        torch = _torch()
        pt = self.pt
        maps = torch.empty((self.n_rhs, pt.ncomp * pt.n_pix), dtype=torch.float64, device=pt.device)
        xs = torch.empty((self.n_rhs, max(1, pt.ncomp * pt.n_kept)), dtype=torch.float64, device=pt.device)
        infos = (SolveInfo * self.n_rhs)()
        hl = max(self.opts.max_iter, self.opts.fixed_iter, self.opts.max_outer) + 1
        hist = np.zeros(hl) if history else None
        rc = load().mm_solver_finish(self.handle, _ptr(maps), _ptr(xs), infos,
                                     None if hist is None else hist.ctypes.data_as(_pf64), 0 if hist is None else hl)
        _check(rc, allow=(MM_OK, MM_NOTCONVERGED))
        out = {"maps": maps, "x": xs[:, :pt.ncomp * pt.n_kept], "info": [i.as_dict() for i in infos], "status": rc}
        if hist is not None:
            i0 = out["info"][0]
            out["history"] = hist[: (i0["outer_iters"] + 1 if self.opts.mixed else i0["iters"] + 1)]
        return out

    def snapshot(self, device=None):
        """The solve's state after the last step, as a uint8 tensor (host
        memory unless a device is given); blocks until the stream is idle."""
        torch = _torch()
        sz = _c.c_size_t()
        _check(load().mm_solver_snapshot_size(self.handle, _c.byref(sz)))
        buf = torch.empty(sz.value, dtype=torch.uint8, device=device if device is not None else "cpu")
        _check(load().mm_solver_snapshot(self.handle, _ptr(buf), sz.value))
        return buf

    def restore(self, buf):
        """Continue from a snapshot of a solve of the same problem."""
        _check(load().mm_solver_restore(self.handle, _ptr(buf), buf.numel()))
        self.done = False

    def close(self):
        if getattr(self, "handle", None):
            load().mm_solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
