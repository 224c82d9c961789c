"""Python binding of libwd (include/wd.h): conjugate gradient for the
Wilson-Dirac operator on AMD MI355X (gfx950), arXiv 2111.14958.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libwd.so.  Fields are PyTorch tensors on the GPU (complex128 in the
canonical layouts of wd.h, or uint8 buffers in the packed layouts); streams are
PyTorch's current stream.  If libwd.so has not been built the import of the
binding fails with an error saying so -- there is no fallback.

The C functions are exposed with their C names (lib().wd_dslash, ...) and through
thin helpers with the same names minus the prefix.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwd.so")

F64, F32, F16N = 0, 1, 2
METHOD_CGNE, METHOD_BICGSTAB = 0, 1
PRECOND_NONE, PRECOND_EO = 0, 1
PACKED = 1
STREAM_READ, STREAM_COPY, STREAM_WRITE = 0, 1, 2
GAUGE_RECON12 = 1 << 8   # wd_gauge_create: also keep a two-row (reconstruct-12) FP32 copy
GAUGE_F64, GAUGE_F32, GAUGE_F16 = 1, 2, 4

WD_OK, WD_EINVAL, WD_ENODEV, WD_EHIP, WD_ENOMEM = 0, -1, -2, -3, -4
WD_ENOTCONV, WD_EBREAKDOWN, WD_ETOOBIG, WD_ENOTFOUND = -5, -6, -7, -8

# every symbol declared in include/wd.h
EXPORTS = [
    "wd_version", "wd_strerror", "wd_last_error_detail", "wd_device_info",
    "wd_gauge_create", "wd_gauge_destroy", "wd_gauge_info",
    "wd_spinor_bytes", "wd_pack_spinor", "wd_unpack_spinor",
    "wd_dslash", "wd_dslash_dag", "wd_dslash_noalloc",
    "wd_coo_create", "wd_coo_destroy", "wd_coo_info", "wd_coo_export", "wd_coo_spmv",
    "wd_cg_default_params", "wd_cg_workspace_bytes", "wd_cg_solve", "wd_cg_solve_batch",
    "wd_tune_dslash", "wd_tune_lookup", "wd_tune_cg", "wd_shape_set", "wd_shape_get",
    "wd_profile_enable", "wd_profile_reset", "wd_profile_read", "wd_cg_graph_stats", "wd_stream",
    "wd_serve_footprint", "wd_serve_create", "wd_serve_submit", "wd_serve_poll",
    "wd_serve_stats_get", "wd_serve_destroy",
]


class WDError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        l = lib()
        msg = l.wd_strerror(code).decode()
        detail = l.wd_last_error_detail().decode()
        super().__init__(f"{where}: {msg} ({code})" + (f": {detail}" if detail else ""))


class CGParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("reliable_every", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("use_x0", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("method", ctypes.c_int32),
                ("precondition", ctypes.c_int32), ("max_cus", ctypes.c_int32)]


class CGReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("true_rel_res", ctypes.c_double), ("iter_rel_res", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_ if f[0] != "reserved"}


class TuneResult(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("rhs_per_thread", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("hop_order", ctypes.c_int32),
                ("rhs_loop", ctypes.c_int32), ("site_order", ctypes.c_int32),
                ("us", ctypes.c_double), ("gbps", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes_total", ctypes.c_double)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("arena_dev", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("device", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("t_sign", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("m0", ctypes.c_double),
                ("gauge_dev", ctypes.c_void_p), ("src_dev", ctypes.c_void_p),
                ("sol_dev", ctypes.c_void_p), ("params", CGParams)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("arena_high_water", ctypes.c_uint64), ("active", ctypes.c_int32),
                ("pending", ctypes.c_int32), ("arena_capacity", ctypes.c_uint64)]


_lib = None


def lib():
    """The loaded libwd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2111_14958_amd.build` (there is no fallback)")
        l = ctypes.CDLL(LIB_PATH)
        P, I32, U32, D, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                              ctypes.c_double, ctypes.c_size_t)
        sig = {
            "wd_version": ([], ctypes.c_int),
            "wd_strerror": ([ctypes.c_int], ctypes.c_char_p),
            "wd_last_error_detail": ([], ctypes.c_char_p),
            "wd_device_info": ([ctypes.c_int, ctypes.c_char_p, SZ, ctypes.POINTER(I32)], ctypes.c_int),
            "wd_gauge_create": ([ctypes.POINTER(I32), I32, P, U32, P, ctypes.POINTER(P)], ctypes.c_int),
            "wd_gauge_destroy": ([P], ctypes.c_int),
            "wd_gauge_info": ([P, ctypes.POINTER(I32), ctypes.POINTER(I32),
                               ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(U32)], ctypes.c_int),
            "wd_spinor_bytes": ([P, I32, I32], SZ),
            "wd_pack_spinor": ([P, I32, P, P, I32, P], ctypes.c_int),
            "wd_unpack_spinor": ([P, I32, P, P, I32, P], ctypes.c_int),
            "wd_dslash": ([P, D, I32, P, P, I32, U32, P], ctypes.c_int),
            "wd_dslash_dag": ([P, D, I32, P, P, I32, U32, P], ctypes.c_int),
            "wd_dslash_noalloc": ([P, D, I32, I32, P, P, I32, P], ctypes.c_int),
            "wd_coo_create": ([P, D, I32, I32, P, ctypes.POINTER(P)], ctypes.c_int),
            "wd_coo_destroy": ([P], ctypes.c_int),
            "wd_coo_info": ([P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(SZ)], ctypes.c_int),
            "wd_coo_export": ([P, P, P, P, P], ctypes.c_int),
            "wd_coo_spmv": ([P, P, P, I32, P], ctypes.c_int),
            "wd_cg_default_params": ([ctypes.POINTER(CGParams)], None),
            "wd_cg_workspace_bytes": ([P, I32, ctypes.POINTER(CGParams)], SZ),
            "wd_cg_solve": ([P, D, P, P, ctypes.POINTER(CGParams), P, SZ,
                             ctypes.POINTER(CGReport), P], ctypes.c_int),
            "wd_cg_solve_batch": ([P, D, P, P, I32, ctypes.POINTER(CGParams), P, SZ,
                                   ctypes.POINTER(CGReport), P], ctypes.c_int),
            "wd_tune_dslash": ([P, I32, I32, I32, ctypes.POINTER(TuneResult), P], ctypes.c_int),
            "wd_tune_cg": ([P, D, I32, P, I32, I32, ctypes.POINTER(TuneResult), P], ctypes.c_int),
            "wd_tune_lookup": ([P, I32, I32, I32, ctypes.POINTER(TuneResult)], ctypes.c_int),
            "wd_shape_set": ([P, I32, I32, I32, I32, ctypes.POINTER(TuneResult)], ctypes.c_int),
            "wd_shape_get": ([P, I32, I32, I32, I32, ctypes.POINTER(TuneResult)], ctypes.c_int),
            "wd_profile_enable": ([I32], ctypes.c_int),
            "wd_profile_reset": ([], ctypes.c_int),
            "wd_profile_read": ([ctypes.POINTER(KernelStat), I32, ctypes.POINTER(I32)], ctypes.c_int),
            "wd_cg_graph_stats": ([ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(I32)], ctypes.c_int),
            "wd_stream": ([I32, P, P, SZ, P], ctypes.c_int),
            "wd_serve_footprint": ([ctypes.POINTER(Request)], SZ),
            "wd_serve_create": ([ctypes.POINTER(ServeConfig), ctypes.POINTER(P)], ctypes.c_int),
            "wd_serve_submit": ([P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
            "wd_serve_poll": ([P, ctypes.c_uint64, ctypes.POINTER(CGReport), ctypes.POINTER(I32)], ctypes.c_int),
            "wd_serve_stats_get": ([P, ctypes.POINTER(ServeStats)], ctypes.c_int),
            "wd_serve_destroy": ([P], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def _check(rc: int, where: str):
    if rc != WD_OK:
        raise WDError(rc, where)


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _require_cuda(t, dtype=None, name="tensor"):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t


def version() -> int:
    return lib().wd_version()


def device_info(device: int = 0):
    arch = ctypes.create_string_buffer(64)
    ncu = ctypes.c_int32(0)
    rc = lib().wd_device_info(device, arch, 64, ctypes.byref(ncu))
    _check(rc, "wd_device_info")
    return arch.value.decode(), ncu.value


class Gauge:
    """Device-resident packed links (wd_gauge).  U: complex128 GPU tensor
    [Lt, Lz, Ly, Lx, 4, 3, 3]; dims = (Lx, Ly, Lz, Lt)."""

    def __init__(self, U, dims, t_sign: int = -1, precs=(F64, F32, F16N), recon12: bool = False):
        torch = _torch()
        _require_cuda(U, torch.complex128, "U")
        self.dims = tuple(int(d) for d in dims)
        self.t_sign = int(t_sign)
        self.sites = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        if U.numel() != self.sites * 36:
            raise ValueError("U does not match dims")
        mask = GAUGE_RECON12 if recon12 else 0
        for p in precs:
            mask |= 1 << p
        d = (ctypes.c_int32 * 4)(*self.dims)
        h = ctypes.c_void_p()
        _check(lib().wd_gauge_create(d, self.t_sign, _ptr(U), mask, _stream(), ctypes.byref(h)),
               "wd_gauge_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().wd_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def spinor_bytes(self, prec: int, nrhs: int) -> int:
        return int(lib().wd_spinor_bytes(self.handle, prec, nrhs))


def empty_packed(g: Gauge, prec: int, nrhs: int):
    torch = _torch()
    return torch.empty(g.spinor_bytes(prec, nrhs), dtype=torch.uint8, device="cuda")


def pack_spinor(g: Gauge, psi, prec: int, out=None):
    """canonical complex128 [nrhs, ..., 4, 3] -> packed uint8 buffer."""
    torch = _torch()
    _require_cuda(psi, torch.complex128, "psi")
    nrhs = psi.numel() // (g.sites * 12)
    out = empty_packed(g, prec, nrhs) if out is None else out
    _check(lib().wd_pack_spinor(g.handle, prec, _ptr(psi), _ptr(out), nrhs, _stream()),
           "wd_pack_spinor")
    return out


def unpack_spinor(g: Gauge, buf, prec: int, nrhs: int, out=None):
    torch = _torch()
    lt, lz, ly, lx = g.dims[3], g.dims[2], g.dims[1], g.dims[0]
    if out is None:
        out = torch.empty((nrhs, lt, lz, ly, lx, 4, 3), dtype=torch.complex128, device="cuda")
    _check(lib().wd_unpack_spinor(g.handle, prec, _ptr(buf), _ptr(out), nrhs, _stream()),
           "wd_unpack_spinor")
    return out


def dslash(g: Gauge, m0: float, psi, prec: int = F64, dagger: bool = False,
           packed: bool = False, nrhs: int | None = None, out=None):
    """out = D psi (or D^dagger psi).  Canonical complex128 unless packed=True,
    in which case psi/out are packed buffers and nrhs must be given."""
    torch = _torch()
    if packed:
        if nrhs is None:
            raise ValueError("nrhs is required for packed buffers")
        out = empty_packed(g, prec, nrhs) if out is None else out
    else:
        _require_cuda(psi, torch.complex128, "psi")
        nrhs = psi.numel() // (g.sites * 12)
        out = torch.empty_like(psi) if out is None else out
    fn = lib().wd_dslash_dag if dagger else lib().wd_dslash
    _check(fn(g.handle, float(m0), prec, _ptr(psi), _ptr(out), nrhs,
              PACKED if packed else 0, _stream()), "wd_dslash_dag" if dagger else "wd_dslash")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20   # WD_NOALLOC_SCRATCH_BYTES


def dslash_noalloc(g: Gauge, m0: float, psi, prec: int = F64, dagger: bool = False, out=None):
    """wd_dslash_noalloc: out = D psi (or D^dagger psi) on canonical complex128
    fields, the packed temporaries held in the library's static device scratch."""
    torch = _torch()
    _require_cuda(psi, torch.complex128, "psi")
    nrhs = psi.numel() // (g.sites * 12)
    out = torch.empty_like(psi) if out is None else out
    _check(lib().wd_dslash_noalloc(g.handle, float(m0), prec, 1 if dagger else 0, _ptr(psi),
                                   _ptr(out), nrhs, _stream()), "wd_dslash_noalloc")
    return out


class Coo:
    """D (or D^dagger) in the coordinate format of Sec. 2 (wd_coo_*)."""

    def __init__(self, g: Gauge, m0: float, prec: int = F64, dagger: bool = False):
        h = ctypes.c_void_p()
        _check(lib().wd_coo_create(g.handle, float(m0), prec, 1 if dagger else 0, _stream(),
                                   ctypes.byref(h)), "wd_coo_create")
        self.handle, self.prec, self.sites = h, prec, g.sites
        nnz, rows, nb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_size_t()
        _check(lib().wd_coo_info(h, ctypes.byref(nnz), ctypes.byref(rows), ctypes.byref(nb)),
               "wd_coo_info")
        self.nnz, self.rows, self.bytes = nnz.value, rows.value, nb.value

    def export(self):
        torch = _torch()
        vdt = torch.complex128 if self.prec == F64 else torch.complex64
        val = torch.empty(self.nnz, dtype=vdt, device="cuda")
        row = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        col = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        _check(lib().wd_coo_export(self.handle, _ptr(val), _ptr(row), _ptr(col), _stream()),
               "wd_coo_export")
        return val, row, col

    def spmv(self, x, out=None):
        torch = _torch()
        vdt = torch.complex128 if self.prec == F64 else torch.complex64
        _require_cuda(x, vdt, "x")
        nrhs = x.numel() // self.rows
        out = torch.empty_like(x) if out is None else out
        _check(lib().wd_coo_spmv(self.handle, _ptr(x), _ptr(out), nrhs, _stream()), "wd_coo_spmv")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().wd_coo_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cg_default_params(**kw) -> CGParams:
    p = CGParams()
    lib().wd_cg_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def cg_workspace_bytes(g: Gauge, nrhs: int, params: CGParams) -> int:
    return int(lib().wd_cg_workspace_bytes(g.handle, nrhs, ctypes.byref(params)))


def cg_solve_batch(g: Gauge, m0: float, src, sol=None, params: CGParams | None = None,
                   ws=None, raise_on_error: bool = True):
    """Solve D x = src for every field of src ([nrhs, ..., 4, 3] complex128).
    Returns (sol, reports list of dicts, rc)."""
    torch = _torch()
    _require_cuda(src, torch.complex128, "src")
    params = params or cg_default_params()
    nrhs = src.numel() // (g.sites * 12)
    if sol is None:
        sol = torch.zeros_like(src)
    nb = cg_workspace_bytes(g, nrhs, params)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    reps = (CGReport * nrhs)()
    rc = lib().wd_cg_solve_batch(g.handle, float(m0), _ptr(src), _ptr(sol), nrhs,
                                 ctypes.byref(params), _ptr(ws), ws.numel(), reps, _stream())
    if raise_on_error and rc not in (WD_OK, WD_ENOTCONV, WD_EBREAKDOWN):
        _check(rc, "wd_cg_solve_batch")
    return sol, [r.as_dict() for r in reps], rc


def cg_solve(g: Gauge, m0: float, src, sol=None, params: CGParams | None = None, ws=None,
             raise_on_error: bool = True):
    """Single-field solve through wd_cg_solve; src is [..., 4, 3] complex128."""
    torch = _torch()
    _require_cuda(src, torch.complex128, "src")
    params = params or cg_default_params()
    if src.numel() != g.sites * 12:
        raise ValueError("cg_solve takes one field")
    if sol is None:
        sol = torch.zeros_like(src)
    nb = cg_workspace_bytes(g, 1, params)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    rep = CGReport()
    rc = lib().wd_cg_solve(g.handle, float(m0), _ptr(src), _ptr(sol), ctypes.byref(params),
                           _ptr(ws), ws.numel(), ctypes.byref(rep), _stream())
    if raise_on_error and rc not in (WD_OK, WD_ENOTCONV, WD_EBREAKDOWN):
        _check(rc, "wd_cg_solve")
    return sol, rep.as_dict(), rc


def tune_dslash(g: Gauge, prec: int, nrhs: int, dagger: bool = False) -> dict:
    r = TuneResult()
    _check(lib().wd_tune_dslash(g.handle, prec, nrhs, 1 if dagger else 0, ctypes.byref(r),
                                _stream()), "wd_tune_dslash")
    return {f[0]: getattr(r, f[0]) for f in r._fields_ if f[0] != "reserved"}


def tune_cg(g: Gauge, m0: float, inner: int, src, iters: int = 30) -> dict:
    """Autotune the CG phase kernels on the fields src ([nrhs, ..., 4, 3]
    complex128, as cg_solve_batch takes them); returns the stored shape."""
    torch = _torch()
    _require_cuda(src, torch.complex128, "src")
    nrhs = src.numel() // (g.sites * 12)
    r = TuneResult()
    _check(lib().wd_tune_cg(g.handle, float(m0), inner, _ptr(src), nrhs, iters, ctypes.byref(r), _stream()),
           "wd_tune_cg")
    out = {f[0]: getattr(r, f[0]) for f in r._fields_ if f[0] != "gbps"}
    out["strip"] = r.site_order & 0xFFF
    out["xy_planes"] = max(1, (r.site_order >> 12) & 7)
    out["xy_lds"] = (r.site_order >> 17) & 1
    return out


def tune_lookup(g: Gauge, prec: int, nrhs: int, dagger: bool = False) -> dict:
    r = TuneResult()
    _check(lib().wd_tune_lookup(g.handle, prec, nrhs, 1 if dagger else 0, ctypes.byref(r)),
           "wd_tune_lookup")
    return {f[0]: getattr(r, f[0]) for f in r._fields_ if f[0] != "reserved"}


FAMILY_DSLASH, FAMILY_CG_A, FAMILY_CG_B, FAMILY_CG_R = 0, 1, 2, 3


def shape_set(g: Gauge, prec: int, nrhs: int, dagger: bool, family: int, block: int,
              rhs_per_thread: int = 1, xcd_remap: int = 1, hop_order: int = 1, rhs_loop: int = 1,
              strip: int = 0, group_major: int = 0, xy_lds: int = 0, max_blocks_per_cu: int = 0,
              rhs_pass: int = 0, xy_planes: int = 1):
    r = TuneResult(block=block, rhs_per_thread=rhs_per_thread, xcd_remap=xcd_remap,
                   hop_order=hop_order, rhs_loop=rhs_loop,
                   site_order=strip | ((xy_planes if xy_planes > 1 else 0) << 12) | (group_major << 16) |
                   ((1 if xy_lds else 0) << 17) | (max_blocks_per_cu << 18) |
                   ((1 if xy_lds == 2 else 0) << 24) | (rhs_pass << 25))
    _check(lib().wd_shape_set(g.handle, prec, nrhs, 1 if dagger else 0, family, ctypes.byref(r)),
           "wd_shape_set")


def shape_get(g: Gauge, prec: int, nrhs: int, dagger: bool, family: int) -> dict:
    r = TuneResult()
    _check(lib().wd_shape_get(g.handle, prec, nrhs, 1 if dagger else 0, family, ctypes.byref(r)),
           "wd_shape_get")
    out = {f[0]: getattr(r, f[0]) for f in r._fields_ if f[0] not in ("us", "gbps")}
    out["strip"] = r.site_order & 0xFFF
    out["xy_planes"] = max(1, (r.site_order >> 12) & 7)
    out["group_major"] = (r.site_order >> 16) & 1
    out["xy_lds"] = (1 + ((r.site_order >> 24) & 1)) if (r.site_order >> 17) & 1 else 0
    out["max_blocks_per_cu"] = (r.site_order >> 18) & 0x3F
    out["rhs_pass"] = (r.site_order >> 25) & 0x3F
    return out


def profile_enable(on: bool = True):
    _check(lib().wd_profile_enable(1 if on else 0), "wd_profile_enable")


def profile_reset():
    _check(lib().wd_profile_reset(), "wd_profile_reset")


def profile_read() -> dict:
    arr = (KernelStat * 16)()
    n = ctypes.c_int32(0)
    _check(lib().wd_profile_read(arr, 16, ctypes.byref(n)), "wd_profile_read")
    out = {}
    for i in range(min(n.value, 16)):
        k = arr[i]
        out[k.name.decode()] = {"launches": k.launches, "total_ms": k.total_ms,
                                "bytes_total": k.bytes_total}
    return out


def cg_graph_stats():
    """(chunk graphs captured since load, graphs cached now)"""
    built, cached = ctypes.c_int64(0), ctypes.c_int32(0)
    _check(lib().wd_cg_graph_stats(ctypes.byref(built), ctypes.byref(cached)), "wd_cg_graph_stats")
    return built.value, cached.value


def stream(kind: int, src, dst, nbytes: int):
    """One streaming kernel (STREAM_READ / STREAM_COPY / STREAM_WRITE) over nbytes
    of the GPU tensors src and dst (src may be None for STREAM_WRITE)."""
    _check(lib().wd_stream(kind, None if src is None else _ptr(src), _ptr(dst), int(nbytes), _stream()),
           "wd_stream")


@dataclass
class Ticket:
    id: int
    nrhs: int


class Server:
    """Continuous-batching solve server (wd_serve_*) over a caller-owned arena."""

    def __init__(self, arena, max_slots: int = 16, chunk: int = 0, device: int = 0):
        torch = _torch()
        _require_cuda(arena, torch.uint8, "arena")
        self.arena = arena
        cfg = ServeConfig(arena_dev=arena.data_ptr(), arena_bytes=arena.numel(),
                          max_slots=max_slots, chunk=chunk, device=device, reserved=0)
        h = ctypes.c_void_p()
        _check(lib().wd_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "wd_serve_create")
        self.handle = h
        self._keep = {}

    @staticmethod
    def request(dims, nrhs, m0, gauge, src, sol, params: CGParams | None = None, t_sign=-1):
        req = Request()
        req.dims[:] = [int(d) for d in dims]
        req.t_sign = int(t_sign)
        req.nrhs = int(nrhs)
        req.m0 = float(m0)
        req.gauge_dev = gauge.data_ptr()
        req.src_dev = src.data_ptr()
        req.sol_dev = sol.data_ptr()
        req.params = params or cg_default_params()
        return req

    @staticmethod
    def footprint(req: Request) -> int:
        return int(lib().wd_serve_footprint(ctypes.byref(req)))

    def submit(self, req: Request, keep=None) -> Ticket:
        """Queue a request.  The server reads the fields on its own stream, so
        the caller's stream is synchronised first (the fields must be ready)."""
        _torch().cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        _check(lib().wd_serve_submit(self.handle, ctypes.byref(req), ctypes.byref(t)),
               "wd_serve_submit")
        if keep is not None:
            self._keep[t.value] = keep
        return Ticket(t.value, req.nrhs)

    def poll(self, ticket: Ticket):
        reps = (CGReport * ticket.nrhs)()
        done = ctypes.c_int32(0)
        _check(lib().wd_serve_poll(self.handle, ticket.id, reps, ctypes.byref(done)),
               "wd_serve_poll")
        if done.value:
            self._keep.pop(ticket.id, None)
            return [r.as_dict() for r in reps]
        return None

    def stats(self) -> dict:
        st = ServeStats()
        _check(lib().wd_serve_stats_get(self.handle, ctypes.byref(st)), "wd_serve_stats_get")
        return {f[0]: getattr(st, f[0]) for f in st._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().wd_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
