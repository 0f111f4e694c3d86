"""MI355X Sparse Bessel Decomposition (SBD) matvec: thin Python binding.

Every computation runs in the HIP library ``libsbd.so`` (C ABI in
``include/sbd.h``); this module only marshals arguments.  PyTorch provides
device memory and streams.  There is no CPU fallback: if the library is
missing, every call raises.

Functions mirror the C ABI names: ``sbd_plan``, ``sbd_apply``,
``sbd_apply_parts``, ``sbd_plan_info``, ``sbd_plan_export``,
``sbd_workspace_bytes``, ``sbd_plan_bytes``, ``sbd_free``, ``sbd_fft2``.
``Plan`` wraps a plan handle.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _abi
from ._abi import (SBD_LAPLACE, SBD_HELMHOLTZ, SBD_GENERAL, SBD_F64, SBD_F32, SBD_C128, SBD_C64, SBD_PART_FAR,
                   SBD_PART_NEAR, SBD_PART_ALL, SBD_IO_SORTED, SBD_ARR_PERM, SBD_ARR_ROWPTR, SBD_ARR_COL, SBD_ARR_VAL,
                   SBD_ARR_COEF, SBD_ARR_RADII, SBD_ARR_M, SBD_ARR_KEYS, SBD_ARR_TPERM, SBD_ARR_TKEYS, SBD_OK,
                   SBD_EINVAL, SBD_ENOMEM, SBD_EDUP, SBD_EFLOOR, SBD_EHIP, SBD_EUNSUPPORTED, SBD_ENOCONV)

__all__ = ["SbdError", "Plan", "load_library", "sbd_plan", "sbd_plan_targets", "sbd_apply", "sbd_apply_noalloc",
           "sbd_apply_parts", "sbd_plan_info",
           "sbd_plan_export", "sbd_workspace_bytes", "sbd_plan_bytes", "sbd_free", "sbd_fft2", "sbd_launch_times", "sbd_set_timing",
           "sbd_gmres", "sbd_gmres_workspace_bytes",
           "SBD_LAPLACE", "SBD_HELMHOLTZ", "SBD_GENERAL", "general_kernel", "SBD_PART_FAR", "SBD_PART_NEAR", "SBD_PART_ALL"]

_LIB = None


class SbdError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load_library()
        msg = lib.sbd_strerror(status).decode()
        detail = lib.sbd_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}) {detail}")
        self.status = status


def load_library(path: str | None = None):
    """Load libsbd.so (built in-tree).  torch is imported first so that the process
    uses a single HIP runtime."""
    global _LIB
    if _LIB is not None:
        return _LIB
    import torch  # noqa: F401  (loads the HIP runtime torch was built with)
    path = path or _abi.LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"SBD HIP library not built: {path} (run paper_1711_07877_amd/build.py)")
    _LIB = _abi.declare(ctypes.CDLL(path))
    return _LIB


def _check(st: int, where: str):
    if st != 0:
        raise SbdError(st, where)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


_DTYPES = None


def _dtype_code(t):
    import torch
    global _DTYPES
    if _DTYPES is None:
        _DTYPES = {torch.float64: SBD_F64, torch.float32: SBD_F32, torch.complex128: SBD_C128,
                   torch.complex64: SBD_C64}
    if t.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return _DTYPES[t.dtype]


def general_kernel(c_log=0.0, terms=(), enforce=0) -> dict:
    """SBD_GENERAL kernel G(r) = c_log log r + sum_j r^m_j (a_j sin(w_j r) + b_j cos(w_j r)),
    terms = [(m, w, a, b), ...], with the multi-Dirichlet condition enforced to order
    `enforce` (Section 4.3).  Pass as sbd_plan(..., kind=SBD_GENERAL, general=...)."""
    return {"c_log": float(c_log), "terms": [tuple(float(v) for v in t) for t in terms], "enforce": int(enforce)}


def _kernel(kind, wavenumber, general):
    ker = _abi.sbd_kernel(int(kind), float(wavenumber))
    if int(kind) == SBD_GENERAL:
        if general is None:
            raise ValueError("SBD_GENERAL needs general=general_kernel(...)")
        flat = [v for t in general["terms"] for v in t]
        buf = (ctypes.c_double * max(1, len(flat)))(*flat)
        ker.c_log = general["c_log"]
        ker.nterms = len(general["terms"])
        ker.terms = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
        ker.enforce = general["enforce"]
        ker._buf = buf          # keeps the term array alive for the call
    return ker


def sbd_plan(points, kind=SBD_LAPLACE, eps=1e-3, wavenumber=0.0, delta_min=0.0, precision=0, max_rhs=1,
             nufft_tol=0.0, sigma=0.0, force_order=0, tile=0, byte_cap=0, timing=0, fit_reuse=0,
             stream=None, general=None, near_fp32=0, deterministic=0, near_assembly=0) -> "Plan":
    """Off-line part.  points: CUDA float64 tensor [N, 2] (contiguous)."""
    import torch
    lib = load_library()
    if not (points.is_cuda and points.dtype == torch.float64 and points.dim() == 2 and points.shape[1] == 2):
        raise TypeError("points must be a CUDA float64 tensor of shape [N, 2]")
    points = points.contiguous()
    opt = _options(lib, delta_min, precision, max_rhs, nufft_tol, sigma, force_order, tile, byte_cap, timing,
                   fit_reuse, near_fp32, deterministic, near_assembly)
    ker = _kernel(kind, wavenumber, general)
    h = ctypes.c_void_p()
    st = lib.sbd_plan(ctypes.c_void_p(points.data_ptr()), points.shape[0], ctypes.byref(ker), float(eps),
                      ctypes.byref(opt), _stream_ptr(stream), ctypes.byref(h))
    _check(st, "sbd_plan")
    return Plan(h, points.shape[0], int(kind), int(max_rhs))


def _options(lib, delta_min, precision, max_rhs, nufft_tol, sigma, force_order, tile, byte_cap, timing, fit_reuse,
             near_fp32=0, deterministic=0, near_assembly=0):
    opt = _abi.sbd_options()
    lib.sbd_default_options(ctypes.byref(opt))
    opt.delta_min = float(delta_min)
    opt.precision = int(precision)
    opt.max_rhs = int(max_rhs)
    opt.nufft_tol = float(nufft_tol)
    opt.sigma = float(sigma)
    opt.force_order = int(force_order)
    opt.tile = int(tile)
    opt.byte_cap = int(byte_cap)
    opt.fit_reuse = int(fit_reuse)
    opt.timing = int(timing)
    opt.near_fp32 = int(near_fp32)
    opt.deterministic = int(deterministic)
    opt.near_assembly = int(near_assembly)
    return opt


def sbd_plan_targets(targets, sources, kind=SBD_LAPLACE, eps=1e-3, wavenumber=0.0, delta_min=0.0, precision=0,
                     max_rhs=1, nufft_tol=0.0, sigma=0.0, force_order=0, tile=0, byte_cap=0, timing=0, fit_reuse=0,
                     stream=None, general=None, near_fp32=0, deterministic=0, near_assembly=0) -> "Plan":
    """Off-line part for q_k = sum_l G(x_k - y_l) f_l with separate targets x [M, 2] and
    sources y [N, 2] (CUDA float64 tensors)."""
    import torch
    lib = load_library()
    for t in (targets, sources):
        if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.shape[1] == 2):
            raise TypeError("targets and sources must be CUDA float64 tensors of shape [*, 2]")
    targets = targets.contiguous()
    sources = sources.contiguous()
    opt = _options(lib, delta_min, precision, max_rhs, nufft_tol, sigma, force_order, tile, byte_cap, timing,
                   fit_reuse, near_fp32, deterministic, near_assembly)
    ker = _kernel(kind, wavenumber, general)
    h = ctypes.c_void_p()
    st = lib.sbd_plan_targets(ctypes.c_void_p(targets.data_ptr()), targets.shape[0],
                              ctypes.c_void_p(sources.data_ptr()), sources.shape[0], ctypes.byref(ker), float(eps),
                              ctypes.byref(opt), _stream_ptr(stream), ctypes.byref(h))
    _check(st, "sbd_plan_targets")
    return Plan(h, sources.shape[0], int(kind), int(max_rhs), n_targets=targets.shape[0])


def _require_device(where, **tensors):
    """Every tensor must live in device memory on one device: the library reads and writes
    these buffers from GPU kernels, where a host pointer is a memory fault."""
    dev = None
    for name, t in tensors.items():
        if t is None:
            continue
        if not getattr(t, "is_cuda", False):
            raise TypeError(f"{where}: {name} must be a CUDA tensor (got {getattr(t, 'device', type(t))})")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise TypeError(f"{where}: {name} is on {t.device}, expected {dev}")


def sbd_apply_parts(plan: "Plan", f, q, parts=SBD_PART_ALL, workspace=None, stream=None):
    lib = load_library()
    _require_device("sbd_apply", f=f, q=q, workspace=workspace)
    if f.dim() == 1:
        nrhs = 1
    else:
        nrhs = f.shape[0]
    if (f.shape[-1] != plan.n or q.shape[:-1] != f.shape[:-1] or q.shape[-1] != plan.n_targets or q.dtype != f.dtype
            or not (f.is_contiguous() and q.is_contiguous())):
        raise ValueError("f [nrhs, N] and q [nrhs, M] must be contiguous tensors of the same dtype")
    ws = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    st = lib.sbd_apply_parts(plan.handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr()), nrhs,
                             _dtype_code(f), int(parts), ws, wsb, _stream_ptr(stream))
    _check(st, "sbd_apply")
    return q


def sbd_apply(plan: "Plan", f, q, workspace=None, stream=None):
    return sbd_apply_parts(plan, f, q, SBD_PART_ALL, workspace, stream)


def sbd_apply_noalloc(plan: "Plan", f, q, stream=None):
    """sbd_apply on the library's static per-device scratch (no allocation in the call);
    f [nrhs, N] and q [nrhs, M] contiguous CUDA tensors of one dtype."""
    lib = load_library()
    _require_device("sbd_apply_noalloc", f=f, q=q)
    nrhs = 1 if f.dim() == 1 else f.shape[0]
    if (f.shape[-1] != plan.n or q.shape[:-1] != f.shape[:-1] or q.shape[-1] != plan.n_targets or q.dtype != f.dtype
            or not (f.is_contiguous() and q.is_contiguous())):
        raise ValueError("f [nrhs, N] and q [nrhs, M] must be contiguous tensors of the same dtype")
    st = lib.sbd_apply_noalloc(plan.handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr()), nrhs,
                               _dtype_code(f), _stream_ptr(stream))
    _check(st, "sbd_apply_noalloc")
    return q


def sbd_plan_info(plan: "Plan") -> dict:
    lib = load_library()
    info = _abi.sbd_info()
    _check(lib.sbd_plan_info(plan.handle, ctypes.byref(info)), "sbd_plan_info")
    return {name: getattr(info, name) for name, _ in _abi.sbd_info._fields_}


_EXPORT = {SBD_ARR_PERM: (np.int32, "n"), SBD_ARR_ROWPTR: (np.int64, "m1"), SBD_ARR_COL: (np.int32, "nnz"),
           SBD_ARR_VAL: (np.float64, "nnz"), SBD_ARR_COEF: (np.float64, "P"), SBD_ARR_RADII: (np.float64, "P"),
           SBD_ARR_M: (np.int64, "P"), SBD_ARR_KEYS: (np.int64, "n"), SBD_ARR_TPERM: (np.int32, "m"),
           SBD_ARR_TKEYS: (np.int64, "m")}


def sbd_plan_export(plan: "Plan", which: int) -> np.ndarray:
    lib = load_library()
    info = sbd_plan_info(plan)
    dt, what = _EXPORT[which]
    count = {"n": info["n"], "m": info["n_targets"], "m1": info["n_targets"] + 1, "nnz": info["nnz"],
             "P": info["P"]}[what]
    out = np.empty(count, dtype=dt)
    _check(lib.sbd_plan_export(plan.handle, int(which), out.ctypes.data_as(ctypes.c_void_p), out.nbytes),
           "sbd_plan_export")
    return out


def sbd_workspace_bytes(plan: "Plan", nrhs: int = 1) -> int:
    return int(load_library().sbd_workspace_bytes(plan.handle, int(nrhs)))


def sbd_set_cache_limit(nbytes: int):
    """Keep up to nbytes of released large device blocks for reuse by later plans (0: off)."""
    _check(load_library().sbd_set_cache_limit(int(nbytes)), "sbd_set_cache_limit")


def sbd_cache_bytes() -> int:
    return int(load_library().sbd_cache_bytes())


def sbd_prefit(eps: float, a: float, kind=SBD_LAPLACE, wavenumber=0.0, delta_max=1.0, force_order=0,
               general=None) -> int:
    """Fit the SBD series for (kernel, eps, annulus ratio a) into the shared fit cache that
    plans made with fit_reuse=1 use (host only).  Returns the number of Bessel terms P."""
    lib = load_library()
    ker = _kernel(kind, wavenumber, general)
    p = ctypes.c_int(0)
    _check(lib.sbd_prefit(ctypes.byref(ker), float(eps), float(a), float(delta_max), int(force_order),
                          ctypes.byref(p)), "sbd_prefit")
    return int(p.value)


def sbd_plan_bytes(plan: "Plan") -> int:
    return int(load_library().sbd_plan_bytes(plan.handle))


def sbd_free(plan: "Plan"):
    if plan.handle is not None and plan.handle.value:
        load_library().sbd_free(plan.handle)
    plan.handle = None


def sbd_set_timing(plan: "Plan", enable: bool = True):
    load_library().sbd_set_timing(plan.handle, int(bool(enable)))


def sbd_launch_times(plan: "Plan") -> dict:
    """{kernel label: (ms per sbd_apply call, algorithmic bytes per call)} since the last read."""
    lib = load_library()
    buf = ctypes.create_string_buffer(4096)
    ms = (ctypes.c_double * 64)()
    by = (ctypes.c_double * 64)()
    n = lib.sbd_launch_times(plan.handle, buf, 4096, ms, by, 64)
    if n < 0:
        raise SbdError(-1, "sbd_launch_times")
    names = buf.value.decode().split("\n")[:n]
    return {nm: (ms[k], by[k]) for k, nm in enumerate(names)}


def sbd_fft2(data, direction=-1, stream=None):
    """In-place 2-D complex FFT of a CUDA complex tensor [ny, nx] (library kernels, natural order)."""
    lib = load_library()
    _require_device("sbd_fft2", data=data)
    if not data.is_contiguous() or data.dim() != 2:
        raise ValueError("contiguous 2-D tensor required")
    _check(lib.sbd_fft2(ctypes.c_void_p(data.data_ptr()), data.shape[0], data.shape[1], _dtype_code(data),
                        int(direction), _stream_ptr(stream)), "sbd_fft2")
    return data


def sbd_gmres_workspace_bytes(plan: "Plan", restart: int = 30) -> int:
    return int(load_library().sbd_gmres_workspace_bytes(plan.handle, int(restart)))


def sbd_gmres(plan: "Plan", b, x=None, weights=None, diag=None, restart=30, max_restarts=100, rtol=1e-6,
              workspace=None, stream=None, check=True):
    """Solve (sbd_apply(w o x) + d o x) = b with restarted GMRES (Laplace plans).

    b, x, weights, diag: CUDA float64 tensors [N].  x=None starts from zero.
    Returns (x, iterations, relres); with check=True a solve that stops above
    rtol raises SbdError(SBD_ENOCONV).
    """
    import torch
    lib = load_library()
    _require_device("sbd_gmres", b=b, x=x, weights=weights, diag=diag, workspace=workspace)
    for t in (b, x, weights, diag):
        if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == plan.n):
            raise ValueError("b, x, weights and diag must be contiguous CUDA float64 tensors of length N")
    opt = _abi.sbd_gmres_options(int(restart), int(max_restarts), float(rtol), 1 if x is None else 0)
    if x is None:
        x = torch.empty_like(b)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    ws = ptr(workspace)
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    its = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = lib.sbd_gmres(plan.handle, ptr(weights), ptr(diag), ptr(b), ptr(x), ctypes.byref(opt), ws, wsb,
                       _stream_ptr(stream), ctypes.byref(its), ctypes.byref(rel))
    if st != SBD_OK and (check or st != SBD_ENOCONV):
        _check(st, "sbd_gmres")
    return x, its.value, rel.value


class Plan:
    """Handle of an SBD plan (off-line part); ``apply`` runs the on-line part."""

    def __init__(self, handle, n, kind, max_rhs, n_targets=None):
        self.handle = handle
        self.n = n
        self.n_targets = n if n_targets is None else n_targets
        self.kind = kind
        self.max_rhs = max_rhs

    def info(self) -> dict:
        return sbd_plan_info(self)

    def export(self, which: int) -> np.ndarray:
        return sbd_plan_export(self, which)

    def apply(self, f, out=None, parts=SBD_PART_ALL, workspace=None, stream=None, sorted_io=False):
        """q = A f.  sorted_io: f and q in the plan's sorted order (SBD_IO_SORTED)."""
        import torch
        _require_device("Plan.apply", f=f, out=out, workspace=workspace)
        if sorted_io:
            parts = parts | SBD_IO_SORTED
        q = out if out is not None else torch.empty(tuple(f.shape[:-1]) + (self.n_targets,), dtype=f.dtype,
                                                     device=f.device)
        return sbd_apply_parts(self, f, q, parts, workspace, stream)

    def workspace_bytes(self, nrhs=1) -> int:
        return sbd_workspace_bytes(self, nrhs)

    def gmres(self, b, x=None, weights=None, diag=None, **kw):
        return sbd_gmres(self, b, x, weights, diag, **kw)

    def gmres_workspace_bytes(self, restart=30) -> int:
        return sbd_gmres_workspace_bytes(self, restart)

    def plan_bytes(self) -> int:
        return sbd_plan_bytes(self)

    def launch_times(self) -> dict:
        return sbd_launch_times(self)

    def set_timing(self, enable=True):
        sbd_set_timing(self, enable)

    def free(self):
        sbd_free(self)

    def __del__(self):
        try:
            if self.handle is not None:
                sbd_free(self)
        except Exception:
            pass
