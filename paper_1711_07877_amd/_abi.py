"""ctypes mirror of include/sbd.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbd.so")

(SBD_OK, SBD_EINVAL, SBD_ENOMEM, SBD_EDUP, SBD_EFLOOR, SBD_EHIP, SBD_EUNSUPPORTED,
 SBD_ENOCONV) = 0, -1, -2, -3, -4, -5, -6, -7
SBD_LAPLACE, SBD_HELMHOLTZ, SBD_GENERAL = 0, 1, 2
SBD_F64, SBD_F32, SBD_C128, SBD_C64 = 0, 1, 2, 3
SBD_PART_FAR, SBD_PART_NEAR, SBD_PART_ALL = 1, 2, 3
SBD_IO_SORTED = 4
SBD_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024
(SBD_ARR_PERM, SBD_ARR_ROWPTR, SBD_ARR_COL, SBD_ARR_VAL, SBD_ARR_COEF, SBD_ARR_RADII, SBD_ARR_M,
 SBD_ARR_KEYS, SBD_ARR_TPERM, SBD_ARR_TKEYS) = range(10)


class sbd_kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("wavenumber", ctypes.c_double), ("c_log", ctypes.c_double),
                ("nterms", ctypes.c_int), ("terms", ctypes.POINTER(ctypes.c_double)), ("enforce", ctypes.c_int)]


class sbd_options(ctypes.Structure):
    _fields_ = [("delta_min", ctypes.c_double), ("precision", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("nufft_tol", ctypes.c_double), ("sigma", ctypes.c_double), ("force_order", ctypes.c_int),
                ("tile", ctypes.c_int), ("timing", ctypes.c_int), ("byte_cap", ctypes.c_size_t),
                ("fit_reuse", ctypes.c_int), ("near_fp32", ctypes.c_int), ("deterministic", ctypes.c_int),
                ("near_assembly", ctypes.c_int)]


class sbd_gmres_options(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_restarts", ctypes.c_int), ("rtol", ctypes.c_double),
                ("zero_guess", ctypes.c_int)]


class sbd_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("kind", ctypes.c_int), ("precision", ctypes.c_int), ("P", ctypes.c_int),
                ("n_xi", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("eps", ctypes.c_double), ("delta_min", ctypes.c_double), ("delta_max", ctypes.c_double),
                ("center_x", ctypes.c_double), ("center_y", ctypes.c_double), ("fit_error", ctypes.c_double),
                ("h", ctypes.c_double), ("w", ctypes.c_int), ("beta", ctypes.c_double), ("sigma", ctypes.c_double),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("Mx", ctypes.c_int64), ("My", ctypes.c_int64),
                ("tile", ctypes.c_int), ("ntx", ctypes.c_int64), ("nty", ctypes.c_int64),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("inv_c", ctypes.c_double),
                ("ncx", ctypes.c_int64), ("ncy", ctypes.c_int64), ("nsub", ctypes.c_int),
                ("d2max", ctypes.c_double), ("plan_seconds", ctypes.c_double), ("fit_seconds", ctypes.c_double),
                ("plan_bytes", ctypes.c_size_t), ("n_targets", ctypes.c_int64), ("bipartite", ctypes.c_int),
                ("near_fp32", ctypes.c_int), ("deterministic", ctypes.c_int), ("colconv", ctypes.c_int),
                ("near_assembly", ctypes.c_int), ("pd_grid", ctypes.c_int), ("pd_tol", ctypes.c_double),
                ("near_seconds", ctypes.c_double), ("assembly_seconds", ctypes.c_double),
                ("bin_seconds", ctypes.c_double), ("symbol_seconds", ctypes.c_double), ("row_pairs", ctypes.c_int)]


def declare(lib):
    P = ctypes.c_void_p
    i64, i32, dbl, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    lib.sbd_default_options.argtypes = [ctypes.POINTER(sbd_options)]
    lib.sbd_default_options.restype = None
    lib.sbd_plan.argtypes = [P, i64, ctypes.POINTER(sbd_kernel), dbl, ctypes.POINTER(sbd_options), P,
                             ctypes.POINTER(P)]
    lib.sbd_plan.restype = i32
    lib.sbd_plan_targets.argtypes = [P, i64, P, i64, ctypes.POINTER(sbd_kernel), dbl, ctypes.POINTER(sbd_options), P,
                                     ctypes.POINTER(P)]
    lib.sbd_plan_targets.restype = i32
    lib.sbd_set_cache_limit.argtypes = [sz]
    lib.sbd_set_cache_limit.restype = i32
    lib.sbd_cache_bytes.argtypes = []
    lib.sbd_cache_bytes.restype = sz
    lib.sbd_prefit.argtypes = [ctypes.POINTER(sbd_kernel), dbl, dbl, dbl, i32, ctypes.POINTER(i32)]
    lib.sbd_prefit.restype = i32
    lib.sbd_workspace_bytes.argtypes = [P, i32]
    lib.sbd_workspace_bytes.restype = sz
    lib.sbd_plan_bytes.argtypes = [P]
    lib.sbd_plan_bytes.restype = sz
    lib.sbd_apply.argtypes = [P, P, P, i32, i32, P, sz, P]
    lib.sbd_apply.restype = i32
    lib.sbd_apply_noalloc.argtypes = [P, P, P, i32, i32, P]
    lib.sbd_apply_noalloc.restype = i32
    lib.sbd_apply_parts.argtypes = [P, P, P, i32, i32, i32, P, sz, P]
    lib.sbd_apply_parts.restype = i32
    lib.sbd_plan_info.argtypes = [P, ctypes.POINTER(sbd_info)]
    lib.sbd_plan_info.restype = i32
    lib.sbd_plan_export.argtypes = [P, i32, P, sz]
    lib.sbd_plan_export.restype = i32
    lib.sbd_free.argtypes = [P]
    lib.sbd_free.restype = None
    lib.sbd_strerror.argtypes = [i32]
    lib.sbd_strerror.restype = ctypes.c_char_p
    lib.sbd_last_error.argtypes = []
    lib.sbd_last_error.restype = ctypes.c_char_p
    lib.sbd_set_timing.argtypes = [P, i32]
    lib.sbd_set_timing.restype = i32
    lib.sbd_launch_times.argtypes = [P, ctypes.c_char_p, sz, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), i32]
    lib.sbd_launch_times.restype = i32
    lib.sbd_fft2.argtypes = [P, i64, i64, i32, i32, P]
    lib.sbd_fft2.restype = i32
    lib.sbd_gmres_workspace_bytes.argtypes = [P, i32]
    lib.sbd_gmres_workspace_bytes.restype = sz
    lib.sbd_gmres.argtypes = [P, P, P, P, P, ctypes.POINTER(sbd_gmres_options), P, sz, P,
                              ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    lib.sbd_gmres.restype = i32
    return lib
