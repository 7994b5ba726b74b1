"""ctypes view of libhdi.so: the structs and signatures of include/hdi.h."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdi.so")

HDI_OK, HDI_ERR_ARG, HDI_ERR_EMPTY_MASK, HDI_ERR_NO_CONVERGENCE, HDI_ERR_WORKSPACE, HDI_ERR_HIP, HDI_ERR_BUDGET = range(7)
HDI_FLAG_NO_FMG = 1
HDI_FLAG_CG = 2


class hdi_image(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("channels", ctypes.c_int32)]


class hdi_solve_params(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("local_iters", ctypes.c_int32), ("coarse_iters", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("small_from", ctypes.c_int32), ("robin", ctypes.c_float),
                ("local_stop", ctypes.c_float), ("mid_iters", ctypes.c_int32)]


class hdi_solve_report(ctypes.Structure):
    _fields_ = [("rel_residual", ctypes.c_double * 3), ("outer_iters", ctypes.c_int32),
                ("vcycles", ctypes.c_int32), ("ms", ctypes.c_float)]


class hdi_tonal_params(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("local_outer", ctypes.c_int32), ("local_inner", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("inner", hdi_solve_params), ("mse_gain", ctypes.c_double),
                ("block", ctypes.c_int32)]


class hdi_tonal_report(ctypes.Structure):
    _fields_ = [("mse_initial", ctypes.c_double), ("mse_final", ctypes.c_double),
                ("rel_normal_residual", ctypes.c_double), ("outer_iters", ctypes.c_int32),
                ("inner_solves", ctypes.c_int32), ("inner_vcycles", ctypes.c_int32), ("ms", ctypes.c_float)]


HDI_JOB_INPAINT, HDI_JOB_TONAL = 0, 1


class hdi_job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("img", hdi_image), ("mask", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("tonal", ctypes.POINTER(hdi_tonal_params)),
                ("tonal_report", ctypes.POINTER(hdi_tonal_report))]


class hdi_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("flags", ctypes.c_int32), ("img", hdi_image), ("mask", ctypes.c_void_p),
                ("f", ctypes.c_void_p), ("out", ctypes.c_void_p), ("solve", hdi_solve_params),
                ("tonal", ctypes.POINTER(hdi_tonal_params))]


class hdi_request_report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("inner_solves", ctypes.c_int32), ("max_running", ctypes.c_int32),
                ("rel_residual", ctypes.c_double * 3), ("mse_initial", ctypes.c_double),
                ("mse_final", ctypes.c_double), ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double)]


class hdi_spatial_params(ctypes.Structure):
    _fields_ = [("density", ctypes.c_double), ("t", ctypes.c_double), ("n0", ctypes.c_int64),
                ("n_steps", ctypes.c_int32), ("partition", ctypes.c_int32), ("solve", hdi_solve_params)]


class hdi_spatial_report(ctypes.Structure):
    _fields_ = [("initial_count", ctypes.c_int64), ("final_count", ctypes.c_int64), ("solve_rounds", ctypes.c_int32),
                ("rel_residual", ctypes.c_double * 3), ("ms", ctypes.c_float)]


HDI_VINIT_TRACE = 64


class hdi_vinit_params(ctypes.Structure):
    _fields_ = [("weighting", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("tau", ctypes.c_double),
                ("flags", ctypes.c_int32), ("solve", hdi_solve_params)]


class hdi_vinit_report(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("best", ctypes.c_int32), ("solves", ctypes.c_int32),
                ("mse", ctypes.c_double * HDI_VINIT_TRACE), ("ms", ctypes.c_float)]


HDI_STEP_HOOK = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_float),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.c_void_p)

HDI_REQ_INPAINT, HDI_REQ_TONAL = 0, 1
HDI_REQ_HOST_IO = 1
HDI_SERVER_PLAIN = 1
HDI_SERVER_TONAL_SHARED = 2
HDI_TONAL_PCG_RAS, HDI_TONAL_RAS, HDI_TONAL_CGNR = 0, 1, 2
HDI_TONAL_INIT_FROM_F = 1
HDI_TONAL_TRACE = 2
HDI_PART_DELAUNAY, HDI_PART_VORONOI = 0, 1
HDI_PART_JFA = 4
HDI_VINIT_DIRECT, HDI_VINIT_VORONOI, HDI_VINIT_VORONOI_LOG = 0, 1, 2
HDI_VINIT_FROM_F, HDI_VINIT_NO_STOP = 1, 2

_P = ctypes.c_void_p
_SIGS = {
    "hdi_inpaint_workspace_bytes": (ctypes.c_size_t, [hdi_image]),
    "inpaint_solve": (ctypes.c_int32, [hdi_image, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                       ctypes.POINTER(hdi_solve_params), ctypes.POINTER(hdi_solve_report), _P]),
    "hdi_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "inpaint_solve_noalloc": (ctypes.c_int32, [hdi_image, _P, _P, _P, _P, ctypes.POINTER(hdi_solve_params),
                                               ctypes.POINTER(hdi_solve_report), _P]),
    "hdi_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.POINTER(hdi_job)]),
    "hdi_solve_batch": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(hdi_job), _P, ctypes.c_size_t,
                                         ctypes.POINTER(hdi_solve_params), ctypes.POINTER(hdi_solve_report), _P]),
    "hdi_tonal_workspace_bytes": (ctypes.c_size_t, [hdi_image]),
    "tonal_optimize": (ctypes.c_int32, [hdi_image, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                        ctypes.POINTER(hdi_tonal_params), ctypes.POINTER(hdi_tonal_report), _P]),
    "hdi_vinit_workspace_bytes": (ctypes.c_size_t, [hdi_image]),
    "voronoi_init": (ctypes.c_int32, [hdi_image, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                      ctypes.POINTER(hdi_vinit_params), ctypes.POINTER(hdi_vinit_report), _P]),
    "hdi_error_map": (ctypes.c_int32, [hdi_image, _P, _P, _P, _P]),
    "hdi_initial_mask_workspace_bytes": (ctypes.c_size_t, [hdi_image]),
    "hdi_initial_mask": (ctypes.c_int32, [hdi_image, _P, _P, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_int64), _P,
                                          ctypes.c_size_t, _P]),
    "hdi_spatial_workspace_bytes": (ctypes.c_size_t, [hdi_image]),
    "spatial_optimize": (ctypes.c_int32, [hdi_image, _P, _P, ctypes.POINTER(hdi_spatial_params), _P, _P, _P,
                                          ctypes.c_size_t, ctypes.POINTER(hdi_spatial_report), HDI_STEP_HOOK, _P, _P]),
    "hdi_densify_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "hdi_labels_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "hdi_voronoi_labels": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_uint64), _P, ctypes.c_size_t, _P]),
    "densify_step": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_int32, _P,
                                      ctypes.POINTER(ctypes.c_int64), _P, ctypes.c_size_t, _P]),
    "hdi_autotune": (ctypes.c_int32, [hdi_image, _P, _P, _P, ctypes.c_size_t, ctypes.POINTER(hdi_solve_params),
                                      ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_float), _P]),
    "hdi_request_bytes": (ctypes.c_size_t, [ctypes.POINTER(hdi_request)]),
    "hdi_server_create": (_P, [_P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "hdi_server_submit": (ctypes.c_int32, [_P, ctypes.POINTER(hdi_request), ctypes.POINTER(ctypes.c_uint64)]),
    "hdi_server_poll": (ctypes.c_int32, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(hdi_request_report)]),
    "hdi_server_drain": (ctypes.c_int32, [_P]),
    "hdi_server_destroy": (None, [_P]),
    "hdi_block_count": (ctypes.c_int64, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "hdi_stats_enable": (None, [ctypes.c_int32]),
    "hdi_stats_reset": (None, []),
    "hdi_stats_get": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "hdi_stats_get_lds": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "hdi_lds_calibrate": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_void_p]),
    "hdi_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "hdi_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libhdi.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2401_06747_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


class HdiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().hdi_status_string(status).decode()}: {msg}")
        self.status = status


def check(status):
    if status != HDI_OK:
        raise HdiError(status, lib().hdi_last_error().decode())
