"""ctypes declarations of libswvis.so (include/swvis.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libswvis.so")

SWV_OK, SWV_EINVAL, SWV_EDOMAIN, SWV_ENOMEM, SWV_EHIP, SWV_ENOTSUP = 0, -1, -2, -3, -4, -5
SWV_FP64, SWV_F32C = 0, 1
SWV_ROUTE_DIRECT, SWV_ROUTE_TREE = 0, 1
SWV_MAX_LEVEL = 29
SWV_HOGBOM_ABS = 1
SWV_HOGBOM_SINGLE = 2
PREDICTORS = {"tree": 0, "degrid": 1, "direct": 2}
SWV_CLEAN_MAX_CYCLES = 64
# kernel families of the tuning table (swv_tune_get / swv_tune_set)
FAM_DIRECT64, FAM_DIRECT32, FAM_TREE, FAM_ADJOINT, FAM_GRAD = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "SWV_OK", -1: "SWV_EINVAL", -2: "SWV_EDOMAIN", -3: "SWV_ENOMEM",
                -4: "SWV_EHIP", -5: "SWV_ENOTSUP"}


class SwvError(RuntimeError):
    """A libswvis call returned a negative status."""

    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code
        self.message = message


class TreeStats(C.Structure):
    _fields_ = [("J", C.c_int), ("n_comp", C.c_int64), ("n_leaves", C.c_int64),
                ("n_internal", C.c_int64), ("n_nodes", C.c_int64 * (SWV_MAX_LEVEL + 1)),
                ("n_records", C.c_int64), ("sparsity", C.c_double),
                ("build_seconds", C.c_double), ("max_branching", C.c_int)]


class Peaks(C.Structure):
    _fields_ = [("fp64_fma_tflops", C.c_double), ("fp32_fma_tflops", C.c_double),
                ("sincos_f32_gops", C.c_double), ("cis2pi_f64_gops", C.c_double)]


class PlanStats(C.Structure):
    _fields_ = [("n_instances", C.c_int64), ("n_items", C.c_int64),
                ("total_terms", C.c_int64), ("tile_rows", C.c_int),
                ("grid_blocks", C.c_int), ("block_threads", C.c_int)]


class Instance(C.Structure):
    _fields_ = [("route", C.c_int), ("prec", C.c_int), ("sign", C.c_int),
                ("n_vis", C.c_int64), ("u", C.c_void_p), ("v", C.c_void_p), ("w", C.c_void_p),
                ("n_comp", C.c_int64), ("l", C.c_void_p), ("m", C.c_void_p),
                ("flux", C.c_void_p), ("tree", C.c_void_p), ("vis_out", C.c_void_p)]


class CycleInstance(C.Structure):
    _fields_ = [("route", C.c_int), ("sign", C.c_int), ("n_vis", C.c_int64),
                ("u", C.c_void_p), ("v", C.c_void_p), ("w", C.c_void_p),
                ("vis_obs", C.c_void_p), ("vis_model", C.c_void_p), ("resid", C.c_void_p),
                ("chi2", C.c_void_p), ("inv_sigma2", C.c_double), ("n_pix", C.c_int64),
                ("pix_l", C.c_void_p), ("pix_m", C.c_void_p), ("pix_nm1", C.c_void_p),
                ("image", C.c_void_p), ("comp_cap", C.c_int64), ("tree_level_cap", C.c_int),
                ("d_flux", C.c_void_p), ("d_l", C.c_void_p), ("d_m", C.c_void_p)]


class CleanParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("cell", C.c_double), ("J", C.c_int),
                ("ra_p", C.c_double), ("dec_p", C.c_double), ("gain", C.c_double),
                ("threshold", C.c_double), ("minor_iter", C.c_int64), ("n_major", C.c_int),
                ("flags", C.c_int), ("sign", C.c_int), ("predictor", C.c_int),
                ("support", C.c_int), ("image_prec", C.c_int)]


_NC = SWV_CLEAN_MAX_CYCLES


class CleanStats(C.Structure):
    _fields_ = [("n_cycles", C.c_int), ("found", C.c_int64 * _NC), ("leaves", C.c_int64 * _NC),
                ("chi2", C.c_double * _NC), ("ms_minor", C.c_double * _NC),
                ("ms_build", C.c_double * _NC), ("ms_predict", C.c_double * _NC),
                ("ms_image", C.c_double * _NC), ("ms_beam", C.c_double),
                ("ms_dirty", C.c_double)]


class DegridStats(C.Structure):
    _fields_ = [("n_planes", C.c_int64), ("grid_nx", C.c_int), ("grid_ny", C.c_int),
                ("w0", C.c_double), ("dw", C.c_double), ("c", C.c_double),
                ("plane_bytes", C.c_int64), ("host_ms", C.c_double)]


_vp, _i64, _int, _dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
_pvp = C.POINTER(C.c_void_p)

SIGNATURES = {
    "swv_version": [C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "swv_ctx_create": [_int, _vp, _pvp],
    "swv_ctx_set_stream": [_vp, _vp],
    "swv_ctx_synchronize": [_vp],
    "swv_ctx_destroy": [_vp],
    "swv_predict_direct": [_vp, _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _int, _int, _vp],
    "swv_tree_build": [_int, _dbl, _dbl, _i64, _vp, _vp, _vp, _pvp],
    "swv_tree_stats": [_vp, C.POINTER(TreeStats)],
    "swv_tree_leaves": [_vp, _vp, _vp, _vp, _vp, _vp],
    "swv_tree_level": [_vp, _int, _vp, _vp, _vp, _vp],
    "swv_predict_tree": [_vp, _vp, _i64, _vp, _vp, _vp, _int, _int, _vp],
    "swv_tree_set_flux": [_vp, _vp],
    "swv_predict_tree_leaves": [_vp, _vp, _i64, _vp, _vp, _vp, _int, _int, _vp],
    "swv_tree_destroy": [_vp],
    "swv_ang2pix": [_int, _dbl, _dbl, _i64, _vp, _vp, _vp],
    "swv_pixel_centres": [_int, _dbl, _dbl, _i64, _vp, _vp, _vp, _vp],
    "swv_pixels_in_disk": [_int, _dbl, _dbl, _dbl, _i64, _vp, _vp, _vp, _vp, C.POINTER(_i64)],
    "swv_residual_chi2": [_vp, _i64, _vp, _vp, _dbl, _vp, _vp],
    "swv_adjoint": [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _int, _int, _vp],
    "swv_adjoint_noalloc": [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _int, _int,
                            _vp],
    "swv_grad_direct": [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _int, _dbl,
                        _vp, _vp, _vp],
    "swv_batch_plan": [_vp, _int, C.POINTER(Instance), _pvp],
    "swv_plan_stats": [_vp, C.POINTER(PlanStats)],
    "swv_batch_run": [_vp],
    "swv_graph_capture": [_vp, _pvp],
    "swv_graph_launch": [_vp],
    "swv_graph_destroy": [_vp],
    "swv_plan_destroy": [_vp],
    "swv_tree_threshold": [_vp, _dbl, _pvp],
    "swv_tree_prune": [_vp, _i64, _vp, _pvp],
    "swv_tree_kept": [_vp, _i64, _vp, C.POINTER(_i64), C.POINTER(_i64)],
    "swv_cycle_create": [_vp, _int, C.POINTER(CycleInstance), _pvp],
    "swv_cycle_set_components": [_vp, _int, _i64, _vp, _vp, _vp],
    "swv_cycle_set_tree": [_vp, _int, _vp],
    "swv_cycle_run": [_vp],
    "swv_cycle_capture": [_vp],
    "swv_cycle_launch": [_vp],
    "swv_cycle_destroy": [_vp],
    "swv_autotune": [_vp, C.c_char_p, _int],
    "swv_tune_load": [_vp, C.c_char_p],
    "swv_tune_get": [_vp, _int, _int, C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "swv_tune_set": [_vp, _int, _int, _int, _int],
    "swv_measure_peaks": [_vp, _vp],
    "swv_image_grid": [_vp, _int, _int, _int, _int, _dbl, _vp, _vp, _vp],
    "swv_dirty_image": [_vp, _i64, _vp, _vp, _vp, _vp, _int, _int, _int, _int, _dbl, _int, _int,
                        _vp],
    "swv_hogbom": [_vp, _int, _int, _vp, _vp, _dbl, _dbl, _i64, _int, _vp, _vp, _vp],
    "swv_cross_reference": [_int, _dbl, _dbl, _int, _int, _dbl, _vp],
    "swv_tree_build_pixels": [_int, _dbl, _dbl, _i64, _vp, _vp, _pvp],
    "swv_fit_clean_beam": [_int, _int, _vp, _vp],
    "swv_restore": [_vp, _int, _int, _i64, _vp, _vp, _vp, _vp, _vp],
    "swv_predict_degrid": [_vp, _int, _int, _dbl, _vp, _i64, _vp, _vp, _vp, _int, _int, _vp,
                           C.POINTER(DegridStats)],
    "swv_wavelet_clean": [_vp, C.POINTER(CleanParams), _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                          _i64, _vp, _vp, C.POINTER(_i64), C.POINTER(CleanStats)],
}

_lib = None


def lib() -> C.CDLL:
    """The loaded library.  Raises if it is not built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run "
                               "`python paper_1909_03956_amd/build.py` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.swv_last_error.argtypes = []
        L.swv_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != SWV_OK:
        raise SwvError(rc, lib().swv_last_error().decode(errors="replace"))
