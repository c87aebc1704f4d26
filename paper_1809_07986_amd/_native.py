"""ctypes declarations of libsgm.so (the C ABI in include/sgm.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgm.so")

SGM_OK, SGM_EINVAL, SGM_ENOMEM, SGM_EHIP, SGM_ESTATE = 0, -1, -2, -3, -4
FLAG_PRED, FLAG_RESET, FLAG_FULLWIN, FLAG_GATEFAIL = 1, 2, 4, 8
WIN_KSIGMA, WIN_LEARNED = 0, 1
LEARNED_WMAX = 32
DEBUG_STAGES, DEBUG_SHORT_SEGMENTS, DEBUG_ALT_HORIZONTAL, DEBUG_DENSE_RERUN = 1, 2, 4, 8
CNN_NPARAMS = 19394
(STAGE_CENSUS_L, STAGE_CENSUS_R, STAGE_LO, STAGE_HI, STAGE_OFFSETS, STAGE_COST, STAGE_SUM, STAGE_DHAT,
 STAGE_PM, STAGE_FLAGS, STAGE_DSTAR, STAGE_DZ, STAGE_STATUS) = range(13)
STAGE_PATH0 = 16
(STAGE_NU, STAGE_NU_W, STAGE_FEATURES, STAGE_CNN_OUT, STAGE_HALFWIDTH, STAGE_RPIX, STAGE_KAPPA,
 STAGE_RERUN) = range(32, 40)

# every symbol include/sgm.h declares
EXPORTS = ("sgm_default_params", "sgm_paper_params", "sgm_create", "sgm_destroy", "sgm_full_frame", "sgm_reduced_frame",
           "sgm_get_disparity", "sgm_get_variance", "sgm_get_motion_mask", "sgm_get_disparity_median",
           "sgm_get_state", "sgm_set_state",
           "sgm_match_windows", "sgm_get_stage", "sgm_cost_cells", "sgm_set_debug", "sgm_set_profiling",
           "sgm_read_profile", "sgm_batch_create", "sgm_batch_destroy", "sgm_batch_context", "sgm_batch_full",
           "sgm_batch_step", "sgm_batch_step_graph", "sgm_batch_set_schedule", "sgm_batch_autotune", "sgm_autotune",
           "sgm_set_window_model", "sgm_get_features", "sgm_learned_targets", "sgm_cnn_create", "sgm_cnn_destroy",
           "sgm_cnn_set_params", "sgm_cnn_get_params", "sgm_cnn_forward", "sgm_cnn_loss", "sgm_cnn_backward",
           "sgm_cnn_get_grads", "sgm_cnn_adam", "sgm_cnn_train_step", "sgm_detect_default_params",
           "sgm_detector_create", "sgm_detector_destroy", "sgm_detector_windows", "sgm_detect", "sgm_detect_frame",
           "sgm_detector_stage", "sgm_detect_noalloc", "sgm_last_error")
PROF_STAGES = ("census", "predict", "cost", "agg_h", "agg_v", "wta", "cnn", "rerun")


class SgmParams(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("max_disp", ctypes.c_int32),
                ("census_w", ctypes.c_int32), ("census_h", ctypes.c_int32), ("path_mask", ctypes.c_uint32),
                ("p1", ctypes.c_int32), ("p2", ctypes.c_int32),
                ("k_sigma", ctypes.c_double), ("q", ctypes.c_double), ("r", ctypes.c_double),
                ("chi2_gate", ctypes.c_double), ("disc_thresh", ctypes.c_double),
                ("f", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("baseline", ctypes.c_double), ("window_mode", ctypes.c_int32), ("gate_rerun", ctypes.c_int32),
                ("r_curv", ctypes.c_double)]


class SgmDetectParams(ctypes.Structure):
    _fields_ = [("top", ctypes.c_int32), ("n_sizes", ctypes.c_int32), ("sizes", (ctypes.c_int32 * 2) * 8),
                ("scale", ctypes.c_int32), ("cap", ctypes.c_int32), ("thresh", ctypes.c_int32),
                ("max_detections", ctypes.c_int32), ("min_area", ctypes.c_int64), ("merge_iou", ctypes.c_double)]


DSTAGE_SAT, DSTAGE_FIRED = 0, 1
DETECT_MAX = 2048

_lib = None


def load(path: str = LIB_PATH):
    """Load libsgm.so and declare its functions (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "sgm_default_params": [ctypes.POINTER(SgmParams), I32, I32, I32],
        "sgm_paper_params": [ctypes.POINTER(SgmParams), I32, I32, I32],
        "sgm_create": [ctypes.POINTER(SgmParams), ctypes.POINTER(P)],
        "sgm_destroy": [P],
        "sgm_full_frame": [P, P, P, I32, P],
        "sgm_reduced_frame": [P, P, P, I32, ctypes.POINTER(ctypes.c_double), P],
        "sgm_get_disparity": [P, P, I32, P],
        "sgm_get_variance": [P, P, I32, P],
        "sgm_get_motion_mask": [P, P, I32, P],
        "sgm_get_disparity_median": [P, P, I32, P],
        "sgm_get_state": [P, P, P, P, P],
        "sgm_set_state": [P, P, P, P, P],
        "sgm_match_windows": [P, P, P, I32, P, P, P, P, P],
        "sgm_get_stage": [P, I32, P, SZ, P],
        "sgm_cost_cells": [P, ctypes.POINTER(I64), P],
        "sgm_set_debug": [P, I32],
        "sgm_set_profiling": [P, I32],
        "sgm_read_profile": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64), P],
        "sgm_batch_create": [I32, ctypes.POINTER(SgmParams), ctypes.POINTER(P), ctypes.POINTER(P),
                             ctypes.POINTER(I32), ctypes.POINTER(P)],
        "sgm_batch_destroy": [P],
        "sgm_batch_context": [P, I32],
        "sgm_batch_full": [P, P],
        "sgm_batch_step": [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double),
                           P],
        "sgm_batch_step_graph": [P, ctypes.POINTER(ctypes.c_double), P],
        "sgm_batch_set_schedule": [P, I32, I32],
        "sgm_batch_autotune": [P, ctypes.POINTER(ctypes.c_double), I32, ctypes.POINTER(I32), P],
        "sgm_autotune": [P, I32],
        "sgm_set_window_model": [P, ctypes.POINTER(ctypes.c_float), I32],
        "sgm_get_features": [P, P, I32, P, P],
        "sgm_learned_targets": [P, P, P, P, P],
        "sgm_cnn_create": [I32, I32, I32, ctypes.POINTER(P)],
        "sgm_cnn_destroy": [P],
        "sgm_cnn_set_params": [P, ctypes.POINTER(ctypes.c_float), I32],
        "sgm_cnn_get_params": [P, ctypes.POINTER(ctypes.c_float), I32],
        "sgm_cnn_forward": [P, P, I32, P, P],
        "sgm_cnn_loss": [P, P, P, P],
        "sgm_cnn_backward": [P, P],
        "sgm_cnn_get_grads": [P, ctypes.POINTER(ctypes.c_float), I32],
        "sgm_cnn_adam": [P, ctypes.c_float, P],
        "sgm_cnn_train_step": [P, P, P, I32, ctypes.c_float, P, P],
        "sgm_detect_default_params": [ctypes.POINTER(SgmDetectParams), I32, I32],
        "sgm_detector_create": [I32, I32, ctypes.POINTER(SgmDetectParams), P],
        "sgm_detector_destroy": [P],
        "sgm_detector_windows": [P, ctypes.POINTER(I64)],
        "sgm_detect": [P, P, P, P, P, P, P],
        "sgm_detect_frame": [P, P, P, P, P],
        "sgm_detector_stage": [P, I32, P, SZ, P],
        "sgm_detect_noalloc": [I32, I32, ctypes.POINTER(SgmDetectParams), P, P, P, P, P, P],
        "sgm_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.sgm_destroy.restype = None
    lib.sgm_batch_destroy.restype = None
    lib.sgm_cnn_destroy.restype = None
    lib.sgm_detector_destroy.restype = None
    lib.sgm_batch_context.restype = ctypes.c_void_p
    lib.sgm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib
