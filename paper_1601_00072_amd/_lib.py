"""ctypes declarations of include/fcm.h and the loader of the in-tree libfcm.so.

Argument marshalling only: every step of the computation runs in the HIP
library.  There is no fallback -- if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfcm.so")

FCM_OK = 0
FCM_NOT_CONVERGED = 1
FCM_RUNNING = 2
FCM_EINVAL = -1
FCM_ENOMEM = -2
FCM_EDEVICE = -3
FCM_ESTATE = -4
FCM_ENUMERIC = -5
FCM_EUNSUPPORTED = -6
FCM_EIO = -7

FCM_MAX_CLUSTERS = 8
FCM_INIT_LINSPACE = 0
FCM_INIT_GIVEN = 1
FCM_INIT_DEVICE = 2
FCM_INIT_RANDOM_U = 3
FCM_MLP_FP32 = 0
FCM_MLP_BF16 = 1
FCM_F_KAHAN_ONLY = 1 << 0
FCM_F_TIMING = 1 << 1
FCM_DRIVER_LOOP = 0
FCM_DRIVER_GRAPH = 1
FCM_DRIVER_PERSISTENT = 2
FCM_DRIVER_HISTOGRAM = 3
FCM_EXCHANGE_AUTO = 0
FCM_EXCHANGE_LEADER = 1
FCM_EXCHANGE_ALLGATHER = 2
FCM_LAUNCH_COOPERATIVE = 0
FCM_LAUNCH_RESIDENT = 1

# every symbol include/fcm.h declares
EXPORTS = (
    "fcm_init", "fcm_reset", "fcm_set_tuning", "fcm_get_tuning", "fcm_iterate", "fcm_solve", "fcm_labels",
    "fcm_centroids", "fcm_trajectory", "fcm_destroy", "fcm_strerror", "fcm_last_error", "fcm_version",
    "fcm_batch_init", "fcm_batch_set_tiling", "fcm_batch_solve", "fcm_batch_labels", "fcm_batch_trajectory",
    "fcm_batch_destroy", "fcm_mlp_param_count", "fcm_mlp_create", "fcm_mlp_get_params", "fcm_mlp_set_params",
    "fcm_mlp_forward", "fcm_mlp_loss_grad", "fcm_mlp_train", "fcm_mlp_destroy", "fcm_histogram",
    "fcm_warm_centroids", "fcm_solve_warm", "fcm_batch_set_start", "fcm_autotune", "fcm_batch_autotune",
    "fcm_confusion", "fcm_dice", "fcm_paper_solve", "fcm_solve_async", "fcm_solve_wait",
    "fcm_mlp_save", "fcm_mlp_load", "fcm_batch_solve_warm", "fcm_batch_targets", "fcm_set_wait_limit",
    "fcm_batch_timeline", "fcm_batch_set_tail_tiling", "fcm_histogram_noalloc", "fcm_batch_set_block",
)


class FcmParams(ctypes.Structure):
    _fields_ = [
        ("n_clusters", ctypes.c_int32),
        ("m", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("init", ctypes.c_int32),
        ("init_centroids", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]


class FcmTuning(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("grid", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("driver", ctypes.c_int32),
        ("graph_k", ctypes.c_int32),
        ("exchange", ctypes.c_int32),
        ("launch", ctypes.c_int32),
    ]


class FcmResult(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("passes", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("n_clusters", ctypes.c_int32),
        ("delta", ctypes.c_double),
        ("J", ctypes.c_double),
        ("centroids", ctypes.c_double * FCM_MAX_CLUSTERS),
        ("kernel_ms", ctypes.c_double),
        ("lo", ctypes.c_int32),
        ("hi", ctypes.c_int32),
    ]


class FcmPaperStats(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double),
        ("kernels_ms", ctypes.c_double),
        ("copy_ms", ctypes.c_double),
        ("host_ms", ctypes.c_double),
        ("launches", ctypes.c_int64),
    ]


class FcmTrainCfg(ctypes.Structure):
    _fields_ = [
        ("epochs", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("lr", ctypes.c_float),
        ("pad", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libfcm.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1601_00072_amd.build`")
    try:
        import torch  # noqa: F401  (brings in the HIP runtime the tensors live in)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.fcm_init.argtypes = [ctypes.POINTER(vp), vp, i64, ctypes.POINTER(FcmParams), vp]
    lib.fcm_init.restype = ctypes.c_int
    lib.fcm_reset.argtypes = [vp]
    lib.fcm_reset.restype = ctypes.c_int
    lib.fcm_set_tuning.argtypes = [vp, ctypes.POINTER(FcmTuning)]
    lib.fcm_set_tuning.restype = ctypes.c_int
    lib.fcm_get_tuning.argtypes = [vp, ctypes.POINTER(FcmTuning)]
    lib.fcm_get_tuning.restype = ctypes.c_int
    lib.fcm_iterate.argtypes = [vp, i32, ctypes.POINTER(FcmResult)]
    lib.fcm_iterate.restype = ctypes.c_int
    lib.fcm_solve.argtypes = [vp, ctypes.POINTER(FcmResult)]
    lib.fcm_solve.restype = ctypes.c_int
    lib.fcm_labels.argtypes = [vp, vp]
    lib.fcm_labels.restype = ctypes.c_int
    lib.fcm_centroids.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.fcm_centroids.restype = ctypes.c_int
    lib.fcm_trajectory.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.fcm_trajectory.restype = ctypes.c_int
    lib.fcm_destroy.argtypes = [vp]
    lib.fcm_destroy.restype = None
    lib.fcm_strerror.argtypes = [ctypes.c_int]
    lib.fcm_strerror.restype = ctypes.c_char_p
    lib.fcm_last_error.argtypes = []
    lib.fcm_last_error.restype = ctypes.c_char_p
    lib.fcm_version.argtypes = []
    lib.fcm_version.restype = ctypes.c_int
    lib.fcm_batch_init.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(i64), i32, ctypes.POINTER(FcmParams), vp]
    lib.fcm_batch_init.restype = ctypes.c_int
    lib.fcm_batch_set_tiling.argtypes = [vp, i32, i32]
    lib.fcm_batch_set_tiling.restype = ctypes.c_int
    lib.fcm_batch_set_tail_tiling.argtypes = [vp, i32, i32]
    lib.fcm_batch_set_tail_tiling.restype = ctypes.c_int
    lib.fcm_batch_set_block.argtypes = [vp, i32]
    lib.fcm_batch_set_block.restype = ctypes.c_int
    lib.fcm_batch_solve.argtypes = [vp, ctypes.POINTER(FcmResult)]
    lib.fcm_batch_solve.restype = ctypes.c_int
    lib.fcm_batch_labels.argtypes = [vp, vp]
    lib.fcm_batch_labels.restype = ctypes.c_int
    lib.fcm_batch_trajectory.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.fcm_batch_trajectory.restype = ctypes.c_int
    lib.fcm_batch_destroy.argtypes = [vp]
    lib.fcm_batch_destroy.restype = None
    f32p, f64p = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
    lib.fcm_mlp_param_count.argtypes = [i32]
    lib.fcm_mlp_param_count.restype = i32
    lib.fcm_mlp_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.c_uint64, vp]
    lib.fcm_mlp_create.restype = ctypes.c_int
    lib.fcm_mlp_get_params.argtypes = [vp, f32p]
    lib.fcm_mlp_get_params.restype = ctypes.c_int
    lib.fcm_mlp_set_params.argtypes = [vp, f32p]
    lib.fcm_mlp_set_params.restype = ctypes.c_int
    lib.fcm_mlp_forward.argtypes = [vp, vp, i32, vp, i32]
    lib.fcm_mlp_forward.restype = ctypes.c_int
    lib.fcm_mlp_loss_grad.argtypes = [vp, vp, vp, i32, f64p, f32p]
    lib.fcm_mlp_loss_grad.restype = ctypes.c_int
    lib.fcm_mlp_train.argtypes = [vp, vp, vp, i32, ctypes.POINTER(FcmTrainCfg), f64p]
    lib.fcm_mlp_train.restype = ctypes.c_int
    lib.fcm_mlp_destroy.argtypes = [vp]
    lib.fcm_mlp_destroy.restype = None
    lib.fcm_mlp_save.argtypes = [vp, ctypes.c_char_p]
    lib.fcm_mlp_save.restype = ctypes.c_int
    lib.fcm_mlp_load.argtypes = [vp, ctypes.c_char_p]
    lib.fcm_mlp_load.restype = ctypes.c_int
    lib.fcm_batch_solve_warm.argtypes = [vp, vp, i32, ctypes.POINTER(FcmResult), ctypes.POINTER(FcmResult),
                                         ctypes.POINTER(ctypes.c_uint8)]
    lib.fcm_batch_solve_warm.restype = ctypes.c_int
    lib.fcm_set_wait_limit.argtypes = [vp, ctypes.c_double, ctypes.POINTER(i32)]
    lib.fcm_set_wait_limit.restype = ctypes.c_int
    lib.fcm_batch_timeline.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]
    lib.fcm_batch_timeline.restype = ctypes.c_int
    lib.fcm_batch_targets.argtypes = [vp, i32, vp]
    lib.fcm_batch_targets.restype = ctypes.c_int
    lib.fcm_histogram.argtypes = [vp, ctypes.POINTER(i64), i32, vp, vp]
    lib.fcm_histogram.restype = ctypes.c_int
    lib.fcm_histogram_noalloc.argtypes = [vp, ctypes.POINTER(i64), i32, vp, vp]
    lib.fcm_histogram_noalloc.restype = ctypes.c_int
    lib.fcm_paper_solve.argtypes = [vp, i64, ctypes.POINTER(FcmParams), vp, ctypes.POINTER(FcmResult), vp, vp, vp,
                                    ctypes.POINTER(FcmPaperStats)]
    lib.fcm_paper_solve.restype = ctypes.c_int
    lib.fcm_solve_async.argtypes = [vp, vp]
    lib.fcm_solve_async.restype = ctypes.c_int
    lib.fcm_solve_wait.argtypes = [vp, ctypes.POINTER(FcmResult), ctypes.POINTER(i64)]
    lib.fcm_solve_wait.restype = ctypes.c_int
    lib.fcm_confusion.argtypes = [vp, vp, i64, i32, i32, vp, vp]
    lib.fcm_confusion.restype = ctypes.c_int
    lib.fcm_dice.argtypes = [vp, i32, i32, ctypes.POINTER(i32), vp, vp]
    lib.fcm_dice.restype = ctypes.c_int
    lib.fcm_warm_centroids.argtypes = [vp, vp, i32, vp, vp]
    lib.fcm_warm_centroids.restype = ctypes.c_int
    lib.fcm_solve_warm.argtypes = [vp, vp, i32, ctypes.POINTER(FcmResult), ctypes.POINTER(FcmResult),
                                   ctypes.POINTER(i32)]
    lib.fcm_solve_warm.restype = ctypes.c_int
    lib.fcm_batch_set_start.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint8)]
    lib.fcm_batch_set_start.restype = ctypes.c_int
    lib.fcm_autotune.argtypes = [vp, ctypes.c_char_p, i32, ctypes.POINTER(FcmTuning), f64p]
    lib.fcm_autotune.restype = ctypes.c_int
    lib.fcm_batch_autotune.argtypes = [vp, ctypes.c_char_p, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32), f64p]
    lib.fcm_batch_autotune.restype = ctypes.c_int
    _lib = lib
    return lib
