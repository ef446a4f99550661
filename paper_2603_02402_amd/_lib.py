"""ctypes binding of ``librsc.so`` (argument marshalling only).

Every call takes torch tensors that live on the current HIP device and
enqueues the library's kernels on torch's current stream.  Nothing here
computes: there is no CPU fallback, and importing this module on a machine
without the built library raises.
"""

from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsc.so")

RSC_OK = 0
STATUS_NAMES = {
    0: "RSC_OK",
    -1: "RSC_ERR_INVALID_ARG",
    -2: "RSC_ERR_HIP",
    -3: "RSC_ERR_NO_MEMORY",
    -4: "RSC_ERR_CAPACITY",
    -5: "RSC_ERR_OVERFLOW",
    -6: "RSC_ERR_UNSUPPORTED",
    -7: "RSC_ERR_WORKSPACE",
    -8: "RSC_ERR_BAD_GRAPH",
}
RSC_FP32, RSC_BF16, RSC_FP8_E4M3 = 0, 1, 2
RSC_EUCLIDEAN, RSC_COSINE = 0, 1
RSC_BATCH_POLICIES = 6
RSC_BATCH_TRIALS = 32

# Every symbol include/rsc.h declares, with (restype, argtypes).
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_SZ = ctypes.c_size_t


class KnnOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("screen", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("fp8_residual", ctypes.c_int32)]


class KnnStats(ctypes.Structure):
    _fields_ = [("escalated_rows", ctypes.c_int64), ("rescanned_rows", ctypes.c_int64),
                ("max_err_ratio", ctypes.c_float),
                ("max_ref_norm", ctypes.c_float)]


class LeidenStats(ctypes.Structure):
    _fields_ = [("quality", ctypes.c_double), ("n_communities", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("move_bytes", ctypes.c_int64)]


class RoutedStats(ctypes.Structure):
    _fields_ = [("routed_rows", ctypes.c_int64), ("low_mass_rows", ctypes.c_int64),
                ("uncertified_rows", ctypes.c_int64), ("escalated_rows", ctypes.c_int64),
                ("rescanned_rows", ctypes.c_int64), ("mean_probed_rows", ctypes.c_double),
                ("mean_screened_rows", ctypes.c_double)]


_U64 = ctypes.c_uint64
_F = ctypes.c_float

SIGNATURES = {
    "rsc_abi_version": (ctypes.c_int, []),
    "rsc_last_error": (ctypes.c_char_p, []),
    "rsc_knn_workspace_bytes": (_SZ, [_I64, _I64, _I32, _I32, _P]),
    "rsc_knn": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "rsc_knn_opt": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _P, _P, _P, _SZ, _P]),
    "rsc_knn_ex": (ctypes.c_int, [_P, _I64, _P, _I64, _I32, _I32, _P, _P, _P, _P, _SZ, _P]),
    "rsc_knn_read_escalated": (ctypes.c_int, [_P, _SZ, _I64, _I64, _I32, _I32, _P, _I32, _P, _I64, _P, _P]),
    "rsc_knn_read_stats": (ctypes.c_int, [_P, _SZ, _P, _P]),
    "rsc_knn_batched_workspace_bytes": (_SZ, [_P, _I32, _I32, _I32]),
    "rsc_knn_batched": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "rsc_knn_batched_autotune": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P, _SZ, _P, _P, _P]),
    "rsc_batch_policy_name": (ctypes.c_char_p, [_I32]),
    "rsc_batch_trial_name": (ctypes.c_char_p, [_I32]),
    "rsc_connectivities_workspace_bytes": (_SZ, [_I64, _I32]),
    "rsc_connectivities": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P, _I64, _P, _P, _P, _P, _SZ, _P]),
    "rsc_connectivities_noalloc_max_bytes": (_SZ, []),
    "rsc_connectivities_noalloc": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P, _I64, _P, _P, _P, _P]),
    "rsc_connectivities_batched_workspace_bytes": (_SZ, [_P, _I32, _I32]),
    "rsc_connectivities_batched": (ctypes.c_int, [_P, _P, _P, _I32, _I32, _P, _P, _P, _I64, _P, _P, _SZ, _P]),
    "rsc_partition_kmeans_workspace_bytes": (_SZ, [_I64, _I32, _I32]),
    "rsc_partition_kmeans": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "rsc_partition_labels": (ctypes.c_int, [_P, _I64, _I32, _P, _I64, _P, _P]),
    "rsc_partition_lists_workspace_bytes": (_SZ, [_I32]),
    "rsc_partition_lists": (ctypes.c_int, [_P, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "rsc_router_create": (ctypes.c_int, [_P, _I32, _I32, _I32, _U64]),
    "rsc_router_destroy": (None, [_P]),
    "rsc_router_info": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "rsc_router_train_workspace_bytes": (_SZ, [_P, _I32, _I64]),
    "rsc_router_train": (ctypes.c_int, [_P, _P, _I64, _P, _I32, _I32, _I32, _F, _P, _P, _SZ, _P]),
    "rsc_router_gradients_workspace_bytes": (_SZ, [_P, _I64]),
    "rsc_router_gradients": (ctypes.c_int, [_P, _P, _I64, _P, _I32, _P, _P, _P, _SZ, _P]),
    "rsc_router_infer_workspace_bytes": (_SZ, [_P]),
    "rsc_router_logits": (ctypes.c_int, [_P, _P, _I64, _P, _P, _SZ, _P]),
    "rsc_router_probe": (ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "rsc_router_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "rsc_router_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "rsc_knn_probed_workspace_bytes": (_SZ, [_I64, _I32, _I32, _I32, _I32]),
    "rsc_knn_probed": (ctypes.c_int, [_P, _I64, _I32, _I32, _P, _P, _I32, _P, _I32, _P, _P, _P, _P, _P, _P, _SZ,
                                      _P]),
    "rsc_knn_routed_workspace_bytes": (_SZ, [_P, _I64, _I32, _I32, _I32, _I32]),
    "rsc_knn_routed": (ctypes.c_int, [_P, _P, _I64, _I32, _I32, _P, _P, _I32, _I32, _F, _P, _P, _P, _P, _P, _SZ,
                                      _P]),
    "rsc_edistance_groups_workspace_bytes": (_SZ, [_I64, _I64]),
    "rsc_edistance_groups": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _P, _SZ, _P]),
    "rsc_edistance_sums_workspace_bytes": (_SZ, [_I64, _I64, _I64, _I32]),
    "rsc_edistance_sums": (ctypes.c_int, [_P, _I64, _I32, _P, _I64, _P, _P, _I64, _P, _P, _SZ, _P]),
    "rsc_edistance_pairwise_workspace_bytes": (_SZ, [_I64, _I64, _I32]),
    "rsc_edistance_pairwise": (ctypes.c_int, [_P, _I64, _I32, _P, _I64, _P, _P, _P, _P, _SZ, _P]),
    "rsc_edistance_onesided_workspace_bytes": (_SZ, [_I64, _I64, _I32]),
    "rsc_edistance_onesided": (ctypes.c_int, [_P, _I64, _I32, _P, _I64, _P, _I64, _P, _P, _SZ, _P]),
    "rsc_pca_workspace_bytes": (_SZ, [_I64, _I32, _I32]),
    "rsc_pca_covariance": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "rsc_pca": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "rsc_leiden_workspace_bytes": (_SZ, [_I64, _I64]),
    "rsc_leiden": (ctypes.c_int, [_P, _P, _P, _I64, _I64, ctypes.c_double, _P, _P, _P, _SZ, _P]),
    "rsc_umap_workspace_bytes": (_SZ, [_I64, _I64, _I32, _I32]),
    "rsc_umap_layout": (ctypes.c_int, [_P, _P, _P, _I64, _I64, _I32, _P, _I32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _I32, _U64, _P, _SZ, _P]),
    "rsc_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "rsc_profile_reset": (ctypes.c_int, []),
    "rsc_profile_get": (ctypes.c_int, [ctypes.c_char_p, _P, _P]),
}

_lock = threading.Lock()
_lib = None


class RscError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


def load(path: str = LIB_PATH):
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise ImportError(
                    f"{path} is missing: build it with `python -m paper_2603_02402_amd.build` "
                    "(the kNN graph has no CPU fallback)")
            lib = ctypes.CDLL(path)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(status: int) -> None:
    if status != RSC_OK:
        msg = load().rsc_last_error()
        raise RscError(status, msg.decode() if msg else "")
