"""ctypes declarations of the C ABI in include/bt_si_sq.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbtsisq.so")

BT_OK, BT_ERR_INVALID, BT_ERR_OOM, BT_ERR_SINGULAR, BT_ERR_HIP, BT_ERR_STATE, BT_ERR_TOLERANCE = range(7)
BT_FP64, BT_MIXED = 0, 1
BT_DIAG_ONLY, BT_PLAIN, BT_GRAPH, BT_SIGMA_ANTIHERMITIAN, BT_FUSED = 0x1, 0x2, 0x4, 0x8, 0x10
STATUS_NAMES = {0: "BT_OK", 1: "BT_ERR_INVALID", 2: "BT_ERR_OOM", 3: "BT_ERR_SINGULAR",
                4: "BT_ERR_HIP", 5: "BT_ERR_STATE", 6: "BT_ERR_TOLERANCE"}

BT_TILE_SHAPES = 3
BT_TUNE_SIZE_CLASSES = 6
BT_TUNE_WORK_CLASSES = 14
BT_TUNE_ENTRIES = 2 * BT_TUNE_SIZE_CLASSES * BT_TUNE_WORK_CLASSES

EXPORTED = [
    "bt_si_sq_workspace_bytes", "bt_si_sq_partition_bounds", "bt_si_sq_flops",
    "bt_si_sq_create", "bt_si_sq_factor", "bt_si_sq_selected_solve", "bt_si_sq_solve",
    "bt_si_sq_sync", "bt_si_sq_destroy", "bt_si_sq_last_error", "bt_si_sq_last_launch_count",
    "bt_si_sq_profile", "bt_si_sq_profile_stats",
    "bt_si_sq_batch_workspace_bytes", "bt_si_sq_batch_create", "bt_si_sq_batch_create_in",
    "bt_si_sq_batch_solve",
    "bt_si_sq_batch_count", "bt_si_sq_batch_selected_solve",
    "bt_si_sq_autotune", "bt_si_sq_tune_table",
    "bt_si_sq_diag_gemm", "bt_si_sq_diag_inverse", "bt_si_sq_diag_schedule",
    "bt_si_sq_diag_inverse_noalloc", "bt_si_sq_diag_inverse_noalloc_max_bytes",
]

KERNEL_NAMES = {0: "product_fp64", 1: "product_mixed", 2: "inv_panel", 3: "inv_init",
                4: "inv_finish", 5: "sum", 6: "norm", 7: "fused"}


class bt_desc(C.Structure):
    _fields_ = [("n", C.c_int32), ("b", C.c_int32), ("a", C.c_int32),
                ("partitions", C.c_int32), ("part_bounds", C.POINTER(C.c_int32)),
                ("precision", C.c_int32), ("tol", C.c_double), ("flags", C.c_uint32),
                ("block_sizes", C.POINTER(C.c_int32)), ("reduced_parts", C.c_int32)]


class bt_blocks(C.Structure):
    _fields_ = [("diag", C.c_void_p), ("upper", C.c_void_p), ("lower", C.c_void_p),
                ("arrow_right", C.c_void_p), ("arrow_bottom", C.c_void_p), ("tip", C.c_void_p)]


class bt_kernel_stat(C.Structure):
    _fields_ = [("kind", C.c_int32), ("launches", C.c_int32), ("total_ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


class BTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class BTToleranceError(BTError):
    """BT_ERR_TOLERANCE: the FP64 re-run of a mixed-precision solve still has an
    error estimate above tol.  The results are written; err and fallback hold
    the estimates and fallback flags the call returned."""

    def __init__(self, msg: str, err, fallback):
        super().__init__(BT_ERR_TOLERANCE, msg)
        self.err = err
        self.fallback = fallback


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} missing "
                          "(run python -m paper_2601_04904_amd.build)")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    L.bt_si_sq_workspace_bytes.argtypes = [C.POINTER(bt_desc)]
    L.bt_si_sq_workspace_bytes.restype = C.c_size_t
    L.bt_si_sq_partition_bounds.argtypes = [C.POINTER(bt_desc), C.POINTER(C.c_int32)]
    L.bt_si_sq_partition_bounds.restype = C.c_int
    L.bt_si_sq_flops.argtypes = [C.POINTER(bt_desc), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.bt_si_sq_flops.restype = C.c_int
    L.bt_si_sq_create.argtypes = [C.POINTER(bt_desc), C.c_void_p, C.POINTER(H)]
    L.bt_si_sq_create.restype = C.c_int
    L.bt_si_sq_factor.argtypes = [H, C.POINTER(bt_blocks), C.POINTER(bt_blocks)]
    L.bt_si_sq_factor.restype = C.c_int
    L.bt_si_sq_selected_solve.argtypes = [H, C.POINTER(bt_blocks), C.POINTER(bt_blocks),
                                          C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.bt_si_sq_selected_solve.restype = C.c_int
    L.bt_si_sq_solve.argtypes = [H, C.POINTER(bt_blocks), C.POINTER(bt_blocks), C.POINTER(bt_blocks),
                                 C.POINTER(bt_blocks), C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.bt_si_sq_solve.restype = C.c_int
    L.bt_si_sq_sync.argtypes = [H]
    L.bt_si_sq_sync.restype = C.c_int
    L.bt_si_sq_destroy.argtypes = [H]
    L.bt_si_sq_destroy.restype = C.c_int
    L.bt_si_sq_last_error.argtypes = [H]
    L.bt_si_sq_last_error.restype = C.c_char_p
    L.bt_si_sq_last_launch_count.argtypes = [H]
    L.bt_si_sq_last_launch_count.restype = C.c_int32
    L.bt_si_sq_profile.argtypes = [H, C.c_int32]
    L.bt_si_sq_profile.restype = C.c_int
    L.bt_si_sq_profile_stats.argtypes = [H, C.POINTER(bt_kernel_stat), C.c_int32,
                                         C.POINTER(C.c_int32)]
    L.bt_si_sq_profile_stats.restype = C.c_int
    L.bt_si_sq_batch_workspace_bytes.argtypes = [C.c_int32, C.POINTER(bt_desc)]
    L.bt_si_sq_batch_workspace_bytes.restype = C.c_size_t
    L.bt_si_sq_batch_create.argtypes = [C.c_int32, C.POINTER(bt_desc), C.c_void_p, C.POINTER(H)]
    L.bt_si_sq_batch_create.restype = C.c_int
    L.bt_si_sq_batch_create_in.argtypes = [C.c_int32, C.POINTER(bt_desc), C.c_void_p, C.c_void_p,
                                           C.c_size_t, C.POINTER(H)]
    L.bt_si_sq_batch_create_in.restype = C.c_int
    L.bt_si_sq_batch_solve.argtypes = [H, C.POINTER(bt_blocks), C.POINTER(bt_blocks),
                                       C.POINTER(bt_blocks), C.POINTER(bt_blocks),
                                       C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.bt_si_sq_batch_solve.restype = C.c_int
    L.bt_si_sq_batch_selected_solve.argtypes = [H, C.POINTER(bt_blocks), C.POINTER(bt_blocks),
                                                C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.bt_si_sq_batch_selected_solve.restype = C.c_int
    L.bt_si_sq_batch_count.argtypes = [H]
    L.bt_si_sq_batch_count.restype = C.c_int32
    L.bt_si_sq_autotune.argtypes = [C.c_void_p, C.c_char_p, C.c_size_t]
    L.bt_si_sq_autotune.restype = C.c_int
    L.bt_si_sq_tune_table.argtypes = [C.POINTER(C.c_int32), C.c_int32]
    L.bt_si_sq_tune_table.restype = C.c_int
    dp = C.POINTER(C.c_double)
    L.bt_si_sq_diag_gemm.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, C.c_void_p, C.c_int32,
                                     C.c_int32, C.c_void_p, C.c_int32, C.c_int32, dp, C.c_void_p,
                                     C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_void_p]
    L.bt_si_sq_diag_gemm.restype = C.c_int
    L.bt_si_sq_diag_inverse.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                        C.POINTER(C.c_int32), C.c_void_p]
    L.bt_si_sq_diag_inverse.restype = C.c_int
    L.bt_si_sq_diag_inverse_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                                C.POINTER(C.c_int32), C.c_void_p]
    L.bt_si_sq_diag_inverse_noalloc.restype = C.c_int
    L.bt_si_sq_diag_inverse_noalloc_max_bytes.argtypes = []
    L.bt_si_sq_diag_inverse_noalloc_max_bytes.restype = C.c_size_t
    L.bt_si_sq_diag_schedule.argtypes = [C.POINTER(bt_desc), C.c_char_p, C.c_size_t]
    L.bt_si_sq_diag_schedule.restype = C.c_size_t
    _lib = L
    return L


def make_desc(n: int, b: int, a: int = 0, partitions: int = 1, bounds=None,
              precision: int = BT_FP64, tol: float = 1e-4, flags: int = 0, sizes=None,
              reduced_parts: int = 0):
    """bt_desc; sizes: per-block sizes (then b is ignored) or None;
    reduced_parts: parts of the reduced system's recursive partitioned solve
    (0: the default two)."""
    d = bt_desc()
    d.n, d.b, d.a, d.partitions = n, b, a, partitions
    keep = None
    if bounds is not None:
        keep = (C.c_int32 * len(bounds))(*bounds)
        d.part_bounds = C.cast(keep, C.POINTER(C.c_int32))
    keep_sizes = None
    if sizes is not None:
        if len(sizes) != n:
            raise ValueError(f"sizes has {len(sizes)} entries, n = {n}")
        keep_sizes = (C.c_int32 * n)(*[int(v) for v in sizes])
        d.block_sizes = C.cast(keep_sizes, C.POINTER(C.c_int32))
    d.precision, d.tol, d.flags = precision, tol, flags
    d.reduced_parts = reduced_parts
    d._keep = (keep, keep_sizes)  # keep the arrays alive with the descriptor
    return d


def check_tol(status: int, handle, err, fallback):
    """check(), except that BT_ERR_TOLERANCE raises BTToleranceError with the
    call's estimates and fallback flags attached."""
    if status == BT_ERR_TOLERANCE:
        msg = lib().bt_si_sq_last_error(handle)
        raise BTToleranceError(msg.decode() if msg else "", err, fallback)
    check(status, handle)


def check(status: int, handle=None):
    if status != BT_OK:
        msg = lib().bt_si_sq_last_error(handle)
        raise BTError(status, msg.decode() if msg else "")
