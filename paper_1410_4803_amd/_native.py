"""ctypes binding of libpg.so: argument marshalling only.

Every statistic is computed by the library's HIP kernels; this module
allocates device buffers with PyTorch, passes raw pointers and the current
HIP stream, and turns status codes into exceptions.  There is no fallback: if
libpg.so is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpg.so")

PG_OK, PG_EINVAL, PG_ENOMEM, PG_EDEVICE, PG_EUNSUPPORTED = 0, -1, -2, -3, -4
PG_TRI_UPPER, PG_FULL = 0, 1
PG_PATH_AUTO, PG_PATH_POPC, PG_PATH_MFMA, PG_PATH_SPARSE = 0, 1, 2, 3

LAYOUTS = {"tri": PG_TRI_UPPER, "full": PG_FULL}
PATHS = {"auto": PG_PATH_AUTO, "popc": PG_PATH_POPC, "mfma": PG_PATH_MFMA,
         "sparse": PG_PATH_SPARSE}

# ABI symbols (include/pg.h)
SYMBOLS = ("pg_status_str", "pg_last_error", "pg_version", "pg_profile_events",
           "pg_ibs_workspace_bytes", "pg_ibs_matrix", "pg_ld_workspace_bytes", "pg_ld_window",
           "pg_prune_workspace_bytes", "pg_ld_prune", "pg_grm_workspace_bytes", "pg_grm_matrix",
           "pg_ibs_distance", "pg_cluster_workspace_bytes", "pg_ibs_cluster", "pg_peak_rates",
           "pg_batch_plan", "pg_batch_workspace_bytes", "pg_batch_tiles", "pg_batch_upload",
           "pg_batch_launch", "pg_plan_free", "pg_batch_capture", "pg_graph_launch",
           "pg_graph_destroy", "pg_ibs_matrix_noalloc", "pg_noalloc_scratch_bytes", "pg_resolve_path",
           "pg_ibs_similarity", "pg_genome_workspace_bytes", "pg_ibs_genome")
PG_KIND_IBS, PG_KIND_LD = 0, 1
PG_COUNTS_U16 = 0x100    # out_layout flag: 16-bit IBS counts

LD_PAIR = np.dtype([("a", "<i4"), ("b", "<i4"), ("n", "<i8"), ("sx", "<i8"), ("sy", "<i8"),
                    ("sxx", "<i8"), ("syy", "<i8"), ("sxy", "<i8"), ("r2", "<f8")])
assert LD_PAIR.itemsize == 64

MERGE = np.dtype([("a", "<i4"), ("b", "<i4"), ("height", "<f8")])
assert MERGE.itemsize == 16


class PgError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {status_str(status)} ({status}): {detail}")
        self.status = status


class Genotypes(ctypes.Structure):
    """Mirror of pg_genotypes."""
    _fields_ = [("bed", ctypes.c_void_p), ("n_samples", ctypes.c_int64),
                ("n_variants", ctypes.c_int64), ("bytes_per_variant", ctypes.c_int64),
                ("missing_mask", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    """Mirror of pg_problem."""
    _fields_ = [("kind", ctypes.c_int), ("path", ctypes.c_int), ("g", Genotypes),
                ("sample_idx", ctypes.c_void_p), ("n_sel", ctypes.c_int64),
                ("v_begin", ctypes.c_int64), ("v_end", ctypes.c_int64),
                ("out_layout", ctypes.c_int), ("ibs0", ctypes.c_void_p),
                ("ibs1", ctypes.c_void_p), ("ibs2", ctypes.c_void_p), ("nonmiss", ctypes.c_void_p),
                ("window", ctypes.c_int32), ("r2_min", ctypes.c_double), ("out", ctypes.c_void_p),
                ("capacity", ctypes.c_int64), ("n_out", ctypes.c_void_p)]


assert ctypes.sizeof(Problem) == 160

_lib = None


def load():
    """Load libpg.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1410_4803_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    i64, i32, dbl, p, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    gp = ctypes.POINTER(Genotypes)
    lib.pg_status_str.argtypes = [ctypes.c_int]
    lib.pg_status_str.restype = ctypes.c_char_p
    lib.pg_last_error.argtypes = []
    lib.pg_last_error.restype = ctypes.c_char_p
    lib.pg_version.argtypes = []
    lib.pg_version.restype = ctypes.c_int
    lib.pg_profile_events.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    lib.pg_profile_events.restype = ctypes.c_int
    lib.pg_ibs_workspace_bytes.argtypes = [gp, i64, i64, i64, ctypes.c_int, ctypes.POINTER(sz)]
    lib.pg_ibs_workspace_bytes.restype = ctypes.c_int
    lib.pg_ibs_matrix.argtypes = [gp, p, i64, i64, i64, ctypes.c_int, ctypes.c_int, p, p, p, p, p,
                                  sz, p]
    lib.pg_ibs_matrix.restype = ctypes.c_int
    lib.pg_ibs_matrix_noalloc.argtypes = [gp, p, i64, i64, i64, ctypes.c_int, ctypes.c_int, p, p,
                                          p, p, p]
    lib.pg_ibs_matrix_noalloc.restype = ctypes.c_int
    lib.pg_noalloc_scratch_bytes.argtypes = [ctypes.POINTER(sz)]
    lib.pg_noalloc_scratch_bytes.restype = ctypes.c_int
    lib.pg_resolve_path.argtypes = [ctypes.c_int, i64, i64, i32, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)]
    lib.pg_resolve_path.restype = ctypes.c_int
    lib.pg_ld_workspace_bytes.argtypes = [gp, i64, i64, i64, i32, ctypes.c_int, ctypes.POINTER(sz)]
    lib.pg_ld_workspace_bytes.restype = ctypes.c_int
    lib.pg_ld_window.argtypes = [gp, p, i64, i64, i64, i32, dbl, p, i64, p, ctypes.c_int, p, sz, p]
    lib.pg_ld_window.restype = ctypes.c_int
    lib.pg_prune_workspace_bytes.argtypes = [gp, i64, i64, i64, i32, ctypes.c_int,
                                             ctypes.POINTER(sz)]
    lib.pg_prune_workspace_bytes.restype = ctypes.c_int
    lib.pg_ld_prune.argtypes = [gp, p, i64, i64, i64, i32, i32, dbl, p, p, ctypes.c_int, p, sz, p]
    lib.pg_ld_prune.restype = ctypes.c_int
    lib.pg_grm_workspace_bytes.argtypes = [gp, i64, i64, i64, ctypes.POINTER(sz)]
    lib.pg_grm_workspace_bytes.restype = ctypes.c_int
    lib.pg_grm_matrix.argtypes = [gp, p, i64, i64, i64, ctypes.c_int, ctypes.c_int, p, p, p, sz,
                                  p]
    lib.pg_grm_matrix.restype = ctypes.c_int
    lib.pg_ibs_distance.argtypes = [p, p, p, i64, p, p]
    lib.pg_ibs_distance.restype = ctypes.c_int
    lib.pg_cluster_workspace_bytes.argtypes = [i64, ctypes.POINTER(sz)]
    lib.pg_cluster_workspace_bytes.restype = ctypes.c_int
    lib.pg_ibs_cluster.argtypes = [p, p, p, i64, p, p, sz, p]
    lib.pg_ibs_cluster.restype = ctypes.c_int
    lib.pg_ibs_similarity.argtypes = [p, p, p, i64, p, p]
    lib.pg_ibs_similarity.restype = ctypes.c_int
    lib.pg_genome_workspace_bytes.argtypes = [gp, i64, i64, i64, ctypes.POINTER(sz)]
    lib.pg_genome_workspace_bytes.restype = ctypes.c_int
    lib.pg_ibs_genome.argtypes = [gp, p, i64, i64, i64, p, p, p, i64, p, p, p, p, p, sz, p]
    lib.pg_ibs_genome.restype = ctypes.c_int
    lib.pg_peak_rates.argtypes = [p, sz, p]
    lib.pg_peak_rates.restype = ctypes.c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.pg_batch_plan.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, pp]
    lib.pg_batch_plan.restype = ctypes.c_int
    lib.pg_batch_workspace_bytes.argtypes = [p, ctypes.POINTER(sz)]
    lib.pg_batch_workspace_bytes.restype = ctypes.c_int
    lib.pg_batch_tiles.argtypes = [p, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int)]
    lib.pg_batch_tiles.restype = ctypes.c_int
    lib.pg_batch_upload.argtypes = [p, p, sz, p]
    lib.pg_batch_upload.restype = ctypes.c_int
    lib.pg_batch_launch.argtypes = [p, p, sz, p]
    lib.pg_batch_launch.restype = ctypes.c_int
    lib.pg_plan_free.argtypes = [p]
    lib.pg_plan_free.restype = None
    lib.pg_batch_capture.argtypes = [p, p, sz, p, pp]
    lib.pg_batch_capture.restype = ctypes.c_int
    lib.pg_graph_launch.argtypes = [p, p]
    lib.pg_graph_launch.restype = ctypes.c_int
    lib.pg_graph_destroy.argtypes = [p]
    lib.pg_graph_destroy.restype = ctypes.c_int
    _lib = lib
    return lib


def status_str(status: int) -> str:
    return load().pg_status_str(status).decode()


def last_error() -> str:
    return load().pg_last_error().decode()


def check(status: int, where: str) -> None:
    if status != PG_OK:
        raise PgError(status, where, last_error())
