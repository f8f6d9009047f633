"""ctypes declarations of libpodcg (include/podcg.h).  Marshalling only."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpodcg.so")

OK, NOT_CONVERGED, RANK_REDUCED = 0, 1, 2
ERR_INVALID_ARG, ERR_HIP, ERR_OOM, ERR_NOT_SPD, ERR_NONFINITE, ERR_NO_MATRIX, ERR_SIZE = (
    -1, -2, -3, -4, -5, -6, -7)
MAX_BASIS = 32

EXPORTED = [
    "podcg_default_options", "podcg_create", "podcg_destroy", "podcg_set_matrix",
    "podcg_push_snapshot", "podcg_reset_snapshots", "podcg_build_pod", "podcg_set_basis",
    "podcg_get_basis", "podcg_get_reduced", "podcg_get_pod_spectrum", "podcg_get_format", "podcg_solve",
    "podcg_solve_plain", "podcg_solve_noalloc", "podcg_matvec", "podcg_pattern_outer", "podcg_stream_triad",
    "podcg_strerror", "podcg_last_error",
    "podcg_batch_default_options", "podcg_batch_create", "podcg_batch_destroy",
    "podcg_batch_set_options", "podcg_batch_get_options", "podcg_batch_solve", "podcg_batch_tune",
    "podcg_batch_set_values", "podcg_batch_push_build", "podcg_batch_last_error",
    "podcg_ts_default_options", "podcg_ts_enable", "podcg_ts_solve", "podcg_ts_get_state",
    "podcg_ts_set_state",
]


class Options(C.Structure):
    _fields_ = [("omega", C.c_int32), ("rank_max", C.c_int32), ("maxit", C.c_int32),
                ("check_every", C.c_int32), ("weights", C.c_int32), ("timing", C.c_int32),
                ("rank_rtol", C.c_double), ("energy", C.c_double), ("precision", C.c_int32),
                ("max_refine", C.c_int32), ("inner_rtol", C.c_double), ("spmv_grid", C.c_int32),
                ("update_grid", C.c_int32), ("dir_grid", C.c_int32), ("projection", C.c_int32),
                ("lds_solve", C.c_int32)]


class BatchOptions(C.Structure):
    _fields_ = [("slices_per_item", C.c_int32), ("rows_per_item", C.c_int32), ("grid", C.c_int32),
                ("graph_iters", C.c_int32), ("check_every", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class TsOptions(C.Structure):
    _fields_ = [("ybar", C.c_int32), ("y_trunc", C.c_int32), ("w_max", C.c_int32), ("w_cap", C.c_int32),
                ("stage2_maxit", C.c_int32), ("cap", C.c_int32), ("weights", C.c_int32),
                ("stage3_gram", C.c_int32), ("energy_y", C.c_double), ("energy_w", C.c_double),
                ("rho", C.c_double), ("stage2_factor", C.c_double), ("phi", C.c_int32),
                ("inner_maxit", C.c_int32), ("inner_rtol", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class TsStats(C.Structure):
    _fields_ = [("w", C.c_int32), ("m", C.c_int32), ("k2", C.c_int32), ("k3", C.c_int32),
                ("matvecs", C.c_int32), ("truncated", C.c_int32), ("m_next", C.c_int32),
                ("w_next", C.c_int32), ("status", C.c_int32), ("jacobi_sweeps", C.c_int32),
                ("stage1_relres", C.c_double), ("stage2_relres", C.c_double), ("relres", C.c_double),
                ("true_relres", C.c_double), ("bnorm", C.c_double), ("stage12_ms", C.c_double),
                ("stage3_ms", C.c_double), ("accum_ms", C.c_double), ("k_in", C.c_int32),
                ("projections", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("matvecs", C.c_int32), ("rank", C.c_int32),
                ("status", C.c_int32), ("stage1_relres", C.c_double), ("relres", C.c_double),
                ("true_relres", C.c_double), ("bnorm", C.c_double), ("cond_G", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("timed_iters", C.c_int32),
                ("polls", C.c_int32), ("spmv_ms", C.c_double), ("update_ms", C.c_double),
                ("dir_ms", C.c_double), ("refine_steps", C.c_int32), ("path", C.c_int32),
                ("first_inner_relres", C.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libpodcg.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1512_05820_amd.build.build()")
    L = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "podcg_default_options": ([C.POINTER(Options)], None),
        "podcg_create": ([C.POINTER(P), I64, C.POINTER(Options), P], C.c_int),
        "podcg_destroy": ([P], C.c_int),
        "podcg_set_matrix": ([P, I64, P, P, P], C.c_int),
        "podcg_push_snapshot": ([P, P], C.c_int),
        "podcg_reset_snapshots": ([P], C.c_int),
        "podcg_build_pod": ([P, C.POINTER(I32)], C.c_int),
        "podcg_set_basis": ([P, P, I32], C.c_int),
        "podcg_get_basis": ([P, P, C.POINTER(I32)], C.c_int),
        "podcg_get_reduced": ([P, P, P, C.POINTER(I32)], C.c_int),
        "podcg_get_pod_spectrum": ([P, P, C.POINTER(I32)], C.c_int),
        "podcg_get_format": ([P, P], C.c_int),
        "podcg_solve": ([P, P, P, D, C.POINTER(Stats)], C.c_int),
        "podcg_solve_plain": ([P, P, P, D, C.POINTER(Stats)], C.c_int),
        "podcg_solve_noalloc": ([P, P, P, D, C.POINTER(Stats)], C.c_int),
        "podcg_matvec": ([P, P, P], C.c_int),
        "podcg_pattern_outer": ([P, P, P, D, P], C.c_int),
        "podcg_stream_triad": ([P, P, P, P, I64, D, I32, C.POINTER(D)], C.c_int),
        "podcg_strerror": ([C.c_int], C.c_char_p),
        "podcg_last_error": ([P], C.c_char_p),
        "podcg_batch_default_options": ([C.POINTER(BatchOptions)], None),
        "podcg_batch_create": ([C.POINTER(P), I32, C.POINTER(P), C.POINTER(BatchOptions)], C.c_int),
        "podcg_batch_destroy": ([P], C.c_int),
        "podcg_batch_set_options": ([P, C.POINTER(BatchOptions)], C.c_int),
        "podcg_batch_get_options": ([P, C.POINTER(BatchOptions)], C.c_int),
        "podcg_batch_solve": ([P, C.POINTER(P), C.POINTER(P), C.POINTER(D), I32, C.POINTER(Stats)],
                              C.c_int),
        "podcg_batch_tune": ([P, C.POINTER(P), C.POINTER(P), I32, C.POINTER(BatchOptions),
                             C.POINTER(D)], C.c_int),
        "podcg_batch_set_values": ([P, C.POINTER(C.c_int64), C.POINTER(P)], C.c_int),
        "podcg_batch_push_build": ([P, C.POINTER(P)], C.c_int),
        "podcg_batch_last_error": ([P], C.c_char_p),
        "podcg_ts_default_options": ([C.POINTER(TsOptions)], None),
        "podcg_ts_enable": ([P, C.POINTER(TsOptions)], C.c_int),
        "podcg_ts_solve": ([P, P, P, D, C.POINTER(TsStats)], C.c_int),
        "podcg_ts_get_state": ([P, P, C.POINTER(I32), P, C.POINTER(I32)], C.c_int),
        "podcg_ts_set_state": ([P, P, I32, P, I32, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L
