"""ctypes declarations of the C ABI in include/sparsink.h.

Loads ``libsparsink.so`` from this package directory.  torch is imported
first so that the HIP runtime torch already uses (same soname) is the one the
library binds to; device pointers and streams then cross the boundary freely.
There is no fallback: if the library is missing this import fails.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, \
    c_uint32, c_uint64, c_void_p

import torch  # noqa: F401  (binds the process to torch's HIP runtime first)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsparsink.so")

SS_OK = 0
SS_NOT_CONVERGED = 1
SS_E_INVALID_ARG = -1
SS_E_HIP = -2
SS_E_WORKSPACE = -3
SS_E_NONFINITE = -4
SS_E_EMPTY = -5
SS_E_CAPACITY = -6

PRECISION = {"f64": 0, "f32": 1, "f32_log": 2}
COST = {"maxnorm": 0, "plain": 1, "wfr": 2, "euclid": 3}
STOP = {"marginal": 0, "delta": 1}
EMPTY = {"auto": 0, "renormalize": 1, "zero": 2, "fail": 3}


class SsProblem(ctypes.Structure):
    _fields_ = [("n", c_int64), ("m", c_int64), ("d", c_int32), ("problem_index", c_uint32),
                ("x", c_void_p), ("y", c_void_p), ("a", c_void_p), ("b", c_void_p)]


class SsOptions(ctypes.Structure):
    _fields_ = [("eps", c_double), ("lambda_", c_double), ("s", c_double), ("tol", c_double),
                ("seed", c_uint64), ("max_iter", c_int32), ("precision", c_int32),
                ("cost", c_int32), ("stop_rule", c_int32), ("empty_policy", c_int32),
                ("block_threads", c_int32), ("graph_iters", c_int32), ("reserved0", c_int32),
                ("init_log_u", c_void_p), ("init_log_v", c_void_p), ("u_out", c_void_p),
                ("v_out", c_void_p), ("err_hist", c_void_p), ("shrink", c_double),
                ("eta", c_double)]


class SsResult(ctypes.Structure):
    _fields_ = [("estimate", c_double), ("transport", c_double), ("neg_entropy", c_double),
                ("kl_a", c_double), ("kl_b", c_double), ("sparse_objective", c_double),
                ("marginal_err", c_double), ("cmax", c_double), ("z_norm", c_double),
                ("dropped_mass_a", c_double), ("dropped_mass_b", c_double),
                ("nnz", c_int64), ("empty_rows", c_int64), ("empty_cols", c_int64),
                ("iters", c_int32), ("status", c_int32),
                ("t_prep_ms", c_float), ("t_sample_ms", c_float), ("t_iter_ms", c_float),
                ("t_obj_ms", c_float), ("warm_start", c_int32), ("reserved", c_int32)]


class SsSparse(ctypes.Structure):
    _fields_ = [("mask", c_void_p), ("row_ptr", c_void_p), ("col_idx", c_void_p),
                ("val", c_void_p), ("col_ptr", c_void_p), ("row_idx", c_void_p),
                ("val_t", c_void_p), ("row_fac", c_void_p), ("col_fac", c_void_p),
                ("capacity", c_int64), ("nnz", c_int64), ("cmax", c_double),
                ("z_norm", c_double), ("z_in", c_double)]


class SsBatch(ctypes.Structure):
    _fields_ = [("count", c_int32), ("d", c_int32), ("n", c_void_p), ("m", c_void_p),
                ("s", c_void_p), ("problem_index", c_void_p), ("x", c_void_p), ("y", c_void_p),
                ("a", c_void_p), ("b", c_void_p)]


class SsSchedule(ctypes.Structure):
    _fields_ = [("lanes_per_line", c_int32), ("block_threads", c_int32)]


BATCH_MAX_SIDE = 4096
NOALLOC_SCRATCH_BYTES = 32 << 20
MLP_PARAMS = 133889


class SsMlp(ctypes.Structure):
    _fields_ = [("params", c_void_p), ("bf16", c_void_p), ("w2t", c_void_p), ("adam_m", c_void_p),
                ("adam_v", c_void_p), ("step", c_int32), ("reserved", c_int32)]


class SsIbpProblem(ctypes.Structure):
    _fields_ = [("n", c_int64), ("d", c_int32), ("count", c_int32), ("x", c_void_p),
                ("b", c_void_p), ("w", c_void_p)]


class SsIbpResult(ctypes.Structure):
    _fields_ = [("err", c_double), ("cmax", c_double), ("nnz", c_int64),
                ("empty_rows", c_int64), ("empty_cols", c_int64), ("iters", c_int32),
                ("status", c_int32), ("t_sample_ms", c_float), ("t_iter_ms", c_float)]


IBP_MAX_MEASURES = 64


class SsDivergence(ctypes.Structure):
    _fields_ = [("value", c_double), ("value_sparse", c_double), ("ot_xy", c_double),
                ("ot_xx", c_double), ("ot_yy", c_double), ("sparse_xy", c_double),
                ("sparse_xx", c_double), ("sparse_yy", c_double), ("nnz", c_int64),
                ("iters_xy", c_int32), ("iters_xx", c_int32), ("iters_yy", c_int32),
                ("status", c_int32)]


# Every symbol the header declares, with its signature.
SIGNATURES = {
    "ss_workspace_size": (c_int, [POINTER(SsProblem), POINTER(SsOptions), POINTER(c_size_t)]),
    "ss_sample": (c_int, [POINTER(SsProblem), POINTER(SsOptions), POINTER(SsSparse), c_void_p,
                          c_size_t, c_void_p]),
    "spar_sink_ot": (c_int, [POINTER(SsProblem), POINTER(SsOptions), c_void_p, c_size_t,
                             c_void_p, POINTER(SsResult)]),
    "spar_sink_uot": (c_int, [POINTER(SsProblem), POINTER(SsOptions), c_void_p, c_size_t,
                              c_void_p, POINTER(SsResult)]),
    "spar_sink_ot_noalloc": (c_int, [POINTER(SsProblem), POINTER(SsOptions), c_void_p,
                                     POINTER(SsResult)]),
    "dense_sinkhorn": (c_int, [POINTER(SsProblem), POINTER(SsOptions), c_void_p, c_size_t,
                               c_void_p, POINTER(SsResult)]),
    "ss_time_iterations": (c_int, [POINTER(SsProblem), POINTER(SsOptions), c_void_p, c_size_t,
                                   c_void_p, c_int32, POINTER(c_double)]),
    "ss_batch_workspace_size": (c_int, [POINTER(SsBatch), POINTER(SsOptions), POINTER(c_size_t)]),
    "spar_sink_batched": (c_int, [POINTER(SsBatch), POINTER(SsOptions), POINTER(SsSchedule),
                                  c_void_p, c_size_t, c_void_p, POINTER(SsResult)]),
    "ss_batch_learned_workspace_size": (c_int, [POINTER(SsBatch), POINTER(SsOptions),
                                                POINTER(c_size_t)]),
    "spar_sink_batched_learned": (c_int, [POINTER(SsBatch), POINTER(SsOptions),
                                          POINTER(SsSchedule), POINTER(SsMlp), c_void_p,
                                          c_size_t, c_void_p, POINTER(SsResult)]),
    "ss_autotune_batched": (c_int, [POINTER(SsBatch), POINTER(SsOptions), c_void_p, c_size_t,
                                    c_void_p, POINTER(SsSchedule), POINTER(c_float),
                                    POINTER(c_int32)]),
    "ss_mlp_sync": (c_int, [POINTER(SsMlp), c_void_p]),
    "ss_warmstart_workspace_size": (c_int, [POINTER(SsBatch), POINTER(c_size_t)]),
    "ss_warmstart_predict": (c_int, [POINTER(SsMlp), POINTER(SsBatch), c_double, c_int32,
                                     c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ss_warmstart_train_step": (c_int, [POINTER(SsMlp), POINTER(SsBatch), c_double, c_int32,
                                        c_void_p, c_void_p, c_float, c_void_p, c_size_t, c_void_p,
                                        POINTER(c_float), c_void_p]),
    "ss_ibp_workspace_size": (c_int, [POINTER(SsIbpProblem), POINTER(SsOptions),
                                      POINTER(c_size_t)]),
    "spar_ibp": (c_int, [POINTER(SsIbpProblem), POINTER(SsOptions), c_void_p, c_void_p, c_size_t,
                         c_void_p, POINTER(SsIbpResult)]),
    "ss_ibp_sample": (c_int, [POINTER(SsIbpProblem), POINTER(SsOptions), c_int32,
                              POINTER(SsSparse), c_void_p, c_size_t, c_void_p]),
    "ss_ibp_time_iterations": (c_int, [POINTER(SsIbpProblem), POINTER(SsOptions), c_void_p,
                                       c_size_t, c_void_p, c_int32, POINTER(c_double),
                                       POINTER(c_int64)]),
    "ss_divergence_workspace_size": (c_int, [POINTER(SsProblem), POINTER(SsOptions),
                                             POINTER(c_size_t)]),
    "ss_sinkhorn_divergence": (c_int, [POINTER(SsProblem), POINTER(SsOptions), c_void_p,
                                       c_void_p, c_void_p, c_size_t, c_void_p,
                                       POINTER(SsDivergence)]),
    "ss_status_string": (c_char_p, [c_int]),
    "ss_last_error": (c_char_p, []),
    "ss_version": (c_int, []),
}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_2306_06581_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


class SparSinkError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.ss_last_error().decode() or lib.ss_status_string(code).decode()
        super().__init__(f"{where}: status {code} ({lib.ss_status_string(code).decode()}): {msg}")
        self.code = code
