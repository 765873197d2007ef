"""ctypes declarations of libmq.so (the C ABI in include/mq.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmq.so")

MQ_OK = 0
MQ_WARN_NOT_CONVERGED = 1
MQ_ERR_INVALID_ARG = -1
MQ_ERR_NO_DEVICE = -2
MQ_ERR_OUT_OF_MEMORY = -3
MQ_ERR_DEVICE = -4
MQ_ERR_NONFINITE = -5
MQ_ERR_BUSY = -6
MQ_ERR_CANCELLED = -7

MQ_MAT_LOGNORMAL_SCALAR, MQ_MAT_KL, MQ_MAT_NONLINEAR = 0, 1, 2
MQ_PREC_FP64, MQ_PREC_MIXED = 0, 1
MQ_APPLY_A, MQ_APPLY_M, MQ_APPLY_K = 0, 1, 2
MQ_PATH_AUTO, MQ_PATH_RESIDENT, MQ_PATH_STREAMING, MQ_PATH_WIDE = 0, 1, 2, 3
MQ_PRECOND_AUTO, MQ_PRECOND_JACOBI, MQ_PRECOND_MULTIGRID = 0, 1, 2
MQ_MEM_DEVICE, MQ_MEM_HOST = 0, 1
MQ_NOALLOC_WORKSPACE_BYTES = 268435456
MQ_MASS_CONSISTENT, MQ_MASS_LUMPED = 0, 1
MQ_FLAG_NOT_CONVERGED, MQ_FLAG_FAILED, MQ_FLAG_PICARD_CAP, MQ_FLAG_PARAREAL_KMAX = 1, 2, 4, 8


class ProblemDesc(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("material", C.c_int32), ("precision", C.c_int32), ("path", C.c_int32),
        ("conductor", C.c_double * 4), ("strip", C.c_double * 2),
        ("J0", C.c_double), ("freq", C.c_double),
        ("sigma0", C.c_double), ("nu_cond", C.c_double), ("nu_air", C.c_double),
        ("s_sigma", C.c_double), ("s_nu", C.c_double),
        ("n_modes", C.c_int32), ("picard_max", C.c_int32),
        ("corr_len", C.c_double), ("s_kl", C.c_double),
        ("k1", C.c_double), ("k2", C.c_double), ("k3", C.c_double), ("s_k", C.c_double),
        ("picard_tol", C.c_double),
        ("tol", C.c_double), ("inner_rtol", C.c_double),
        ("max_iter", C.c_int32), ("max_sweeps", C.c_int32),
        ("precond", C.c_int32), ("tile", C.c_int32), ("mg_omega", C.c_double),
        ("mg_levels", C.c_int32), ("mg_coarse_sweeps", C.c_int32),
        ("split_steps", C.c_int32), ("mg_block_min", C.c_int32), ("mem_kind", C.c_int32),
        ("mass", C.c_int32),
    ]


class ProblemInfo(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_dof", C.c_int32), ("pitch", C.c_int32), ("n_xi", C.c_int32),
        ("box", C.c_int32 * 4), ("resident_ok", C.c_int32), ("lds_bytes", C.c_int32),
        ("precond", C.c_int32), ("mg_levels", C.c_int32),
        ("n_modes_used", C.c_int32), ("kl_lambda", C.c_double * 16),
        ("tile", C.c_int32), ("block", C.c_int32),
    ]


class RunStats(C.Structure):
    _fields_ = [
        ("n_instances", C.c_int64), ("sample_steps", C.c_int64), ("inner_iters", C.c_int64),
        ("sweeps", C.c_int64), ("picard_iters", C.c_int64),
        ("max_inner_per_step", C.c_int32), ("n_not_converged", C.c_int32), ("n_failed", C.c_int32),
        ("path", C.c_int32), ("grid", C.c_int32), ("block", C.c_int32),
        ("kernel_ms", C.c_double), ("total_ms", C.c_double),
        ("lat_p50_ms", C.c_double), ("lat_p99_ms", C.c_double), ("lat_max_ms", C.c_double),
        ("phase_ms", C.c_double * 8), ("busy_ms", C.c_double), ("n_pieces", C.c_int64),
    ]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        return d


class LevelDesc(C.Structure):
    _fields_ = [("steps_per_period", C.c_int32), ("coarse_steps_per_period", C.c_int32),
                ("n_periods", C.c_int32), ("reserved", C.c_int32)]


class PararealDesc(C.Structure):
    _fields_ = [("n_periods", C.c_int32), ("n_slices", C.c_int32),
                ("fine_steps_per_slice", C.c_int32), ("coarse_steps_per_slice", C.c_int32),
                ("k_max", C.c_int32), ("fixed_k", C.c_int32), ("tol", C.c_double)]


class AdaptiveDesc(C.Structure):
    _fields_ = [("target_rmse", C.c_double), ("var_fraction", C.c_double), ("n_pilot", C.c_int32),
                ("max_rounds", C.c_int32)]


class ServerDesc(C.Structure):
    _fields_ = [("base", ProblemDesc), ("hbm_budget_bytes", C.c_int64), ("max_inflight", C.c_int32),
                ("n_streams", C.c_int32), ("max_batch", C.c_int32), ("chunk_steps", C.c_int32),
                ("wide_min_nodes", C.c_int32), ("wide_queue", C.c_int32), ("wide_load_limit", C.c_int32),
                ("reserved", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("steps_per_period", C.c_int32), ("n_periods", C.c_int32),
                ("n_xi", C.c_int32), ("xi", C.c_double * 16), ("user_id", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("user_id", C.c_uint64), ("q", C.c_double),
                ("status", C.c_int32), ("inner_iters", C.c_int32), ("sweeps", C.c_int32), ("path", C.c_int32),
                ("t_submit_ns", C.c_int64), ("t_start_ns", C.c_int64), ("t_done_ns", C.c_int64),
                ("message", C.c_char * 64)]


class CombinedDesc(C.Structure):
    _fields_ = [("n_slices", C.c_int32), ("coarse_steps_per_period", C.c_int32), ("k_max", C.c_int32),
                ("reserved", C.c_int32), ("tol", C.c_double)]


class CombinedStats(C.Structure):
    _fields_ = [("n_slices", C.c_int32), ("coarse_steps_per_period", C.c_int32), ("n_cores", C.c_int32),
                ("n_c_para", C.c_int32), ("ms_levels", C.c_double), ("ms_parareal", C.c_double),
                ("ms_total", C.c_double), ("para_fine_steps", C.c_int64), ("para_coarse_steps", C.c_int64),
                ("mean_k", C.c_double), ("max_k", C.c_int32), ("level_slots", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class CostIn(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("K", C.c_int32), ("M", C.c_int32), ("n_cores", C.c_int32),
                ("C", C.c_double * 16), ("N", C.c_double * 16)]


class CostOut(C.Structure):
    _fields_ = [("tau_para", C.c_double), ("effort_para", C.c_double), ("tau_ref", C.c_double),
                ("effort_ref", C.c_double), ("tau_comb", C.c_double), ("effort_comb", C.c_double),
                ("speedup", C.c_double), ("s_inf", C.c_double), ("eps_inf", C.c_double), ("r", C.c_double),
                ("kappa", C.c_int32), ("n_c_para", C.c_int32), ("batches", C.c_int32 * 16), ("s_nc", C.c_double)]


VP = C.c_void_p
PD = C.POINTER(C.c_double)

# name -> (restype, argtypes); this is the complete exported C ABI
SIGNATURES = {
    "mq_last_error": (C.c_char_p, []),
    "mq_version": (C.c_int, []),
    "mq_last_flags": (C.c_int, [C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int64)]),
    "fem_setup": (C.c_int, [C.POINTER(ProblemDesc), VP, C.POINTER(VP)]),
    "mq_problem_destroy": (C.c_int, [VP]),
    "mq_ndof": (C.c_int, [VP, C.POINTER(C.c_int64)]),
    "mq_problem_info_get": (C.c_int, [VP, C.POINTER(ProblemInfo)]),
    "mq_set_initial_state": (C.c_int, [VP, VP]),
    "mlmc_level_run": (C.c_int, [VP, C.POINTER(LevelDesc), C.c_int32, VP, VP, VP, VP, C.POINTER(RunStats)]),
    "mlmc_level_run_noalloc": (C.c_int, [VP, C.POINTER(LevelDesc), C.c_int32, VP, VP, VP, VP,
                                         C.POINTER(RunStats)]),
    "mlmc_multilevel_run": (C.c_int, [VP, C.c_int32, C.POINTER(LevelDesc), C.POINTER(C.c_int32),
                                      C.POINTER(VP), C.POINTER(VP), C.POINTER(VP), C.POINTER(RunStats)]),
    "parareal_run": (C.c_int, [VP, C.POINTER(PararealDesc), C.c_int32, VP, VP, VP, VP, C.POINTER(RunStats)]),
    "mlmc_multimesh_run": (C.c_int, [C.c_int32, C.POINTER(VP), C.POINTER(LevelDesc), C.POINTER(C.c_int32),
                                     C.POINTER(VP), C.POINTER(VP), C.POINTER(VP), C.POINTER(RunStats)]),
    "mlmc_adaptive_run": (C.c_int, [VP, C.c_int32, C.POINTER(LevelDesc), C.POINTER(C.c_int32), C.POINTER(VP),
                                    C.POINTER(VP), C.POINTER(VP), C.POINTER(AdaptiveDesc), C.POINTER(C.c_int32),
                                    PD, C.POINTER(RunStats)]),
    "mlmc_combined_run": (C.c_int, [VP, C.c_int32, C.POINTER(LevelDesc), C.POINTER(C.c_int32), C.POINTER(VP),
                                    C.POINTER(CombinedDesc), C.POINTER(VP), C.POINTER(VP), VP, C.POINTER(RunStats),
                                    C.POINTER(CombinedStats)]),
    "mq_cost_model": (C.c_int, [C.POINTER(CostIn), C.POINTER(CostOut)]),
    "mq_plan_split": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                PD, C.POINTER(C.c_int32)]),
    "mlmc_estimate": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(VP), C.POINTER(VP), VP, VP]),
    "mq_debug_apply": (C.c_int, [VP, C.c_int32, C.c_double, C.c_int32, VP, VP, VP]),
    "mq_server_create": (C.c_int, [C.POINTER(ServerDesc), VP, C.POINTER(VP)]),
    "mq_submit": (C.c_int, [VP, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "mq_poll": (C.c_int, [VP, C.POINTER(Result), C.c_int32, C.POINTER(C.c_int32)]),
    "mq_server_pending": (C.c_int, [VP, C.POINTER(C.c_int32)]),
    "mq_server_destroy": (C.c_int, [VP]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libmq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libmq.so not built ({path}); run __graft_entry__.build() or "
                           "python paper_2507_19246_amd/build.py")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmq error {code}: {msg}")
        self.code = code


def check(code: int) -> int:
    if code < 0:
        raise MQError(code, load().mq_last_error().decode(errors="replace"))
    return code
