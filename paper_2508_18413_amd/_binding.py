"""ctypes binding of libpmcmc (include/pmcmc.h).  Argument marshalling only:
every step of the computation runs in the library's HIP kernels.  Torch is
used for device memory and the current stream.  There is no fallback: if the
library or a GPU is missing, calls raise."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmcmc.so")

PMC_OK, PMC_ERR_INVALID, PMC_ERR_UNSUPPORTED, PMC_ERR_OOM, PMC_ERR_HIP, PMC_NOT_CONVERGED, \
    PMC_ERR_NONFINITE = range(7)
STATUS_NAMES = {0: "PMC_OK", 1: "PMC_ERR_INVALID", 2: "PMC_ERR_UNSUPPORTED", 3: "PMC_ERR_OOM",
                4: "PMC_ERR_HIP", 5: "PMC_NOT_CONVERGED", 6: "PMC_ERR_NONFINITE"}
PMC_F32, PMC_F64 = 0, 1
PMC_SAMPLER_MALA, PMC_SAMPLER_ULA, PMC_SAMPLER_HMC = 0, 1, 2
PMC_TARGET_GAUSSIAN, PMC_TARGET_BANANA, PMC_TARGET_LOGREG, PMC_TARGET_FUNNEL = 0, 1, 2, 3
PMC_DEER_DENSE, PMC_QDEER_DIAG, PMC_QDEER_BLOCK2, PMC_PICARD = 0, 1, 2, 3
PMC_JAC_F32, PMC_JAC_BF16 = 0, 1
PMC_GATE_FROZEN, PMC_GATE_SURROGATE = 0, 1
PMC_PRODUCTS_AUTO, PMC_PRODUCTS_F32, PMC_PRODUCTS_SPLIT16, PMC_PRODUCTS_REFINE = 0, 1, 2, 3


class pmc_target_desc(C.Structure):
    _fields_ = [("kind", C.c_int), ("dim", C.c_int), ("dtype", C.c_int), ("mean", C.c_void_p),
                ("prec", C.c_void_p), ("X", C.c_void_p), ("y", C.c_void_p), ("n_data", C.c_int),
                ("prior_var", C.c_double), ("theta", C.c_double), ("products", C.c_int)]


class pmc_problem(C.Structure):
    _fields_ = [("sampler", C.c_int), ("target", C.c_void_p), ("step_size", C.c_double),
                ("n_chains", C.c_int), ("offsets", C.POINTER(C.c_int64)), ("n_steps", C.c_int64),
                ("s0", C.c_void_p), ("noise", C.c_void_p), ("uniforms", C.c_void_p),
                ("init_guess", C.c_void_p), ("out_states", C.c_void_p),
                ("out_accept", C.c_void_p), ("out_gtilde", C.c_void_p), ("n_leapfrog", C.c_int),
                ("inv_mass", C.c_void_p)]


class pmc_options(C.Structure):
    _fields_ = [("variant", C.c_int), ("jac_prec", C.c_int), ("gate", C.c_int),
                ("atol", C.c_double), ("rtol", C.c_double), ("max_iter", C.c_int),
                ("damping", C.c_double), ("clip", C.c_double), ("clip_inf_norm", C.c_int),
                ("skip_converged_prefix", C.c_int), ("graph_sweeps", C.c_int),
                ("trace_out", C.c_void_p), ("trace_bytes", C.c_size_t), ("floor_stall", C.c_int),
                ("profile_kernels", C.c_int), ("jac_probes", C.c_int), ("probe_seed", C.c_uint64),
                ("basis", C.c_void_p), ("window_width", C.c_int), ("tie_band", C.c_double)]


class pmc_result(C.Structure):
    _fields_ = [("sweeps_per_chain", C.POINTER(C.c_int32)), ("n_converged", C.c_int),
                ("sweeps_total", C.c_int), ("n_floor", C.c_int), ("n_accept", C.c_int64), ("resid_inf", C.c_double),
                ("resid_l2", C.c_double), ("max_ratio", C.c_double), ("nonfinite", C.c_int64),
                ("elapsed_ms", C.c_float), ("eval_ms", C.c_float), ("scan_ms", C.c_float),
                ("eval_steps", C.c_int64), ("chain_state", C.POINTER(C.c_int8))]


_lib = None


def lib():
    """Loads libpmcmc.so (built in-tree by paper_2508_18413_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libpmcmc.so not built ({LIB_PATH}); run python paper_2508_18413_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, st = C.c_void_p, C.c_int64, C.c_int
        sig = {
            "pmc_create": [C.POINTER(vp), C.c_int, vp],
            "pmc_destroy": [vp],
            "pmc_set_stream": [vp, vp],
            "pmc_target_create": [vp, C.POINTER(pmc_target_desc), C.POINTER(vp)],
            "pmc_target_destroy": [vp],
            "pmc_workspace_size": [vp, C.POINTER(pmc_problem), C.POINTER(pmc_options),
                                   C.POINTER(C.c_size_t)],
            "pmc_default_options": [C.POINTER(pmc_options), C.c_int],
            "pmc_solve": [vp, C.POINTER(pmc_problem), C.POINTER(pmc_options), vp, C.c_size_t,
                          C.POINTER(pmc_result)],
            "pmc_solve_noalloc": [vp, C.POINTER(pmc_problem), C.POINTER(pmc_options), C.POINTER(pmc_result)],
            "pmc_sample_sequential": [vp, C.POINTER(pmc_problem), C.POINTER(pmc_result)],
            "pmc_hmc_sample": [vp, vp, C.c_double, C.c_int, C.c_int, vp, vp, vp,
                               C.POINTER(pmc_options), C.c_int, vp, vp, vp, C.POINTER(C.c_int32),
                               C.POINTER(pmc_result)],
            "pmc_adjoint": [vp, C.POINTER(pmc_problem), vp, vp, vp, C.POINTER(C.c_double),
                            C.POINTER(C.c_double)],
            "pmc_linrec_diag": [vp, C.c_int, C.c_int, i64, vp, vp, vp],
            "pmc_linrec_block2": [vp, C.c_int, i64, vp, vp, vp],
            "pmc_linrec_dense": [vp, C.c_int, C.c_int, C.c_int, i64, vp, vp, vp],
            "pmc_autotune": [vp, C.POINTER(pmc_problem), C.POINTER(pmc_options), C.c_char_p],
            "pmc_set_scan_timing": [vp, C.c_int],
            "pmc_last_scan_ms": [vp, C.POINTER(C.c_float)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = st
        L.pmc_last_error.restype = C.c_char_p
        L.pmc_last_error.argtypes = []
        L.pmc_version.restype = C.c_char_p
        L.pmc_version.argtypes = []
        _lib = L
    return _lib


class PMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, allow=()):
    if status == PMC_OK or status in allow:
        return status
    raise PMCError(status, lib().pmc_last_error().decode())


def exported_symbols(header_path: str) -> list[str]:
    """Names of the functions declared in a pmcmc header."""
    import re
    txt = open(header_path).read()
    return sorted(set(re.findall(r"\b(pmc_[a-z0-9_]+)\s*\(", txt)))
