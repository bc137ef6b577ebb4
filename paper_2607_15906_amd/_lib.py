"""ctypes loader for libgocp.so: declares every C ABI entry point of gocp.h."""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# GOCP_PHASE_TRACE=1 selects the measurement build that records the
# energy+screen launch's phase trace (python -m paper_2607_15906_amd.build
# --phase-trace); the product library otherwise
LIB_PATH = os.path.join(_HERE, "libgocp_trace.so" if os.environ.get("GOCP_PHASE_TRACE") == "1" else "libgocp.so")

GOCP_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESHAPE",
          -5: "ENOTSUP", -6: "EBUSY", -7: "ENUMERIC", -8: "ECANCELED"}
GOCP_EBUSY = -6


class GocpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class AdaptParams(C.Structure):
    _fields_ = [("grad_tol", C.c_double), ("max_iter", C.c_int32), ("use_graph", C.c_int32),
                ("schedule", C.c_int32), ("reserved", C.c_int32)]


class ReoptParams(C.Structure):
    _fields_ = [("grad_tol", C.c_double), ("max_iter", C.c_int32), ("bfgs_max_iter", C.c_int32),
                ("bfgs_gtol", C.c_double)]


class ReoptResult(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("converged", C.c_int32),
                ("energies", C.POINTER(C.c_double)), ("ops", C.POINTER(C.c_int32)),
                ("thetas", C.POINTER(C.c_double)), ("gnorms", C.POINTER(C.c_double)),
                ("bfgs_steps", C.POINTER(C.c_int32)), ("bfgs_evals", C.POINTER(C.c_int32))]


class RequestInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_qubits", C.c_int32), ("t_submit_ns", C.c_int64),
                ("t_admit_ns", C.c_int64), ("t_done_ns", C.c_int64)]


class AdaptResult(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("converged", C.c_int32),
                ("energies", C.POINTER(C.c_double)), ("ops", C.POINTER(C.c_int32)),
                ("thetas", C.POINTER(C.c_double)), ("gnorms", C.POINTER(C.c_double)),
                ("gmax", C.POINTER(C.c_double)), ("substeps", C.POINTER(C.c_int32))]


_P = C.c_void_p
_PP = C.POINTER(C.c_void_p)
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_U32P = C.POINTER(C.c_uint32)
_U64P = C.POINTER(C.c_uint64)
_F64P = C.POINTER(C.c_double)

# name -> argtypes (restype is int for every call except gocp_last_error)
SIGNATURES = {
    "gocp_version": [],
    "pauli_hamiltonian_load": [C.c_int, _F64P, _F64P, C.c_double, C.c_int, _PP],
    "pauli_hamiltonian_load_terms": [C.c_int, C.c_int64, _U32P, _U32P, _F64P, _PP],
    "gocp_ham_info": [_P, _I32P, _I64P, _I32P],
    "gocp_ham_terms": [_P, C.c_int64, _U32P, _U32P, _F64P],
    "gocp_ham_free": [_P],
    "pool_build": [C.c_int, C.c_int, C.c_int, _PP],
    "pool_build_pauli": [C.c_int, C.c_int, C.c_int, _PP],
    "gocp_pool_info": [_P, _I32P, _I32P, _I32P],
    "gocp_pool_op": [_P, C.c_int32, _I32P, _I32P, _U32P],
    "gocp_pool_strings": [_P, _I32P, _U32P, _F64P],
    "gocp_pool_free": [_P],
    "gocp_partition": [_P, _I32P, _I32P, _I32P],
    "gocp_conflict_degrees": [_P, _I64P, _I32P],
    "gocp_hf_index": [C.c_int, C.c_int, C.c_int, _U64P],
    "gocp_basis_occupation": [C.c_int, C.c_int, C.c_uint64, _U64P],
    "gocp_state_hf": [_P, C.c_int, C.c_int, C.c_int, _P, C.c_int],
    "gocp_sector_weight": [_P, C.c_int, C.c_int, C.c_int, _P, C.c_int, _F64P],
    "gocp_ctx_create": [C.c_int, _P, _PP],
    "gocp_ctx_destroy": [_P],
    "gocp_ctx_set_stream": [_P, _P],
    "gocp_ctx_synchronize": [_P],
    "gocp_state_basis": [_P, C.c_int, C.c_uint64, _P, C.c_int],
    "energy": [_P, _P, _P, C.c_int, _F64P],
    "gocp_apply_hamiltonian": [_P, _P, _P, C.c_int, _P, _F64P],
    "pool_gradients": [_P, _P, _P, _P, C.c_int, _F64P, C.c_int],
    "pool_gradients_noalloc": [_P, _P, _P, _P, C.c_int, _F64P],
    "taylor5_apply": [_P, _P, C.c_int32, C.c_double, _P, C.c_int, _I32P],
    "taylor5_apply_family": [_P, _P, C.c_int32, _I32P, C.POINTER(C.c_double), _P, C.c_int, _I32P],
    "adapt_solve": [_P, _P, _P, _P, C.c_int, C.POINTER(AdaptParams), C.POINTER(AdaptResult)],
    "adapt_reopt_solve": [_P, _P, _P, _P, C.c_int, C.POINTER(ReoptParams), C.POINTER(ReoptResult)],
    "gocp_batch_create": [_P, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                          C.POINTER(C.c_void_p), C.c_int, C.POINTER(AdaptParams), _PP],
    "gocp_batch_step": [_P, C.c_int32],
    "gocp_batch_step_timed": [_P, C.c_int32, C.c_int32, C.c_int32, _F64P, _F64P],
    "gocp_batch_run": [_P],
    "gocp_batch_poll": [_P, _I32P],
    "gocp_batch_result": [_P, C.c_int32, C.POINTER(AdaptResult)],
    "gocp_batch_time_kernel": [_P, C.c_int32, C.c_int32, _F64P],
    "gocp_batch_schedule": [_P, _I32P],
    "gocp_batch_destroy": [_P],
    "gocp_request_footprint": [C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int, _I64P],
    "gocp_request_bytes": [_P, _P, C.c_int32, C.c_int, _I64P],
    "gocp_server_create": [_P, C.c_int64, C.c_int32, C.c_int, C.c_int32, C.c_int32, _PP],
    "gocp_server_submit": [_P, _P, _P, C.c_int32, C.c_double, _U64P],
    "gocp_server_poll": [_P, C.c_uint64, C.POINTER(AdaptResult), C.POINTER(RequestInfo)],
    "gocp_server_stats": [_P, _I32P, _I32P, _I64P, _I64P, _I64P],
    "gocp_server_destroy": [_P],
    "gocp_phase_trace": [_P, C.POINTER(C.c_uint64), C.c_int32, _I32P],
}

_lib = None


def load():
    """Load libgocp.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{os.path.basename(LIB_PATH)} not built at {LIB_PATH}; run "
                          "`python -m paper_2607_15906_amd.build` (with --phase-trace for the trace build)")
    lib = C.CDLL(LIB_PATH)
    lib.gocp_last_error.restype = C.c_char_p
    lib.gocp_last_error.argtypes = []
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = C.c_int
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != GOCP_OK:
        msg = load().gocp_last_error().decode(errors="replace")
        raise GocpError(code, msg)
