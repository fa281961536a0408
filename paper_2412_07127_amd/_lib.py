"""ctypes declarations of the C ABI in include/icpcg.h (argument marshalling only).

The shared library libicpcg.so is built in-tree by build.py. Loading fails
loudly when it is missing: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libicpcg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "icpcg.h")

OK, E_INVALID, E_PIVOT, E_BREAKDOWN, E_MAXITER, E_NONFINITE, E_DEVICE, E_NOMEM, E_TRUE_RESIDUAL = range(9)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_PIVOT", 3: "E_BREAKDOWN", 4: "E_MAXITER",
                5: "E_NONFINITE", 6: "E_DEVICE", 7: "E_NOMEM", 8: "E_TRUE_RESIDUAL"}
F64, F32, BF16 = 0, 1, 2
PREC_FACTOR, PREC_JACOBI, PREC_NONE = 0, 1, 2


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class FactorOpts(C.Structure):
    _fields_ = [("max_restarts", C.c_int), ("alpha_min", C.c_double)]


class FactorInfo(C.Structure):
    _fields_ = [("alpha", C.c_double), ("restarts", C.c_int), ("min_pivot", C.c_double),
                ("nlevels", C.c_int64)]


class PrecInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("nlevels_L", C.c_int64),
                ("nlevels_U", C.c_int64), ("nsupernodes_L", C.c_int64),
                ("nsupernodes_U", C.c_int64), ("nsn_levels_L", C.c_int64),
                ("nsn_levels_U", C.c_int64), ("dtype", C.c_int), ("kind", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int64), ("max_replace", C.c_int),
                ("block_width", C.c_int), ("check_every", C.c_int), ("use_graph", C.c_int)]


class ColInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("replacements", C.c_int), ("status", C.c_int),
                ("relres", C.c_double), ("true_relres", C.c_double)]


class TuneInfo(C.Structure):
    _fields_ = [("block_width", C.c_int), ("ms_per_step", C.c_double * 5), ("ms_per_rhs", C.c_double)]


_lib = None


def load():
    """Load libicpcg.so (raises RuntimeError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    st = C.c_int
    i64 = C.c_int64
    sig = {
        "icpcg_create": ([C.POINTER(P), P], st),
        "icpcg_destroy": ([P], st),
        "icpcg_set_stream": ([P, P], st),
        "icpcg_last_error": ([P], C.c_char_p),
        "icpcg_status_string": ([st], C.c_char_p),
        "icpcg_tril_nnz": ([P, C.POINTER(Csr), C.POINTER(i64)], st),
        "icpcg_factor": ([P, C.POINTER(Csr), P, P, P, C.POINTER(FactorOpts), C.POINTER(FactorInfo)], st),
        "icpcg_prec_create": ([P, C.POINTER(Csr), st, C.POINTER(P)], st),
        "icpcg_prec_destroy": ([P], st),
        "icpcg_dropout": ([P, C.POINTER(Csr), C.c_double, P, P, P, C.POINTER(i64)], st),
        "icpcg_prec_create_simple": ([P, C.POINTER(Csr), st, C.POINTER(P)], st),
        "icpcg_prec_update_values": ([P, P, P], st),
        "icpcg_prec_get_info": ([P, P, C.POINTER(PrecInfo)], st),
        "icpcg_prec_levels": ([P, P, P, P, P, P, P, P], st),
        "icpcg_prec_transpose": ([P, P, P, P, P], st),
        "icpcg_spmv": ([P, C.POINTER(Csr), P, P, i64], st),
        "icpcg_trsv": ([P, P, st, P, st, P, i64], st),
        "icpcg_apply": ([P, P, P, st, P, P, i64], st),
        "icpcg_apply_rz": ([P, P, P, P, P, P, i64], st),
        "icpcg_apply_rz_noalloc": ([P, P, P, P, P, P, i64], st),
        "icpcg_trsv_rz": ([P, P, P, P, P, P, i64], st),
        "icpcg_apply_backward": ([P, P, P, P, P, P, P, P, i64], st),
        "icpcg_solve": ([P, C.POINTER(Csr), P, P, P, i64, C.POINTER(SolveOpts), C.POINTER(ColInfo)], st),
        "icpcg_sync": ([P], st),
        "icpcg_mat_create": ([P, C.POINTER(Csr), C.POINTER(P)], st),
        "icpcg_mat_destroy": ([P], st),
        "icpcg_mat_spmv": ([P, P, P, P, i64], st),
        "icpcg_solve_mat": ([P, P, P, P, P, i64, C.POINTER(SolveOpts), C.POINTER(ColInfo)], st),
        "icpcg_autotune": ([P, P, P, i64, C.POINTER(TuneInfo)], st),
        "icpcg_step_timing": ([P, st], st),
        "icpcg_step_timing_get": ([P, P, C.POINTER(i64)], st),
        "icpcg_color_order": ([P, C.POINTER(Csr), C.c_uint64, P, C.POINTER(C.c_int32)], st),
        "icpcg_block_color_order": ([P, C.POINTER(Csr), P, C.c_int32, P, C.POINTER(C.c_int32)], st),
        "icpcg_permute_matrix": ([P, C.POINTER(Csr), P, P, P, P], st),
        "icpcg_permute_rows": ([P, P, i64, i64, P, P, st], st),
        "icpcg_gnn_num_params": ([], i64),
        "icpcg_gnn_create": ([P, C.POINTER(Csr), P, C.POINTER(P)], st),
        "icpcg_gnn_destroy": ([P], st),
        "icpcg_gnn_inputs": ([P, P, P, P, C.POINTER(C.c_double)], st),
        "icpcg_gnn_forward": ([P, P, P, P], st),
        "icpcg_gnn_loss_grad": ([P, P, P, P, P, P, st], st),
        "icpcg_adam_step": ([P, P, P, P, P, i64, i64, C.c_double, C.c_double, C.c_double, C.c_double], st),
        "icpcg_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def declared_symbols(header: str = HEADER):
    """Names of the functions declared in include/icpcg.h."""
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(icpcg_[a-z_0-9]+)\s*\(", txt)))
