"""ctypes binding of libfsimg.so (argument marshalling only).

All computation happens in the native library; this module converts Python
objects to the C structures of include/fsi_mg.h and include/fsi_problem.h.
Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsimg.so")

FSI_OK, FSI_NOT_CONVERGED, FSI_PENDING = 0, 1, 2
FSI_E_INVALID, FSI_E_OOM, FSI_E_SINGULAR, FSI_E_DEVICE = -1, -2, -3, -4
FSI_E_NONFINITE, FSI_E_CAPACITY, FSI_E_UNKNOWN_TICKET = -5, -6, -7
PREC = {"fp64": 0, "bf16": 1, "fp16": 2, "fp32": 3}
ORTH = {"cgs2": 0, "cgs": 1}
SIDE = {"right": 0, "left": 1}


class FsiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Csr(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int64),
                ("rowptr", C.POINTER(C.c_int64)), ("colind", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class Patches(C.Structure):
    _fields_ = [("npatch", C.c_int32), ("ptr", C.POINTER(C.c_int64)), ("dof", C.POINTER(C.c_int32)),
                ("owned", C.POINTER(C.c_uint8)), ("kind", C.POINTER(C.c_uint8))]


class LevelC(C.Structure):
    _fields_ = [("J", Csr), ("P", Csr), ("R", Csr), ("patches", Patches),
                ("dirichlet", C.POINTER(C.c_uint8))]


class MgOpts(C.Structure):
    _fields_ = [("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("omega", C.c_double),
                ("precision", C.c_int32), ("solid_precision", C.c_int32),
                ("refine_sweeps", C.c_int32), ("use_graph", C.c_int32), ("tuning_db", C.c_char_p),
                ("fluid_ilu", C.c_int32)]


class KrylovOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("rtol", C.c_double), ("maxit", C.c_int32),
                ("orth", C.c_int32), ("x0_nonzero", C.c_int32), ("history", C.POINTER(C.c_double)),
                ("fixed_iters", C.c_int32), ("side", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("true_relres", C.c_double), ("est_relres", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("rho", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ProblemSpecC(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("levels", C.c_int32), ("patch", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("solid_lo", C.c_double * 3), ("solid_hi", C.c_double * 3),
                ("rho", C.c_double), ("mu", C.c_double), ("mu_s", C.c_double),
                ("u_peak", C.c_double), ("amp", C.c_double), ("kmax", C.c_int32),
                ("coeffs", C.POINTER(C.c_double)), ("transient", C.c_int32), ("dt", C.c_double),
                ("rho_s", C.c_double), ("amp_d", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("device", C.c_int32),
                ("batch_vcycles", C.c_int32), ("reserved", C.c_int32)]


class ElementData(C.Structure):
    _fields_ = [("dim", C.c_int32), ("ne", C.c_int32), ("nl", C.c_int32), ("na", C.c_int32),
                ("np", C.c_int32), ("nq", C.c_int32), ("ncolor", C.c_int32), ("ndof", C.c_int64),
                ("l2g", C.POINTER(C.c_int32)), ("tgt", C.POINTER(C.c_int32)), ("solid", C.POINTER(C.c_uint8)),
                ("color_ptr", C.POINTER(C.c_int32)), ("color_elems", C.POINTER(C.c_int32)),
                ("N", C.POINTER(C.c_double)), ("dN", C.POINTER(C.c_double)), ("psi", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("vol", C.c_double), ("dirichlet", C.POINTER(C.c_uint8)),
                ("dval", C.POINTER(C.c_double)), ("y_prev", C.POINTER(C.c_double)),
                ("mu", C.c_double), ("rho", C.c_double), ("mu_s", C.c_double), ("dt", C.c_double),
                ("rho_s", C.c_double)]


class NewtonOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("tol", C.c_double)]


class NewtonInfo(C.Structure):
    _fields_ = [("steps", C.c_int32), ("converged", C.c_int32), ("krylov_iters", C.c_int32),
                ("last_update", C.c_double), ("res0", C.c_double), ("res_last", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol the headers declare (checked by the CPU tests)
EXPORTS = [
    "fsi_abi_version", "fsi_status_string", "fsi_last_error", "fsi_mg_setup", "fsi_mg_vcycle",
    "fsi_mg_vcycle_batch", "fsi_mg_set_jvalues", "fsi_mg_galerkin",
    "fsi_fgmres_solve", "fsi_fgmres_solve_noalloc", "fsi_mg_apply", "fsi_mg_export_patches", "fsi_mg_level_info",
    "fsi_mg_refactor", "fsi_mg_jvalues", "fsi_mg_profile", "fsi_mg_autotune",
    "fsi_mg_destroy", "fsi_server_create", "fsi_serve_submit", "fsi_serve_poll",
    "fsi_server_stats", "fsi_server_destroy", "fsi_stream_read", "fsi_stream_read_blocks",
    "fsi_problem_build", "fsi_problem_nlevels", "fsi_problem_levels", "fsi_problem_vectors",
    "fsi_problem_dirichlet", "fsi_problem_residual", "fsi_problem_destroy", "fsi_problem_last_error",
    "fsi_problem_element_data", "fsi_assembly_create", "fsi_assembly_run", "fsi_newton_solve",
    "fsi_cn_steps", "fsi_fmg_solve", "fsi_assembly_destroy",
]

_lib = None


def lib():
    """The loaded native library (raises when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"native library not built: {LIB_PATH} (run paper_1709_05660_amd.build)")
    # torch's HIP runtime has the same SONAME as the one the library links;
    # loading torch first makes the library bind to that single runtime.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "fsi_abi_version": (C.c_int32, []),
        "fsi_status_string": (C.c_char_p, [C.c_int32]),
        "fsi_last_error": (C.c_char_p, []),
        "fsi_mg_setup": (C.c_int32, [C.POINTER(LevelC), C.c_int32, C.POINTER(MgOpts), P, C.POINTER(P)]),
        "fsi_mg_vcycle": (C.c_int32, [P, P, P, P]),
        "fsi_mg_vcycle_batch": (C.c_int32, [C.POINTER(P), C.c_int32, C.POINTER(P), C.POINTER(P), P]),
        "fsi_mg_set_jvalues": (C.c_int32, [P, C.c_int32, P, P]),
        "fsi_mg_galerkin": (C.c_int32, [P, P]),
        "fsi_fgmres_solve": (C.c_int32, [P, P, P, C.POINTER(KrylovOpts), C.POINTER(SolveInfo), P]),
        "fsi_fgmres_solve_noalloc": (C.c_int32, [P, P, P, C.POINTER(KrylovOpts), C.POINTER(SolveInfo), P]),
        "fsi_mg_apply": (C.c_int32, [P, C.c_int32, C.c_int32, P, P, P, P]),
        "fsi_mg_export_patches": (C.c_int32, [P, C.c_int32, P, P, P, P]),
        "fsi_mg_level_info": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_int64)]),
        "fsi_mg_destroy": (C.c_int32, [P]),
        "fsi_mg_refactor": (C.c_int32, [P, P]),
        "fsi_mg_autotune": (C.c_int32, [P, C.c_char_p, P, C.POINTER(C.c_int32)]),
        "fsi_mg_jvalues": (C.c_int32, [P, C.c_int32, C.POINTER(C.POINTER(C.c_double))]),
        "fsi_mg_profile": (C.c_int32, [P, C.c_int32, C.POINTER(C.c_double)]),
        "fsi_stream_read": (C.c_int32, [P, C.c_int64, P, P]),
        "fsi_stream_read_blocks": (C.c_int32, []),
        "fsi_server_create": (C.c_int32, [C.POINTER(ServerOpts), C.POINTER(P)]),
        "fsi_serve_submit": (C.c_int32, [P, C.POINTER(LevelC), C.c_int32, P, C.POINTER(MgOpts),
                                         C.POINTER(KrylovOpts), C.POINTER(C.c_uint64)]),
        "fsi_serve_poll": (C.c_int32, [P, C.c_uint64, P, C.POINTER(SolveInfo)]),
        "fsi_server_stats": (C.c_int32, [P, C.POINTER(C.c_int64)]),
        "fsi_server_destroy": (C.c_int32, [P]),
        "fsi_problem_build": (C.c_int32, [C.POINTER(ProblemSpecC), C.POINTER(P)]),
        "fsi_problem_nlevels": (C.c_int32, [P]),
        "fsi_problem_levels": (C.c_int32, [P, C.POINTER(LevelC)]),
        "fsi_problem_vectors": (C.c_int32, [P, C.POINTER(C.POINTER(C.c_double)),
                                            C.POINTER(C.POINTER(C.c_double)), C.POINTER(C.c_int64)]),
        "fsi_problem_dirichlet": (C.c_int32, [P, C.c_int32, C.POINTER(C.POINTER(C.c_uint8))]),
        "fsi_problem_residual": (C.c_int32, [P, P, P]),
        "fsi_problem_destroy": (C.c_int32, [P]),
        "fsi_problem_last_error": (C.c_char_p, []),
        "fsi_problem_element_data": (C.c_int32, [P, C.POINTER(ElementData)]),
        "fsi_assembly_create": (C.c_int32, [C.POINTER(ElementData), C.POINTER(Csr), P, C.POINTER(P)]),
        "fsi_assembly_run": (C.c_int32, [P, P, P, P, P]),
        "fsi_newton_solve": (C.c_int32, [P, P, P, C.POINTER(NewtonOpts), C.POINTER(KrylovOpts),
                                         C.POINTER(NewtonInfo), P]),
        "fsi_cn_steps": (C.c_int32, [P, P, P, C.c_int32, C.POINTER(NewtonOpts), C.POINTER(KrylovOpts),
                                     C.POINTER(NewtonInfo), P]),
        "fsi_fmg_solve": (C.c_int32, [C.c_int32, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(P),
                                      C.POINTER(C.c_int32), C.POINTER(NewtonOpts), C.POINTER(KrylovOpts),
                                      C.POINTER(NewtonInfo), P]),
        "fsi_assembly_destroy": (C.c_int32, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status, what=""):
    if status < 0:
        msg = lib().fsi_last_error().decode()
        raise FsiError(status, f"{what}: {msg}" if what else msg)
    return status


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))
