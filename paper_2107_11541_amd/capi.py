"""ctypes declarations of the C ABI in include/feasm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfeasm.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EBADMESH, FE_EBADELEM, FE_ENOCONV, FE_EBREAKDOWN, FE_EDEVICE, FE_EBUSY = range(9)
STATUS_NAMES = {0: "FE_OK", 1: "FE_EINVAL", 2: "FE_ENOMEM", 3: "FE_EBADMESH", 4: "FE_EBADELEM",
                5: "FE_ENOCONV", 6: "FE_EBREAKDOWN", 7: "FE_EDEVICE", 8: "FE_EBUSY"}
FE_TET04, FE_PYR05, FE_PEN06, FE_HEX08 = 4, 5, 6, 8
FE_FP64, FE_MIXED = 0, 1
FE_OP_MOMENTUM, FE_OP_SCALAR, FE_OP_POISSON = 0, 1, 2
FE_UPLOAD_RENUMBER = 1
FE_UPLOAD_COLOURED = 2
FE_UPLOAD_GENERAL_SPMV = 4
FE_FORM_FULL_STRESS, FE_FORM_EMAC = 1, 2

P = C.c_void_p
i32, i64, dbl, sz = C.c_int32, C.c_int64, C.c_double, C.c_size_t


class Fields(C.Structure):
    _fields_ = [("op", C.c_int), ("dt", dbl), ("u", P), ("rho", P), ("mu", P),
                ("n_scalars", i32), ("Y", P), ("D", P)]


class StepInfo(C.Structure):
    _fields_ = [("cg_iterations", i32), ("cg_true_rel_residual", dbl)]


class AsmInfo(C.Structure):
    _fields_ = [("min_detJ", dbl), ("first_bad_elem", i64)]


class CGInfo(C.Structure):
    _fields_ = [("iterations", i32), ("outer_iterations", i32), ("rel_residual", dbl),
                ("true_rel_residual", dbl), ("symmetric_spmv", i32)]


class MeshDesc(C.Structure):
    _fields_ = [("nen", i32), ("n_nodes", i64), ("n_elems", i64), ("nnz", i64), ("rowptr", P),
                ("colidx", P), ("n_blocks", i64), ("n_colors", i32), ("max_row", i32),
                ("n_dirichlet", i64), ("device_bytes", sz)]


class PlanDesc(C.Structure):
    _fields_ = [("n_nodes", i64), ("n_elems", i64), ("nnz", i64), ("n_blocks", i64), ("n_colors", i32),
                ("max_row", i32), ("max_block_nodes", i32), ("max_block_slots", i32), ("max_phases", i32)]


class Job(C.Structure):
    _fields_ = [("type", C.c_int), ("n_nodes", i64), ("coords", P), ("n_elems", i64), ("conn", P),
                ("n_dirichlet", i64), ("dirichlet_nodes", P), ("dt", dbl), ("u", P), ("rho", P), ("mu", P),
                ("rtol", dbl), ("max_iter", i32), ("x", P), ("mom_rhs", P), ("elem_types", P)]


class JobResult(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", i32), ("rel_residual", dbl), ("true_rel_residual", dbl),
                ("min_detJ", dbl), ("first_bad_elem", i64), ("plan_ms", dbl), ("wait_ms", dbl),
                ("run_ms", dbl), ("total_ms", dbl), ("message", C.c_char * 128)]


# name -> (restype, argtypes); every symbol include/feasm.h declares
SIGNATURES = {
    "fe_ctx_create": (C.c_int, [C.c_int, P, C.POINTER(P)]),
    "fe_ctx_destroy": (None, [P]),
    "fe_ctx_last_error": (C.c_char_p, [P]),
    "fe_ctx_set_stream": (C.c_int, [P, P]),
    "fe_mesh_upload": (C.c_int, [P, C.c_int, i64, P, i64, P, i64, P, C.c_uint32, C.POINTER(P)]),
    "fe_mesh_upload_mixed": (C.c_int, [P, i64, P, i64, P, P, i64, P, C.c_uint32, C.POINTER(P)]),
    "fe_mesh_info": (C.c_int, [P, C.POINTER(MeshDesc)]),
    "fe_mesh_perm": (C.c_int, [P, P, P]),
    "fe_mesh_pattern_host": (C.c_int, [P, P, P]),
    "fe_mesh_to_mesh_order": (C.c_int, [P, P, P, i32]),
    "fe_mesh_to_user_order": (C.c_int, [P, P, P, i32]),
    "fe_mesh_free": (None, [P]),
    "fe_assemble": (C.c_int, [P, C.POINTER(Fields), C.c_int, P, P, C.POINTER(AsmInfo)]),
    "fe_assemble_block": (C.c_int, [P, C.c_uint32, dbl, P, P, P, P, P, C.POINTER(AsmInfo)]),
    "fe_apply_dirichlet": (C.c_int, [P, P, P, P]),
    "fe_spmv": (C.c_int, [P, P, P, P]),
    "fe_dot": (C.c_int, [P, i64, P, P, C.POINTER(dbl)]),
    "fe_axpy": (C.c_int, [P, i64, dbl, P, P]),
    "fe_cg_solve": (C.c_int, [P, P, P, P, dbl, i32, C.c_int, C.POINTER(CGInfo)]),
    "fe_cg_solve_noalloc": (C.c_int, [P, P, P, P, dbl, i32, C.POINTER(CGInfo)]),
    "fe_residual": (C.c_int, [P, P, P, P, C.c_uint32, P]),
    "fe_gradient": (C.c_int, [P, P, P]),
    "fe_scalar_residual": (C.c_int, [P, P, P, P, dbl, P]),
    "fe_scalar_step": (C.c_int, [P, dbl, P, P, dbl, P]),
    "fe_wall_faces": (C.c_int, [P, i64, P, P, dbl]),
    "fe_wall_traction": (C.c_int, [P, P, P, P, P]),
    "fe_divergence": (C.c_int, [P, dbl, P, P, P]),
    "fe_fractional_step": (C.c_int, [P, dbl, P, P, P, C.c_uint32, P, P, dbl, i32, C.c_int, C.POINTER(StepInfo)]),
    "fe_serve_create": (C.c_int, [P, sz, i32, i32, C.POINTER(P)]),
    "fe_serve_submit": (C.c_int, [P, C.POINTER(Job), C.POINTER(i64)]),
    "fe_serve_poll": (C.c_int, [P, i64, C.POINTER(i32), C.POINTER(JobResult)]),
    "fe_serve_wait": (C.c_int, [P, i64, C.POINTER(JobResult)]),
    "fe_serve_stats": (C.c_int, [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
    "fe_serve_destroy": (None, [P]),
    "fe_ctx_profile": (C.c_int, [P, C.c_int]),
    "fe_ctx_profile_read": (C.c_int, [P, C.c_int, C.POINTER(i64), C.POINTER(dbl)]),
    "fe_plan_create": (C.c_int, [C.c_int, i64, P, i64, P, C.c_uint32, C.POINTER(P)]),
    "fe_plan_create_mixed": (C.c_int, [i64, P, i64, P, P, C.c_uint32, C.POINTER(P)]),
    "fe_plan_export_types": (C.c_int, [P, P, P, P, C.POINTER(i64)]),
    "fe_plan_export_color_blocks": (C.c_int, [P, P]),
    "fe_plan_info": (C.c_int, [P, C.POINTER(PlanDesc)]),
    "fe_plan_export": (C.c_int, [P, P, P, P, P, P, P, P, P]),
    "fe_plan_owner_info": (C.c_int, [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(i32), C.POINTER(i32)]),
    "fe_plan_export_owner": (C.c_int, [P, P, P, P, P, P, P, P, P]),
    "fe_plan_free": (None, [P]),
    "fe_plan_last_error": (C.c_char_p, []),
    "fe_pack_layout": (C.c_int, [i64, i32, C.POINTER(i64), C.POINTER(i64)]),
}

_lib = None


def load(build_if_missing: bool = True):
    """Load libfeasm.so; build it first only if no library exists."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise ImportError(f"{LIB_PATH} is not built (python -m paper_2107_11541_amd.build)")
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
