"""ctypes declarations of the C ABI in include/oasis.h.

Loading fails loudly when liboasis.so has not been built: there is no CPU
fallback for anything the library computes.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OASIS_LIB") or os.path.join(HERE, "liboasis.so")

OK, EINVAL, EHIP, ENOTCONV, EBREAKDOWN, ENAN, EWORKSPACE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
FORM_MASS, FORM_STIFF, FORM_GRAD_X, FORM_GRAD_Y, FORM_GRAD_Z, FORM_CONV = range(6)
KRYLOV_TIME = 1
KRYLOV_NULLSPACE_CONST = 2
ASSEMBLE_ROWS, ASSEMBLE_COLORS = 0, 1
PSTART_PREV, PSTART_ZERO = 0, 1
UPDATE_LUMPED, UPDATE_CONSISTENT, UPDATE_GRADIENT = 0, 1, 2
CONV_ABCN, CONV_ABE = 0, 1
MAX_SCALARS = 4
AMG_THETA = 0.125
INSPECT_A, INSPECT_DIAG_A, INSPECT_RHS = 100, 101, 102
STORAGE_AUTO, STORAGE_ELL, STORAGE_CSR = 0, 1, 2
PCG_NOALLOC_BYTES = 64 << 20
CG_FORM_AUTO, CG_FORM_TWO, CG_FORM_SINGLE = 0, 1, 2
MPNN_IN, MPNN_HID, MPNN_LAYERS = 6, 32, 3
MPNN_NPARAM = 32 * 6 + 32 + 3 * 32 * 32 * 2 + 3 * 32 + 32 + 1
MPNN_LOSS_MSE, MPNN_LOSS_KNORM = 0, 1
AMG_HALF_LEVEL0 = 4

i32 = C.c_int32
i64 = C.c_int64
f64 = C.c_double
f32 = C.c_float
vp = C.c_void_p
sz = C.c_size_t
P = C.POINTER


class Csr(C.Structure):
    _fields_ = [("n", i32), ("nnz", i32), ("row_ptr", vp), ("col_idx", vp), ("val", vp), ("dtype", i32)]


class Mesh(C.Structure):
    _fields_ = [("dim", i32), ("n_vert", i32), ("n_cell", i32), ("n_dof", i32), ("coords", vp),
                ("cells", vp), ("vert2dof", vp), ("n_colors", i32), ("color_ptr", P(i32)),
                ("color_cells", vp)]


class Tuning(C.Structure):
    _fields_ = [("storage", i32), ("grid_cap", i32), ("cg_form", i32)]


class KrylovOpts(C.Structure):
    _fields_ = [("rtol", f64), ("maxit", i32), ("precision", i32), ("inner_rtol", f64),
                ("max_outer", i32), ("check_every", i32), ("flags", i32), ("tuning", Tuning)]


class KrylovStats(C.Structure):
    _fields_ = [("iters", i32), ("outer_iters", i32), ("status", i32), ("restarts", i32),
                ("rel_res", f64), ("kernel_ms", f64), ("kernel_count", i32), ("ell_patterns", i32)]


class AmgParams(C.Structure):
    _fields_ = [("theta", f64), ("coarse_size", i32), ("max_levels", i32), ("precision", i32), ("flags", i32),
                ("tuning", Tuning)]


class AmgLevelInfo(C.Structure):
    _fields_ = [("n", i32), ("nnz", i32), ("row_ptr", P(i32)), ("col_idx", P(i32)), ("val", P(f64)),
                ("near_null", P(f64)), ("omega", f64), ("n_agg", i32), ("agg", P(i32)), ("p_nnz", i32),
                ("p_row_ptr", P(i32)), ("p_col_idx", P(i32)), ("p_val", P(f64)), ("coarse_inv", P(f64))]


class IpcsParams(C.Structure):
    _fields_ = [("dt", f64), ("nu", f64), ("f", f64 * 3), ("n_bc", i32), ("bc_dofs", vp),
                ("rtol_u", f64), ("rtol_p", f64), ("maxit", i32), ("precision", i32),
                ("inner_rtol", f64), ("assembly", i32), ("pressure_start", i32),
                ("pressure_delta", f64), ("tuning", Tuning), ("inner_iters", i32), ("velocity_update", i32),
                ("n_scalars", i32), ("diffusivity", f64 * 4), ("scalar_source", f64 * 4), ("convection", i32)]


class State(C.Structure):
    _fields_ = [("U1", vp * 3), ("U2", vp * 3), ("Un", vp * 3), ("p", vp), ("phi", vp),
                ("UI", vp * 3), ("b_phi", vp), ("C1", vp * 4), ("Cn", vp * 4), ("C_bc", vp * 4)]


class StepStats(C.Structure):
    _fields_ = [("iters_u", i32 * 3), ("iters_p", i32), ("outer_u", i32), ("outer_p", i32),
                ("status", i32), ("guess_used", i32), ("res_u", f64 * 3), ("res_p", f64),
                ("ms_assemble", f64), ("ms_velocity", f64), ("ms_pressure", f64),
                ("ms_update", f64), ("ms_total", f64), ("iters_m", i32 * 3), ("iters_c", i32 * 4),
                ("res_c", f64 * 4), ("ms_scalars", f64)]


_SIGS = {
    "oasis_graph_workspace_size": (i32, [P(Mesh), P(sz)]),
    "oasis_p1_pattern": (i32, [vp, P(Mesh), vp, vp, i64, P(i32), vp, sz]),
    "oasis_color_cells": (i32, [vp, P(Mesh), vp, vp, P(i32), vp, sz]),
    "oasis_color_classes": (i32, [vp, i32, vp, i32, P(i32), vp, vp, sz]),
    "oasis_rcm_workspace_size": (i32, [i32, P(sz)]),
    "oasis_rcm": (i32, [vp, i32, vp, vp, vp, vp, vp, sz]),
    "oasis_relabel": (i32, [vp, i32, vp, vp, vp]),
    "oasis_assemble_p1": (i32, [vp, P(Mesh), i32, P(vp), f64, P(Csr), P(Csr)]),
    "oasis_spmv": (i32, [vp, P(Csr), vp, vp, f64, f64]),
    "oasis_krylov_workspace_size": (i32, [i32, i32, i32, P(KrylovOpts), P(sz)]),
    "oasis_pcg": (i32, [vp, P(Csr), vp, vp, P(KrylovOpts), vp, sz, P(KrylovStats)]),
    "oasis_pcg_noalloc": (i32, [vp, P(Csr), vp, vp, P(KrylovOpts), P(KrylovStats)]),
    "oasis_bicgstab": (i32, [vp, P(Csr), i32, vp, vp, P(KrylovOpts), vp, sz, P(KrylovStats)]),
    "oasis_amg_setup": (i32, [vp, P(Csr), vp, P(AmgParams), P(vp)]),
    "oasis_amg_workspace_size": (i32, [vp, P(sz)]),
    "oasis_amg_upload": (i32, [vp, vp, vp, sz]),
    "oasis_amg_levels": (i32, [vp, P(i32)]),
    "oasis_amg_level": (i32, [vp, i32, P(AmgLevelInfo)]),
    "oasis_amg_vcycle": (i32, [vp, vp, vp, vp]),
    "oasis_amg_pcg": (i32, [vp, vp, vp, vp, P(KrylovOpts), P(KrylovStats)]),
    "oasis_amg_destroy": (i32, [vp]),
    "oasis_ipcs_set_amg": (i32, [vp, vp]),
    "oasis_ipcs_workspace_size": (i32, [P(Mesh), i32, P(IpcsParams), P(sz)]),
    "oasis_ipcs_create": (i32, [vp, P(Mesh), vp, vp, i32, P(IpcsParams), vp, sz, P(vp)]),
    "oasis_ipcs_step": (i32, [vp, vp, P(State), vp, vp, P(StepStats)]),
    "oasis_ipcs_matrix": (i32, [vp, i32, P(vp), P(vp)]),
    "oasis_ipcs_destroy": (i32, [vp]),
    "oasis_ipcs_set_warmstart": (i32, [vp, vp, vp, vp, sz]),
    "oasis_mpnn_workspace_size": (i32, [i32, P(sz)]),
    "oasis_mpnn_forward": (i32, [vp, P(Csr), vp, i32, vp, vp, vp, vp, vp, vp, vp, sz]),
    "oasis_mpnn_backward": (i32, [vp, P(Csr), vp, vp, vp, vp, vp, i32, P(f64), vp, sz]),
    "oasis_mpnn_adam": (i32, [vp, vp, vp, vp, vp, i32, f32, f32, f32, f32]),
    "oasis_strerror": (C.c_char_p, [i32]),
    "oasis_last_hip_error": (i32, []),
    "oasis_version": (C.c_char_p, []),
}

_lib = None


def load():
    """Load liboasis.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("liboasis.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7)
    # as the one liboasis links; whichever is loaded first serves the whole
    # process, so load torch's first: device memory and streams come from
    # torch, and the library must share its runtime.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class OasisError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        msg = lib.oasis_strerror(code).decode()
        if code == EHIP:
            msg += " (hipError %d)" % lib.oasis_last_hip_error()
        super().__init__("%s: %s [%d]" % (where, msg, code))
        self.code = code


def check(code, where, allow=()):
    if code != OK and code not in allow:
        raise OasisError(code, where)
    return code
