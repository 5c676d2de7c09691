"""MI355X (gfx950) hot path of the P1-P1 IPCS_ABCN Navier-Stokes scheme.

The compute lives in liboasis.so (hand-written HIP kernels behind the C ABI
of include/oasis.h); this package is its ctypes binding plus a small
time-stepping driver.  Importing it loads the library and fails loudly if
it has not been built.
"""
from . import _lib
from ._lib import (OK, EINVAL, EHIP, ENOTCONV, EBREAKDOWN, ENAN, EWORKSPACE, EUNSUPPORTED, F32, F64,
                   FORM_CONV, FORM_GRAD_X, FORM_GRAD_Y, FORM_GRAD_Z, FORM_MASS, FORM_STIFF, PSTART_PREV,
                   PSTART_ZERO, ASSEMBLE_ROWS, ASSEMBLE_COLORS, INSPECT_A, INSPECT_DIAG_A, INSPECT_RHS,
                   STORAGE_AUTO, STORAGE_ELL, STORAGE_CSR, CG_FORM_AUTO, CG_FORM_TWO, CG_FORM_SINGLE,
                   UPDATE_LUMPED, UPDATE_CONSISTENT, UPDATE_GRADIENT, CONV_ABCN, CONV_ABE, MAX_SCALARS,
                   MPNN_LOSS_MSE, MPNN_LOSS_KNORM, AMG_HALF_LEVEL0, OasisError)

_lib.load()

from .api import (AMG, IPCS, MPNN, DeviceCSR, DeviceMesh, assemble_p1, bicgstab, color_cells,  # noqa: E402
                  color_classes, colorize, p1_pattern, pcg, pcg_noalloc, rcm, relabel, spmv)

__all__ = ["AMG", "IPCS", "MPNN", "DeviceCSR", "DeviceMesh", "assemble_p1", "bicgstab", "color_cells", "color_classes",
           "colorize", "p1_pattern", "pcg", "pcg_noalloc", "rcm", "relabel", "spmv", "OasisError",
           "OK", "EINVAL", "EHIP", "ENOTCONV", "EBREAKDOWN", "ENAN", "EWORKSPACE", "EUNSUPPORTED", "F32", "F64",
           "FORM_MASS", "FORM_STIFF", "FORM_GRAD_X", "FORM_GRAD_Y", "FORM_GRAD_Z", "FORM_CONV", "PSTART_PREV",
           "PSTART_ZERO", "ASSEMBLE_ROWS", "ASSEMBLE_COLORS", "INSPECT_A", "INSPECT_DIAG_A", "INSPECT_RHS",
           "STORAGE_AUTO", "STORAGE_ELL", "STORAGE_CSR", "CG_FORM_AUTO", "CG_FORM_TWO", "CG_FORM_SINGLE",
           "UPDATE_LUMPED", "UPDATE_CONSISTENT", "UPDATE_GRADIENT", "CONV_ABCN", "CONV_ABE", "MAX_SCALARS",
           "MPNN_LOSS_MSE", "MPNN_LOSS_KNORM", "AMG_HALF_LEVEL0"]
