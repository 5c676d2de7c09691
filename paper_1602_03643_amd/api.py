"""Python binding of the C ABI: the same entry points, taking torch tensors.

Argument marshalling only: every operation runs in liboasis.so on the GPU.
Device memory (including every workspace) is allocated here with torch and
handed to the library; the library itself never allocates.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


def _lib():
    return L.load()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(device=None):
    return torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)


def _workspace(nbytes, device=None):
    # 256-byte aligned by the caching allocator
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=_dev(device))


# ---------------------------------------------------------------------------
# data holders

@dataclass
class DeviceCSR:
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor | None = None

    @property
    def n(self):
        return self.row_ptr.numel() - 1

    @property
    def nnz(self):
        return self.col_idx.numel()

    def with_values(self, val):
        return DeviceCSR(self.row_ptr, self.col_idx, val)

    def c(self):
        v = self.val
        dt = L.F64 if (v is None or v.dtype == torch.float64) else L.F32
        return L.Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                     None if v is None else v.data_ptr(), dt)


@dataclass
class DeviceMesh:
    dim: int
    coords: torch.Tensor          # float64 [n_vert, dim]
    cells: torch.Tensor           # int32 [n_cell, dim+1]
    vert2dof: torch.Tensor        # int32 [n_vert]
    n_dof: int
    color_ptr: np.ndarray | None = None       # host int32 [n_colors+1]
    color_cells: torch.Tensor | None = None   # int32 [n_cell]
    _cptr: object = field(default=None, repr=False)

    @classmethod
    def from_arrays(cls, dim, coords, cells, vert2dof, n_dof, device=None):
        d = _dev(device)
        return cls(int(dim), torch.as_tensor(np.ascontiguousarray(coords), dtype=torch.float64).to(d),
                   torch.as_tensor(np.ascontiguousarray(cells), dtype=torch.int32).to(d),
                   torch.as_tensor(np.ascontiguousarray(vert2dof), dtype=torch.int32).to(d), int(n_dof))

    @property
    def n_vert(self):
        return self.coords.shape[0]

    @property
    def n_cell(self):
        return self.cells.shape[0]

    @property
    def n_colors(self):
        return 0 if self.color_ptr is None else len(self.color_ptr) - 1

    def c(self):
        if self.color_ptr is not None:
            self._cptr = (C.c_int32 * len(self.color_ptr))(*[int(v) for v in self.color_ptr])
            cp = C.cast(self._cptr, C.POINTER(C.c_int32))
        else:
            cp = None
        return L.Mesh(self.dim, self.n_vert, self.n_cell, self.n_dof, self.coords.data_ptr(),
                      self.cells.data_ptr(), self.vert2dof.data_ptr(), self.n_colors, cp,
                      None if self.color_cells is None else self.color_cells.data_ptr())


# ---------------------------------------------------------------------------
# graph set-up

def p1_pattern(mesh: DeviceMesh, stream=None) -> DeviceCSR:
    lib = _lib()
    cm = mesh.c()
    nb = C.c_size_t()
    L.check(lib.oasis_graph_workspace_size(C.byref(cm), C.byref(nb)), "oasis_graph_workspace_size")
    ws = _workspace(nb.value, mesh.coords.device)
    row_ptr = torch.empty(mesh.n_dof + 1, dtype=torch.int32, device=mesh.coords.device)
    nnz = C.c_int32()
    L.check(lib.oasis_p1_pattern(_stream(stream), C.byref(cm), _p(row_ptr), None, 0, C.byref(nnz),
                                 _p(ws), ws.numel()), "oasis_p1_pattern")
    col_idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=mesh.coords.device)[: nnz.value]
    L.check(lib.oasis_p1_pattern(_stream(stream), C.byref(cm), _p(row_ptr), _p(col_idx), nnz.value,
                                 C.byref(nnz), _p(ws), ws.numel()), "oasis_p1_pattern")
    return DeviceCSR(row_ptr, col_idx)


def color_cells(mesh: DeviceMesh, priority: torch.Tensor, stream=None):
    lib = _lib()
    cm = mesh.c()
    nb = C.c_size_t()
    L.check(lib.oasis_graph_workspace_size(C.byref(cm), C.byref(nb)), "oasis_graph_workspace_size")
    ws = _workspace(nb.value, mesh.coords.device)
    color = torch.empty(mesh.n_cell, dtype=torch.int32, device=mesh.coords.device)
    nc = C.c_int32()
    L.check(lib.oasis_color_cells(_stream(stream), C.byref(cm), _p(priority.to(torch.int32).contiguous()),
                                  _p(color), C.byref(nc), _p(ws), ws.numel()), "oasis_color_cells")
    return color, nc.value


def color_classes(mesh: DeviceMesh, color: torch.Tensor, n_colors: int, stream=None):
    lib = _lib()
    cm = mesh.c()
    nb = C.c_size_t()
    L.check(lib.oasis_graph_workspace_size(C.byref(cm), C.byref(nb)), "oasis_graph_workspace_size")
    ws = _workspace(nb.value, mesh.coords.device)
    cptr = (C.c_int32 * (n_colors + 1))()
    cells = torch.empty(mesh.n_cell, dtype=torch.int32, device=mesh.coords.device)
    L.check(lib.oasis_color_classes(_stream(stream), mesh.n_cell, _p(color), n_colors, cptr, _p(cells),
                                    _p(ws), ws.numel()), "oasis_color_classes")
    return np.array(cptr[:], dtype=np.int32), cells


def colorize(mesh: DeviceMesh, priority: torch.Tensor, stream=None) -> torch.Tensor:
    """Colour the cells and attach the colour classes to `mesh`."""
    color, nc = color_cells(mesh, priority, stream)
    mesh.color_ptr, mesh.color_cells = color_classes(mesh, color, nc, stream)
    return color


def rcm(pattern: DeviceCSR, stream=None):
    lib = _lib()
    n = pattern.n
    nb = C.c_size_t()
    L.check(lib.oasis_rcm_workspace_size(n, C.byref(nb)), "oasis_rcm_workspace_size")
    ws = _workspace(nb.value, pattern.row_ptr.device)
    perm = torch.empty(n, dtype=torch.int32, device=pattern.row_ptr.device)
    order = torch.empty_like(perm)
    L.check(lib.oasis_rcm(_stream(stream), n, _p(pattern.row_ptr), _p(pattern.col_idx), _p(perm), _p(order),
                          _p(ws), ws.numel()), "oasis_rcm")
    return perm, order


def relabel(x: torch.Tensor, perm: torch.Tensor, stream=None) -> torch.Tensor:
    out = torch.empty_like(x)
    L.check(_lib().oasis_relabel(_stream(stream), x.numel(), _p(x), _p(perm), _p(out)), "oasis_relabel")
    return out


# ---------------------------------------------------------------------------
# assembly and products

def assemble_p1(mesh: DeviceMesh, pattern: DeviceCSR, form: int, uab=None, alpha=1.0, base=None,
                out=None, stream=None) -> torch.Tensor:
    val = torch.empty(pattern.nnz, dtype=torch.float64, device=pattern.row_ptr.device) if out is None else out
    A = pattern.with_values(val).c()
    B = pattern.with_values(base).c() if base is not None else None
    arr = None
    if uab is not None:
        arr = (C.c_void_p * 3)(*[u.data_ptr() for u in uab] + [None] * (3 - len(uab)))
    L.check(_lib().oasis_assemble_p1(_stream(stream), C.byref(mesh.c()), form, arr, float(alpha),
                                     None if B is None else C.byref(B), C.byref(A)), "oasis_assemble_p1")
    return val


def spmv(A: DeviceCSR, x: torch.Tensor, y: torch.Tensor, alpha=1.0, beta=0.0, stream=None):
    L.check(_lib().oasis_spmv(_stream(stream), C.byref(A.c()), _p(x), _p(y), float(alpha), float(beta)),
            "oasis_spmv")
    return y


def _tuning(storage=L.STORAGE_AUTO, grid_cap=0, cg_form=L.CG_FORM_AUTO):
    return L.Tuning(int(storage), int(grid_cap), int(cg_form))


def _opts(rtol, maxit, precision, inner_rtol, max_outer, check_every, time_kernel, tuning=None):
    return L.KrylovOpts(float(rtol), int(maxit), int(precision), float(inner_rtol), int(max_outer),
                        int(check_every), L.KRYLOV_TIME if time_kernel else 0,
                        tuning if tuning is not None else _tuning())


def _stats(st):
    return dict(iters=st.iters, outer_iters=st.outer_iters, status=st.status, restarts=st.restarts,
                rel_res=st.rel_res, kernel_ms=st.kernel_ms, kernel_count=st.kernel_count,
                ell_patterns=st.ell_patterns)


def pcg(A: DeviceCSR, b, x, rtol=1e-8, maxit=10000, precision=L.F64, inner_rtol=0.1, max_outer=50,
        check_every=0, time_kernel=False, ws=None, stream=None, raise_on=True, nullspace_const=False,
        storage=L.STORAGE_AUTO, grid_cap=0, cg_form=L.CG_FORM_AUTO):
    """F32 mode: FP32 iterations with reliable updates every `inner_rtol`
    reduction of the residual.  storage, grid_cap, cg_form: oasis_tuning."""
    lib = _lib()
    o = _opts(rtol, maxit, precision, inner_rtol, max_outer, check_every, time_kernel,
              _tuning(storage, grid_cap, cg_form))
    if nullspace_const:
        o.flags |= L.KRYLOV_NULLSPACE_CONST
    nb = C.c_size_t()
    L.check(lib.oasis_krylov_workspace_size(A.n, A.nnz, 1, C.byref(o), C.byref(nb)), "oasis_krylov_workspace_size")
    if ws is None or ws.numel() < nb.value:
        ws = _workspace(nb.value, b.device)
    st = L.KrylovStats()
    rc = lib.oasis_pcg(_stream(stream), C.byref(A.c()), _p(b), _p(x), C.byref(o), _p(ws), ws.numel(), C.byref(st))
    if raise_on:
        L.check(rc, "oasis_pcg", allow=(L.ENOTCONV, L.EBREAKDOWN, L.ENAN))
    out = _stats(st)
    out["rc"] = rc
    return out


def pcg_noalloc(A: DeviceCSR, b, x, rtol=1e-8, maxit=10000, precision=L.F64, inner_rtol=0.1, check_every=0,
                stream=None, raise_on=True, nullspace_const=False, storage=L.STORAGE_ELL, grid_cap=0,
                cg_form=L.CG_FORM_AUTO):
    """oasis_pcg with the library's own scratch array as workspace (no
    device allocation here or in the library)."""
    o = _opts(rtol, maxit, precision, inner_rtol, 0, check_every, False, _tuning(storage, grid_cap, cg_form))
    if nullspace_const:
        o.flags |= L.KRYLOV_NULLSPACE_CONST
    st = L.KrylovStats()
    rc = _lib().oasis_pcg_noalloc(_stream(stream), C.byref(A.c()), _p(b), _p(x), C.byref(o), C.byref(st))
    if raise_on:
        L.check(rc, "oasis_pcg_noalloc", allow=(L.ENOTCONV, L.EBREAKDOWN, L.ENAN))
    out = _stats(st)
    out["rc"] = rc
    return out


def bicgstab(A: DeviceCSR, b, x, rtol=1e-8, maxit=10000, precision=L.F64, inner_rtol=1e-4, max_outer=50,
             check_every=0, time_kernel=False, ws=None, stream=None, raise_on=True,
             storage=L.STORAGE_AUTO, grid_cap=0):
    """b, x: [nrhs, n] (or [n]) float64 tensors; x holds x0 on entry."""
    lib = _lib()
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    o = _opts(rtol, maxit, precision, inner_rtol, max_outer, check_every, time_kernel,
              _tuning(storage, grid_cap))
    nb = C.c_size_t()
    L.check(lib.oasis_krylov_workspace_size(A.n, A.nnz, nrhs, C.byref(o), C.byref(nb)),
            "oasis_krylov_workspace_size")
    if ws is None or ws.numel() < nb.value:
        ws = _workspace(nb.value, b.device)
    st = (L.KrylovStats * nrhs)()
    rc = lib.oasis_bicgstab(_stream(stream), C.byref(A.c()), nrhs, _p(b), _p(x), C.byref(o), _p(ws), ws.numel(),
                            st)
    if raise_on:
        L.check(rc, "oasis_bicgstab", allow=(L.ENOTCONV, L.EBREAKDOWN, L.ENAN))
    return [dict(_stats(s), rc=rc) for s in st]


# ---------------------------------------------------------------------------
# algebraic multigrid

class AMG:
    """Handle for oasis_amg_setup/upload/vcycle/pcg/destroy: the
    smoothed-aggregation hierarchy of an F64 CSR matrix (set up on the host
    by the library) and its device image in a torch-allocated workspace."""

    def __init__(self, A: DeviceCSR, B=None, precision=L.F64, singular=False, theta=0.0, coarse_size=0,
                 max_levels=0, storage=L.STORAGE_AUTO, grid_cap=0, stream=None, half_level0=False):
        """half_level0: an FP32 cycle reads level 0's values stored as FP16
        (OASIS_AMG_HALF_LEVEL0)."""
        lib = _lib()
        self.A, self.B = A, B
        self.n = A.n
        flags = (L.KRYLOV_NULLSPACE_CONST if singular else 0) | (L.AMG_HALF_LEVEL0 if half_level0 else 0)
        self.params = L.AmgParams(float(theta), int(coarse_size), int(max_levels), int(precision), flags,
                                  _tuning(storage, grid_cap))
        self._csr = A.c()
        h = C.c_void_p()
        L.check(lib.oasis_amg_setup(_stream(stream), C.byref(self._csr), _p(B), C.byref(self.params), C.byref(h)),
                "oasis_amg_setup")
        self.handle = h
        nb = C.c_size_t()
        L.check(lib.oasis_amg_workspace_size(h, C.byref(nb)), "oasis_amg_workspace_size")
        self.ws = _workspace(nb.value, A.row_ptr.device)
        L.check(lib.oasis_amg_upload(_stream(stream), h, _p(self.ws), self.ws.numel()), "oasis_amg_upload")

    def n_levels(self):
        v = C.c_int32()
        L.check(_lib().oasis_amg_levels(self.handle, C.byref(v)), "oasis_amg_levels")
        return v.value

    def level(self, l):
        """Host copy of level l: dict of numpy arrays (matrix, near-null vector,
        omega, aggregation, prolongator; coarse_inv on the coarsest level)."""
        info = L.AmgLevelInfo()
        L.check(_lib().oasis_amg_level(self.handle, int(l), C.byref(info)), "oasis_amg_level")
        n, nnz = info.n, info.nnz
        arr = lambda ptr, cnt: np.ctypeslib.as_array(ptr, shape=(cnt,)).copy()  # noqa: E731
        out = dict(n=n, row_ptr=arr(info.row_ptr, n + 1), col_idx=arr(info.col_idx, nnz), val=arr(info.val, nnz),
                   near_null=arr(info.near_null, n), omega=info.omega, n_agg=info.n_agg)
        if info.n_agg > 0:
            out.update(agg=arr(info.agg, n), p_row_ptr=arr(info.p_row_ptr, n + 1),
                       p_col_idx=arr(info.p_col_idx, info.p_nnz), p_val=arr(info.p_val, info.p_nnz))
        else:
            out["coarse_inv"] = arr(info.coarse_inv, n * n).reshape(n, n)
        return out

    def vcycle(self, r, z=None, stream=None):
        z = torch.empty_like(r) if z is None else z
        L.check(_lib().oasis_amg_vcycle(_stream(stream), self.handle, _p(r), _p(z)), "oasis_amg_vcycle")
        return z

    def pcg(self, b, x, rtol=1e-8, maxit=1000, check_every=0, time_kernel=False, stream=None, raise_on=True,
            precision=L.F64, inner_rtol=0.0):
        """precision F32 (FP32 handles): the mixed-precision CG, whose FP64
        residual replaces the recursive one every inner_rtol reduction
        (0: the library's default)."""
        o = _opts(rtol, maxit, precision, inner_rtol, 0, check_every, time_kernel)
        st = L.KrylovStats()
        rc = _lib().oasis_amg_pcg(_stream(stream), self.handle, _p(b), _p(x), C.byref(o), C.byref(st))
        if raise_on:
            L.check(rc, "oasis_amg_pcg", allow=(L.ENOTCONV, L.EBREAKDOWN, L.ENAN))
        out = _stats(st)
        out["rc"] = rc
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib().oasis_amg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# the IPCS step

class IPCS:
    """Handle for oasis_ipcs_create/step/destroy on one mesh."""

    def __init__(self, mesh: DeviceMesh, pattern: DeviceCSR, dt, nu, f, bc_dofs: torch.Tensor,
                 rtol_u=1e-8, rtol_p=1e-8, maxit=10000, precision=L.F64, inner_rtol=0.0,
                 assembly=L.ASSEMBLE_ROWS, pressure_start=L.PSTART_PREV, pressure_delta=0.0,
                 storage=L.STORAGE_AUTO, grid_cap=0, cg_form=L.CG_FORM_AUTO, inner_iters=1,
                 velocity_update=L.UPDATE_LUMPED, diffusivity=(), scalar_source=None, convection=L.CONV_ABCN,
                 stream=None):
        lib = _lib()
        self.mesh, self.pattern = mesh, pattern
        self.dim, self.n = mesh.dim, mesh.n_dof
        self.bc_dofs = bc_dofs.to(torch.int32).contiguous()
        fv = (C.c_double * 3)(*([float(v) for v in f] + [0.0] * (3 - len(f))))
        nsc = len(diffusivity)
        if nsc > L.MAX_SCALARS:
            raise ValueError("at most %d scalars" % L.MAX_SCALARS)
        src = list(scalar_source) if scalar_source is not None else [0.0] * nsc
        dv = (C.c_double * 4)(*([float(v) for v in diffusivity] + [0.0] * (4 - nsc)))
        sv = (C.c_double * 4)(*([float(v) for v in src] + [0.0] * (4 - len(src))))
        self.n_scalars = nsc
        self.params = L.IpcsParams(float(dt), float(nu), fv, int(self.bc_dofs.numel()),
                                   self.bc_dofs.data_ptr() if self.bc_dofs.numel() else None,
                                   float(rtol_u), float(rtol_p), int(maxit), int(precision), float(inner_rtol),
                                   int(assembly), int(pressure_start), float(pressure_delta),
                                   _tuning(storage, grid_cap, cg_form), int(inner_iters), int(velocity_update),
                                   nsc, dv, sv, int(convection))
        cm = mesh.c()
        nb = C.c_size_t()
        L.check(lib.oasis_ipcs_workspace_size(C.byref(cm), pattern.nnz, C.byref(self.params), C.byref(nb)),
                "oasis_ipcs_workspace_size")
        self.ws = _workspace(nb.value, mesh.coords.device)
        h = C.c_void_p()
        L.check(lib.oasis_ipcs_create(_stream(stream), C.byref(cm), _p(pattern.row_ptr), _p(pattern.col_idx),
                                      pattern.nnz, C.byref(self.params), _p(self.ws), self.ws.numel(),
                                      C.byref(h)), "oasis_ipcs_create")
        self.handle = h
        self._mesh_c = cm

    def step(self, U1, U2, Un, p, phi, bc_values=None, phi_guess=None, UI=None, b_phi=None, stream=None,
             raise_on=True, C1=None, Cn=None, C_bc=None):
        """U1, U2, Un: [dim, n] float64; p, phi: [n] (updated in place).
        Scalars: C1, Cn [n_scalars, n], C_bc [n_scalars, n_bc]."""
        st = L.State()

        def rows(t, count):
            # the addresses of t[0], t[1], ... without building row views
            if t.dim() == 1:
                return [t.data_ptr()]
            base, step = t.data_ptr(), t.stride(0) * t.element_size()
            return [base + k * step for k in range(count)]

        if self.n_scalars:
            c1, cn = rows(C1, self.n_scalars), rows(Cn, self.n_scalars)
            cb = rows(C_bc, self.n_scalars) if C_bc is not None else None
            for a in range(self.n_scalars):
                st.C1[a], st.Cn[a] = c1[a], cn[a]
                if cb is not None:
                    st.C_bc[a] = cb[a]
        u1, u2, un = rows(U1, self.dim), rows(U2, self.dim), rows(Un, self.dim)
        ui = rows(UI, self.dim) if UI is not None else None
        for k in range(self.dim):
            st.U1[k], st.U2[k], st.Un[k] = u1[k], u2[k], un[k]
            if ui is not None:
                st.UI[k] = ui[k]
        st.p = p.data_ptr()
        st.phi = phi.data_ptr()
        st.b_phi = None if b_phi is None else b_phi.data_ptr()
        stats = L.StepStats()
        rc = _lib().oasis_ipcs_step(_stream(stream), self.handle, C.byref(st), _p(bc_values), _p(phi_guess),
                                    C.byref(stats))
        if raise_on:
            L.check(rc, "oasis_ipcs_step", allow=(L.ENOTCONV,))
        d = dict(iters_u=list(stats.iters_u)[: self.dim], iters_p=stats.iters_p, outer_u=stats.outer_u,
                 outer_p=stats.outer_p, status=stats.status, guess_used=stats.guess_used,
                 res_u=list(stats.res_u)[: self.dim], res_p=stats.res_p, ms_assemble=stats.ms_assemble,
                 ms_velocity=stats.ms_velocity, ms_pressure=stats.ms_pressure, ms_update=stats.ms_update,
                 ms_total=stats.ms_total, iters_m=list(stats.iters_m)[: self.dim],
                 iters_c=list(stats.iters_c)[: self.n_scalars], res_c=list(stats.res_c)[: self.n_scalars],
                 ms_scalars=stats.ms_scalars, rc=rc)
        return d

    def pressure_amg(self, precision=L.F64, theta=0.0, coarse_size=0, max_levels=0, stream=None,
                     half_level0=False):
        """Build a multigrid hierarchy on the handle's scaled pressure matrix,
        upload it and attach it to the pressure solve (oasis_ipcs_set_amg)."""
        Ks, s = self.matrix(L.FORM_STIFF, copy=False)     # the hierarchy keeps these by reference
        amg = AMG(self.pattern.with_values(Ks), s, precision=precision, singular=True, theta=theta,
                  coarse_size=coarse_size, max_levels=max_levels, stream=stream, half_level0=half_level0)
        self.set_amg(amg)
        return amg

    def set_amg(self, amg):
        """Attach an AMG handle built on this handle's pressure matrix (None
        detaches it: Jacobi again)."""
        L.check(_lib().oasis_ipcs_set_amg(self.handle, None if amg is None else amg.handle), "oasis_ipcs_set_amg")
        self._amg = amg

    def set_warmstart(self, params, coords):
        """Attach a learned pressure warm start (params: float32 [MPNN.NPARAM],
        coords: float64 [n, dim], both on the device); None detaches it."""
        lib = _lib()
        if params is None:
            L.check(lib.oasis_ipcs_set_warmstart(self.handle, None, None, None, 0), "oasis_ipcs_set_warmstart")
            self._warm = None
            return
        params = params.to(torch.float32).contiguous()
        coords = coords.to(torch.float64).contiguous()
        nb = C.c_size_t()
        L.check(lib.oasis_mpnn_workspace_size(self.n, C.byref(nb)), "oasis_mpnn_workspace_size")
        ws = _workspace(nb.value, params.device)
        L.check(lib.oasis_ipcs_set_warmstart(self.handle, _p(params), _p(coords), _p(ws), ws.numel()),
                "oasis_ipcs_set_warmstart")
        self._warm = (params, coords, ws)   # kept alive while attached

    def matrix(self, which, count=None, copy=True):
        """A handle matrix's values on the pattern as a device tensor: a copy,
        or (copy=False) a view of the handle's own memory."""
        val = C.c_void_p()
        sq = C.c_void_p()
        L.check(_lib().oasis_ipcs_matrix(self.handle, int(which), C.byref(val), C.byref(sq)), "oasis_ipcs_matrix")
        n = self.pattern.nnz if count is None else count
        out = _from_ptr(val.value, n, self.ws, copy)
        sqt = _from_ptr(sq.value, self.n, self.ws, copy) if sq.value else None
        return out, sqt

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _lib().oasis_ipcs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _from_ptr(ptr, count, ws, copy=True):
    """`count` doubles at device address ptr (inside ws): a new tensor, or a
    view of ws."""
    base = ws.data_ptr()
    off = ptr - base
    if off < 0 or off % 8 or off + 8 * count > ws.numel():
        raise ValueError("pointer outside the workspace")
    v = ws[off: off + 8 * count].view(torch.float64)
    return v.clone() if copy else v


# ---------------------------------------------------------------------------
# learned warm start

class MPNN:
    """Workspace holder for oasis_mpnn_forward / backward / adam on one graph.

    Ks, s: the scaled pressure matrix (unit diagonal) and sqrt(diag K), as an
    IPCS handle holds them (IPCS.matrix(FORM_STIFF))."""

    NPARAM = L.MPNN_NPARAM

    def __init__(self, Ks: DeviceCSR, s: torch.Tensor, coords: torch.Tensor | None = None):
        lib = _lib()
        self.Ks, self.s = Ks, s
        self.coords = coords
        self.dim = 0 if coords is None else int(coords.shape[1])
        nb = C.c_size_t()
        L.check(lib.oasis_mpnn_workspace_size(Ks.n, C.byref(nb)), "oasis_mpnn_workspace_size")
        self.ws = _workspace(nb.value, s.device)

    def forward(self, params, b_phi, phi_prev, guess=None, delta=None, stream=None):
        L.check(_lib().oasis_mpnn_forward(_stream(stream), C.byref(self.Ks.c()), _p(self.s), self.dim,
                                          _p(self.coords), _p(b_phi), _p(phi_prev), _p(params), _p(guess),
                                          _p(delta), _p(self.ws), self.ws.numel()), "oasis_mpnn_forward")
        return guess, delta

    def backward(self, params, phi, phi_prev, grad, loss_kind=L.MPNN_LOSS_MSE, stream=None):
        """Loss of the last forward pass (MPNN_LOSS_MSE or MPNN_LOSS_KNORM)
        and its parameter gradient into grad."""
        loss = C.c_double()
        L.check(_lib().oasis_mpnn_backward(_stream(stream), C.byref(self.Ks.c()), _p(self.s), _p(phi),
                                           _p(phi_prev), _p(params), _p(grad), int(loss_kind), C.byref(loss),
                                           _p(self.ws), self.ws.numel()), "oasis_mpnn_backward")
        return loss.value

    @staticmethod
    def adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        L.check(_lib().oasis_mpnn_adam(_stream(stream), _p(params), _p(grad), _p(m), _p(v), int(t), float(lr),
                                       float(beta1), float(beta2), float(eps)), "oasis_mpnn_adam")
