"""MI355X (gfx950) finite-element assembly + Jacobi-PCG, Python binding.

Every step of the path runs in the HIP kernels of libfeasm.so; this module
only marshals arguments through the C ABI (include/feasm.h).  PyTorch is used
for device memory and the stream.  There is no CPU fallback: without the
built library or a GPU the calls raise.

    ctx  = Context()                                   # device 0, torch's current stream
    mesh = Mesh(ctx, HEX08, coords, conn, dirichlet)   # host numpy arrays, user numbering
    u_m  = mesh.to_mesh(u_user)                         # device arrays are in mesh numbering
    values, rhs, info = assemble(mesh, MOMENTUM, dt, u=u_m, rho=rho_m, mu=mu_m)
    apply_dirichlet(mesh, L, f)
    x, cg = cg_solve(mesh, L, f, rtol=1e-8)
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref

import numpy as np

from . import capi
from .capi import (FE_FP64, FE_HEX08, FE_MIXED, FE_OP_MOMENTUM, FE_OP_POISSON, FE_OP_SCALAR,
                   FE_PEN06, FE_PYR05, FE_TET04, FE_UPLOAD_RENUMBER)

HEX08, PEN06, PYR05, TET04 = FE_HEX08, FE_PEN06, FE_PYR05, FE_TET04
HYBRID = 0   # mixed element types: Mesh(..., types=...) with conn [E, 8]
MOMENTUM, SCALAR, POISSON = FE_OP_MOMENTUM, FE_OP_SCALAR, FE_OP_POISSON
FP64, MIXED = FE_FP64, FE_MIXED

__all__ = ["Context", "Mesh", "Plan", "Server", "assemble", "assemble_block", "apply_dirichlet", "spmv", "dot", "axpy", "cg_solve",
           "cg_solve_noalloc", "residual", "gradient", "divergence", "fractional_step", "wall_traction", "scalar_residual",
           "scalar_step", "FULL_STRESS", "EMAC",
           "FeError", "HEX08", "PEN06", "PYR05", "TET04", "HYBRID", "MOMENTUM", "SCALAR", "POISSON", "FP64", "MIXED", "pack_layout"]


class FeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{capi.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_dev(t, dtype, n, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{name}: need a contiguous {dtype} tensor with >= {n} entries")


_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def _close_all():
    # Release device objects while the HIP runtime is still up (atexit runs
    # before the runtime's own teardown); destroying a context frees its meshes.
    for c in list(_LIVE_CONTEXTS):
        c.close()


class Context:
    """One device and one stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = capi.load()
        self.device = device
        with torch.cuda.device(device):
            s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = C.c_void_p()
        st = self.lib.fe_ctx_create(device, C.c_void_p(s.cuda_stream), C.byref(h))
        if st != capi.FE_OK:
            raise FeError(st, "fe_ctx_create failed")
        self.h = h
        self._meshes = weakref.WeakSet()
        self._servers = weakref.WeakSet()
        _LIVE_CONTEXTS.add(self)

    def error(self) -> str:
        return self.lib.fe_ctx_last_error(self.h).decode()

    def check(self, st: int):
        if st != capi.FE_OK:
            raise FeError(st, self.error())

    def profile(self, enable: bool = True):
        self.check(self.lib.fe_ctx_profile(self.h, 1 if enable else 0))

    def profile_read(self, slot: int):
        n = C.c_int64()
        ms = C.c_double()
        self.check(self.lib.fe_ctx_profile_read(self.h, slot, C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)

    def close(self):
        if getattr(self, "h", None):
            for sv in list(self._servers):
                sv.close()          # servers first: they use the context's device
            for m in list(self._meshes):
                m.h = None          # freed by fe_ctx_destroy
            self.lib.fe_ctx_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check usable while module globals
        # are torn down at interpreter exit
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """A preprocessed, device-resident mesh (fe_mesh_upload)."""

    def __init__(self, ctx: Context, elem_type: int, coords, conn, dirichlet=None, renumber: bool = True,
                 types=None, coloured: bool = False, symmetric_spmv: bool = True):
        """elem_type: HEX08, PEN06, PYR05, TET04 (conn [E, nen]) or HYBRID with
        types [E] node counts and conn [E, 8] (fe_mesh_upload_mixed).
        coloured: HEX08 matrix assembly by coloured element blocks (the
        serving runtime's form) instead of owner groups.
        symmetric_spmv=False: FE_UPLOAD_GENERAL_SPMV (a mesh solved once)."""
        self.ctx = ctx
        lib = ctx.lib
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        width = 8 if elem_type == HYBRID else elem_type
        if coords.ndim != 2 or coords.shape[1] != 3 or conn.ndim != 2 or conn.shape[1] != width:
            raise ValueError("coords must be [N,3] and conn [E,nen] ([E,8] for a hybrid mesh)")
        if (elem_type == HYBRID) != (types is not None):
            raise ValueError("types are given exactly for a HYBRID mesh")
        d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.int32)
        nd, dp = (0, None) if d is None else (d.shape[0], d.ctypes.data)
        flags = ((FE_UPLOAD_RENUMBER if renumber else 0) | (capi.FE_UPLOAD_COLOURED if coloured else 0) |
                 (0 if symmetric_spmv else capi.FE_UPLOAD_GENERAL_SPMV))
        h = C.c_void_p()
        if types is None:
            st = lib.fe_mesh_upload(ctx.h, elem_type, coords.shape[0], coords.ctypes.data, conn.shape[0],
                                    conn.ctypes.data, nd, dp, flags, C.byref(h))
        else:
            types = np.ascontiguousarray(types, dtype=np.uint8)
            if types.shape != (conn.shape[0],):
                raise ValueError("types must be [E]")
            st = lib.fe_mesh_upload_mixed(ctx.h, coords.shape[0], coords.ctypes.data, conn.shape[0],
                                          types.ctypes.data, conn.ctypes.data, nd, dp, flags, C.byref(h))
        ctx.check(st)
        self.h = h
        ctx._meshes.add(self)
        desc = capi.MeshDesc()
        ctx.check(lib.fe_mesh_info(h, C.byref(desc)))
        self.desc = desc
        self.nen = desc.nen
        self.n_nodes = desc.n_nodes
        self.n_elems = desc.n_elems
        self.nnz = desc.nnz
        self.node_perm = np.zeros(self.n_nodes, dtype=np.int32)
        self.elem_perm = np.zeros(self.n_elems, dtype=np.int32)
        ctx.check(lib.fe_mesh_perm(h, self.node_perm.ctypes.data, self.elem_perm.ctypes.data))

    def set_wall(self, face_nen, face_conn, delta: float):
        """fe_wall_faces: register the wall faces (face_nen [F] 3 or 4, face_conn
        [F, 4] user node ids) at exchange distance delta; F = 0 clears them."""
        nen = np.ascontiguousarray(face_nen, dtype=np.uint8)
        conn = np.ascontiguousarray(face_conn, dtype=np.int32)
        if conn.ndim != 2 or conn.shape[1] != 4 or nen.shape != (conn.shape[0],):
            raise ValueError("face_nen must be [F] and face_conn [F, 4]")
        self.ctx.check(self.ctx.lib.fe_wall_faces(self.h, conn.shape[0], nen.ctypes.data, conn.ctypes.data,
                                                  float(delta)))

    def info(self) -> dict:
        d = capi.MeshDesc()
        self.ctx.check(self.ctx.lib.fe_mesh_info(self.h, C.byref(d)))
        return {k: getattr(d, k) for k, _ in capi.MeshDesc._fields_ if k not in ("rowptr", "colidx")}

    def pattern_host(self):
        """(rowptr, colidx) copied to host numpy arrays, mesh numbering."""
        rp = np.empty(self.n_nodes + 1, dtype=np.int32)
        ci = np.empty(self.nnz, dtype=np.int32)
        self.ctx.check(self.ctx.lib.fe_mesh_pattern_host(self.h, rp.ctypes.data, ci.ctypes.data))
        return rp, ci

    def to_mesh(self, t_user, ncomp: int = None):
        """Device [ncomp][N] user-numbered array -> mesh numbering (new tensor)."""
        torch = _torch()
        t_user = t_user.contiguous()
        nc = ncomp or max(1, t_user.numel() // self.n_nodes)
        out = torch.empty_like(t_user)
        self.ctx.check(self.ctx.lib.fe_mesh_to_mesh_order(self.h, _ptr(t_user), _ptr(out), nc))
        return out

    def to_user(self, t_mesh, ncomp: int = None):
        torch = _torch()
        t_mesh = t_mesh.contiguous()
        nc = ncomp or max(1, t_mesh.numel() // self.n_nodes)
        out = torch.empty_like(t_mesh)
        self.ctx.check(self.ctx.lib.fe_mesh_to_user_order(self.h, _ptr(t_mesh), _ptr(out), nc))
        return out

    def close(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx.lib.fe_mesh_free(self.h)
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check usable while module globals
        # are torn down at interpreter exit
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


FULL_STRESS, EMAC = capi.FE_FORM_FULL_STRESS, capi.FE_FORM_EMAC


def residual(mesh: Mesh, u, rho, mu, out=None, form: int = 0):
    """fe_residual: out[4, N] = -(C(u) + K_mu) u (3 rows) and the lumped
    rho-mass; form: FULL_STRESS and/or EMAC operator variants."""
    torch = _torch()
    N = mesh.n_nodes
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(rho, torch.float64, N, "rho")
    _check_dev(mu, torch.float64, N, "mu")
    if out is None:
        out = torch.empty((4, N), dtype=torch.float64, device=u.device)
    _check_dev(out, torch.float64, 4 * N, "out")
    mesh.ctx.check(mesh.ctx.lib.fe_residual(mesh.h, _ptr(u), _ptr(rho), _ptr(mu), int(form), _ptr(out)))
    return out


def scalar_residual(mesh: Mesh, u, rho, Y, D: float, out=None):
    """fe_scalar_residual: out[2, N] = -(C(u) + K_{rho D}) Y and the lumped rho-mass."""
    torch = _torch()
    N = mesh.n_nodes
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(rho, torch.float64, N, "rho")
    _check_dev(Y, torch.float64, N, "Y")
    if out is None:
        out = torch.empty((2, N), dtype=torch.float64, device=u.device)
    _check_dev(out, torch.float64, 2 * N, "out")
    mesh.ctx.check(mesh.ctx.lib.fe_scalar_residual(mesh.h, _ptr(u), _ptr(rho), _ptr(Y), float(D), _ptr(out)))
    return out


def scalar_step(mesh: Mesh, dt: float, u, rho, D: float, Y):
    """fe_scalar_step: one explicit SSP-RK3 step of the scalar Y [N] (in place)."""
    torch = _torch()
    N = mesh.n_nodes
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(rho, torch.float64, N, "rho")
    _check_dev(Y, torch.float64, N, "Y")
    mesh.ctx.check(mesh.ctx.lib.fe_scalar_step(mesh.h, float(dt), _ptr(u), _ptr(rho), float(D), _ptr(Y)))
    return Y


def gradient(mesh: Mesh, p, out=None):
    """fe_gradient: out[3, N] = int N_a grad p."""
    torch = _torch()
    N = mesh.n_nodes
    _check_dev(p, torch.float64, N, "p")
    if out is None:
        out = torch.empty((3, N), dtype=torch.float64, device=p.device)
    _check_dev(out, torch.float64, 3 * N, "out")
    mesh.ctx.check(mesh.ctx.lib.fe_gradient(mesh.h, _ptr(p), _ptr(out)))
    return out


def wall_traction(mesh: Mesh, u, rho, mu, out=None):
    """fe_wall_traction: out[3, N] = the wall model's traction (nodal vector)."""
    torch = _torch()
    N = mesh.n_nodes
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(rho, torch.float64, N, "rho")
    _check_dev(mu, torch.float64, N, "mu")
    if out is None:
        out = torch.empty((3, N), dtype=torch.float64, device=u.device)
    _check_dev(out, torch.float64, 3 * N, "out")
    mesh.ctx.check(mesh.ctx.lib.fe_wall_traction(mesh.h, _ptr(u), _ptr(rho), _ptr(mu), _ptr(out)))
    return out


def divergence(mesh: Mesh, dt: float, u, rho, out=None):
    """fe_divergence: out[N] = (1/dt) int grad N_a . (rho u)."""
    torch = _torch()
    N = mesh.n_nodes
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(rho, torch.float64, N, "rho")
    if out is None:
        out = torch.empty(N, dtype=torch.float64, device=u.device)
    _check_dev(out, torch.float64, N, "out")
    mesh.ctx.check(mesh.ctx.lib.fe_divergence(mesh.h, float(dt), _ptr(u), _ptr(rho), _ptr(out)))
    return out


def fractional_step(mesh: Mesh, dt: float, rho, mu, L, u, p, rtol: float = 1e-8, max_iter: int = 20000,
                    form: int = 0, precision: int = FP64):
    """fe_fractional_step: advances u [3, N] and p [N] in place (device,
    mesh numbering); L is the Poisson matrix after apply_dirichlet.
    Returns {"cg_iterations", "cg_true_rel_residual"}."""
    torch = _torch()
    N = mesh.n_nodes
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(p, torch.float64, N, "p")
    _check_dev(rho, torch.float64, N, "rho")
    _check_dev(mu, torch.float64, N, "mu")
    _check_dev(L, torch.float64, mesh.nnz, "L")
    info = capi.StepInfo()
    mesh.ctx.check(mesh.ctx.lib.fe_fractional_step(mesh.h, float(dt), _ptr(rho), _ptr(mu), _ptr(L), int(form),
                                                   _ptr(u), _ptr(p), float(rtol), int(max_iter), int(precision),
                                                   C.byref(info)))
    return {"cg_iterations": info.cg_iterations, "cg_true_rel_residual": info.cg_true_rel_residual}


def assemble(mesh: Mesh, op: int, dt: float, u, rho, mu=None, Y=None, D=None, precision: int = FP64,
             values=None, rhs=None):
    """fe_assemble.  Returns (values[n_mat, nnz], rhs[n_rhs, N], info dict)."""
    torch = _torch()
    N, nnz = mesh.n_nodes, mesh.nnz
    dev = u.device
    ns = 0
    if op == SCALAR:
        ns = int(Y.shape[0])
        Dh = np.ascontiguousarray(np.asarray(D, dtype=np.float64))
        if Dh.shape[0] != ns:
            raise ValueError("D must have one entry per scalar")
    n_mat = ns if op == SCALAR else 1
    n_rhs = 3 if op == MOMENTUM else (ns if op == SCALAR else 1)
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(rho, torch.float64, N, "rho")
    if op == MOMENTUM:
        _check_dev(mu, torch.float64, N, "mu")
    if op == SCALAR:
        _check_dev(Y, torch.float64, ns * N, "Y")
    if values is None:
        values = torch.empty((n_mat, nnz), dtype=torch.float64, device=dev)
    if rhs is None:
        rhs = torch.empty((n_rhs, N), dtype=torch.float64, device=dev)
    _check_dev(values, torch.float64, n_mat * nnz, "values")
    _check_dev(rhs, torch.float64, n_rhs * N, "rhs")
    f = capi.Fields()
    f.op = op
    f.dt = float(dt)
    f.u = u.data_ptr()
    f.rho = rho.data_ptr()
    f.mu = mu.data_ptr() if mu is not None else None
    f.n_scalars = ns
    f.Y = Y.data_ptr() if Y is not None else None
    f.D = Dh.ctypes.data if ns else None
    info = capi.AsmInfo()
    st = mesh.ctx.lib.fe_assemble(mesh.h, C.byref(f), precision, _ptr(values), _ptr(rhs), C.byref(info))
    out = {"min_detJ": info.min_detJ, "first_bad_elem": info.first_bad_elem, "status": st}
    if st != capi.FE_OK:
        raise FeError(st, mesh.ctx.error())
    return values, rhs, out


def assemble_block(mesh: Mesh, form: int, dt: float, u, rho, mu, values=None, rhs=None):
    """fe_assemble_block: the momentum operator with the full-stress viscous
    term (form FULL_STRESS) and EMAC's (div u) term (form EMAC) as 3x3 blocks.
    Returns (values[nnz, 3, 3], rhs[3, N], info dict)."""
    torch = _torch()
    N, nnz = mesh.n_nodes, mesh.nnz
    _check_dev(u, torch.float64, 3 * N, "u")
    _check_dev(rho, torch.float64, N, "rho")
    _check_dev(mu, torch.float64, N, "mu")
    if values is None:
        values = torch.empty((nnz, 3, 3), dtype=torch.float64, device=u.device)
    if rhs is None:
        rhs = torch.empty((3, N), dtype=torch.float64, device=u.device)
    _check_dev(values, torch.float64, 9 * nnz, "values")
    _check_dev(rhs, torch.float64, 3 * N, "rhs")
    info = capi.AsmInfo()
    st = mesh.ctx.lib.fe_assemble_block(mesh.h, int(form), float(dt), _ptr(u), _ptr(rho), _ptr(mu), _ptr(values),
                                        _ptr(rhs), C.byref(info))
    out = {"min_detJ": info.min_detJ, "first_bad_elem": info.first_bad_elem, "status": st}
    if st != capi.FE_OK:
        raise FeError(st, mesh.ctx.error())
    return values, rhs, out


def apply_dirichlet(mesh: Mesh, values, rhs, g=None):
    torch = _torch()
    _check_dev(values, torch.float64, mesh.nnz, "values")
    _check_dev(rhs, torch.float64, mesh.n_nodes, "rhs")
    if g is not None:
        _check_dev(g, torch.float64, mesh.n_nodes, "g")
    mesh.ctx.check(mesh.ctx.lib.fe_apply_dirichlet(mesh.h, _ptr(values), _ptr(rhs), _ptr(g)))


def spmv(mesh: Mesh, values, x, y=None):
    torch = _torch()
    _check_dev(values, torch.float64, mesh.nnz, "values")
    _check_dev(x, torch.float64, mesh.n_nodes, "x")
    if y is None:
        y = torch.empty(mesh.n_nodes, dtype=torch.float64, device=x.device)
    mesh.ctx.check(mesh.ctx.lib.fe_spmv(mesh.h, _ptr(values), _ptr(x), _ptr(y)))
    return y


def dot(ctx: Context, x, y) -> float:
    torch = _torch()
    n = x.numel()
    _check_dev(x, torch.float64, n, "x")
    _check_dev(y, torch.float64, n, "y")
    out = C.c_double()
    ctx.check(ctx.lib.fe_dot(ctx.h, n, _ptr(x), _ptr(y), C.byref(out)))
    return float(out.value)


def axpy(ctx: Context, a: float, x, y):
    torch = _torch()
    n = x.numel()
    _check_dev(x, torch.float64, n, "x")
    _check_dev(y, torch.float64, n, "y")
    ctx.check(ctx.lib.fe_axpy(ctx.h, n, float(a), _ptr(x), _ptr(y)))
    return y


def cg_solve(mesh: Mesh, values, rhs, x=None, rtol: float = 1e-8, max_iter: int = 10000,
             precision: int = FP64, raise_on_noconv: bool = True):
    """fe_cg_solve.  Returns (x, info dict); info['status'] is the fe_status."""
    torch = _torch()
    _check_dev(values, torch.float64, mesh.nnz, "values")
    _check_dev(rhs, torch.float64, mesh.n_nodes, "rhs")
    if x is None:
        x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device=rhs.device)
    _check_dev(x, torch.float64, mesh.n_nodes, "x")
    info = capi.CGInfo()
    st = mesh.ctx.lib.fe_cg_solve(mesh.h, _ptr(values), _ptr(rhs), _ptr(x), float(rtol), int(max_iter),
                                  precision, C.byref(info))
    out = {"status": st, "iterations": info.iterations, "outer_iterations": info.outer_iterations,
           "rel_residual": info.rel_residual, "true_rel_residual": info.true_rel_residual,
           "symmetric_spmv": bool(info.symmetric_spmv)}
    if st != capi.FE_OK and (raise_on_noconv or st != capi.FE_ENOCONV):
        raise FeError(st, mesh.ctx.error())
    return x, out


def cg_solve_noalloc(mesh: Mesh, values, rhs, x=None, rtol: float = 1e-8, max_iter: int = 10000,
                     raise_on_noconv: bool = True):
    """fe_cg_solve_noalloc: FP64 PCG with its work buffers in the library's
    fixed device area (no device allocation).  Returns (x, info dict)."""
    torch = _torch()
    _check_dev(values, torch.float64, mesh.nnz, "values")
    _check_dev(rhs, torch.float64, mesh.n_nodes, "rhs")
    if x is None:
        x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device=rhs.device)
    _check_dev(x, torch.float64, mesh.n_nodes, "x")
    info = capi.CGInfo()
    st = mesh.ctx.lib.fe_cg_solve_noalloc(mesh.h, _ptr(values), _ptr(rhs), _ptr(x), float(rtol), int(max_iter),
                                          C.byref(info))
    out = {"status": st, "iterations": info.iterations, "outer_iterations": info.outer_iterations,
           "rel_residual": info.rel_residual, "true_rel_residual": info.true_rel_residual,
           "symmetric_spmv": bool(info.symmetric_spmv)}
    if st != capi.FE_OK and (raise_on_noconv or st != capi.FE_ENOCONV):
        raise FeError(st, mesh.ctx.error())
    return x, out


class Server:
    """Continuous-batching service of assemble + solve requests (fe_serve_*).

    A request is one mesh with its fields: momentum and Poisson assembly,
    Dirichlet elimination and the Jacobi-PCG pressure solve, all on the GPU.
    The host arrays of a request are kept alive here until it completes.
    """

    def __init__(self, ctx: Context, hbm_budget: int = 8 << 30, max_slots: int = 16, host_threads: int = 4):
        self.ctx = ctx
        self.lib = ctx.lib
        h = C.c_void_p()
        ctx.check(self.lib.fe_serve_create(ctx.h, int(hbm_budget), int(max_slots), int(host_threads),
                                           C.byref(h)))
        self.h = h
        self._pending = {}
        ctx._servers.add(self)

    def submit(self, elem_type: int, coords, conn, dirichlet, dt: float, u, rho, mu, rtol: float = 1e-8,
               max_iter: int = 10000, want_mom_rhs: bool = False, types=None) -> int:
        """Queue one request; a hybrid mesh passes elem_type HYBRID, conn [E, 8]
        and types [E] (node counts)."""
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        n = coords.shape[0]
        width = 8 if elem_type == HYBRID else elem_type
        if coords.ndim != 2 or coords.shape[1] != 3 or conn.ndim != 2 or conn.shape[1] != width:
            raise ValueError("coords must be [N,3] and conn [E,nen] ([E,8] for a hybrid mesh)")
        if (elem_type == HYBRID) != (types is not None):
            raise ValueError("types are given exactly for a HYBRID mesh")
        ty = None if types is None else np.ascontiguousarray(types, dtype=np.uint8)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, n)
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(n)
        mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(n)
        d = np.ascontiguousarray(dirichlet if dirichlet is not None else np.zeros(0), dtype=np.int32)
        x = np.zeros(n, dtype=np.float64)
        mr = np.zeros((3, n), dtype=np.float64) if want_mom_rhs else None
        job = capi.Job(type=elem_type, n_nodes=n, coords=coords.ctypes.data, n_elems=conn.shape[0],
                       conn=conn.ctypes.data, n_dirichlet=d.shape[0], dirichlet_nodes=d.ctypes.data if d.size else None,
                       dt=float(dt), u=u.ctypes.data, rho=rho.ctypes.data, mu=mu.ctypes.data, rtol=float(rtol),
                       max_iter=int(max_iter), x=x.ctypes.data, mom_rhs=None if mr is None else mr.ctypes.data,
                       elem_types=None if ty is None else ty.ctypes.data)
        t = C.c_int64()
        st = self.lib.fe_serve_submit(self.h, C.byref(job), C.byref(t))
        if st != capi.FE_OK:
            raise FeError(st, "fe_serve_submit failed")
        self._pending[t.value] = (job, coords, conn, d, u, rho, mu, x, mr, ty)
        return t.value

    def _result(self, ticket, r):
        keep = self._pending.pop(ticket)
        return {"status": int(r.status), "status_name": capi.STATUS_NAMES.get(r.status, str(r.status)),
                "iterations": int(r.iterations), "rel_residual": r.rel_residual,
                "true_rel_residual": r.true_rel_residual, "min_detJ": r.min_detJ,
                "first_bad_elem": int(r.first_bad_elem), "plan_ms": r.plan_ms, "wait_ms": r.wait_ms,
                "run_ms": r.run_ms, "total_ms": r.total_ms, "message": r.message.decode(errors="replace"),
                "x": keep[7], "mom_rhs": keep[8]}

    def poll(self, ticket: int):
        done = C.c_int32()
        r = capi.JobResult()
        st = self.lib.fe_serve_poll(self.h, ticket, C.byref(done), C.byref(r))
        if st != capi.FE_OK:
            raise FeError(st, "fe_serve_poll: unknown ticket")
        return self._result(ticket, r) if done.value else None

    def wait(self, ticket: int) -> dict:
        r = capi.JobResult()
        st = self.lib.fe_serve_wait(self.h, ticket, C.byref(r))
        if st != capi.FE_OK:
            raise FeError(st, "fe_serve_wait: unknown ticket")
        return self._result(ticket, r)

    def stats(self) -> dict:
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        if self.lib.fe_serve_stats(self.h, C.byref(a), C.byref(b), C.byref(c)) != capi.FE_OK:
            raise FeError(capi.FE_EINVAL, "fe_serve_stats failed")
        return {"completed": a.value, "batches": b.value, "batched_requests": c.value,
                "mean_batch": c.value / b.value if b.value else 0.0}

    def close(self):
        if getattr(self, "h", None):
            self.lib.fe_serve_destroy(self.h)
            self.h = None
            self._pending.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check usable while module globals
        # are torn down at interpreter exit
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Host-only preprocessing (fe_plan_create): no device needed."""

    def __init__(self, elem_type: int, coords, conn, renumber: bool = True, types=None):
        self.lib = capi.load()
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        flags = FE_UPLOAD_RENUMBER if renumber else 0
        h = C.c_void_p()
        if types is None:
            st = self.lib.fe_plan_create(elem_type, coords.shape[0], coords.ctypes.data, conn.shape[0],
                                         conn.ctypes.data, flags, C.byref(h))
        else:
            types = np.ascontiguousarray(types, dtype=np.uint8)
            st = self.lib.fe_plan_create_mixed(coords.shape[0], coords.ctypes.data, conn.shape[0],
                                               types.ctypes.data, conn.ctypes.data, flags, C.byref(h))
        if st != capi.FE_OK:
            raise FeError(st, self.lib.fe_plan_last_error().decode())
        self.h = h
        d = capi.PlanDesc()
        self.lib.fe_plan_info(h, C.byref(d))
        self.desc = {k: getattr(d, k) for k, _ in capi.PlanDesc._fields_}

    def export(self) -> dict:
        d = self.desc
        N, E, nnz, nb = d["n_nodes"], d["n_elems"], d["nnz"], d["n_blocks"]
        out = {"node_perm": np.zeros(N, np.int32), "elem_perm": np.zeros(E, np.int32),
               "rowptr": np.zeros(N + 1, np.int32), "colidx": np.zeros(nnz, np.int32),
               "block_elem_ptr": np.zeros(nb + 1, np.int32), "block_color": np.zeros(nb, np.int32),
               "block_node_ptr": np.zeros(nb + 1, np.int32)}
        # first pass to size block_nodes
        self.lib.fe_plan_export(self.h, None, None, None, None, None, None,
                                out["block_node_ptr"].ctypes.data, None)
        out["block_nodes"] = np.zeros(int(out["block_node_ptr"][-1]), np.int32)
        a = [out[k].ctypes.data for k in ("node_perm", "elem_perm", "rowptr", "colidx", "block_elem_ptr",
                                          "block_color", "block_node_ptr", "block_nodes")]
        self.lib.fe_plan_export(self.h, *a)
        nl = C.c_int64()
        out["elem_types"] = np.zeros(E, np.uint8)
        out["block_types"] = np.zeros(nb, np.uint8)
        self.lib.fe_plan_export_types(self.h, None, None, None, C.byref(nl))
        out["launches"] = np.zeros((nl.value, 3), np.int32)
        self.lib.fe_plan_export_types(self.h, out["elem_types"].ctypes.data, out["block_types"].ctypes.data,
                                      out["launches"].ctypes.data, C.byref(nl))
        out["color_blocks"] = np.zeros(nb, np.int32)
        self.lib.fe_plan_export_color_blocks(self.h, out["color_blocks"].ctypes.data)
        return out

    def export_owner(self) -> dict:
        """The owner plan of the matrix assembly (single-type meshes)."""
        G, T = C.c_int64(), C.c_int64()
        ra, lns, offs, priv = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        st = self.lib.fe_plan_owner_info(self.h, C.byref(G), C.byref(T), C.byref(ra), C.byref(lns), C.byref(offs),
                                         C.byref(priv))
        if st != capi.FE_OK:
            raise FeError(st, "no owner plan (hybrid mesh)")
        G, T = G.value, T.value
        out = {"rows_per_task": ra.value, "ln_stride": lns.value, "off_stride": offs.value,
               "wave_private": bool(priv.value),
               "groups": np.zeros((G, 4), np.int32), "node_ptr": np.zeros(G + 1, np.int32),
               "nphase": np.zeros(G, np.uint8), "task_elem": np.zeros(T, np.int32),
               "task_ln": np.zeros((T, lns.value), np.uint16), "task_off": np.zeros((T, offs.value), np.uint8),
               "task_phase": np.zeros(T, np.uint8)}
        self.lib.fe_plan_export_owner(self.h, None, out["node_ptr"].ctypes.data, None, None, None, None, None, None)
        out["nodes"] = np.zeros(int(out["node_ptr"][-1]), np.int32)
        a = [out[k].ctypes.data for k in ("groups", "node_ptr", "nodes", "nphase", "task_elem", "task_ln",
                                          "task_off", "task_phase")]
        self.lib.fe_plan_export_owner(self.h, *a)
        return out

    def __del__(self):
        try:
            if self.h:
                self.lib.fe_plan_free(self.h)
                self.h = None
        except Exception:
            pass


def pack_layout(n_elems: int, vector_size: int):
    lib = capi.load()
    p = C.c_int64()
    q = C.c_int64()
    st = lib.fe_pack_layout(n_elems, vector_size, C.byref(p), C.byref(q))
    if st != capi.FE_OK:
        raise FeError(st, "bad pack layout arguments")
    return int(p.value), int(q.value)
