"""Helpers shared by the GPU tests: marshalling between the user numbering of
the generators / oracle and the mesh numbering of the library."""
import numpy as np


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def mesh_fields(mesh, case):
    """Nodal fields of a case moved to the device in mesh numbering."""
    out = {"u": mesh.to_mesh(dev(case.u)), "rho": mesh.to_mesh(dev(case.rho)),
           "mu": mesh.to_mesh(dev(case.mu))}
    if case.Y.shape[0]:
        out["Y"] = mesh.to_mesh(dev(case.Y))
    return out


def user_order(mesh):
    """Permutation that maps mesh-CSR entries to the user canonical CSR."""
    rp, ci = mesh.pattern_host()
    perm = mesh.node_perm.astype(np.int64)
    rows = np.repeat(perm, np.diff(rp))
    cols = perm[ci]
    order = np.lexsort((cols, rows))
    return order, rows[order], cols[order]


def values_user(mesh, vals_mesh, order=None):
    if order is None:
        order, _, _ = user_order(mesh)
    return vals_mesh[..., order]


def rhs_user(mesh, rhs_mesh):
    out = np.empty_like(rhs_mesh)
    out[..., mesh.node_perm] = rhs_mesh
    return out


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def row_scaled_err(rowptr, got, ref):
    """max over entries of |got - ref| / max_j |ref_ij| of its row."""
    rows = np.repeat(np.arange(rowptr.shape[0] - 1), np.diff(rowptr))
    scale = np.maximum.reduceat(np.abs(ref), rowptr[:-1]) if ref.size else np.zeros(0)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(got - ref) / scale[rows])) if ref.size else 0.0


def submesh_rows(case, nodes):
    """Elements touching `nodes`, relabelled compactly.

    Returns (coords, conn, local_of_global, global_of_local); the rows of
    `nodes` assembled on this submesh are complete."""
    conn = case.conn
    mark = np.zeros(case.n_nodes, bool)
    mark[nodes] = True
    emask = mark[conn].any(axis=1)
    sub = conn[emask]
    glob = np.unique(sub)
    loc = np.full(case.n_nodes, -1, np.int64)
    loc[glob] = np.arange(glob.size)
    return case.coords[glob], loc[sub].astype(np.int32), loc, glob


def make_mesh(ctx, case, renumber=True, coloured=False):
    """Upload a case: fe_mesh_upload, or fe_mesh_upload_mixed for a hybrid one
    (always coloured element blocks)."""
    import paper_2107_11541_amd as fe
    if case.types is None:
        return fe.Mesh(ctx, case.nen, case.coords, case.conn, case.dirichlet, renumber=renumber, coloured=coloured)
    return fe.Mesh(ctx, fe.HYBRID, case.coords, case.conn, case.dirichlet, renumber=renumber, types=case.types)


def submesh_rows_typed(case, nodes):
    """submesh_rows for a mesh with per-element types (padded connectivity).

    Returns (coords, conn, types, local_of_global, global_of_local)."""
    conn = case.conn
    types = case.types if case.types is not None else np.full(case.n_elems, case.nen, np.uint8)
    valid = np.arange(conn.shape[1])[None, :] < types[:, None]
    safe = np.where(valid, conn, 0)
    mark = np.zeros(case.n_nodes, bool)
    mark[nodes] = True
    emask = (mark[safe] & valid).any(axis=1)
    sub, sv = safe[emask], valid[emask]
    glob = np.unique(sub[sv])
    loc = np.full(case.n_nodes, -1, np.int64)
    loc[glob] = np.arange(glob.size)
    sconn = np.where(sv, loc[sub], -1).astype(np.int32)
    return case.coords[glob], sconn, types[emask], loc, glob
