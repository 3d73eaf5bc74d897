"""GPU parity on prism (PEN06), pyramid (PYR05) and hybrid meshes: the HIP
assembly through the C ABI (fe_mesh_upload for one type,
fe_mesh_upload_mixed for mixed types) against the FP64 oracle.

Same bar as the single-type tests: FP64 assembly to 1e-12 relative (norm and
per entry, scaled by its row's largest entry), mixed precision to 1e-5,
bitwise determinism, PCG to the oracle's solution.  The full-size case is
the 128^3 hybrid cube (7.9 M elements of all four types), checked on sampled
rows assembled by the oracle on the elements around them.
"""
import numpy as np
import pytest

import meshgen
import oracle
from tests.gpu_helpers import (dev, host, make_mesh, mesh_fields, rel, rhs_user, row_scaled_err,
                               submesh_rows_typed, user_order, values_user)

pytestmark = pytest.mark.gpu

MOM, SCA, POI = oracle.OP_MOMENTUM, oracle.OP_SCALAR, oracle.OP_POISSON
TOL = 1e-12
KINDS = {"pen": meshgen.PEN06, "pyr": meshgen.PYR05, "hybrid": meshgen.HYBRID}


@pytest.fixture(scope="module")
def fe_ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_11541_amd as fe
    ctx = fe.Context(0)
    yield ctx
    torch.cuda.synchronize()


def _fe():
    import paper_2107_11541_amd as fe
    return fe


def gpu_assemble(ctx, case, op, precision=0, renumber=True, mesh=None):
    fe = _fe()
    if mesh is None:
        mesh = make_mesh(ctx, case, renumber)
    f = mesh_fields(mesh, case)
    kw = {"Y": f["Y"], "D": case.D} if op == SCA else {}
    v, b, info = fe.assemble(mesh, op, case.dt, f["u"], f["rho"], f["mu"], precision=precision, **kw)
    return mesh, host(v), host(b), info


def oracle_assemble(case, op):
    kw = {"Y": case.Y, "D": case.D} if op == SCA else {}
    return oracle.assemble(case.coords, case.conn, op, case.dt, case.u, case.rho, case.mu, types=case.types, **kw)


def check_parity(mesh, case, op, v, b, tol=TOL):
    rp, ci, V, B = oracle_assemble(case, op)
    order, rows, cols = user_order(mesh)
    assert np.array_equal(cols, ci), "pattern differs from the oracle's"
    vu = values_user(mesh, v, order)
    bu = rhs_user(mesh, b)
    for k in range(V.shape[0]):
        assert rel(vu[k], V[k]) <= tol, (k, rel(vu[k], V[k]))
        assert row_scaled_err(rp, vu[k], V[k]) <= tol
    for k in range(B.shape[0]):
        assert rel(bu[k], B[k]) <= tol, (k, rel(bu[k], B[k]))


@pytest.mark.parametrize("op", [MOM, POI])
@pytest.mark.parametrize("kind,n", [("pen", 1), ("pen", 7), ("pyr", 1), ("pyr", 6), ("hybrid", 4),
                                    ("hybrid", 9)])
def test_assembly_parity(fe_ctx, kind, n, op):
    case = meshgen.make_case(n, KINDS[kind], 0.12, case_id=60 + n, shuffle=True, temperature=True)
    print(f"{kind} n={n} E={case.n_elems} op={op}", flush=True)
    mesh, v, b, info = gpu_assemble(fe_ctx, case, op)
    check_parity(mesh, case, op, v, b)
    assert info["first_bad_elem"] == -1 and info["min_detJ"] > 0


@pytest.mark.parametrize("kind", ["pen", "pyr", "hybrid"])
def test_scalar_operator_parity(fe_ctx, kind):
    case = meshgen.make_case(5, KINDS[kind], 0.1, case_id=70, shuffle=True, n_scalars=3)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, SCA)
    check_parity(mesh, case, SCA, v, b)


def test_hybrid_without_renumbering(fe_ctx):
    # user order interleaves the types: blocks close at every type change
    case = meshgen.make_case(5, meshgen.HYBRID, 0.1, case_id=71, shuffle=True)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, MOM, renumber=False)
    assert np.array_equal(mesh.node_perm, np.arange(case.n_nodes))
    check_parity(mesh, case, MOM, v, b)


def test_hybrid_mixed_precision_error_bound(fe_ctx):
    case = meshgen.make_case(6, meshgen.HYBRID, 0.1, case_id=72, shuffle=True, temperature=True)
    for op in (MOM, POI):
        mesh, v, b, _ = gpu_assemble(fe_ctx, case, op, precision=1)
        rp, ci, V, B = oracle_assemble(case, op)
        vu, bu = values_user(mesh, v), rhs_user(mesh, b)
        ev, eb = rel(vu[0], V[0]), rel(bu, B)
        assert ev <= 1e-5 and eb <= 1e-5, (op, ev, eb)
        assert ev > 1e-12
        assert row_scaled_err(rp, vu[0], V[0]) <= 1e-4


def test_hybrid_bitwise_deterministic(fe_ctx):
    case = meshgen.make_case(10, meshgen.HYBRID, 0.15, case_id=73, shuffle=True)
    mesh, v1, b1, _ = gpu_assemble(fe_ctx, case, MOM)
    for _ in range(3):
        _, v2, b2, _ = gpu_assemble(fe_ctx, case, MOM, mesh=mesh)
        assert np.array_equal(v1, v2) and np.array_equal(b1, b2)


def test_hybrid_bad_element_reported(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(4, meshgen.HYBRID, 0.0, case_id=74, shuffle=True)
    e = int(np.flatnonzero(case.types == 5)[0])
    X = case.coords.copy()
    apex = case.conn[e, 4]
    X[apex] = 2 * X[case.conn[e, 0]] - X[apex]      # push a pyramid's apex through its base
    case.coords = X
    with pytest.raises(oracle.AssembleError) as oe:
        oracle_assemble(case, MOM)
    mesh = make_mesh(fe_ctx, case, renumber=False)
    f = mesh_fields(mesh, case)
    import ctypes as C
    import torch
    import paper_2107_11541_amd.capi as capi
    info = capi.AsmInfo()
    fld = capi.Fields(op=MOM, dt=case.dt, u=f["u"].data_ptr(), rho=f["rho"].data_ptr(),
                      mu=f["mu"].data_ptr(), n_scalars=0, Y=None, D=None)
    vals = torch.empty(mesh.nnz, dtype=torch.float64, device="cuda")
    rhs = torch.empty(3 * mesh.n_nodes, dtype=torch.float64, device="cuda")
    st = fe_ctx.lib.fe_assemble(mesh.h, C.byref(fld), 0, C.c_void_p(vals.data_ptr()),
                                C.c_void_p(rhs.data_ptr()), C.byref(info))
    assert st == capi.FE_EBADELEM
    assert info.first_bad_elem == oe.value.bad_elem and info.min_detJ <= 0


def test_mixed_upload_argument_errors(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(4, meshgen.HYBRID, 0.1, case_id=75)
    bad = case.types.copy()
    bad[0] = 3
    with pytest.raises(fe.FeError) as ei:
        fe.Mesh(fe_ctx, fe.HYBRID, case.coords, case.conn, case.dirichlet, types=bad)
    assert ei.value.status == 1


def test_hybrid_pcg_matches_oracle(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(8, meshgen.HYBRID, 0.1, case_id=76, shuffle=True, temperature=True)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, POI)
    L, f = dev(v[0]), dev(b[0])
    fe.apply_dirichlet(mesh, L, f)
    x, info = fe.cg_solve(mesh, L, f, rtol=1e-10, max_iter=3000)
    rp, ci, Lr, fr = oracle_assemble(case, POI)
    Lr, fr = Lr[0].copy(), fr[0].copy()
    oracle.dirichlet(rp, ci, Lr, fr, case.dirichlet)
    xo, st, it, rr, tr = oracle.pcg(rp, ci, Lr, fr, rtol=1e-10)
    assert info["status"] == 0 and st == oracle.OK
    assert abs(info["iterations"] - it) <= 2, (info["iterations"], it)
    assert rel(rhs_user(mesh, host(x)), xo) <= 1e-8
    x32, i32 = fe.cg_solve(mesh, L, f, rtol=1e-8, max_iter=3000, precision=1)
    assert i32["status"] == 0 and i32["true_rel_residual"] <= 1e-8


def test_full_size_hybrid_sampled_rows(fe_ctx):
    """The 128^3 hybrid cube: momentum and Poisson at full size, 64 sampled
    rows (plus the first and last user node) against the oracle on the
    elements around them."""
    fe = _fe()
    case = meshgen.hybrid()
    print(f"full-size hybrid: N={case.n_nodes} E={case.n_elems}", flush=True)
    mesh = make_mesh(fe_ctx, case)
    f = mesh_fields(mesh, case)
    rp_m, ci_m = mesh.pattern_host()
    perm = mesh.node_perm
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(perm.size, dtype=perm.dtype)
    rng = np.random.default_rng(5)
    pyr = case.conn[np.flatnonzero(case.types == 5)[0], :5]     # the sparse pyramid slab
    nodes = np.unique(np.concatenate([rng.integers(0, case.n_nodes, 64), [0, case.n_nodes - 1], pyr]))
    sc, sconn, st, loc, glob = submesh_rows_typed(case, nodes)
    assert set(np.unique(st)) == {4, 5, 6, 8}
    for op in (MOM, POI):
        v, b, _ = fe.assemble(mesh, op, case.dt, f["u"], f["rho"], f["mu"])
        v, b = host(v)[0], host(b)
        rp, ci, V, B = oracle.assemble(sc, sconn, op, case.dt, case.u[:, glob], case.rho[glob],
                                       case.mu[glob], types=st)
        for i in nodes:
            li, im = loc[i], iperm[i]
            ocols = glob[ci[rp[li]:rp[li + 1]]]
            ovals = V[0][rp[li]:rp[li + 1]]
            gcols = perm[ci_m[rp_m[im]:rp_m[im + 1]]]
            gvals = v[rp_m[im]:rp_m[im + 1]]
            o = np.argsort(gcols)
            assert np.array_equal(gcols[o], ocols)
            assert np.abs(gvals[o] - ovals).max() <= TOL * np.abs(ovals).max()
            for r in range(B.shape[0]):
                rms = np.sqrt(np.mean(B[r] ** 2))
                assert abs(b[r][im] - B[r][li]) <= TOL * max(abs(B[r][li]), rms)
    mesh.close()
