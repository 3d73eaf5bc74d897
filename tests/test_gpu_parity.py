"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances: FP64 assembly, relative Frobenius and RHS error <= 1e-12 and
per-entry error <= 1e-12 of its row's largest entry (some entries cancel to
~0); solver kernels <= 1e-13; CG to its residual bound; mixed precision to
the stated bound of 1e-5 relative (FP32 quadrature), well above the ~1e-7 observed.
"""
import numpy as np
import pytest

import meshgen
import oracle
from tests.gpu_helpers import (dev, host, mesh_fields, rel, rhs_user, row_scaled_err, submesh_rows,
                               user_order, values_user)

pytestmark = pytest.mark.gpu

MOM, SCA, POI = oracle.OP_MOMENTUM, oracle.OP_SCALAR, oracle.OP_POISSON
TOL = 1e-12


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


def gpu_assemble(ctx, case, op, precision=0, renumber=True, mesh=None, coloured=False):
    fe = _fe()
    if mesh is None:
        mesh = fe.Mesh(ctx, case.nen, case.coords, case.conn, case.dirichlet, renumber=renumber, coloured=coloured)
    f = mesh_fields(mesh, case)
    kw = {}
    if op == SCA:
        kw = {"Y": f["Y"], "D": case.D}
    v, b, info = fe.assemble(mesh, op, case.dt, f["u"], f["rho"], f["mu"], precision=precision, **kw)
    return mesh, host(v), host(b), info


def oracle_assemble(case, op):
    kw = {"Y": case.Y, "D": case.D} if op == SCA else {}
    return oracle.assemble(case.coords, case.conn, op, case.dt, case.u, case.rho, case.mu, **kw)


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
    return rp, ci, V, B, vu, bu


# --- assembly ------------------------------------------------------------------

@pytest.mark.parametrize("coloured", [False, True])
@pytest.mark.parametrize("op", [MOM, POI])
def test_hex_cfg0_assembly_parity(fe_ctx, op, coloured):
    """Owner groups (the HEX08 default) and coloured element blocks (the
    served form) against the oracle."""
    case = meshgen.cfg0()
    mesh, v, b, info = gpu_assemble(fe_ctx, case, op, coloured=coloured)
    check_parity(mesh, case, op, v, b)
    assert info["first_bad_elem"] == -1 and info["min_detJ"] > 0


@pytest.mark.parametrize("precision", [0, 1])
def test_hex_owner_and_coloured_forms_agree(fe_ctx, precision):
    """The two HEX08 assembly forms on a jittered, shuffled 12^3 mesh: the
    same sums in another order (FP64 1e-13, mixed 1e-6 of the row scale)."""
    case = meshgen.make_case(12, meshgen.HEX08, 0.15, case_id=45, shuffle=True)
    for op in (MOM, POI):
        m1, v1, b1, _ = gpu_assemble(fe_ctx, case, op, precision=precision)
        m2, v2, b2, _ = gpu_assemble(fe_ctx, case, op, precision=precision, coloured=True)
        assert np.array_equal(m1.node_perm, m2.node_perm)
        tol = 1e-13 if precision == 0 else 1e-6
        assert rel(v1, v2) <= tol and rel(b1, b2) <= tol
        m1.close()
        m2.close()


@pytest.mark.parametrize("n,shuffle,renumber", [(1, False, True), (3, True, True), (7, True, True),
                                                (6, True, False), (13, True, True)])
def test_hex_ragged_and_unrenumbered_parity(fe_ctx, n, shuffle, renumber):
    case = meshgen.make_case(n, meshgen.HEX08, 0.12, case_id=20 + n, shuffle=shuffle)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, MOM, renumber=renumber)
    check_parity(mesh, case, MOM, v, b)


@pytest.mark.parametrize("op", [MOM, POI])
@pytest.mark.parametrize("n", [1, 5])
def test_tet_assembly_parity(fe_ctx, op, n):
    case = meshgen.make_case(n, meshgen.TET04, 0.10, case_id=30 + n, shuffle=True, temperature=True)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, op)
    check_parity(mesh, case, op, v, b)


@pytest.mark.parametrize("kind", [meshgen.HEX08, meshgen.TET04])
def test_scalar_operator_parity(fe_ctx, kind):
    case = meshgen.make_case(5, kind, 0.1, case_id=40, shuffle=True, n_scalars=3)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, SCA)
    check_parity(mesh, case, SCA, v, b)


def test_assembly_is_bitwise_deterministic(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(12, meshgen.HEX08, 0.15, case_id=41, shuffle=True)
    mesh, v1, b1, _ = gpu_assemble(fe_ctx, case, MOM)
    for _ in range(3):
        _, v2, b2, _ = gpu_assemble(fe_ctx, case, MOM, mesh=mesh)
        assert np.array_equal(v1, v2) and np.array_equal(b1, b2)
    # values are overwritten, not accumulated: garbage in the output is ignored
    import torch
    f = mesh_fields(mesh, case)
    vals = torch.full((1, mesh.nnz), 7.0, dtype=torch.float64, device="cuda")
    rhs = torch.full((3, mesh.n_nodes), -3.0, dtype=torch.float64, device="cuda")
    fe.assemble(mesh, MOM, case.dt, f["u"], f["rho"], f["mu"], values=vals, rhs=rhs)
    assert np.array_equal(host(vals), v1) and np.array_equal(host(rhs), b1)


def test_mixed_precision_assembly_error_bound(fe_ctx):
    case = meshgen.make_case(6, meshgen.TET04, 0.10, case_id=42, shuffle=True, temperature=True)
    for op in (MOM, POI):
        mesh, v, b, _ = gpu_assemble(fe_ctx, case, op, precision=1)
        rp, ci, V, B = oracle_assemble(case, op)
        vu = values_user(mesh, v)
        bu = rhs_user(mesh, b)
        ev, eb = rel(vu[0], V[0]), rel(bu, B)
        # FP32 quadrature: ~ (terms) * 2^-24 relative; stated bound 1e-5
        assert ev <= 1e-5 and eb <= 1e-5, (op, ev, eb)
        assert ev > 1e-12   # it really is FP32 quadrature
        assert row_scaled_err(rp, vu[0], V[0]) <= 1e-4


def test_bad_element_reported_with_user_index(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(4, meshgen.HEX08, 0.0, case_id=43, shuffle=True)
    bad_e = 17
    c = case.conn[bad_e]
    X = case.coords.copy()
    X[[c[0], c[6]]] = X[[c[6], c[0]]]      # fold element 17 (and its neighbours)
    case.coords = X
    mesh = fe.Mesh(fe_ctx, 8, case.coords, case.conn, None)
    f = mesh_fields(mesh, case)
    with pytest.raises(fe.FeError) as ei:
        fe.assemble(mesh, MOM, case.dt, f["u"], f["rho"], f["mu"])
    assert ei.value.status == 4
    try:
        oracle_assemble(case, MOM)
    except oracle.AssembleError as err:
        first = err.bad_elem
    # the GPU reports the smallest mesh index; it must be one of the folded elements
    # and at least as early in user order as the oracle's first when no renumbering
    mesh2 = fe.Mesh(fe_ctx, 8, case.coords, case.conn, None, renumber=False)
    f2 = mesh_fields(mesh2, case)
    with pytest.raises(fe.FeError):
        fe.assemble(mesh2, MOM, case.dt, f2["u"], f2["rho"], f2["mu"])
    import paper_2107_11541_amd.capi as capi
    import ctypes as C
    info = capi.AsmInfo()
    fld = capi.Fields(op=MOM, dt=case.dt, u=f2["u"].data_ptr(), rho=f2["rho"].data_ptr(),
                      mu=f2["mu"].data_ptr(), n_scalars=0, Y=None, D=None)
    import torch
    vals = torch.empty(mesh2.nnz, dtype=torch.float64, device="cuda")
    rhs = torch.empty(3 * mesh2.n_nodes, dtype=torch.float64, device="cuda")
    st = fe_ctx.lib.fe_assemble(mesh2.h, C.byref(fld), 0, C.c_void_p(vals.data_ptr()),
                                C.c_void_p(rhs.data_ptr()), C.byref(info))
    assert st == 4 and info.first_bad_elem == first and info.min_detJ <= 0


def test_assemble_argument_errors(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(2, meshgen.HEX08, 0.0, case_id=44)
    mesh = fe.Mesh(fe_ctx, 8, case.coords, case.conn, None)
    f = mesh_fields(mesh, case)
    with pytest.raises(fe.FeError) as ei:
        fe.assemble(mesh, MOM, -1.0, f["u"], f["rho"], f["mu"])
    assert ei.value.status == 1
    with pytest.raises(fe.FeError) as ei:
        fe.assemble(mesh, MOM, 0.1, f["u"], f["rho"], f["mu"], precision=5)
    assert ei.value.status == 1


# --- Dirichlet, solver kernels, PCG -------------------------------------------

def poisson_gpu(ctx, case, mesh=None):
    fe = _fe()
    mesh, v, b, _ = gpu_assemble(ctx, case, POI, mesh=mesh)
    L = dev(v[0])
    f = dev(b[0])
    fe.apply_dirichlet(mesh, L, f)
    return mesh, L, f


def poisson_oracle(case):
    rp, ci, L, f = oracle_assemble(case, POI)
    L, f = L[0].copy(), f[0].copy()
    oracle.dirichlet(rp, ci, L, f, case.dirichlet)
    return rp, ci, L, f


def test_dirichlet_parity(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(8, meshgen.HEX08, 0.1, case_id=50, shuffle=True)
    mesh, L, f = poisson_gpu(fe_ctx, case)
    rp, ci, Lr, fr = poisson_oracle(case)
    order, _, _ = user_order(mesh)
    assert rel(host(L)[order], Lr) <= TOL
    assert rel(rhs_user(mesh, host(f)), fr) <= TOL
    # non-zero Dirichlet data
    rng = np.random.default_rng(1)
    g = rng.normal(0, 1, case.n_nodes)
    _, v, b, _ = gpu_assemble(fe_ctx, case, POI, mesh=mesh)
    L2, f2 = dev(v[0]), dev(b[0])
    fe.apply_dirichlet(mesh, L2, f2, mesh.to_mesh(dev(g)))
    _, _, Lo, fo = oracle_assemble(case, POI)
    Lo, fo = Lo[0].copy(), fo[0].copy()
    oracle.dirichlet(rp, ci, Lo, fo, case.dirichlet, g)
    assert rel(host(L2)[order], Lo) <= TOL
    assert rel(rhs_user(mesh, host(f2)), fo) <= TOL


def test_spmv_dot_axpy_parity(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(9, meshgen.HEX08, 0.1, case_id=51, shuffle=True)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, MOM)
    rng = np.random.default_rng(2)
    x = rng.normal(0, 1, case.n_nodes)
    y = fe.spmv(mesh, dev(v[0]), mesh.to_mesh(dev(x)))
    rp, ci, V, _ = oracle_assemble(case, MOM)
    yr = oracle.spmv(rp, ci, V[0], x)
    assert rel(rhs_user(mesh, host(y)), yr) <= 1e-13
    for n in (1, 255, 256, 1000, 262145):
        a = rng.normal(0, 1, n)
        c = rng.normal(0, 1, n)
        d = fe.dot(fe_ctx, dev(a), dev(c))
        assert abs(d - oracle.dot(a, c)) <= 1e-13 * np.abs(a * c).sum()
        yy = dev(c)
        fe.axpy(fe_ctx, 0.37, dev(a), yy)
        assert rel(host(yy), c + 0.37 * a) <= 1e-15
    assert fe.dot(fe_ctx, dev(np.zeros(0)), dev(np.zeros(0))) == 0.0


def _spmv_blocks(mesh):
    """The SpMV row blocks of the documented rule (<= 64 rows, <= 1021
    nonzeros, <= 256 distinct columns, rows taken greedily), simulated on the
    pattern the library exposes: per block its distinct-column count and
    whether the column limit is what ended it."""
    rp, ci = mesh.pattern_host()
    rp = rp.astype(np.int64)
    n = len(rp) - 1
    ncols, capped, r = [], [], 0
    while r < n:
        cols = set(ci[rp[r]:rp[r + 1]].tolist())
        r1, cap = r + 1, False
        while r1 < n and r1 - r < 64 and rp[r1 + 1] - rp[r] <= 1021:
            more = cols | set(ci[rp[r1]:rp[r1 + 1]].tolist())
            if len(more) > 256:
                cap = True
                break
            cols = more
            r1 += 1
        ncols.append(len(cols))
        capped.append(cap)
        r = r1
    return np.array(ncols), np.array(capped)


def _spmv_forms(mesh, vals_host, x):
    """y from the 16-byte form (aligned values) and from the one-entry form
    (the same values at an 8-byte offset)."""
    fe = _fe()
    import torch
    nnz = mesh.nnz
    va = dev(vals_host)
    buf = torch.empty(nnz + 1, dtype=torch.float64, device="cuda")
    buf[1:] = va
    vm = buf[1:]
    assert va.data_ptr() % 16 == 0 and vm.data_ptr() % 16 == 8
    return fe.spmv(mesh, va, x), fe.spmv(mesh, vm, x)


@pytest.mark.parametrize("etype,n", [(meshgen.HEX08, 8), (meshgen.HEX08, 10), (meshgen.TET04, 3),
                                     (meshgen.HEX08, 9), (meshgen.HEX08, 48)])
def test_spmv_load_forms_agree(fe_ctx, etype, n):
    """16-byte loads (aligned values, one-byte local indices into each row
    block's column set) and one-entry loads (values offset by 8 bytes, plain
    column indices) give bitwise the same y; nnz % 4 = 1, 3, 2, 0 exercises
    the end-of-array handling of the 16-byte form."""
    import torch
    case = meshgen.make_case(n, etype, 0.1, case_id=53, shuffle=True)
    mesh, v, b, _ = gpu_assemble(fe_ctx, case, MOM)
    x = mesh.to_mesh(dev(np.random.default_rng(3).normal(0, 1, case.n_nodes)))
    ya, ym = _spmv_forms(mesh, v[0], x)
    assert torch.equal(ya, ym)
    rp, ci, V, _ = oracle_assemble(case, MOM)
    yr = oracle.spmv(rp, ci, V[0], rhs_user(mesh, host(x)))
    ncols, _ = _spmv_blocks(mesh)
    print(etype, n, "nnz % 4 =", mesh.nnz % 4, "columns per block max", ncols.max(), flush=True)
    assert rel(rhs_user(mesh, host(ya)), yr) <= 1e-13


def test_spmv_blocks_end_at_the_column_limit(fe_ctx):
    """A TET04 mesh with one node in 80 elements (a 241-entry row) next to
    short rows: row blocks end where a 257th distinct column would enter.
    Both load forms against the definition y_i = sum_j A_ij x_j, with A_ij a
    seeded counter-based value of the user ids (i, j) on the element-sharing
    pattern."""
    import math
    import torch
    fe = _fe()
    rng = np.random.default_rng(3)
    nf, tail = 80, 200
    N = 1 + 3 * nf + tail
    conn = [[0, 1 + 3 * k, 2 + 3 * k, 3 + 3 * k] for k in range(nf)]
    extra = list(range(1 + 3 * nf, N))
    conn += [[extra[k], extra[k + 1], extra[k + 2], extra[k + 3]] for k in range(len(extra) - 3)]
    conn = np.array(conn, np.int32)
    coords = rng.random((N, 3))
    mesh = fe.Mesh(fe_ctx, meshgen.TET04, coords, conn, np.zeros(0, np.int32))
    ncols, capped = _spmv_blocks(mesh)
    assert capped.any() and ncols.max() <= 256, (ncols.max(), capped.sum())
    rp_m, ci_m = mesh.pattern_host()
    perm = mesh.node_perm.astype(np.int64)
    vals = _pair_values(np.repeat(perm, np.diff(rp_m)), perm[ci_m], N)
    xu = rng.uniform(-1.0, 1.0, N)
    ya, ym = _spmv_forms(mesh, vals, dev(xu[perm]))
    assert torch.equal(ya, ym)
    y = host(ya)
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(N)
    worst = 0.0
    for i in range(N):
        cols = np.unique(conn[(conn == i).any(axis=1)])
        terms = _pair_values(np.full(cols.size, i), cols, N) * xu[cols]
        worst = max(worst, abs(y[iperm[i]] - math.fsum(terms)) / np.abs(terms).sum())
    print("blocks", ncols.size, "ended by the column limit", int(capped.sum()), "worst", worst, flush=True)
    assert worst <= 1e-13
    mesh.close()


def test_pcg_graph_replays_match_eager_launches(fe_ctx):
    """Runs of 8 PCG iterations are replayed from a recorded HIP graph; with
    profiling on, every kernel is launched on its own.  Each replayed solve,
    with eager library work and synchronisations in between, must give
    bitwise the eager result (fixed and converged iteration counts)."""
    fe = _fe()
    import torch
    case = meshgen.make_case(11, meshgen.HEX08, 0.12, case_id=54, shuffle=True)
    mesh, L, f = poisson_gpu(fe_ctx, case)
    results = {}
    for mode in ("eager", "graph", "graph", "graph"):
        fe_ctx.profile(mode == "eager")
        for rtol, iters in ((0.0, 40), (1e-9, 2000)):
            x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
            x, info = fe.cg_solve(mesh, L, f, x=x, rtol=rtol, max_iter=iters)
            key = (rtol, iters)
            if mode == "eager":
                results[key] = (host(x), info["iterations"])
            else:
                assert np.array_equal(host(x), results[key][0]), key
                assert info["iterations"] == results[key][1], key
        # unrelated eager work between replays
        y = fe.spmv(mesh, L, f)
        fe.dot(fe_ctx, y, y)
        torch.cuda.synchronize()
    fe_ctx.profile(False)
    assert results[(0.0, 40)][1] == 40


def test_pcg_cfg0_matches_direct_solve(fe_ctx):
    fe = _fe()
    case = meshgen.cfg0()
    mesh, L, f = poisson_gpu(fe_ctx, case)
    x, info = fe.cg_solve(mesh, L, f, rtol=1e-10, max_iter=1000)
    rp, ci, Lr, fr = poisson_oracle(case)
    xo, st, it, rr, tr = oracle.pcg(rp, ci, Lr, fr, rtol=1e-10)
    from tests.test_oracle_pins import dense
    xd = np.linalg.solve(dense(rp, ci, Lr, case.n_nodes), fr)
    xu = rhs_user(mesh, host(x))
    assert info["status"] == 0
    assert abs(info["iterations"] - it) <= 2, (info["iterations"], it)
    assert info["true_rel_residual"] <= 2e-10
    assert rel(xu, xd) <= 1e-8
    assert rel(xu, xo) <= 1e-8


def test_pcg_fixed_iterations_follow_the_oracle(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(9, meshgen.HEX08, 0.15, case_id=52, shuffle=True)
    mesh, L, f = poisson_gpu(fe_ctx, case)
    x, info = fe.cg_solve(mesh, L, f, rtol=0.0, max_iter=12)
    assert info["status"] == 0 and info["iterations"] == 12
    assert info["symmetric_spmv"]   # the Poisson matrix is symmetric: the symmetric SpMV ran
    rp, ci, Lr, fr = poisson_oracle(case)
    xo, st, it, rr, tr = oracle.pcg(rp, ci, Lr, fr, rtol=0.0, max_iter=12)
    assert it == 12
    # the same algorithm on the same data: iterates agree to rounding
    assert rel(rhs_user(mesh, host(x)), xo) <= 1e-10
    assert abs(info["rel_residual"] - rr) <= 1e-8 * rr
    # bitwise reproducible
    x2, _ = fe.cg_solve(mesh, L, f, rtol=0.0, max_iter=12)
    assert np.array_equal(host(x), host(x2))


def test_pcg_noconv_and_breakdown(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(6, meshgen.HEX08, 0.1, case_id=53)
    mesh, L, f = poisson_gpu(fe_ctx, case)
    x, info = fe.cg_solve(mesh, L, f, rtol=1e-14, max_iter=3, raise_on_noconv=False)
    assert info["status"] == 5 and info["iterations"] == 3
    with pytest.raises(fe.FeError) as ei:
        fe.cg_solve(mesh, -L, f, rtol=1e-8, max_iter=50)
    assert ei.value.status == 6


def test_pcg_mixed_reaches_fp64_accuracy(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(16, meshgen.HEX08, 0.15, case_id=54, shuffle=True)
    mesh, L, f = poisson_gpu(fe_ctx, case)
    x64, i64 = fe.cg_solve(mesh, L, f, rtol=1e-12, max_iter=5000)
    x32, i32 = fe.cg_solve(mesh, L, f, rtol=1e-8, max_iter=5000, precision=1)
    assert i32["status"] == 0 and i32["true_rel_residual"] <= 1e-8
    assert i32["outer_iterations"] >= 2
    assert rel(host(x32), host(x64)) <= 1e-6


def test_tet_pcg(fe_ctx):
    fe = _fe()
    case = meshgen.make_case(6, meshgen.TET04, 0.1, case_id=55, shuffle=True, temperature=True)
    mesh, L, f = poisson_gpu(fe_ctx, case)
    x, info = fe.cg_solve(mesh, L, f, rtol=1e-10, max_iter=2000)
    rp, ci, Lr, fr = poisson_oracle(case)
    xo, st, it, rr, tr = oracle.pcg(rp, ci, Lr, fr, rtol=1e-10)
    assert abs(info["iterations"] - it) <= 2
    assert rel(rhs_user(mesh, host(x)), xo) <= 1e-8


# --- full-size workloads, sampled rows -----------------------------------------

def sampled_rows_check(ctx, case, ops, n_sample=64, seed=0, n_scalars=1):
    fe = _fe()
    mesh = fe.Mesh(ctx, case.nen, case.coords, case.conn, case.dirichlet)
    f = mesh_fields(mesh, case)
    ns = min(n_scalars, case.Y.shape[0])
    rp_m, ci_m = mesh.pattern_host()
    perm = mesh.node_perm
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(perm.size, dtype=perm.dtype)
    rng = np.random.default_rng(seed)
    nodes = np.unique(rng.integers(0, case.n_nodes, n_sample))
    sc, sconn, loc, glob = submesh_rows(case, nodes)
    for op in ops:
        kw, okw = {}, {}
        if op == SCA:
            kw = {"Y": f["Y"][:ns], "D": case.D[:ns]}
            okw = {"Y": np.ascontiguousarray(case.Y[:ns, glob]), "D": case.D[:ns]}
        v, b, _ = fe.assemble(mesh, op, case.dt, f["u"], f["rho"], f["mu"], **kw)
        v, b = host(v)[0], host(b)
        rp, ci, V, B = oracle.assemble(sc, sconn, op, case.dt, case.u[:, glob], case.rho[glob],
                                       case.mu[glob], **okw)
        for i in nodes:
            li = loc[i]
            ocols = glob[ci[rp[li]:rp[li + 1]]]
            ovals = V[0][rp[li]:rp[li + 1]]
            im = iperm[i]
            gcols = perm[ci_m[rp_m[im]:rp_m[im + 1]]]
            gvals = v[rp_m[im]:rp_m[im + 1]]
            o = np.argsort(gcols)
            assert np.array_equal(gcols[o], ocols)
            scale = np.abs(ovals).max()
            assert np.abs(gvals[o] - ovals).max() <= TOL * scale
            for r in range(B.shape[0]):
                rms = np.sqrt(np.mean(B[r] ** 2))
                assert abs(b[r][im] - B[r][li]) <= TOL * max(abs(B[r][li]), rms)
    return mesh


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
def test_full_size_sampled_rows(fe_ctx, which):
    case = meshgen.cfg1() if which == "cfg1" else meshgen.cfg2()
    print(f"full-size {which}: N={case.n_nodes} E={case.n_elems}", flush=True)
    sampled_rows_check(fe_ctx, case, [MOM, POI])


def test_full_size_cfg4_sampled_rows(fe_ctx):
    """256^3 HEX08 with 5 species: momentum, one scalar operator and the
    Poisson operator at full size, sampled rows against the oracle."""
    case = meshgen.cfg4()
    print(f"full-size cfg4: N={case.n_nodes} E={case.n_elems}", flush=True)
    mesh = sampled_rows_check(fe_ctx, case, [MOM, SCA, POI], n_sample=48, seed=4)
    mesh.close()


def _pair_values(rows, cols, n):
    """A value for every (row, column) pair of user node ids, in [-1, 1):
    the splitmix64 finaliser of the pair index row * n + col (a counter-based
    generator, so either side can evaluate any entry on its own)."""
    z = (rows.astype(np.uint64) * np.uint64(n) + cols.astype(np.uint64)) + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


@pytest.mark.parametrize("which", ["cfg1", "cfg2"])
def test_full_size_spmv_sampled_rows(fe_ctx, which):
    """y = A x at full size through the bench's SpMV launch configuration.
    A has the mesh's pattern and, for entry (i, j), the value of a seeded
    counter-based function of the user ids (i, j); x is seeded.  Sampled rows
    are checked against the definition: row i's columns are the nodes of the
    elements that contain i, and y_i is the exactly rounded sum of
    A_ij x_j over them."""
    import math
    fe = _fe()
    case = meshgen.cfg1() if which == "cfg1" else meshgen.cfg2()
    N = case.n_nodes
    mesh = fe.Mesh(fe_ctx, case.nen, case.coords, case.conn, case.dirichlet)
    rp_m, ci_m = mesh.pattern_host()
    perm = mesh.node_perm.astype(np.int64)
    vals = _pair_values(np.repeat(perm, np.diff(rp_m)), perm[ci_m], N)
    rng = np.random.default_rng(11)
    xu = rng.uniform(-1.0, 1.0, N)
    y = host(fe.spmv(mesh, dev(vals), dev(xu[perm])))
    del vals
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(N)
    nodes = np.unique(rng.integers(0, N, 96))
    nodes = np.unique(np.concatenate([nodes, [0, N - 1]]))
    mark = np.zeros(N, bool)
    mark[nodes] = True
    sub = case.conn[mark[case.conn].any(axis=1)]
    worst = 0.0
    for i in nodes:
        cols = np.unique(sub[(sub == i).any(axis=1)])
        terms = _pair_values(np.full(cols.size, i), cols, N) * xu[cols]
        ref = math.fsum(terms)
        err = abs(y[iperm[i]] - ref) / np.abs(terms).sum()
        worst = max(worst, err)
    print(f"{which}: {nodes.size} rows, worst error {worst:.2e} of sum |A_ij x_j|", flush=True)
    assert worst <= 1e-13
    mesh.close()
