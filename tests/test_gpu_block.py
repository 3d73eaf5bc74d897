"""GPU parity of the 3x3-block momentum operator (Eq. (1) with the viscous
term in its full-stress form -div(2 mu eps(u)) and EMAC's (div u) term)
against the FP64 oracle's or_assemble_block, through the C ABI.

Tolerances: FP64 sums in another order, so the relative Frobenius and
right-hand-side errors must be <= 1e-12 (as for the scalar operators), and
each entry within 1e-12 of its block row's largest magnitude.  At full size
(128^3) sampled block rows are checked against the oracle run on the
elements around them.
"""
import numpy as np
import pytest

import meshgen
import oracle
from tests.gpu_helpers import dev, host, make_mesh, rel, submesh_rows_typed, user_order

pytestmark = pytest.mark.gpu

TOL = 1e-12
KINDS = {"hex": meshgen.HEX08, "tet": meshgen.TET04, "pen": meshgen.PEN06, "pyr": meshgen.PYR05,
         "hybrid": meshgen.HYBRID}


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


def case_of(kind, n, seed):
    c = meshgen.make_case(n, KINDS[kind], 0.12, case_id=160 + seed, sub=KINDS[kind], shuffle=True,
                          temperature=(seed % 2 == 1))
    # a viscosity large enough for the coupling term to matter beside M/dt
    c.mu = np.random.default_rng(seed).uniform(1e-2, 3e-2, c.n_nodes)
    return c


def fields(mesh, c):
    return (mesh.to_mesh(dev(c.u)), mesh.to_mesh(dev(c.rho)), mesh.to_mesh(dev(np.ascontiguousarray(c.mu))))


def block_rows_err(rp, V, Vo):
    """max over entries of |V - Vo| / max |Vo| of its block row."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    a = np.abs(Vo).reshape(-1, 3, 3)
    # block row (node i, component r): the r-th rows of node i's blocks
    worst = 0.0
    for r in range(3):
        mag = np.abs(Vo.reshape(-1, 3, 3)[:, r, :]).max(axis=1)
        scale = np.maximum.reduceat(mag, rp[:-1])
        scale = np.where(scale > 0, scale, 1.0)
        d = np.abs(V.reshape(-1, 3, 3)[:, r, :] - Vo.reshape(-1, 3, 3)[:, r, :]).max(axis=1)
        worst = max(worst, float(np.max(d / scale[rows])))
    del a
    return worst


@pytest.mark.parametrize("form", [0, 1, 2, 3])
@pytest.mark.parametrize("kind,n", [("hex", 5), ("tet", 4), ("pen", 4), ("pyr", 3), ("hybrid", 6)])
def test_block_operator_matches_oracle(fe_ctx, kind, n, form):
    fe = _fe()
    c = case_of(kind, n, seed=n + form)
    print(f"{kind} n={n} form={form} N={c.n_nodes} E={c.n_elems}", flush=True)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = fields(mesh, c)
    V, B, info = fe.assemble_block(mesh, form, c.dt, u, rho, mu)
    order, _, _ = user_order(mesh)
    Vu = host(V).reshape(-1, 9)[order].reshape(-1)
    Bu = np.empty((3, c.n_nodes))
    Bu[:, mesh.node_perm] = host(B)
    rp, ci, Vo, Bo = oracle.assemble_block(c.coords, c.conn, form, c.dt, c.u, c.rho, c.mu, types=c.types)
    assert rel(Vu, Vo.reshape(-1)) <= TOL
    assert rel(Bu, Bo) <= TOL
    assert block_rows_err(rp, Vu, Vo.reshape(-1)) <= 10 * TOL
    assert info["min_detJ"] > 0
    # bitwise reproducible
    V2, B2, _ = fe.assemble_block(mesh, form, c.dt, u, rho, mu)
    import torch
    assert torch.equal(V, V2) and torch.equal(B, B2)
    mesh.close()


def test_block_operator_form0_is_scalar_momentum_times_identity(fe_ctx):
    """form 0: every block is the scalar momentum entry times I, bitwise
    equal between the block and scalar kernels only up to summation order,
    so compared to 1e-12 of the row scale."""
    fe = _fe()
    c = case_of("hex", 6, seed=1)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = fields(mesh, c)
    V, B, _ = fe.assemble_block(mesh, 0, c.dt, u, rho, mu)
    Vs, Bs, _ = fe.assemble(mesh, fe.MOMENTUM, c.dt, u, rho, mu)
    Vb = host(V).reshape(-1, 3, 3)
    vs = host(Vs)[0]
    eye = np.eye(3)
    assert np.abs(Vb - vs[:, None, None] * eye).max() <= TOL * np.abs(vs).max()
    assert rel(host(B), host(Bs)) <= TOL
    mesh.close()


@pytest.mark.parametrize("form", [1, 3])
def test_block_operator_times_u_is_the_residual(fe_ctx, form):
    """b - A u equals rows 0-2 of fe_residual(u, form): the block operator
    and the matrix-free residual pass describe one discrete operator."""
    fe = _fe()
    import torch
    c = case_of("hybrid", 6, seed=3)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = fields(mesh, c)
    V, B, _ = fe.assemble_block(mesh, form, c.dt, u, rho, mu)
    R = fe.residual(mesh, u, rho, mu, form=form)
    rp, ci = mesh.pattern_host()
    Vh = host(V).reshape(-1, 3, 3)
    uh = host(u).reshape(3, -1)
    rows = np.repeat(np.arange(mesh.n_nodes), np.diff(rp))
    Au = np.zeros((3, mesh.n_nodes))
    for i in range(3):
        for k in range(3):
            np.add.at(Au[i], rows, Vh[:, i, k] * uh[k, ci])
    got = host(B) - Au
    ref = host(R)[:3]
    scale = np.abs(host(B)).max()
    assert np.abs(got - ref).max() <= 1e-11 * scale
    mesh.close()


def test_block_operator_errors(fe_ctx):
    fe = _fe()
    c = case_of("hex", 3, seed=2)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = fields(mesh, c)
    with pytest.raises(fe.FeError) as ei:
        fe.assemble_block(mesh, 4, c.dt, u, rho, mu)
    assert ei.value.status == 1
    with pytest.raises(fe.FeError) as ei:
        fe.assemble_block(mesh, 1, -1.0, u, rho, mu)
    assert ei.value.status == 1
    mesh.close()
    # a folded element is reported by its user id
    bad = meshgen.make_case(3, meshgen.HEX08, 0.0, case_id=9)
    e = 13
    conn = bad.conn.copy()
    conn[e] = conn[e][[4, 5, 6, 7, 0, 1, 2, 3]]
    m2 = fe.Mesh(fe_ctx, meshgen.HEX08, bad.coords, conn, bad.dirichlet)
    u2, r2, mu2 = fields(m2, bad)
    with pytest.raises(fe.FeError) as ei:
        fe.assemble_block(m2, 3, bad.dt, u2, r2, mu2)
    assert ei.value.status == 4
    m2.close()


def test_block_operator_full_size_sampled_rows(fe_ctx):
    """128^3 HEX08 (the step's mesh): sampled block rows of the full-stress
    + EMAC operator against the oracle on the elements around them."""
    fe = _fe()
    case = meshgen.cfg1()
    print(f"full-size block operator: N={case.n_nodes} E={case.n_elems}", flush=True)
    mesh = make_mesh(fe_ctx, case)
    u, rho, mu = fields(mesh, case)
    V, B, _ = fe.assemble_block(mesh, 3, case.dt, u, rho, mu)
    rp_m, ci_m = mesh.pattern_host()
    perm = mesh.node_perm.astype(np.int64)
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(perm.size)
    rng = np.random.default_rng(17)
    nodes = rng.choice(case.n_nodes, 64, replace=False)
    sc, sconn, stypes, loc, glob = submesh_rows_typed(case, nodes)
    rp, ci, Vo, Bo = oracle.assemble_block(sc, sconn, 3, case.dt, case.u[:, glob], case.rho[glob], case.mu[glob])
    Vh = host(V).reshape(-1, 3, 3)
    Bh = host(B)
    for i in nodes:
        li, im = loc[i], iperm[i]
        ocols = glob[ci[rp[li]:rp[li + 1]]]
        ovals = Vo[rp[li]:rp[li + 1]]
        gcols = perm[ci_m[rp_m[im]:rp_m[im + 1]]]
        gvals = Vh[rp_m[im]:rp_m[im + 1]]
        o = np.argsort(gcols)
        assert np.array_equal(gcols[o], ocols)
        for r in range(3):
            scale = np.abs(ovals[:, r, :]).max()
            assert np.abs(gvals[o][:, r, :] - ovals[:, r, :]).max() <= TOL * scale
            assert abs(Bh[r][im] - Bo[r][li]) <= TOL * max(abs(Bo[r][li]), np.sqrt(np.mean(Bo[r] ** 2)))
    mesh.close()
