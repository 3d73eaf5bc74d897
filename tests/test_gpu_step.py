"""GPU parity of the explicit-step pieces (Algorithm 1: Runge-Kutta momentum
stages around the assembly, pressure solve, velocity correction) against the
FP64 oracle, through the C ABI.

Tolerances: the element-vector passes (residual, lumped mass, gradient,
divergence) are FP64 sums in another order, 1e-12 relative like the
assembly; a whole step agrees to the pressure solve's tolerance (both sides
solve to 1e-12, the velocity to 1e-9 relative).
"""
import numpy as np
import pytest

import meshgen
import oracle
from tests.gpu_helpers import dev, host, make_mesh, rel, submesh_rows_typed

pytestmark = pytest.mark.gpu

POI = oracle.OP_POISSON
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


def case_of(kind, n, seed=0):
    c = meshgen.make_case(n, KINDS[kind], 0.12, case_id=130 + seed, sub=KINDS[kind], shuffle=True,
                          temperature=(seed % 2 == 1))
    c.mu = np.random.default_rng(seed).uniform(1e-3, 3e-3, c.n_nodes)
    return c


def to_mesh(mesh, a):
    return mesh.to_mesh(dev(np.ascontiguousarray(a)))


def to_user(mesh, t):
    out = np.empty_like(host(t))
    out[..., mesh.node_perm] = host(t)
    return out


@pytest.mark.parametrize("kind,n", [("hex", 5), ("tet", 4), ("pen", 5), ("pyr", 4), ("hybrid", 6)])
def test_element_vector_passes_match_oracle(fe_ctx, kind, n):
    fe = _fe()
    c = case_of(kind, n, seed=n)
    print(f"{kind} n={n} E={c.n_elems}", flush=True)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    out = to_user(mesh, fe.residual(mesh, u, rho, mu))
    r, m = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types)
    for i in range(3):
        assert rel(out[i], r[i]) <= 1e-12, (i, rel(out[i], r[i]))
    assert rel(out[3], m) <= 1e-13
    p = np.random.default_rng(n).normal(size=c.n_nodes)
    g = to_user(mesh, fe.gradient(mesh, to_mesh(mesh, p)))
    gr = oracle.gradient(c.coords, c.conn, p, c.types)
    assert rel(g, gr) <= 1e-12
    dt = 0.013
    f = to_user(mesh, fe.divergence(mesh, dt, u, rho))
    _, _, _, fr = oracle.assemble(c.coords, c.conn, POI, dt, c.u, c.rho, None, types=c.types)
    assert rel(f, fr[0]) <= 1e-12
    mesh.close()


def _poisson(fe, mesh, c, dt):
    u, rho = to_mesh(mesh, c.u), to_mesh(mesh, c.rho)
    L, f, _ = fe.assemble(mesh, fe.POISSON, dt, u, rho)
    fe.apply_dirichlet(mesh, L, f)
    return L[0].contiguous()


def _oracle_poisson(c, dt):
    rp, ci, L, f = oracle.assemble(c.coords, c.conn, POI, dt, c.u, c.rho, None, types=c.types)
    L, f = L[0].copy(), f[0].copy()
    oracle.dirichlet(rp, ci, L, f, c.dirichlet)
    return rp, ci, L


@pytest.mark.parametrize("kind,n", [("hex", 6), ("tet", 5), ("pen", 5), ("pyr", 4), ("hybrid", 6)])
def test_fractional_step_matches_oracle(fe_ctx, kind, n):
    fe = _fe()
    import torch
    c = case_of(kind, n, seed=7)
    dt = 0.4 / n
    mesh = make_mesh(fe_ctx, c)
    L = _poisson(fe, mesh, c, dt)
    u = to_mesh(mesh, c.u)
    p = torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda")
    rho, mu = to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    info = fe.fractional_step(mesh, dt, rho, mu, L, u, p, rtol=1e-12, max_iter=5000)
    un, pn, it = oracle.fractional_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu,
                                        _oracle_poisson(c, dt), rtol=1e-12, types=c.types)
    assert info["cg_true_rel_residual"] <= 1e-11
    assert abs(info["cg_iterations"] - it) <= 3, (info["cg_iterations"], it)
    ug, pg = to_user(mesh, u), to_user(mesh, p)
    assert rel(pg, pn) <= 1e-8, rel(pg, pn)
    assert rel(ug, un) <= 1e-9, rel(ug, un)
    assert np.array_equal(ug[:, c.dirichlet], c.u[:, c.dirichlet])
    # a second step from the first one's state, bitwise reproducible
    u2, p2 = u.clone(), p.clone()
    fe.fractional_step(mesh, dt, rho, mu, L, u, p, rtol=1e-12, max_iter=5000)
    fe.fractional_step(mesh, dt, rho, mu, L, u2, p2, rtol=1e-12, max_iter=5000)
    assert torch.equal(u, u2) and torch.equal(p, p2)
    mesh.close()


def test_step_argument_errors_and_bad_element(fe_ctx):
    fe = _fe()
    import torch
    c = meshgen.make_case(3, meshgen.HEX08, 0.0, case_id=140)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    L = _poisson(fe, mesh, c, 0.1)
    p = torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FeError) as ei:
        fe.fractional_step(mesh, -0.1, rho, mu, L, u, p)
    assert ei.value.status == 1
    with pytest.raises(fe.FeError) as ei:
        fe.divergence(mesh, 0.0, u, rho)
    assert ei.value.status == 1
    mesh.close()
    X = c.coords.copy()
    e = c.conn[5]
    X[[e[0], e[6]]] = X[[e[6], e[0]]]
    c.coords = X
    mesh = make_mesh(fe_ctx, c)
    with pytest.raises(fe.FeError) as ei:
        fe.residual(mesh, to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu))
    assert ei.value.status == 4
    # the fractional step reads its passes' status words back once, at its
    # end, and still reports the folded element by its user id (L: the
    # identity on this mesh's pattern, so the solve itself succeeds)
    rp, ci = mesh.pattern_host()
    Lh = (ci == np.repeat(np.arange(mesh.n_nodes), np.diff(rp))).astype(np.float64)
    ub = to_mesh(mesh, c.u)
    pb = torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FeError) as ei:
        fe.fractional_step(mesh, 0.01, to_mesh(mesh, c.rho), to_mesh(mesh, c.mu), dev(Lh), ub, pb)
    assert ei.value.status == 4 and "element 5 " in str(ei.value)
    mesh.close()


def test_full_size_residual_and_gradient_sampled_rows(fe_ctx):
    """128^3 HEX08 (the bench's mesh): residual, lumped mass and gradient at
    sampled nodes against the oracle on the elements around them."""
    fe = _fe()
    c = meshgen.cfg1()
    print(f"full-size cfg1: N={c.n_nodes} E={c.n_elems}", flush=True)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    p = np.random.default_rng(3).normal(size=c.n_nodes)
    out = to_user(mesh, fe.residual(mesh, u, rho, mu))
    g = to_user(mesh, fe.gradient(mesh, to_mesh(mesh, p)))
    rng = np.random.default_rng(4)
    nodes = np.unique(np.concatenate([rng.integers(0, c.n_nodes, 64), [0, c.n_nodes - 1]]))
    sc, sconn, st, loc, glob = submesh_rows_typed(c, nodes)
    r, m = oracle.residual(sc, sconn[:, :8], c.u[:, glob], c.rho[glob], c.mu[glob])
    gr = oracle.gradient(sc, sconn[:, :8], p[glob])
    li = loc[nodes]
    for i in range(3):
        scale = np.abs(r[i]).max()
        assert np.abs(out[i][nodes] - r[i][li]).max() <= 1e-12 * scale
        assert np.abs(g[i][nodes] - gr[i][li]).max() <= 1e-12 * np.abs(gr[i]).max()
    assert np.abs(out[3][nodes] - m[li]).max() <= 1e-13 * m.max()
    mesh.close()


@pytest.mark.parametrize("form", [1, 2, 3])
@pytest.mark.parametrize("kind,n", [("hex", 5), ("tet", 4), ("hybrid", 6)])
def test_residual_operator_variants_match_oracle(fe_ctx, kind, n, form):
    """Full-stress viscous term (1), EMAC convection (2), both (3)."""
    fe = _fe()
    c = case_of(kind, n, seed=20 + n)
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    out = to_user(mesh, fe.residual(mesh, u, rho, mu, form=form))
    r, m = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types, form)
    r0, _ = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types)
    assert rel(r, r0) > 1e-6                 # the variant changes the residual
    for i in range(3):
        assert rel(out[i], r[i]) <= 1e-12, (i, rel(out[i], r[i]))
    assert rel(out[3], m) <= 1e-13
    with pytest.raises(fe.FeError) as ei:
        fe.residual(mesh, u, rho, mu, form=4)
    assert ei.value.status == 1
    mesh.close()


def test_fractional_step_full_stress_emac_matches_oracle(fe_ctx):
    fe = _fe()
    import torch
    c = case_of("hex", 6, seed=9)
    dt = 0.4 / 6
    mesh = make_mesh(fe_ctx, c)
    L = _poisson(fe, mesh, c, dt)
    u = to_mesh(mesh, c.u)
    p = torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda")
    form = fe.FULL_STRESS | fe.EMAC
    fe.fractional_step(mesh, dt, to_mesh(mesh, c.rho), to_mesh(mesh, c.mu), L, u, p, rtol=1e-12, max_iter=5000,
                       form=form)
    un, pn, _ = oracle.fractional_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu,
                                       _oracle_poisson(c, dt), rtol=1e-12, form=form)
    assert rel(to_user(mesh, p), pn) <= 1e-8
    assert rel(to_user(mesh, u), un) <= 1e-9
    mesh.close()


def test_fractional_step_mixed_pressure_solve(fe_ctx):
    """FE_MIXED solves the pressure in FP32 PCG inside FP64 refinement: the
    step agrees with the FP64 one to the solve's tolerance."""
    fe = _fe()
    import torch
    c = case_of("hybrid", 6, seed=11)
    dt = 0.05
    mesh = make_mesh(fe_ctx, c)
    L = _poisson(fe, mesh, c, dt)
    rho, mu = to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    outs = []
    for prec in (fe.FP64, fe.MIXED):
        u = to_mesh(mesh, c.u)
        p = torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda")
        info = fe.fractional_step(mesh, dt, rho, mu, L, u, p, rtol=1e-10, max_iter=5000, precision=prec)
        assert info["cg_true_rel_residual"] <= 1e-10
        outs.append((host(u), host(p)))
    assert rel(outs[1][1], outs[0][1]) <= 1e-7
    assert rel(outs[1][0], outs[0][0]) <= 1e-9
    mesh.close()


@pytest.mark.parametrize("kind,n", [("hex", 5), ("tet", 4), ("pen", 5), ("pyr", 4), ("hybrid", 6)])
def test_scalar_residual_and_step_match_oracle(fe_ctx, kind, n):
    """The heat/species residual and one explicit scalar step (no solve)."""
    fe = _fe()
    c = case_of(kind, n, seed=30 + n)
    Y = np.random.default_rng(n).uniform(0, 1, c.n_nodes)
    D = 2e-3
    mesh = make_mesh(fe_ctx, c)
    u, rho, Yd = to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, Y)
    out = to_user(mesh, fe.scalar_residual(mesh, u, rho, Yd, D))
    r, m = oracle.scalar_residual(c.coords, c.conn, c.u, c.rho, Y, D, c.types)
    assert rel(out[0], r) <= 1e-12 and rel(out[1], m) <= 1e-13
    dt = 0.2 / n
    fe.scalar_step(mesh, dt, u, rho, D, Yd)
    yo = oracle.scalar_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, Y, D, c.types)
    assert rel(to_user(mesh, Yd), yo) <= 1e-12
    with pytest.raises(fe.FeError) as ei:
        fe.scalar_step(mesh, dt, u, rho, -1.0, Yd)
    assert ei.value.status == 1
    mesh.close()


@pytest.mark.parametrize("kind,n,renumber", [("hex", 1, True), ("tet", 1, True), ("pen", 1, True),
                                             ("pyr", 1, True), ("hex", 2, False), ("hybrid", 4, False),
                                             ("hybrid", 5, False)])
def test_element_vector_passes_edge_cases(fe_ctx, kind, n, renumber):
    """One-cell meshes (a single block, far below a wavefront) and user
    element order (hybrid blocks closed at every type change): residual with
    both operator variants, gradient, divergence and the scalar residual."""
    fe = _fe()
    c = case_of(kind, n, seed=40 + n)
    print(f"{kind} n={n} E={c.n_elems} renumber={renumber}", flush=True)
    mesh = make_mesh(fe_ctx, c, renumber)
    u, rho, mu = to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    out = to_user(mesh, fe.residual(mesh, u, rho, mu, form=3))
    r, m = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types, form=3)
    for i in range(3):
        assert rel(out[i], r[i]) <= 1e-12, (i, rel(out[i], r[i]))
    assert rel(out[3], m) <= 1e-13
    p = np.random.default_rng(n).normal(size=c.n_nodes)
    g = to_user(mesh, fe.gradient(mesh, to_mesh(mesh, p)))
    assert rel(g, oracle.gradient(c.coords, c.conn, p, c.types)) <= 1e-12
    f = to_user(mesh, fe.divergence(mesh, 0.02, u, rho))
    _, _, _, fr = oracle.assemble(c.coords, c.conn, POI, 0.02, c.u, c.rho, None, types=c.types)
    assert rel(f, fr[0]) <= 1e-12
    Y = np.random.default_rng(n + 1).uniform(0, 1, c.n_nodes)
    s = to_user(mesh, fe.scalar_residual(mesh, u, rho, to_mesh(mesh, Y), 2e-3))
    sr, sm = oracle.scalar_residual(c.coords, c.conn, c.u, c.rho, Y, 2e-3, c.types)
    assert rel(s[0], sr) <= 1e-12 and rel(s[1], sm) <= 1e-13
    mesh.close()
