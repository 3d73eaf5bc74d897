"""GPU parity of the wall model's boundary assembly (Algorithm 1) against the
FP64 oracle: the traction's nodal vector on hex (quadrilateral faces), tet
(triangles) and hybrid (both) walls, its use inside the explicit step,
argument errors, determinism, and the 128^3 HEX08 wall at full size.
Tolerance 1e-12 relative: FP64 with the same Newton steps on both sides."""
import numpy as np
import pytest

import meshgen
import oracle
from tests.gpu_helpers import dev, host, make_mesh, rel

pytestmark = pytest.mark.gpu


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


def to_mesh(mesh, a):
    return mesh.to_mesh(dev(np.ascontiguousarray(a)))


def to_user(mesh, t):
    out = np.empty_like(host(t))
    out[..., mesh.node_perm] = host(t)
    return out


def wall_case(kind, n, seed):
    c = meshgen.make_case(n, kind, 0.12, case_id=160 + seed, shuffle=True, walls=True, temperature=True)
    rng = np.random.default_rng(seed)
    c.u = rng.normal(size=(3, c.n_nodes))
    c.mu = rng.uniform(1e-5, 1e-3, c.n_nodes)
    return c


@pytest.mark.parametrize("kind,n", [(meshgen.HEX08, 5), (meshgen.TET04, 4), (meshgen.HYBRID, 6)])
def test_wall_traction_matches_oracle(fe_ctx, kind, n):
    fe = _fe()
    c = wall_case(kind, n, n)
    delta = 0.3 / n
    mesh = make_mesh(fe_ctx, c)
    mesh.set_wall(c.wall_nen, c.wall_conn, delta)
    u, rho, mu = to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)
    t1 = fe.wall_traction(mesh, u, rho, mu)
    t = to_user(mesh, t1)
    ref = oracle.wall_traction(c.coords, c.wall_nen, c.wall_conn, c.u, c.rho, c.mu, delta)
    assert rel(t, ref) <= 1e-12, rel(t, ref)
    off = np.setdiff1d(np.arange(c.n_nodes), np.unique(c.wall_conn[c.wall_conn >= 0]))
    assert np.abs(t[:, off]).max() == 0.0
    # bitwise repeatable; clearing the faces gives zero
    assert np.array_equal(host(fe.wall_traction(mesh, u, rho, mu)), host(t1))
    mesh.set_wall(np.zeros(0, np.uint8), np.zeros((0, 4), np.int32), 0.0)
    assert np.abs(host(fe.wall_traction(mesh, u, rho, mu))).max() == 0.0
    mesh.close()


def test_wall_argument_errors(fe_ctx):
    fe = _fe()
    c = wall_case(meshgen.HEX08, 3, 1)
    mesh = make_mesh(fe_ctx, c)
    bad = c.wall_nen.copy()
    bad[0] = 5
    for args in ((bad, c.wall_conn, 0.1), (c.wall_nen, c.wall_conn, 0.0),
                 (c.wall_nen, np.where(c.wall_conn == c.wall_conn[0, 0], c.n_nodes, c.wall_conn), 0.1)):
        with pytest.raises(fe.FeError) as ei:
            mesh.set_wall(*args)
        assert ei.value.status == 1
    mesh.close()


@pytest.mark.parametrize("kind,form", [(meshgen.HEX08, 0), (meshgen.HYBRID, 3)])
def test_fractional_step_with_wall_matches_oracle(fe_ctx, kind, form):
    """One step with the wall model; on the hybrid cube with the full-stress
    and EMAC operator variants as well."""
    fe = _fe()
    import torch
    c = wall_case(kind, 6, 2)
    c.u *= 0.3
    # the wall nodes are free (the wall model sets their stress), the other
    # boundary nodes stay Dirichlet
    c.dirichlet = c.dirichlet[np.abs(c.coords[c.dirichlet, 2]) > 1e-12]
    dt, delta = 0.02, 0.05
    mesh = make_mesh(fe_ctx, c)
    mesh.set_wall(c.wall_nen, c.wall_conn, delta)
    u, rho = to_mesh(mesh, c.u), to_mesh(mesh, c.rho)
    L, f, _ = fe.assemble(mesh, fe.POISSON, dt, u, rho)
    fe.apply_dirichlet(mesh, L, f)
    p = torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda")
    fe.fractional_step(mesh, dt, rho, to_mesh(mesh, c.mu), L[0].contiguous(), u, p, rtol=1e-12, max_iter=5000,
                      form=form)
    rp, ci, Lo, fo = oracle.assemble(c.coords, c.conn, oracle.OP_POISSON, dt, c.u, c.rho, None, types=c.types)
    Lo, fo = Lo[0].copy(), fo[0].copy()
    oracle.dirichlet(rp, ci, Lo, fo, c.dirichlet)
    un, pn, _ = oracle.fractional_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu, (rp, ci, Lo),
                                       rtol=1e-12, wall=(c.wall_nen, c.wall_conn, delta), types=c.types,
                                       form=form)
    un0, _, _ = oracle.fractional_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu, (rp, ci, Lo),
                                       rtol=1e-12, types=c.types, form=form)
    assert rel(un, un0) > 1e-8            # the wall term matters
    assert rel(to_user(mesh, p), pn) <= 1e-8
    assert rel(to_user(mesh, u), un) <= 1e-9
    mesh.close()


def test_full_size_wall_traction(fe_ctx):
    """The 128^3 HEX08 mesh's z = 0 wall (16,384 quadrilaterals), every wall
    node against the oracle."""
    fe = _fe()
    c = meshgen.cfg1()
    print(f"full-size cfg1 wall: faces={c.wall_nen.shape[0]}", flush=True)
    delta = 1.0 / 128
    mesh = make_mesh(fe_ctx, c)
    mesh.set_wall(c.wall_nen, c.wall_conn, delta)
    t = to_user(mesh, fe.wall_traction(mesh, to_mesh(mesh, c.u), to_mesh(mesh, c.rho), to_mesh(mesh, c.mu)))
    ref = oracle.wall_traction(c.coords, c.wall_nen, c.wall_conn, c.u, c.rho, c.mu, delta)
    wall = np.unique(c.wall_conn)
    assert rel(t[:, wall], ref[:, wall]) <= 1e-12
    off = np.ones(c.n_nodes, bool)
    off[wall] = False
    assert not np.any(t[:, off])
    mesh.close()
