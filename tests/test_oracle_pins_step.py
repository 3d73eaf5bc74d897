"""Pins of the oracle's explicit-step pieces (Algorithm 1: the Runge-Kutta
momentum stages around the assembly, the pressure solve and the velocity
correction) against facts fixed by the mathematics.

- the matrix-free residual equals b - A u from the assembled momentum
  operator (a different path: CSR matrix times vector) on hex, tet and
  hybrid meshes, and the lumped mass equals the mass matrix's row sums;
- the gradient is exact for a linear pressure and is the adjoint of the
  divergence right-hand side: u . G p = dt p . f(u) for rho = 1;
- the Runge-Kutta predictor's local error falls 16x when dt halves (third
  order; a lower-order tableau fails), and the scheme's stages are the
  Shu-Osher ones (a forward-Euler tableau is detected);
- the full step keeps the boundary velocity, solves the pressure system and
  reduces the discrete divergence.
"""
import numpy as np
import pytest

import meshgen
import oracle

MOM, POI = oracle.OP_MOMENTUM, oracle.OP_POISSON
KINDS = {"hex": meshgen.HEX08, "tet": meshgen.TET04, "hybrid": meshgen.HYBRID}


def case_of(kind, n=4, seed=0):
    c = meshgen.make_case(n, KINDS[kind], 0.12, case_id=120 + seed, sub=KINDS[kind], shuffle=True)
    rng = np.random.default_rng(seed)
    c.mu = rng.uniform(1e-3, 3e-3, c.n_nodes)
    return c


@pytest.mark.parametrize("kind", ["hex", "tet", "hybrid"])
def test_residual_is_b_minus_Au(kind):
    c = case_of(kind)
    r, m = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types)
    dt = 0.37
    rp, ci, A, b = oracle.assemble(c.coords, c.conn, MOM, dt, c.u, c.rho, c.mu, types=c.types)
    for i in range(3):
        ref = b[i] - oracle.spmv(rp, ci, A[0], c.u[i])
        assert np.linalg.norm(r[i] - ref) <= 1e-12 * np.linalg.norm(ref)
    N = c.n_nodes
    _, _, M, _ = oracle.assemble(c.coords, c.conn, MOM, 1.0, np.zeros((3, N)), c.rho, np.zeros(N),
                                 pattern_=(rp, ci), types=c.types)
    assert np.abs(m - oracle.spmv(rp, ci, M[0], np.ones(N))).max() <= 1e-14 * m.max()
    assert np.all(m > 0)


@pytest.mark.parametrize("kind", ["hex", "tet", "hybrid"])
def test_gradient_exact_for_linear_pressure_and_adjoint_of_divergence(kind):
    c = case_of(kind, seed=1)
    N = c.n_nodes
    grad = np.array([0.4, -1.3, 2.1])
    p = c.coords @ grad + 0.7
    g = oracle.gradient(c.coords, c.conn, p, c.types)
    _, m1 = oracle.residual(c.coords, c.conn, np.zeros((3, N)), np.ones(N), np.zeros(N), c.types)
    for j in range(3):
        assert np.abs(g[j] - grad[j] * m1).max() <= 1e-13 * np.abs(grad[j] * m1).max()
    rng = np.random.default_rng(2)
    p = rng.normal(size=N)
    u = rng.normal(size=(3, N))
    dt = 0.3
    _, _, _, f = oracle.assemble(c.coords, c.conn, POI, dt, u, np.ones(N), None, types=c.types)
    g = oracle.gradient(c.coords, c.conn, p, c.types)
    lhs = np.sum(u * g)
    assert abs(lhs - dt * p @ f[0]) <= 1e-12 * np.abs(u * g).sum()


def _predictor_error(c, dt, rk=oracle.SSP_RK3):
    one, _ = oracle.rk_predictor(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu, c.types, rk)
    ref = np.array(c.u)
    for _ in range(32):
        ref, _ = oracle.rk_predictor(c.coords, c.conn, c.dirichlet, dt / 32, ref, c.rho, c.mu, c.types)
    return np.linalg.norm(one - ref)


def test_runge_kutta_local_error_is_fourth_order():
    c = case_of("hex", n=4, seed=3)
    e1, e2 = _predictor_error(c, 0.02), _predictor_error(c, 0.01)
    assert 12.0 < e1 / e2 < 20.0, e1 / e2
    # three forward-Euler stages (a first-order tableau) are caught
    euler = ((0.0, 1.0), (0.0, 1.0), (0.0, 1.0))
    f1, f2 = _predictor_error(c, 0.02, euler), _predictor_error(c, 0.01, euler)
    assert f1 / f2 < 6.0


def test_fractional_step_keeps_boundary_and_reduces_divergence():
    c = case_of("hex", n=6, seed=4)
    N = c.n_nodes
    c.rho = np.ones(N)
    dt = 0.02
    rp, ci, L, _ = oracle.assemble(c.coords, c.conn, POI, dt, c.u, c.rho, None)
    L, z = L[0].copy(), np.zeros(N)
    oracle.dirichlet(rp, ci, L, z, c.dirichlet)
    un, p, it = oracle.fractional_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu, (rp, ci, L))
    assert np.array_equal(un[:, c.dirichlet], c.u[:, c.dirichlet])
    assert it > 0 and np.abs(p[c.dirichlet]).max() == 0.0
    us, _ = oracle.rk_predictor(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu)
    free = np.ones(N, bool)
    free[c.dirichlet] = False

    def rhs(v):
        _, _, _, f = oracle.assemble(c.coords, c.conn, POI, dt, v, c.rho, None, pattern_=(rp, ci))
        return f[0]
    # the pressure solves the stated system: L p = f(u*) on the free rows
    f = rhs(us)
    assert np.linalg.norm((oracle.spmv(rp, ci, L, p) - f)[free]) <= 1e-10 * np.linalg.norm(f[free])
    # an approximate projection (lumped mass): the discrete divergence drops,
    # not to zero
    assert np.linalg.norm(rhs(un)[free]) < 0.95 * np.linalg.norm(f[free])


# --- operator variants of Eq. (1): full-stress viscous term, EMAC convection ---

def _lin(c, A, b=None):
    """Nodal values of the linear field u = A x (+ b), [3, N]."""
    u = (c.coords @ np.asarray(A).T).T
    return np.ascontiguousarray(u if b is None else u + np.asarray(b)[:, None])


@pytest.mark.parametrize("kind", ["hex", "tet", "hybrid"])
def test_full_stress_on_rotations_and_strains(kind):
    # rho = 0 isolates the viscous term; constant mu
    c = case_of(kind, seed=5)
    N = c.n_nodes
    zero, mu = np.zeros(N), np.full(N, 1.7e-3)
    W = np.array([[0.0, -0.4, 0.9], [0.4, 0.0, -1.3], [-0.9, 1.3, 0.0]])     # rigid rotation: eps(u) = 0
    r_fs, _ = oracle.residual(c.coords, c.conn, _lin(c, W), zero, mu, c.types, oracle.FULL_STRESS)
    r_lap, _ = oracle.residual(c.coords, c.conn, _lin(c, W), zero, mu, c.types)
    assert np.abs(r_fs).max() <= 1e-14 * np.abs(r_lap).max()
    assert np.abs(r_lap).max() > 1e-6            # the Laplacian form does not vanish there
    S = np.array([[0.7, 0.2, -0.3], [0.2, -0.1, 0.5], [-0.3, 0.5, 0.4]])      # symmetric, trace != 0
    r_fs, _ = oracle.residual(c.coords, c.conn, _lin(c, S), zero, mu, c.types, oracle.FULL_STRESS)
    r_lap, _ = oracle.residual(c.coords, c.conn, _lin(c, S), zero, mu, c.types)
    assert np.abs(r_fs - 2.0 * r_lap).max() <= 1e-13 * np.abs(r_lap).max()
    # symmetric bilinear form: v . V(u) = u . V(v)
    rng = np.random.default_rng(6)
    u, v = rng.normal(size=(3, N)), rng.normal(size=(3, N))
    ru, _ = oracle.residual(c.coords, c.conn, u, zero, mu, c.types, oracle.FULL_STRESS)
    rv, _ = oracle.residual(c.coords, c.conn, v, zero, mu, c.types, oracle.FULL_STRESS)
    assert abs(np.sum(v * ru) - np.sum(u * rv)) <= 1e-12 * np.abs(v * ru).sum()


@pytest.mark.parametrize("kind", ["hex", "tet", "hybrid"])
def test_emac_divergence_term_and_momentum_conservation(kind):
    c = case_of(kind, seed=6)
    N = c.n_nodes
    one, zero = np.ones(N), np.zeros(N)
    # divergence-free linear field: EMAC = advective form
    A = np.array([[0.3, -0.7, 0.2], [0.5, 0.1, -0.4], [0.6, 0.9, -0.4]])    # trace 0
    r_e, _ = oracle.residual(c.coords, c.conn, _lin(c, A, [0.2, -0.1, 0.3]), one, zero, c.types, oracle.EMAC)
    r_a, _ = oracle.residual(c.coords, c.conn, _lin(c, A, [0.2, -0.1, 0.3]), one, zero, c.types)
    assert np.abs(r_e - r_a).max() <= 1e-14 * np.abs(r_a).max()
    # uniform dilatation u = s x: the extra term is -(div u) M u_i = -3 s M u_i
    s = 0.8
    u = _lin(c, s * np.eye(3))
    r_e, _ = oracle.residual(c.coords, c.conn, u, one, zero, c.types, oracle.EMAC)
    r_a, _ = oracle.residual(c.coords, c.conn, u, one, zero, c.types)
    rp, ci, M, _ = oracle.assemble(c.coords, c.conn, MOM, 1.0, np.zeros((3, N)), one, zero, types=c.types)
    for i in range(3):
        ref = -3.0 * s * oracle.spmv(rp, ci, M[0], u[i])
        assert np.abs(r_e[i] - r_a[i] - ref).max() <= 1e-13 * np.abs(ref).max()
    # total momentum is conserved by the divergence (EMAC) form when u . n = 0
    # on the boundary, not by the advective form
    rng = np.random.default_rng(7)
    u = rng.normal(size=(3, N))
    X = c.coords
    for j in range(3):
        on = (np.abs(X[:, j]) < 1e-12) | (np.abs(X[:, j] - 1.0) < 1e-12)
        u[j, on] = 0.0
    r_e, _ = oracle.residual(c.coords, c.conn, u, one, zero, c.types, oracle.EMAC)
    r_a, _ = oracle.residual(c.coords, c.conn, u, one, zero, c.types)
    scale = np.abs(r_e).sum(axis=1)
    assert np.all(np.abs(r_e.sum(axis=1)) <= 1e-13 * scale), r_e.sum(axis=1) / scale
    assert np.any(np.abs(r_a.sum(axis=1)) > 1e-3 * np.abs(r_a).sum(axis=1))


# --- scalar transport (heat, species): the same stages without a solve ---

@pytest.mark.parametrize("kind", ["hex", "tet", "hybrid"])
def test_scalar_residual_is_b_minus_AY(kind):
    c = case_of(kind, seed=8)
    N = c.n_nodes
    Y = np.random.default_rng(9).uniform(0, 1, N)
    D = 3e-3
    r, m = oracle.scalar_residual(c.coords, c.conn, c.u, c.rho, Y, D, c.types)
    dt = 0.21
    rp, ci, A, b = oracle.assemble(c.coords, c.conn, oracle.OP_SCALAR, dt, c.u, c.rho, None, Y=Y[None, :],
                                   D=np.array([D]), types=c.types)
    ref = b[0] - oracle.spmv(rp, ci, A[0], Y)
    assert np.linalg.norm(r - ref) <= 1e-12 * np.linalg.norm(ref)
    _, m_mom = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types)
    assert np.array_equal(m, m_mom)


def test_scalar_step_keeps_constants_and_is_third_order():
    c = case_of("hex", n=4, seed=10)
    N = c.n_nodes
    # a constant scalar is a steady state (C 1 = 0, K 1 = 0)
    y = oracle.scalar_step(c.coords, c.conn, c.dirichlet, 0.01, c.u, c.rho, np.full(N, 0.7), 2e-3)
    assert np.abs(y - 0.7).max() <= 1e-14
    Y = np.random.default_rng(11).uniform(0, 1, N)

    def err(dt):
        one = oracle.scalar_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, Y, 2e-3)
        ref = Y
        for _ in range(32):
            ref = oracle.scalar_step(c.coords, c.conn, c.dirichlet, dt / 32, c.u, c.rho, ref, 2e-3)
        return np.linalg.norm(one - ref)
    e1, e2 = err(0.02), err(0.01)
    assert 12.0 < e1 / e2 < 20.0, e1 / e2
