"""Pins of the FP64 oracle against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: textbook
identities of the reference elements, closed-form elemental matrices,
operator invariants (row sums, symmetry, isoparametric reproduction), a dense
brute-force assembly, a partitioned direct solve for the Dirichlet
elimination, an independent CG implementation and a manufactured solution.
Each is chosen so that a plausible slip (a dropped term, a sign, a transposed
operand, a wrong index or weight) fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import meshgen
import oracle

MOM, SCA, POI = oracle.OP_MOMENTUM, oracle.OP_SCALAR, oracle.OP_POISSON


def dense(rowptr, colidx, vals, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, colidx[rowptr[i]:rowptr[i + 1]]] = vals[rowptr[i]:rowptr[i + 1]]
    return A


def tet_mesh(n, jitter=0.0, seed=0):
    rs = meshgen.streams(99, seed)
    X = meshgen.cube_nodes(n, jitter, rs["jitter"])
    return X, meshgen.kuhn_split(meshgen.hex_conn(n))


def hex_mesh(n, jitter=0.0, seed=0):
    rs = meshgen.streams(98, seed)
    return meshgen.cube_nodes(n, jitter, rs["jitter"]), meshgen.hex_conn(n)


def interior_mask(X, tol=1e-12):
    return np.all((X > tol) & (X < 1 - tol), axis=1)


# --- reference elements -------------------------------------------------------

@pytest.mark.parametrize("nen", [8, 4])
def test_partition_of_unity_and_gradient_sum(nen):
    rng = np.random.default_rng(1)
    for _ in range(20):
        xi = rng.uniform(-1, 1, 3) if nen == 8 else rng.dirichlet(np.ones(4))[:3]
        N, dN = oracle.shape(nen, xi)
        assert abs(N.sum() - 1.0) < 1e-15
        assert np.abs(dN.sum(axis=0)).max() < 1e-15


def test_hex_kronecker_and_tet_kronecker():
    corners = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                        [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], float)
    for b in range(8):
        N, _ = oracle.shape(8, corners[b])
        assert np.allclose(N, np.eye(8)[b], atol=1e-16)
    tv = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    for b in range(4):
        N, _ = oracle.shape(4, tv[b])
        assert np.allclose(N, np.eye(4)[b], atol=1e-16)


def test_hex_gradient_matches_finite_difference():
    rng = np.random.default_rng(2)
    xi = rng.uniform(-0.9, 0.9, 3)
    _, dN = oracle.shape(8, xi)
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1e-6
        Np, _ = oracle.shape(8, xi + e)
        Nm, _ = oracle.shape(8, xi - e)
        assert np.abs((Np - Nm) / 2e-6 - dN[:, j]).max() < 1e-9


def test_gauss_weights_sum_to_reference_volume():
    _, w = oracle.gauss(8)
    assert abs(w.sum() - 8.0) < 1e-15
    _, w = oracle.gauss(4)
    assert abs(w.sum() - 1.0 / 6.0) < 1e-16


def test_hex_gauss_exact_to_degree_three_per_variable():
    pts, w = oracle.gauss(8)
    for p in range(4):
        for q in range(4):
            for r in range(4):
                exact = 1.0
                for k in (p, q, r):
                    exact *= 0.0 if k % 2 else 2.0 / (k + 1)
                got = np.sum(w * pts[:, 0] ** p * pts[:, 1] ** q * pts[:, 2] ** r)
                assert abs(got - exact) < 1e-14, (p, q, r)
    # not exact at degree 4: the rule is the 2-point one, not something richer
    got = np.sum(w * pts[:, 0] ** 4)
    assert abs(got - 8.0 / 5.0) > 0.1


def test_tet_rule_exact_to_total_degree_two():
    pts, w = oracle.gauss(4)
    for p in range(3):
        for q in range(3 - p):
            for r in range(3 - p - q):
                exact = math.factorial(p) * math.factorial(q) * math.factorial(r) / math.factorial(p + q + r + 3)
                got = np.sum(w * pts[:, 0] ** p * pts[:, 1] ** q * pts[:, 2] ** r)
                assert abs(got - exact) < 1e-16, (p, q, r)


# --- closed-form elemental matrices -------------------------------------------

def single(nen, X, op=MOM, dt=1.0, u=None, rho=None, mu=None, **kw):
    conn = np.arange(nen, dtype=np.int32)[None, :]
    rp, ci, v, b = oracle.assemble(X, conn, op, dt, u, rho, mu, **kw)
    return v.reshape(v.shape[0], nen, nen), b


def test_hex_mass_closed_form_undistorted():
    h = 0.37
    X = meshgen.cube_nodes(1)[meshgen.hex_conn(1)[0]] * h
    # momentum with rho = 1, u = 0, mu = 0, dt = 1 is the plain mass matrix
    A, _ = single(8, X, u=np.zeros((3, 8)), rho=np.ones(8), mu=np.zeros(8))
    corners = X / h
    for a in range(8):
        for b in range(8):
            d = int(np.abs(corners[a] - corners[b]).sum())
            exact = h ** 3 / 216.0 * {0: 8, 1: 4, 2: 2, 3: 1}[d]
            assert abs(A[0, a, b] - exact) < 1e-15 * h ** 3


def test_tet_mass_closed_form():
    X = np.array([[0.1, 0.2, 0.0], [1.3, 0.1, 0.2], [0.2, 0.9, 0.1], [0.3, 0.4, 1.1]])
    V = np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])) / 6.0
    assert V > 0
    A, _ = single(4, X, u=np.zeros((3, 4)), rho=np.ones(4), mu=np.zeros(4))
    assert np.abs(A[0] - V / 20.0 * (np.ones((4, 4)) + np.eye(4))).max() < 1e-15


def test_tet_stiffness_closed_form():
    X = np.array([[0.1, 0.2, 0.0], [1.3, 0.1, 0.2], [0.2, 0.9, 0.1], [0.3, 0.4, 1.1]])
    T = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])   # rows: edge vectors
    V = np.linalg.det(T) / 6.0
    # gradients of barycentric coordinates: rows of inverse of T^T
    G = np.linalg.inv(T)                                    # columns are grad lambda_1..3
    grads = np.vstack([-G.sum(axis=1), G.T])
    L, _ = single(4, X, op=POI, u=np.zeros((3, 4)), rho=np.ones(4))
    assert np.abs(L[0] - V * grads @ grads.T).max() < 1e-13


def test_uniform_grid_laplacian_stencil():
    n, mu = 4, 1.8e-5
    h = 1.0 / n
    X, conn = hex_mesh(n)
    N = X.shape[0]
    rp, ci, K, _ = oracle.assemble(X, conn, MOM, 1.0, np.zeros((3, N)), np.zeros(N), np.full(N, mu))
    i = meshgen.node_id(n, 2, 2, 2)
    for p in range(rp[i], rp[i + 1]):
        d = int(np.abs(np.round((X[ci[p]] - X[i]) / h)).sum())
        exact = mu * h * {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[d]
        assert abs(K[0][p] - exact) < 1e-13 * mu * h


# --- operator invariants on distorted meshes ----------------------------------

@pytest.fixture(scope="module", params=["hex", "tet"])
def jittered(request):
    if request.param == "hex":
        X, conn = hex_mesh(4, 0.15, seed=1)
    else:
        X, conn = tet_mesh(3, 0.10, seed=1)
    N = X.shape[0]
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.2, 1.2, N)
    mu = rng.uniform(1e-5, 3e-5, N)
    u = rng.normal(0, 1, (3, N))
    return X, conn, rho, mu, u


def _mat(X, conn, op, dt, u, rho, mu, **kw):
    rp, ci, v, b = oracle.assemble(X, conn, op, dt, u, rho, mu, **kw)
    return rp, ci, v, b


def test_mass_sum_is_domain_volume(jittered):
    X, conn, *_ = jittered
    N = X.shape[0]
    _, _, M, _ = _mat(X, conn, MOM, 1.0, np.zeros((3, N)), np.ones(N), np.zeros(N))
    assert abs(M.sum() - 1.0) < 1e-13


def test_weighted_mass_sum(jittered):
    X, conn, rho, *_ = jittered
    N = X.shape[0]
    rp, ci, M1, _ = _mat(X, conn, MOM, 1.0, np.zeros((3, N)), np.ones(N), np.zeros(N))
    _, _, Mr, _ = _mat(X, conn, MOM, 1.0, np.zeros((3, N)), rho, np.zeros(N))
    rowsum1 = oracle.spmv(rp, ci, M1[0], np.ones(N))
    assert abs(Mr.sum() - rho @ rowsum1) < 1e-13 * abs(Mr.sum())


def test_viscous_rows_sum_to_zero_symmetric_and_patch(jittered):
    X, conn, rho, mu, u = jittered
    N = X.shape[0]
    rp, ci, K, _ = _mat(X, conn, MOM, 1.0, u, np.zeros(N), mu)   # rho = 0 leaves K only
    Kd = dense(rp, ci, K[0], N)
    scale = np.abs(Kd).max(axis=1)
    assert np.all(np.abs(Kd @ np.ones(N)) <= 1e-13 * scale)
    assert np.abs(Kd - Kd.T).max() <= 1e-13 * scale.max()
    # patch test with constant mu: K x_j vanishes on interior rows
    _, _, Kc, _ = _mat(X, conn, MOM, 1.0, u, np.zeros(N), np.full(N, 2e-5))
    Kcd = dense(rp, ci, Kc[0], N)
    inner = interior_mask(X)
    for j in range(3):
        r = Kcd @ X[:, j]
        assert np.all(np.abs(r[inner]) <= 1e-13 * np.abs(Kcd[inner]).max(axis=1))


def test_convection_rows_sum_to_zero_and_reproduce_linear_fields(jittered):
    X, conn, rho, mu, u = jittered
    N = X.shape[0]
    dt = 0.01
    zero = np.zeros(N)
    rp, ci, A, _ = _mat(X, conn, MOM, dt, u, rho, zero)                # M/dt + C
    _, _, A0, _ = _mat(X, conn, MOM, dt, np.zeros((3, N)), rho, zero)  # M/dt
    Cd = dense(rp, ci, A[0] - A0[0], N)
    Md = dense(rp, ci, A0[0], N) * dt
    scale = np.abs(dense(rp, ci, A[0], N)).max(axis=1)
    assert np.all(np.abs(Cd @ np.ones(N)) <= 1e-13 * scale)
    for j in range(3):
        lhs = Cd @ X[:, j]
        rhs = Md @ u[j]
        assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale)
    # C is not symmetric: a transposed operand would be caught here
    assert np.abs(Cd - Cd.T).max() > 1e-3 * np.abs(Cd).max()


def test_momentum_rhs_is_mass_times_velocity_over_dt(jittered):
    X, conn, rho, mu, u = jittered
    N = X.shape[0]
    dt = 0.02
    rp, ci, A, b = _mat(X, conn, MOM, dt, u, rho, mu)
    _, _, M, _ = _mat(X, conn, MOM, 1.0, np.zeros((3, N)), rho, np.zeros(N))
    for i in range(3):
        ref = oracle.spmv(rp, ci, M[0], u[i]) / dt
        assert np.linalg.norm(b[i] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_scalar_operator_is_momentum_with_rho_d(jittered):
    X, conn, rho, mu, u = jittered
    N = X.shape[0]
    dt = 0.03
    rng = np.random.default_rng(7)
    Y = rng.uniform(0, 1, (3, N))
    D = np.array([1e-6, 3e-5, 1e-4])
    rp, ci, S, bs = _mat(X, conn, SCA, dt, u, rho, mu, Y=Y, D=D)
    _, _, M, _ = _mat(X, conn, MOM, 1.0, np.zeros((3, N)), rho, np.zeros(N))
    for k in range(3):
        _, _, Ak, _ = _mat(X, conn, MOM, dt, u, rho, rho * D[k])   # nodal mu_k = rho D_k
        # mu_g = sum N rho_a D_k = D_k rho_g: same operator up to rounding
        assert np.abs(S[k] - Ak[0]).max() <= 1e-13 * np.abs(Ak[0]).max()
        ref = oracle.spmv(rp, ci, M[0], Y[k]) / dt
        assert np.linalg.norm(bs[k] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_poisson_rhs_constant_flux_vanishes_inside(jittered):
    X, conn, *_ = jittered
    N = X.shape[0]
    c = np.array([0.3, -1.2, 0.7])
    u = np.repeat(c[:, None], N, axis=1)
    rp, ci, L, f = _mat(X, conn, POI, 0.5, u, np.ones(N), None)
    inner = interior_mask(X)
    assert np.abs(f[0][inner]).max() <= 1e-14
    assert np.abs(f[0][~inner]).max() > 1e-3   # the boundary terms are not zero


def test_poisson_rhs_divergence_on_undistorted_grid():
    # f_a = (1/dt) int grad N_a . (x, 0, 0) = -(1/dt) int N_a = -(1/dt) (M 1)_a inside
    X, conn = hex_mesh(4)
    N = X.shape[0]
    dt = 0.25
    u = np.zeros((3, N))
    u[0] = X[:, 0]
    rp, ci, L, f = _mat(X, conn, POI, dt, u, np.ones(N), None)
    _, _, M, _ = _mat(X, conn, MOM, 1.0, np.zeros((3, N)), np.ones(N), np.zeros(N))
    ref = -oracle.spmv(rp, ci, M[0], np.ones(N)) / dt
    inner = interior_mask(X)
    assert np.abs(f[0][inner] - ref[inner]).max() <= 1e-14 * np.abs(ref).max()
    # the density multiplies the flux: rho = 2 doubles it
    _, _, _, f2 = _mat(X, conn, POI, dt, u, np.full(N, 2.0), None)
    assert np.abs(f2[0] - 2 * f[0]).max() <= 1e-14 * np.abs(f[0]).max()


def test_bad_element_is_reported():
    X, conn = hex_mesh(2)
    X = X.copy()
    # fold the first element: swap two of its nodes' positions
    c0 = conn[0]
    X[[c0[0], c0[6]]] = X[[c0[6], c0[0]]]
    N = X.shape[0]
    with pytest.raises(oracle.AssembleError) as ei:
        oracle.assemble(X, conn, MOM, 1.0, np.zeros((3, N)), np.ones(N), np.ones(N))
    assert ei.value.status == oracle.EBADELEM
    assert ei.value.bad_elem == 0
    assert ei.value.min_det <= 0


# --- dense brute force --------------------------------------------------------

@pytest.mark.parametrize("kind", ["hex", "tet"])
@pytest.mark.parametrize("op", [MOM, POI])
def test_csr_equals_dense_sum_of_elemental_matrices(kind, op):
    X, conn = hex_mesh(2, 0.1, seed=3) if kind == "hex" else tet_mesh(2, 0.1, seed=3)
    N, nen = X.shape[0], conn.shape[1]
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.2, 1.2, N)
    mu = rng.uniform(1e-5, 2e-5, N)
    u = rng.normal(0, 1, (3, N))
    dt = 0.1
    rp, ci, V, b = oracle.assemble(X, conn, op, dt, u, rho, mu)
    Ad = np.zeros((N, N))
    bd = np.zeros((b.shape[0], N))
    pattern = np.zeros((N, N), bool)
    for e in range(conn.shape[0]):
        c = conn[e]
        Ae, be = single(nen, X[c], op=op, dt=dt, u=u[:, c], rho=rho[c], mu=mu[c])
        Ad[np.ix_(c, c)] += Ae[0]
        bd[:, c] += be
        pattern[np.ix_(c, c)] = True
    got = dense(rp, ci, V[0], N)
    assert np.linalg.norm(got - Ad) <= 1e-14 * np.linalg.norm(Ad)
    assert np.linalg.norm(b - bd) <= 1e-14 * np.linalg.norm(bd)
    # pattern: exactly the node pairs that share an element, columns sorted
    P = np.zeros((N, N), bool)
    for i in range(N):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        P[i, cols] = True
    assert np.array_equal(P, pattern)


def test_pattern_sizes_match_closed_forms():
    for n in (1, 2, 3, 5):
        X, conn = hex_mesh(n)
        rp, ci = oracle.pattern(conn, X.shape[0])
        assert rp[-1] == meshgen.hex_pattern_nnz(n)
        X, conn = tet_mesh(n)
        rp, ci = oracle.pattern(conn, X.shape[0])
        assert rp[-1] == meshgen.kuhn_pattern_nnz(n)


# --- Dirichlet elimination and PCG --------------------------------------------

def poisson_system(case):
    N = case.n_nodes
    rp, ci, L, f = oracle.assemble(case.coords, case.conn, POI, case.dt, case.u, case.rho, None)
    return rp, ci, L[0].copy(), f[0].copy(), N


def test_dirichlet_elimination_equals_partitioned_solve():
    case = meshgen.make_case(5, meshgen.HEX08, 0.1, case_id=7)
    rp, ci, L, f, N = poisson_system(case)
    Ld = dense(rp, ci, L, N)
    rng = np.random.default_rng(3)
    g = rng.normal(0, 1, N)
    D = case.dirichlet
    F = np.setdiff1d(np.arange(N), D)
    # reference: L_FF x_F = f_F - L_FD g_D, x_D = g_D
    xr = np.zeros(N)
    xr[D] = g[D]
    xr[F] = np.linalg.solve(Ld[np.ix_(F, F)], f[F] - Ld[np.ix_(F, D)] @ g[D])
    L2, f2 = L.copy(), f.copy()
    oracle.dirichlet(rp, ci, L2, f2, D, g)
    L2d = dense(rp, ci, L2, N)
    assert np.abs(L2d - L2d.T).max() <= 1e-15 * np.abs(L2d).max()
    assert np.linalg.eigvalsh(L2d).min() > 0
    x = np.linalg.solve(L2d, f2)
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)
    # Dirichlet rows keep their diagonal
    for i in D[:10]:
        p = rp[i] + np.searchsorted(ci[rp[i]:rp[i + 1]], i)
        assert L2[p] == L[p]


def test_pcg_matches_direct_solve_cfg0():
    case = meshgen.cfg0()
    rp, ci, L, f, N = poisson_system(case)
    oracle.dirichlet(rp, ci, L, f, case.dirichlet)
    x, st, it, rr, tr = oracle.pcg(rp, ci, L, f, rtol=1e-12)
    assert st == oracle.OK
    xd = np.linalg.solve(dense(rp, ci, L, N), f)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert tr <= 2e-12 and rr <= 1e-12


def test_pcg_iteration_count_matches_independent_cg():
    case = meshgen.cfg0()
    rp, ci, L, f, N = poisson_system(case)
    oracle.dirichlet(rp, ci, L, f, case.dirichlet)
    A = sp.csr_matrix((L, ci, rp), shape=(N, N))
    dinv = 1.0 / A.diagonal()
    count = [0]

    def cb(_):
        count[0] += 1
    xs, info = spla.cg(A, f, rtol=1e-10, atol=0.0, M=sp.diags(dinv), callback=cb, maxiter=1000)
    assert info == 0
    x, st, it, rr, tr = oracle.pcg(rp, ci, L, f, rtol=1e-10)
    assert st == oracle.OK
    assert abs(it - count[0]) <= 1
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_pcg_fixed_iterations_and_breakdown():
    case = meshgen.make_case(4, meshgen.HEX08, 0.1, case_id=8)
    rp, ci, L, f, N = poisson_system(case)
    oracle.dirichlet(rp, ci, L, f, case.dirichlet)
    x, st, it, rr, tr = oracle.pcg(rp, ci, L, f, rtol=0.0, max_iter=7)
    assert st == oracle.OK and it == 7
    x, st, it, rr, tr = oracle.pcg(rp, ci, L, f, rtol=1e-14, max_iter=3)
    assert st == oracle.ENOCONV and it == 3
    x, st, it, rr, tr = oracle.pcg(rp, ci, -L, f, rtol=1e-8)
    assert st == oracle.EBREAKDOWN


def test_poisson_patch_linear_pressure_reproduced():
    # linear p as Dirichlet data, zero flux: the discrete solution is p exactly
    case = meshgen.make_case(5, meshgen.HEX08, 0.15, case_id=9)
    N = case.n_nodes
    X = case.coords
    p = 0.3 + 1.1 * X[:, 0] - 0.7 * X[:, 1] + 0.4 * X[:, 2]
    rp, ci, L, f = oracle.assemble(X, case.conn, POI, 1.0, np.zeros((3, N)), np.ones(N), None)
    L, f = L[0], f[0]
    oracle.dirichlet(rp, ci, L, f, case.dirichlet, p)
    x, st, it, rr, tr = oracle.pcg(rp, ci, L, f, rtol=1e-13)
    assert st == oracle.OK
    assert np.abs(x - p).max() <= 1e-11


@pytest.mark.parametrize("jitter", [0.0, 0.1])
def test_poisson_manufactured_solution_second_order(jitter):
    errs = []
    for n in (8, 16, 32):
        rs = meshgen.streams(97, n)
        X = meshgen.cube_nodes(n, jitter, rs["jitter"])
        conn = meshgen.hex_conn(n)
        N = X.shape[0]
        pi = math.pi
        s = np.sin(pi * X)
        c = np.cos(pi * X)
        p = s[:, 0] * s[:, 1] * s[:, 2]
        grad = pi * np.stack([c[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * c[:, 1] * s[:, 2], s[:, 0] * s[:, 1] * c[:, 2]])
        # f_a = int grad N_a . grad p  (dt = 1, rho = 1, u = grad p)
        rp, ci, L, f = oracle.assemble(X, conn, POI, 1.0, grad, np.ones(N), None)
        L, f = L[0], f[0]
        oracle.dirichlet(rp, ci, L, f, meshgen.boundary_nodes(n))
        x, st, *_ = oracle.pcg(rp, ci, L, f, rtol=1e-12)
        assert st == oracle.OK
        errs.append(np.sqrt(np.mean((x - p) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.25), rates
