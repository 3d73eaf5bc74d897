"""Pins of the oracle's prism (PEN06) and pyramid (PYR05) elements and of
its mixed-type (hybrid) meshes, against facts fixed by the mathematics.

Reference elements: partition of unity, Kronecker property, reproduction of
linear fields, finite-difference gradients, traces on shared faces (the
pyramid must be linear on its triangles and bilinear on its base to conform
with TET04 and HEX08), and the exactness of each quadrature rule against
closed-form integrals of monomials.  Elemental matrices: closed-form mass of
a right prism and the pyramid's mass against an independent high-order
rule.  Meshes: the operator invariants (volume, row sums, symmetry, patch
tests, rhs identities) on jittered prism, pyramid and hybrid cubes, a dense
brute-force assembly through the padded connectivity, the bad-element
report, and second-order convergence on the hybrid cube.
"""
import math

import numpy as np
import pytest

import meshgen
import oracle

MOM, SCA, POI = oracle.OP_MOMENTUM, oracle.OP_SCALAR, oracle.OP_POISSON

PEN_NODES = np.array([[0, 0, -1], [1, 0, -1], [0, 1, -1], [0, 0, 1], [1, 0, 1], [0, 1, 1]], float)
PYR_NODES = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0], [0, 0, 1]], float)


def random_point(nen, rng):
    if nen == 6:
        l = rng.dirichlet(np.ones(3))
        return np.array([l[1], l[2], rng.uniform(-1, 1)])
    z = rng.uniform(0, 0.95)
    return np.array([rng.uniform(-1, 1) * (1 - z), rng.uniform(-1, 1) * (1 - z), z])


# --- reference elements -------------------------------------------------------

@pytest.mark.parametrize("nen", [6, 5])
def test_partition_of_unity_linear_reproduction(nen):
    nodes = PEN_NODES if nen == 6 else PYR_NODES
    rng = np.random.default_rng(3)
    for _ in range(50):
        xi = random_point(nen, rng)
        N, dN = oracle.shape(nen, xi)
        assert abs(N.sum() - 1.0) < 1e-15
        assert np.abs(dN.sum(axis=0)).max() < 1e-14
        # isoparametric: the reference nodes interpolate the coordinates
        assert np.abs(N @ nodes - xi).max() < 1e-15
        assert np.abs(nodes.T @ dN - np.eye(3)).max() < 1e-14


@pytest.mark.parametrize("nen", [6, 5])
def test_kronecker(nen):
    nodes = PEN_NODES if nen == 6 else PYR_NODES
    for b in range(nen):
        xi = nodes[b].copy()
        if nen == 5 and b == 4:
            xi[2] = 1.0 - 1e-12     # the rational basis is 0/0 at the apex itself
        N, _ = oracle.shape(nen, xi)
        assert np.abs(N - np.eye(nen)[b]).max() < 1e-11


@pytest.mark.parametrize("nen", [6, 5])
def test_gradient_matches_finite_difference(nen):
    rng = np.random.default_rng(4)
    for _ in range(10):
        xi = random_point(nen, rng)
        _, dN = oracle.shape(nen, xi)
        for j in range(3):
            e = np.zeros(3)
            e[j] = 1e-6
            Np, _ = oracle.shape(nen, xi + e)
            Nm, _ = oracle.shape(nen, xi - e)
            assert np.abs((Np - Nm) / 2e-6 - dN[:, j]).max() < 1e-8


def test_pyramid_traces_conform_with_tet_and_hex():
    rng = np.random.default_rng(5)
    # triangular face (0, 1, 4): eta = zeta - 1; the basis is the face's
    # barycentric coordinates there and the two other base nodes vanish
    for _ in range(20):
        l = rng.dirichlet(np.ones(3))
        xi = l[0] * PYR_NODES[0] + l[1] * PYR_NODES[1] + l[2] * PYR_NODES[4]
        if xi[2] > 1 - 1e-9:
            continue
        N, _ = oracle.shape(5, xi)
        assert np.abs(N[[0, 1, 4]] - l).max() < 1e-14
        assert np.abs(N[[2, 3]]).max() < 1e-14
    # base zeta = 0: the bilinear quadrilateral functions
    for _ in range(20):
        s, t = rng.uniform(-1, 1, 2)
        N, _ = oracle.shape(5, np.array([s, t, 0.0]))
        q = 0.25 * (1 + PYR_NODES[:4, 0] * s) * (1 + PYR_NODES[:4, 1] * t)
        assert np.abs(N[:4] - q).max() < 1e-15 and abs(N[4]) < 1e-16


def test_weights_sum_to_reference_volume():
    assert abs(oracle.gauss(6)[1].sum() - 1.0) < 1e-15
    assert abs(oracle.gauss(5)[1].sum() - 4.0 / 3.0) < 1e-15


def _line(k):
    return 0.0 if k % 2 else 2.0 / (k + 1)


def test_prism_rule_exactness():
    pts, w = oracle.gauss(6)
    f = math.factorial
    for p in range(3):
        for q in range(3 - p):
            for r in range(4):
                exact = f(p) * f(q) / f(p + q + 2) * _line(r)
                got = np.sum(w * pts[:, 0] ** p * pts[:, 1] ** q * pts[:, 2] ** r)
                assert abs(got - exact) < 1e-15, (p, q, r)
    # degree 3 on the triangle is beyond the 3-point rule
    got = np.sum(w * pts[:, 0] ** 3)
    assert abs(got - f(3) / f(5) * 2.0) > 1e-3


def test_pyramid_rule_exactness():
    # int over the pyramid of xi^p eta^q zeta^r, with (xi, eta) = (1-zeta)(s, t):
    # [int s^p][int t^q] * B(r + 1, p + q + 3)
    pts, w = oracle.gauss(5)
    f = math.factorial
    for p in range(4):
        for q in range(4 - p):
            for r in range(4 - p - q):
                beta = f(r) * f(p + q + 2) / f(p + q + r + 3)
                exact = _line(p) * _line(q) * beta
                got = np.sum(w * pts[:, 0] ** p * pts[:, 1] ** q * pts[:, 2] ** r)
                assert abs(got - exact) < 1e-15, (p, q, r)
    got = np.sum(w * pts[:, 2] ** 4)
    assert abs(got - 2.0 * 2.0 * f(4) * f(2) / f(7)) > 1e-4


# --- elemental matrices -------------------------------------------------------

def single(nen, X, op=MOM, dt=1.0, u=None, rho=None, mu=None, **kw):
    conn = np.arange(nen, dtype=np.int32)[None, :]
    rp, ci, v, b = oracle.assemble(X, conn, op, dt, u, rho, mu, **kw)
    return v.reshape(v.shape[0], nen, nen), b


def plain_mass(nen, X):
    A, _ = single(nen, X, u=np.zeros((3, nen)), rho=np.ones(nen), mu=np.zeros(nen))
    return A[0]


def test_right_prism_mass_closed_form():
    tri = np.array([[0.1, 0.2], [1.4, 0.3], [0.5, 1.2]])
    H = 0.7
    X = np.vstack([np.c_[tri, np.zeros(3)], np.c_[tri, np.full(3, H)]])
    e1, e2 = tri[1] - tri[0], tri[2] - tri[0]
    area = 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])
    Mt = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
    Ml = H / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    assert np.abs(plain_mass(6, X) - np.kron(Ml, Mt)).max() < 1e-15


def test_pyramid_mass_against_high_order_rule():
    # reference pyramid mapped by an affine map; a 6-point Gauss-Legendre
    # rule per collapsed coordinate (exact here) integrates N_a N_b |J|
    rng = np.random.default_rng(6)
    Amap = np.eye(3) + 0.2 * rng.normal(size=(3, 3))
    c = rng.normal(size=3)
    X = PYR_NODES @ Amap.T + c
    x6, w6 = np.polynomial.legendre.leggauss(6)
    M = np.zeros((5, 5))
    for i, s in enumerate(x6):
        for j, t in enumerate(x6):
            for k, zz in enumerate(x6):
                z = 0.5 * (zz + 1.0)              # [0, 1]
                m = 1.0 - z
                N, _ = oracle.shape(5, np.array([s * m, t * m, z]))
                wt = w6[i] * w6[j] * w6[k] * 0.5 * m * m * abs(np.linalg.det(Amap))
                M += wt * np.outer(N, N)
    assert np.abs(plain_mass(5, X) - M).max() < 1e-14 * np.abs(M).max()


# --- operator invariants on jittered meshes -------------------------------------

@pytest.fixture(scope="module", params=["pen", "pyr", "hybrid"])
def mesh(request):
    et = {"pen": meshgen.PEN06, "pyr": meshgen.PYR05, "hybrid": meshgen.HYBRID}[request.param]
    c = meshgen.make_case(4, et, 0.15, case_id=96, sub=et, shuffle=True)
    N = c.n_nodes
    rng = np.random.default_rng(8)
    c.rho = rng.uniform(0.2, 1.2, N)
    c.mu = rng.uniform(1e-5, 3e-5, N)
    c.u = rng.normal(0, 1, (3, N))
    return c


def _mat(c, op, dt, u, rho, mu, **kw):
    return oracle.assemble(c.coords, c.conn, op, dt, u, rho, mu, types=c.types, **kw)


def dense(rp, ci, v, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return A


def interior(c):
    m = np.ones(c.n_nodes, bool)
    m[c.dirichlet] = False
    return m


def test_mass_sum_is_domain_volume(mesh):
    N = mesh.n_nodes
    _, _, M, _ = _mat(mesh, MOM, 1.0, np.zeros((3, N)), np.ones(N), np.zeros(N))
    assert abs(M.sum() - 1.0) < 1e-13


def test_viscous_rows_symmetry_and_patch(mesh):
    c = mesh
    N = c.n_nodes
    rp, ci, K, _ = _mat(c, MOM, 1.0, c.u, np.zeros(N), c.mu)
    Kd = dense(rp, ci, K[0], N)
    scale = np.abs(Kd).max(axis=1)
    assert np.all(np.abs(Kd @ np.ones(N)) <= 1e-13 * scale)
    assert np.abs(Kd - Kd.T).max() <= 1e-13 * scale.max()
    _, _, Kc, _ = _mat(c, MOM, 1.0, c.u, np.zeros(N), np.full(N, 2e-5))
    Kcd = dense(rp, ci, Kc[0], N)
    inner = interior(c)
    for j in range(3):
        r = Kcd @ c.coords[:, j]
        assert np.all(np.abs(r[inner]) <= 1e-13 * np.abs(Kcd[inner]).max(axis=1))


def test_convection_reproduces_linear_fields(mesh):
    c = mesh
    N = c.n_nodes
    dt = 0.01
    zero = np.zeros(N)
    rp, ci, A, _ = _mat(c, MOM, dt, c.u, c.rho, zero)
    _, _, A0, _ = _mat(c, MOM, dt, np.zeros((3, N)), c.rho, zero)
    Cd = dense(rp, ci, A[0] - A0[0], N)
    Md = dense(rp, ci, A0[0], N) * dt
    scale = np.abs(dense(rp, ci, A[0], N)).max(axis=1)
    assert np.all(np.abs(Cd @ np.ones(N)) <= 1e-13 * scale)
    for j in range(3):
        assert np.all(np.abs(Cd @ c.coords[:, j] - Md @ c.u[j]) <= 1e-13 * scale)
    assert np.abs(Cd - Cd.T).max() > 1e-3 * np.abs(Cd).max()


def test_rhs_identities(mesh):
    c = mesh
    N = c.n_nodes
    dt = 0.02
    rp, ci, A, b = _mat(c, MOM, dt, c.u, c.rho, c.mu)
    _, _, M, _ = _mat(c, MOM, 1.0, np.zeros((3, N)), c.rho, np.zeros(N))
    for i in range(3):
        ref = oracle.spmv(rp, ci, M[0], c.u[i]) / dt
        assert np.linalg.norm(b[i] - ref) <= 1e-13 * np.linalg.norm(ref)
    Y = np.random.default_rng(9).uniform(0, 1, (2, N))
    D = np.array([1e-6, 5e-5])
    _, _, S, bs = _mat(c, SCA, dt, c.u, c.rho, c.mu, Y=Y, D=D)
    for k in range(2):
        _, _, Ak, _ = _mat(c, MOM, dt, c.u, c.rho, c.rho * D[k])
        assert np.abs(S[k] - Ak[0]).max() <= 1e-13 * np.abs(Ak[0]).max()
        ref = oracle.spmv(rp, ci, M[0], Y[k]) / dt
        assert np.linalg.norm(bs[k] - ref) <= 1e-13 * np.linalg.norm(ref)
    # a constant mass flux has no divergence: the Poisson rhs vanishes inside
    u = np.repeat(np.array([0.3, -1.2, 0.7])[:, None], N, axis=1)
    _, _, _, f = _mat(c, POI, 0.5, u, np.ones(N), None)
    assert np.abs(f[0][interior(c)]).max() <= 1e-13
    assert np.abs(f[0][~interior(c)]).max() > 1e-3


@pytest.mark.parametrize("op", [MOM, POI])
def test_csr_equals_dense_sum_of_elemental_matrices(mesh, op):
    c = mesh
    N = c.n_nodes
    dt = 0.1
    rp, ci, V, b = _mat(c, op, dt, c.u, c.rho, c.mu)
    Ad = np.zeros((N, N))
    bd = np.zeros((b.shape[0], N))
    for e in range(c.n_elems):
        nen = c.nen if c.types is None else int(c.types[e])
        q = c.conn[e, :nen]
        Ae, be = single(nen, c.coords[q], op=op, dt=dt, u=c.u[:, q], rho=c.rho[q], mu=c.mu[q])
        Ad[np.ix_(q, q)] += Ae[0]
        bd[:, q] += be
    assert np.linalg.norm(dense(rp, ci, V[0], N) - Ad) <= 1e-14 * np.linalg.norm(Ad)
    assert np.linalg.norm(b - bd) <= 1e-14 * np.linalg.norm(bd)


def test_hybrid_mesh_holds_every_type_and_padding_is_ignored():
    c = meshgen.make_case(4, meshgen.HYBRID, 0.1, case_id=95)
    assert set(np.unique(c.types)) == {4, 5, 6, 8}
    N = c.n_nodes
    base = oracle.assemble(c.coords, c.conn, POI, 1.0, c.u, c.rho, None, types=c.types)
    conn = c.conn.copy()
    for e in range(c.n_elems):
        conn[e, c.types[e]:] = 0          # any value in the unused slots
    got = oracle.assemble(c.coords, conn, POI, 1.0, c.u, c.rho, None, types=c.types)
    assert np.array_equal(base[1], got[1]) and np.array_equal(base[2], got[2])
    with pytest.raises(ValueError):
        oracle.pattern(c.conn, N, np.full(c.n_elems, 7, np.uint8))


def test_hybrid_bad_element_is_reported():
    c = meshgen.make_case(4, meshgen.HYBRID, 0.0, case_id=95)
    X = c.coords.copy()
    e = int(np.flatnonzero(c.types == 5)[0])
    apex = c.conn[e, 4]
    X[apex] = 2 * X[c.conn[e, 0]] - X[apex]       # push the apex through the base
    N = c.n_nodes
    with pytest.raises(oracle.AssembleError) as ei:
        oracle.assemble(X, c.conn, MOM, 1.0, np.zeros((3, N)), np.ones(N), np.ones(N), types=c.types)
    assert ei.value.status == oracle.EBADELEM
    assert ei.value.min_det <= 0


def test_hybrid_poisson_manufactured_solution_second_order():
    errs = []
    for n in (8, 16, 32):
        c = meshgen.make_case(n, meshgen.HYBRID, 0.1, case_id=94, sub=n)
        X = c.coords
        N = c.n_nodes
        pi = math.pi
        s, co = np.sin(pi * X), np.cos(pi * X)
        p = s[:, 0] * s[:, 1] * s[:, 2]
        grad = pi * np.stack([co[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * co[:, 1] * s[:, 2],
                              s[:, 0] * s[:, 1] * co[:, 2]])
        rp, ci, L, f = oracle.assemble(X, c.conn, POI, 1.0, grad, np.ones(N), None, types=c.types)
        L, f = L[0], f[0]
        oracle.dirichlet(rp, ci, L, f, c.dirichlet)
        x, st, *_ = oracle.pcg(rp, ci, L, f, rtol=1e-12)
        assert st == oracle.OK
        errs.append(np.sqrt(np.mean((x - p) ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.3), rates
