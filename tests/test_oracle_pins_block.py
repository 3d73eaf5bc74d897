"""Pins of the oracle's 3x3-block momentum operator (or_assemble_block):
Eq. (1)'s viscous term in its full-stress form -div(2 mu eps(u)), which
couples the velocity components, and EMAC's (div u) u term, linearised
about the nodal velocity.  Facts the mathematics fixes:

 - form 0 is the scalar momentum operator times the 3x3 identity;
 - rigid motions (translations and rotations, eps = 0) lie in the kernel of
   the full-stress viscous part on every row, boundary rows included, while
   the Laplacian form leaves rotations a residue at the boundary;
 - the viscous part is block symmetric: A[(a,i),(b,k)] = A[(b,k),(a,i)];
 - with u constant per component, the rows of the full operator sum to the
   lumped mass / dt on the diagonal block (C.1 = 0, viscous part exact);
 - interior rows reproduce a linear field (patch test);
 - b - A u is the matrix-free residual of the explicit step (a separate
   oracle routine) for every form, on hex, tet and hybrid meshes.

A transposed coupling term (d N_a/d x_i d N_b/d x_k instead of
d N_a/d x_k d N_b/d x_i) breaks the residual identity; a dropped term or a
wrong sign breaks the residual identity or the kernel pins.
"""
import numpy as np
import pytest

import meshgen
import oracle

KINDS = {"hex": meshgen.HEX08, "tet": meshgen.TET04, "hybrid": meshgen.HYBRID}


def case_of(kind, n, seed):
    c = meshgen.make_case(n, KINDS[kind], 0.12, case_id=150 + seed, shuffle=True, temperature=(seed % 2 == 1))
    c.mu = np.random.default_rng(seed).uniform(1e-3, 3e-3, c.n_nodes)
    return c


def block_spmv(rp, ci, V, x):
    """y[i, a] = sum over row a's entries p and k of V[p, i, k] x[k, col_p]."""
    rows = np.repeat(np.arange(rp.shape[0] - 1), np.diff(rp))
    contrib = np.einsum("pik,kp->ip", V, x[:, ci])
    y = np.zeros_like(x)
    for i in range(3):
        np.add.at(y[i], rows, contrib[i])
    return y


def row_scale(rp, V):
    """Largest |entry| of each block row (a, i): [3, N]."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    s = np.zeros((3, n))
    for i in range(3):
        np.maximum.at(s[i], rows, np.abs(V[:, i, :]).max(axis=1))
    return s


@pytest.mark.parametrize("kind,n", [("hex", 4), ("tet", 3), ("hybrid", 4)])
def test_form0_is_scalar_operator_times_identity(kind, n):
    c = case_of(kind, n, 1)
    rp, ci, V, B = oracle.assemble_block(c.coords, c.conn, 0, c.dt, c.u, c.rho, c.mu, types=c.types)
    _, _, S, Bs = oracle.assemble(c.coords, c.conn, oracle.OP_MOMENTUM, c.dt, c.u, c.rho, c.mu, types=c.types)
    scale = np.abs(S[0]).max()
    for i in range(3):
        for k in range(3):
            ref = S[0] if i == k else 0.0
            assert np.abs(V[:, i, k] - ref).max() <= 1e-14 * scale, (i, k)
    assert np.array_equal(B, Bs)


@pytest.mark.parametrize("kind,n", [("hex", 4), ("tet", 3), ("hybrid", 4)])
def test_rigid_motions_in_kernel_of_full_stress(kind, n):
    c = case_of(kind, n, 2)
    zero = np.zeros(c.n_nodes)
    # rho = 0 leaves the viscous part alone
    rp, ci, V, _ = oracle.assemble_block(c.coords, c.conn, oracle.FULL_STRESS, c.dt, c.u, zero, c.mu, types=c.types)
    rng = np.random.default_rng(3)
    t, w = rng.normal(size=3), rng.normal(size=3)
    X = c.coords.T                                       # [3, N]
    rigid = t[:, None] + np.cross(w, X.T).T              # t + w x x
    scale = row_scale(rp, V) * np.abs(rigid).max()
    y = block_spmv(rp, ci, V, rigid)
    assert np.all(np.abs(y) <= 1e-12 * scale)
    # the Laplacian form alone does not annihilate a rotation on the boundary
    rp, ci, V0, _ = oracle.assemble_block(c.coords, c.conn, 0, c.dt, c.u, zero, c.mu, types=c.types)
    rot = np.cross(w, X.T).T
    y0 = block_spmv(rp, ci, V0, rot)
    assert np.abs(y0).max() > 1e-6 * (row_scale(rp, V0) * np.abs(rot).max()).max()


@pytest.mark.parametrize("kind,n", [("hex", 4), ("tet", 3), ("hybrid", 4)])
def test_viscous_part_is_block_symmetric(kind, n):
    c = case_of(kind, n, 4)
    zero = np.zeros(c.n_nodes)
    rp, ci, V, _ = oracle.assemble_block(c.coords, c.conn, oracle.FULL_STRESS, c.dt, c.u, zero, c.mu, types=c.types)
    N = c.n_nodes
    rows = np.repeat(np.arange(N), np.diff(rp))
    dense = np.zeros((N, 3, N, 3))
    for i in range(3):
        for k in range(3):
            dense[rows, i, ci, k] = V[:, i, k]
    d2 = dense.reshape(3 * N, 3 * N)
    assert np.abs(d2 - d2.T).max() <= 1e-15 * np.abs(d2).max()
    # and the coupling is really there (off-diagonal blocks of one entry)
    assert np.abs(V[:, 0, 1]).max() > 0.02 * np.abs(V[:, 0, 0]).max()


@pytest.mark.parametrize("kind,n", [("hex", 4), ("tet", 3), ("hybrid", 4)])
def test_row_sums_are_lumped_mass_over_dt(kind, n):
    c = case_of(kind, n, 5)
    rp, ci, V, _ = oracle.assemble_block(c.coords, c.conn, oracle.FULL_STRESS, c.dt, c.u, c.rho, c.mu,
                                         types=c.types)
    _, mass = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types)
    for k in range(3):
        e = np.zeros((3, c.n_nodes))
        e[k] = 1.0
        y = block_spmv(rp, ci, V, e)
        for i in range(3):
            ref = mass / c.dt if i == k else np.zeros(c.n_nodes)
            assert np.abs(y[i] - ref).max() <= 1e-12 * (mass / c.dt).max(), (i, k)


def test_patch_test_linear_field_interior_rows():
    c = case_of("hex", 5, 6)
    zero = np.zeros(c.n_nodes)
    rp, ci, V, _ = oracle.assemble_block(c.coords, c.conn, oracle.FULL_STRESS, c.dt, c.u, zero,
                                         np.full(c.n_nodes, 2e-3), types=c.types)
    G = np.random.default_rng(7).normal(size=(3, 3))
    ulin = G @ c.coords.T
    y = block_spmv(rp, ci, V, ulin)
    interior = np.ones(c.n_nodes, bool)
    interior[c.dirichlet] = False
    scale = (row_scale(rp, V) * np.abs(ulin).max())[:, interior]
    assert np.all(np.abs(y[:, interior]) <= 1e-12 * scale)
    assert np.abs(y[:, ~interior]).max() > 1e-8      # boundary rows carry the traction


@pytest.mark.parametrize("form", [0, 1, 2, 3])
@pytest.mark.parametrize("kind,n", [("hex", 4), ("tet", 3), ("hybrid", 4)])
def test_b_minus_Au_is_the_matrix_free_residual(kind, n, form):
    c = case_of(kind, n, 8 + form)
    rp, ci, V, B = oracle.assemble_block(c.coords, c.conn, form, c.dt, c.u, c.rho, c.mu, types=c.types)
    r, _ = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types, form)
    got = B - block_spmv(rp, ci, V, c.u)
    scale = np.abs(B).max() + np.abs(block_spmv(rp, ci, np.abs(V), np.abs(c.u))).max()
    assert np.abs(got - r).max() <= 1e-13 * scale, np.abs(got - r).max() / scale
    # each variant changes the operator
    if form:
        _, _, V0, _ = oracle.assemble_block(c.coords, c.conn, 0, c.dt, c.u, c.rho, c.mu, types=c.types)
        assert np.abs(V - V0).max() > 1e-6 * np.abs(V0).max()


def test_bad_form_and_bad_element():
    c = case_of("hex", 2, 12)
    with pytest.raises(oracle.AssembleError):
        oracle.assemble_block(c.coords, c.conn, 4, c.dt, c.u, c.rho, c.mu)
    X = c.coords.copy()
    e = c.conn[3]
    X[[e[0], e[6]]] = X[[e[6], e[0]]]
    with pytest.raises(oracle.AssembleError) as ei:
        oracle.assemble_block(X, c.conn, 1, c.dt, c.u, c.rho, c.mu)
    assert ei.value.bad_elem >= 0
