"""Pins of the oracle's boundary assembly (Algorithm 1: the wall model), an
equilibrium law of the wall (Reichardt, kappa = 0.41) imposed as a traction
on wall faces, against facts fixed by the mathematics:

- the Newton solve returns a friction velocity that satisfies the law;
- the law's limits: viscous sublayer u+ = y+ (tau_w -> mu U / delta) and
  the logarithmic layer u+ = ln(y+)/kappa + ln(kappa)/kappa + 7.8;
- on a flat wall with uniform tangential flow the traction sums to
  -rho u_tau^2 A u/|u|, ignores the normal velocity, and splits over the
  nodes with the face rule's weights int N_a dS (h^2 {1, 1/2, 1/4} on a
  uniform quadrilateral grid);
- triangle and quadrilateral faces integrate the same wall alike.
"""
import math

import numpy as np
import pytest

import meshgen
import oracle

KAPPA = 0.41


def test_newton_solves_the_law():
    for U in (1e-4, 0.03, 1.0, 40.0):
        for nu in (1e-6, 1.5e-5, 1e-3):
            for delta in (1e-3, 0.02):
                ut = oracle.wall_utau(U, nu, delta)
                yp = delta * ut / nu
                up = math.log(1 + KAPPA * yp) / KAPPA + 7.8 * (1 - math.exp(-yp / 11) - yp / 11 * math.exp(-yp / 3))
                assert abs(ut * up - U) <= 1e-12 * U, (U, nu, delta)
    assert oracle.wall_utau(0.0, 1e-5, 0.01) == 0.0


def test_law_limits():
    # viscous sublayer: y+ << 1, u_tau^2 = nu U / delta
    nu, delta = 1e-3, 1e-3
    U = 1e-8
    ut = oracle.wall_utau(U, nu, delta)
    assert delta * ut / nu < 2e-4
    assert abs(ut * ut / (nu * U / delta) - 1.0) < 1e-6
    # logarithmic layer: y+ ~ 1e5
    nu, delta, U = 1e-6, 0.05, 30.0
    ut = oracle.wall_utau(U, nu, delta)
    yp = delta * ut / nu
    assert yp > 1e4
    loglaw = math.log(yp) / KAPPA + math.log(KAPPA) / KAPPA + 7.8
    assert abs(U / ut - loglaw) < 1e-3 * loglaw


@pytest.mark.parametrize("kind", [meshgen.HEX08, meshgen.TET04, meshgen.HYBRID])
def test_flat_wall_total_traction(kind):
    c = meshgen.make_case(4, kind, 0.15, case_id=150, shuffle=True, walls=True)
    N = c.n_nodes
    rho, mu = np.full(N, 1.2), np.full(N, 1.8e-5)
    U = np.array([0.6, -0.8, 0.0])                      # tangential to z = 0, |U| = 1
    u = np.repeat(U[:, None], N, axis=1)
    delta = 0.01
    t = oracle.wall_traction(c.coords, c.wall_nen, c.wall_conn, u, rho, mu, delta)
    ut = oracle.wall_utau(1.0, 1.8e-5 / 1.2, delta)
    ref = -1.2 * ut * ut * 1.0 * U                       # wall area 1
    assert np.abs(t.sum(axis=1) - ref).max() <= 1e-13
    # only wall nodes receive traction, antiparallel to u
    wall = np.unique(c.wall_conn[c.wall_conn >= 0])
    off = np.setdiff1d(np.arange(N), wall)
    assert np.abs(t[:, off]).max() == 0.0
    assert np.all(U @ t[:, wall] < 0)
    # the normal velocity does not change it
    u2 = u.copy()
    u2[2] = 0.7
    t2 = oracle.wall_traction(c.coords, c.wall_nen, c.wall_conn, u2, rho, mu, delta)
    assert np.abs(t2 - t).max() <= 1e-15 * np.abs(t).max()


def test_nodal_weights_on_uniform_quads():
    n = 4
    c = meshgen.make_case(n, meshgen.HEX08, 0.0, case_id=151, walls=True)
    N = c.n_nodes
    u = np.zeros((3, N))
    u[0] = 1.0
    rho, mu = np.ones(N), np.full(N, 1e-3)
    delta = 0.02
    t = oracle.wall_traction(c.coords, c.wall_nen, c.wall_conn, u, rho, mu, delta)
    tau = oracle.wall_utau(1.0, 1e-3, delta) ** 2
    h = 1.0 / n
    X = c.coords
    wall = np.flatnonzero(np.abs(X[:, 2]) < 1e-12)
    for a in wall:
        edges = int(np.isclose(X[a, 0], 0) or np.isclose(X[a, 0], 1)) + int(np.isclose(X[a, 1], 0) or np.isclose(X[a, 1], 1))
        weight = h * h / (2 ** edges)
        assert abs(t[0, a] + tau * weight) <= 1e-15


def test_triangles_and_quadrilaterals_agree_on_a_linear_field():
    # the same wall as 16 quads or 32 triangles: for a velocity field that is
    # linear on the wall the two integrate N_a t exactly only if t were linear;
    # with uniform U they must agree exactly per node sum over the whole wall
    n = 4
    q = meshgen.make_case(n, meshgen.HEX08, 0.1, case_id=152, walls=True)
    t = meshgen.make_case(n, meshgen.TET04, 0.1, case_id=152, walls=True)
    assert np.array_equal(q.coords, t.coords)
    N = q.n_nodes
    u = np.zeros((3, N))
    u[1] = 2.0
    args = (np.ones(N), np.full(N, 1e-4), 0.05)
    tq = oracle.wall_traction(q.coords, q.wall_nen, q.wall_conn, u, *args)
    tt = oracle.wall_traction(t.coords, t.wall_nen, t.wall_conn, u, *args)
    assert abs(tq.sum() - tt.sum()) <= 1e-14 * abs(tq.sum())
    with pytest.raises(ValueError):
        oracle.wall_traction(q.coords, q.wall_nen, q.wall_conn, u, *args[:2], 0.0)
