"""CPU tests of the all-core timing build of the oracle (oracle/omp.py)
against the serial oracle: it must compute the same sums in another order.

 - the colouring is valid (no two elements of a colour share a node) and
   covers every element once;
 - assembly agrees with the serial oracle to FP64 rounding (the colour
   order changes only the order of each row's additions);
 - the Dirichlet elimination is bitwise the serial one (rows independent);
 - the PCG follows the serial recurrence: same iteration count, same
   iterate to rounding after a fixed number of iterations.
"""
import numpy as np
import pytest

import meshgen
import oracle
from oracle import omp

CASES = {
    "hex": lambda: meshgen.make_case(7, meshgen.HEX08, 0.12, case_id=91, shuffle=True),
    "tet": lambda: meshgen.make_case(5, meshgen.TET04, 0.10, case_id=92, shuffle=True, n_scalars=2),
    "hybrid": lambda: meshgen.make_case(6, meshgen.HYBRID, 0.10, case_id=93, shuffle=True, temperature=True),
}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kind", sorted(CASES))
def test_colouring_is_valid(kind):
    c = CASES[kind]()
    nc, order, ptr = omp.colour(c.conn, c.n_nodes, c.types)
    assert ptr[0] == 0 and ptr[-1] == c.n_elems
    assert np.array_equal(np.sort(order), np.arange(c.n_elems))
    types = c.types if c.types is not None else np.full(c.n_elems, c.conn.shape[1], np.uint8)
    for k in range(nc):
        els = order[ptr[k]:ptr[k + 1]]
        nodes = np.concatenate([c.conn[e, :types[e]] for e in els])
        assert np.unique(nodes).size == nodes.size, f"colour {k} shares a node"


@pytest.mark.parametrize("kind", sorted(CASES))
def test_assembly_matches_serial_oracle(kind):
    c = CASES[kind]()
    ops = [oracle.OP_MOMENTUM, oracle.OP_POISSON] + ([oracle.OP_SCALAR] if c.Y.shape[0] else [])
    for op in ops:
        kw = {"Y": c.Y, "D": c.D} if op == oracle.OP_SCALAR else {}
        _, _, V, B = oracle.assemble(c.coords, c.conn, op, c.dt, c.u, c.rho, c.mu, types=c.types, **kw)
        _, _, Vo, Bo = omp.assemble(c.coords, c.conn, op, c.dt, c.u, c.rho, c.mu, types=c.types, **kw)
        assert rel(Vo, V) <= 1e-14 and rel(Bo, B) <= 1e-14, (op, rel(Vo, V), rel(Bo, B))


def test_bad_element_reported():
    c = meshgen.make_case(3, meshgen.HEX08, 0.0, case_id=94)
    X = c.coords.copy()
    e = c.conn[5]
    X[[e[0], e[6]]] = X[[e[6], e[0]]]
    with pytest.raises(oracle.AssembleError) as a:
        oracle.assemble(X, c.conn, oracle.OP_POISSON, c.dt, c.u, c.rho, None)
    with pytest.raises(oracle.AssembleError) as b:
        omp.assemble(X, c.conn, oracle.OP_POISSON, c.dt, c.u, c.rho, None)
    assert a.value.bad_elem == b.value.bad_elem


def test_dirichlet_and_pcg_follow_the_serial_oracle():
    c = CASES["hex"]()
    rp, ci, L, f = oracle.assemble(c.coords, c.conn, oracle.OP_POISSON, c.dt, c.u, c.rho, None)
    L1, f1 = L[0].copy(), f[0].copy()
    L2, f2 = L[0].copy(), f[0].copy()
    oracle.dirichlet(rp, ci, L1, f1, c.dirichlet)
    omp.dirichlet(rp, ci, L2, f2, c.dirichlet)
    assert np.array_equal(L1, L2) and np.array_equal(f1, f2)
    xs, ss, its, rrs, trs = oracle.pcg(rp, ci, L1, f1, rtol=1e-10)
    xo, so, ito, rro, tro = omp.pcg(rp, ci, L1, f1, rtol=1e-10)
    assert ss == so == oracle.OK and abs(its - ito) <= 1
    assert rel(xo, xs) <= 1e-9 and tro <= 2e-10
    xs, *_ = oracle.pcg(rp, ci, L1, f1, rtol=0.0, max_iter=15)
    xo, so, ito, *_ = omp.pcg(rp, ci, L1, f1, rtol=0.0, max_iter=15)
    assert so == oracle.OK and ito == 15
    assert rel(xo, xs) <= 1e-12
