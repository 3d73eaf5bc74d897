"""Host planner on PEN06, PYR05 and hybrid meshes (no GPU): the CSR pattern
against the oracle's, type grouping, single-type blocks, the colouring and
the (colour, type) launch list."""
import numpy as np
import pytest

import meshgen
import oracle
import paper_2107_11541_amd as fe
from paper_2107_11541_amd import capi

KINDS = {"pen": meshgen.PEN06, "pyr": meshgen.PYR05, "hybrid": meshgen.HYBRID}


def plan_of(case, renumber=True):
    if case.types is None:
        return fe.Plan(case.nen, case.coords, case.conn, renumber=renumber)
    return fe.Plan(fe.HYBRID, case.coords, case.conn, renumber=renumber, types=case.types)


@pytest.mark.parametrize("kind,renumber", [("pen", True), ("pyr", True), ("hybrid", True), ("hybrid", False)])
def test_plan_pattern_matches_oracle(kind, renumber):
    case = meshgen.make_case(6, KINDS[kind], 0.1, case_id=21, shuffle=True)
    ex = plan_of(case, renumber).export()
    perm = ex["node_perm"]
    assert np.array_equal(np.sort(perm), np.arange(case.n_nodes))
    assert np.array_equal(np.sort(ex["elem_perm"]), np.arange(case.n_elems))
    rp, ci = oracle.pattern(case.conn, case.n_nodes, case.types)
    rows = np.repeat(perm, np.diff(ex["rowptr"]))
    cols = perm[ex["colidx"]]
    order = np.lexsort((cols, rows))
    orow = np.repeat(np.arange(case.n_nodes), np.diff(rp))
    assert np.array_equal(rows[order], orow) and np.array_equal(cols[order], ci)
    # per-element types follow the element permutation
    want = np.full(case.n_elems, case.nen, np.uint8) if case.types is None else case.types[ex["elem_perm"]]
    assert np.array_equal(ex["elem_types"], want)


@pytest.mark.parametrize("kind,renumber", [("pen", True), ("pyr", True), ("hybrid", True), ("hybrid", False)])
def test_blocks_colours_and_launches(kind, renumber):
    case = meshgen.make_case(9, KINDS[kind], 0.1, case_id=22, shuffle=True)
    P = plan_of(case, renumber)
    ex = P.export()
    d = P.desc
    nb = d["n_blocks"]
    bep, bnp, bn, col = ex["block_elem_ptr"], ex["block_node_ptr"], ex["block_nodes"], ex["block_color"]
    et, bt = ex["elem_types"], ex["block_types"]
    assert bep[0] == 0 and bep[-1] == case.n_elems
    assert np.diff(bep).min() >= 1 and np.diff(bep).max() <= 64
    # renumbering groups the types: HEX08, PEN06, PYR05, TET04 (without it the
    # user order is kept and blocks close at every type change)
    rank = {8: 0, 6: 1, 5: 2, 4: 3}
    ranks = np.array([rank[t] for t in et])
    if renumber:
        assert np.all(np.diff(ranks) >= 0)
    else:
        assert np.array_equal(ex["elem_perm"], np.arange(case.n_elems))
    iperm = np.empty(case.n_nodes, np.int64)
    iperm[ex["node_perm"]] = np.arange(case.n_nodes)
    mconn = case.conn[ex["elem_perm"]]
    for b in range(nb):
        es = np.arange(bep[b], bep[b + 1])
        assert np.all(et[es] == bt[b]), "a block mixes element types"
        t = int(bt[b])
        touched = np.unique(iperm[mconn[es, :t]])
        assert np.array_equal(touched, bn[bnp[b]:bnp[b + 1]])
    for c in range(d["n_colors"]):
        nodes = np.concatenate([bn[bnp[b]:bnp[b + 1]] for b in np.flatnonzero(col == c)])
        assert np.unique(nodes).size == nodes.size
    # launches: consecutive, cover the colour-ordered block list once, one
    # colour and one type each, colour-major
    L, cb = ex["launches"], ex["color_blocks"]
    assert np.array_equal(np.sort(cb), np.arange(nb))
    assert L[0, 1] == 0 and np.all(L[1:, 1] == L[:-1, 1] + L[:-1, 2]) and L[-1, 1] + L[-1, 2] == nb
    prev = (-1, -1)
    for nen, first, count in L:
        blocks = cb[first:first + count]
        assert count >= 1 and np.all(bt[blocks] == nen)
        c = np.unique(col[blocks])
        assert c.size == 1
        key = (int(c[0]), rank[int(nen)])
        assert key > prev
        prev = key
    if kind == "hybrid":
        assert set(np.unique(L[:, 0])) == {4, 5, 6, 8}


def test_single_type_layouts_are_unchanged():
    # a one-type mesh given through the mixed entry point plans like the plain one
    case = meshgen.make_case(5, meshgen.TET04, 0.1, case_id=23, shuffle=True)
    pad = np.full((case.n_elems, 8), -1, np.int32)
    pad[:, :4] = case.conn
    a = fe.Plan(fe.TET04, case.coords, case.conn).export()
    b = fe.Plan(fe.HYBRID, case.coords, pad, types=np.full(case.n_elems, 4, np.uint8)).export()
    for k in ("node_perm", "elem_perm", "rowptr", "colidx", "block_elem_ptr", "block_color", "launches"):
        assert np.array_equal(a[k], b[k]), k


def test_mixed_plan_rejects_bad_types():
    case = meshgen.make_case(4, meshgen.HYBRID, 0.1, case_id=24)
    bad = case.types.copy()
    bad[3] = 7
    with pytest.raises(fe.FeError) as ei:
        fe.Plan(fe.HYBRID, case.coords, case.conn, types=bad)
    assert ei.value.status == capi.FE_EINVAL
    conn = case.conn.copy()
    e = int(np.flatnonzero(case.types == 5)[0])
    conn[e, 4] = case.n_nodes + 3
    with pytest.raises(fe.FeError) as ei:
        fe.Plan(fe.HYBRID, case.coords, conn, types=case.types)
    assert ei.value.status == capi.FE_EBADMESH
    # the slots past an element's node count are ignored
    conn = case.conn.copy()
    conn[case.types == 4, 4:] = 10 ** 6
    fe.Plan(fe.HYBRID, case.coords, conn, types=case.types)
