"""CPU tests of the C ABI: exported symbols, host preprocessing, error paths.

No GPU is needed: fe_plan_* runs the same preprocessing fe_mesh_upload runs,
kept on the host.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import meshgen
import oracle
import paper_2107_11541_amd as fe
from paper_2107_11541_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "feasm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = capi.load()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(capi.SIGNATURES), set(syms) ^ set(capi.SIGNATURES)


def test_pack_layout_paper_example():
    # Section 4.3: 25 TRI03 and 18 QUAD04 in packs of VECTOR_SIZE = 4
    assert fe.pack_layout(25, 4) == (7, 3)
    assert fe.pack_layout(18, 4) == (5, 2)
    assert fe.pack_layout(0, 4) == (0, 0)
    assert fe.pack_layout(64, 64) == (1, 0)
    with pytest.raises(fe.FeError):
        fe.pack_layout(5, 0)


def to_user_pattern(rp, ci, perm):
    """Mesh-numbered CSR -> (row, col) pairs in user numbering, sorted."""
    rows = np.repeat(perm, np.diff(rp))
    cols = perm[ci]
    order = np.lexsort((cols, rows))
    return rows[order], cols[order], order


@pytest.mark.parametrize("kind,renumber", [("hex", True), ("hex", False), ("tet", True)])
def test_plan_pattern_matches_oracle(kind, renumber):
    case = meshgen.make_case(5, meshgen.HEX08 if kind == "hex" else meshgen.TET04, 0.1, case_id=11,
                             shuffle=True)
    P = fe.Plan(case.nen, case.coords, case.conn, renumber=renumber)
    ex = P.export()
    perm = ex["node_perm"]
    assert np.array_equal(np.sort(perm), np.arange(case.n_nodes))
    assert np.array_equal(np.sort(ex["elem_perm"]), np.arange(case.n_elems))
    if not renumber:
        assert np.array_equal(perm, np.arange(case.n_nodes))
    rp, ci = oracle.pattern(case.conn, case.n_nodes)
    r, c, _ = to_user_pattern(ex["rowptr"], ex["colidx"], perm)
    orow = np.repeat(np.arange(case.n_nodes), np.diff(rp))
    assert np.array_equal(r, orow) and np.array_equal(c, ci)
    # columns ascending within each mesh row
    for i in range(0, case.n_nodes, 7):
        row = ex["colidx"][ex["rowptr"][i]:ex["rowptr"][i + 1]]
        assert np.all(np.diff(row) > 0)


@pytest.mark.parametrize("kind", ["hex", "tet"])
def test_plan_blocks_and_colouring_are_valid(kind):
    case = meshgen.make_case(9, meshgen.HEX08 if kind == "hex" else meshgen.TET04, 0.1, case_id=12,
                             shuffle=True)
    P = fe.Plan(case.nen, case.coords, case.conn, renumber=True)
    ex = P.export()
    d = P.desc
    bep, bnp, bn, col = ex["block_elem_ptr"], ex["block_node_ptr"], ex["block_nodes"], ex["block_color"]
    assert bep[0] == 0 and bep[-1] == case.n_elems
    sizes = np.diff(bep)
    assert sizes.min() >= 1 and sizes.max() <= 64
    # mesh-numbered connectivity of the mesh element order
    iperm = np.empty(case.n_nodes, np.int64)
    iperm[ex["node_perm"]] = np.arange(case.n_nodes)
    mconn = iperm[case.conn[ex["elem_perm"]]]
    for b in range(d["n_blocks"]):
        touched = np.unique(mconn[bep[b]:bep[b + 1]])
        assert np.array_equal(touched, bn[bnp[b]:bnp[b + 1]])
    # no two blocks of one colour share a node
    for c in range(d["n_colors"]):
        blocks = np.flatnonzero(col == c)
        nodes = np.concatenate([bn[bnp[b]:bnp[b + 1]] for b in blocks])
        assert np.unique(nodes).size == nodes.size, f"colour {c} has a shared node"
    assert d["max_block_nodes"] == np.diff(bnp).max()
    if kind == "hex":
        assert d["max_phases"] == 1        # structured hexes never share a node at one local position
    assert d["n_colors"] <= 32


def test_renumbering_makes_blocks_compact():
    case = meshgen.make_case(16, meshgen.HEX08, 0.15, case_id=13, shuffle=True)
    with_r = fe.Plan(8, case.coords, case.conn, renumber=True)
    without = fe.Plan(8, case.coords, case.conn, renumber=False)
    # touched rows per element: a Morton block of 64 cells touches 125 nodes
    # (~2 per element); shuffled blocks hit the LDS budget long before 64
    def rows_per_elem(p):
        ex = p.export()
        return ex["block_node_ptr"][-1] / case.n_elems, p.desc["n_blocks"]
    r_r, nb_r = rows_per_elem(with_r)
    r_n, nb_n = rows_per_elem(without)
    assert r_r < 2.0 and r_n > 4.0
    assert nb_r == case.n_elems // 64 and nb_n > 3 * nb_r


def test_plan_rejects_bad_meshes():
    X, conn = meshgen.cube_nodes(2), meshgen.hex_conn(2)
    bad = conn.copy()
    bad[3, 2] = X.shape[0] + 5
    with pytest.raises(fe.FeError) as ei:
        fe.Plan(8, X, bad)
    assert ei.value.status == capi.FE_EBADMESH
    X2 = np.vstack([X, [[2.0, 2.0, 2.0]]])       # a node that belongs to no element
    with pytest.raises(fe.FeError) as ei:
        fe.Plan(8, X2, conn)
    assert ei.value.status == capi.FE_EBADMESH
    with pytest.raises(fe.FeError) as ei:
        fe.Plan(7, X, conn[:, :7])          # no element type has 7 nodes
    assert ei.value.status == capi.FE_EINVAL


def test_ctx_create_without_gpu_fails_cleanly():
    lib = capi.load()
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = lib.fe_ctx_create(0, None, C.byref(h))
    assert st == capi.FE_EDEVICE and not h.value
