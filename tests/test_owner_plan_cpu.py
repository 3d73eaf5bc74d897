"""CPU tests of the owner plan of the matrix assembly (fe_plan_export_owner):
the invariants the owner kernel relies on, checked on small meshes of each
element type.

* groups cut the rows (mesh numbering) into consecutive ranges, and their
  tasks are consecutive;
* a group lists its own rows first, then its other touched nodes, ascending,
  within the kernel's limits (256 tasks, 1024 nodes);
* a task presents its element's nodes in the element's order or, for HEX08,
  in the order of a proper rotation of the reference cube (det J keeps its
  sign); the contributions (element, owned row) of every group are each
  computed by exactly one task;
* in-row offsets point at the right CSR columns;
* the tasks of one phase hold distinct owned rows (conflict-free, fixed-order
  LDS accumulation): over the group for HEX08, within each wavefront of 64
  tasks for the types that accumulate wave-privately.
"""
import numpy as np
import pytest

import meshgen
import paper_2107_11541_amd as fe

HEX_POS = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                    [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], float)
KINDS = {"hex": meshgen.HEX08, "tet": meshgen.TET04, "pen": meshgen.PEN06, "pyr": meshgen.PYR05}


def mesh_conn(case, ex):
    iperm = np.empty_like(ex["node_perm"])
    iperm[ex["node_perm"]] = np.arange(ex["node_perm"].size)
    return iperm[case.conn[ex["elem_perm"]]]


@pytest.mark.parametrize("kind,n,renumber", [("hex", 7, True), ("hex", 5, False), ("tet", 5, True),
                                             ("pen", 4, True), ("pyr", 3, True)])
def test_owner_plan_invariants(kind, n, renumber):
    case = meshgen.make_case(n, KINDS[kind], 0.12, case_id=210 + n, shuffle=True)
    P = fe.Plan(case.nen, case.coords, case.conn, renumber=renumber)
    ex = P.export()
    ow = P.export_owner()
    nen = case.nen
    ra = ow["rows_per_task"]
    assert ra == (4 if nen == 8 else nen)
    priv = ow["wave_private"]
    assert priv == (nen != 8)
    cm = mesh_conn(case, ex)
    rp, ci = ex["rowptr"], ex["colidx"]
    N = rp.size - 1
    groups = ow["groups"]
    # rows and tasks are cut into consecutive ranges
    assert groups[0, 0] == 0 and groups[0, 2] == 0
    assert np.all(groups[1:, 0] == groups[:-1, 0] + groups[:-1, 1])
    assert np.all(groups[1:, 2] == groups[:-1, 2] + groups[:-1, 3])
    assert groups[-1, 2] + groups[-1, 3] == N
    assert groups[-1, 0] + groups[-1, 1] == ow["task_elem"].size
    assert np.all(groups[:, 1] >= 1) and np.all(groups[:, 1] <= 256) and np.all(groups[:, 3] >= 1)
    # element -> its nodes (mesh numbering), node -> its elements
    elems_of = [[] for _ in range(N)]
    for e in range(cm.shape[0]):
        for a in range(nen):
            elems_of[cm[e, a]].append(e)
    for g, (t0, nt, r0, nr) in enumerate(groups):
        nodes = ow["nodes"][ow["node_ptr"][g]:ow["node_ptr"][g + 1]]
        assert nodes.size <= 1024
        assert np.array_equal(nodes[:nr], np.arange(r0, r0 + nr))
        halo = nodes[nr:]
        assert np.all((halo < r0) | (halo >= r0 + nr)) and np.all(np.diff(halo) > 0)
        covered = {}
        rows_in_phase = {}
        for t in range(t0, t0 + nt):
            e = ow["task_elem"][t]
            ln = ow["task_ln"][t, :nen].astype(np.int64)
            tn = nodes[ln]
            if nen == 8:
                # tn[b] = cm[e][sigma(b)] with sigma a proper rotation of the cube
                sigma = np.array([int(np.nonzero(cm[e] == v)[0][0]) for v in tn])
                assert sorted(sigma) == list(range(8))
                R, *_ = np.linalg.lstsq(HEX_POS, HEX_POS[sigma], rcond=None)
                assert np.allclose(HEX_POS @ R, HEX_POS[sigma])
                assert np.isclose(np.linalg.det(R), 1.0)
            else:
                assert np.array_equal(tn, cm[e])
            ph = (int(ow["task_phase"][t]), (t - t0) // 64 if priv else 0)
            for r in range(ra):
                if ln[r] >= nr:
                    continue
                row = tn[r]
                key = (e, row)
                assert key not in covered, f"contribution {key} computed twice"
                covered[key] = t
                assert row not in rows_in_phase.setdefault(ph, set()), "two tasks of a phase share a row"
                rows_in_phase[ph].add(row)
                cols = ci[rp[row]:rp[row + 1]]
                for b in range(nen):
                    assert cols[ow["task_off"][t, r * nen + b]] == tn[b]
        assert ow["nphase"][g] == max(p for p, _ in rows_in_phase) + 1
        # every (element, owned row) contribution of the group is computed once
        want = {(e, row) for row in range(r0, r0 + nr) for e in elems_of[row]}
        assert set(covered) == want


@pytest.mark.parametrize("nen", [4, 8])
def test_owner_plan_high_valence_node(nen):
    """A node in many elements (the planner does not look at the geometry):
    80 TET04 (a 241-entry row), whose tasks the wave-private accumulation
    spreads over waves, or 36 HEX08 (a 253-entry row, near the 255 limit),
    whose shared accumulation needs 36 phases for the row.  The phase
    invariants hold either way."""
    rng = np.random.default_rng(3)
    nf, tail = (80 if nen == 4 else 36), 200
    k = nen - 1
    N = 1 + k * nf + tail
    conn = [[0] + [1 + k * q + j for j in range(k)] for q in range(nf)]
    extra = list(range(1 + k * nf, N))
    conn += [extra[q:q + nen] for q in range(len(extra) - nen + 1)]
    conn = np.array(conn, np.int32)
    P = fe.Plan(nen, rng.random((N, 3)), conn)
    ow = P.export_owner()
    priv = ow["wave_private"]
    assert priv == (nen != 8)
    assert ow["nphase"].max() >= (36 if not priv else 4)
    ex = P.export()
    iperm = np.empty_like(ex["node_perm"])
    iperm[ex["node_perm"]] = np.arange(N)
    cm = iperm[conn[ex["elem_perm"]]]
    ra = ow["rows_per_task"]
    for g, (t0, nt, r0, nr) in enumerate(ow["groups"]):
        nodes = ow["nodes"][ow["node_ptr"][g]:ow["node_ptr"][g + 1]]
        seen = {}
        for t in range(t0, t0 + nt):
            tn = nodes[ow["task_ln"][t, :nen].astype(np.int64)]
            assert sorted(tn) == sorted(cm[ow["task_elem"][t]])
            for r in range(ra):
                if tn[r] < r0 or tn[r] >= r0 + nr:
                    continue
                key = (int(ow["task_phase"][t]), (t - t0) // 64 if priv else 0, int(tn[r]))
                assert key not in seen
                seen[key] = t


def test_owner_plan_hex_tasks_per_element():
    """HEX08: interior elements of a group give two tasks, the others one or
    two; the average stays near the owned-row count's lower bound."""
    case = meshgen.make_case(16, meshgen.HEX08, 0.15, case_id=219, shuffle=True)
    P = fe.Plan(8, case.coords, case.conn)
    ow = P.export_owner()
    T = ow["task_elem"].size
    # each task covers at most 4 of the 8 * E (element, row) contributions
    assert T >= 2 * case.n_elems
    assert T <= 3.2 * case.n_elems
    assert ow["groups"][:, 1].mean() > 160   # groups fill most of a 256-lane work-group


def test_owner_plan_absent_for_hybrid_meshes():
    case = meshgen.make_case(4, meshgen.HYBRID, 0.1, case_id=220)
    P = fe.Plan(fe.HYBRID, case.coords, case.conn, types=case.types)
    with pytest.raises(fe.FeError):
        P.export_owner()
