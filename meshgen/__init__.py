"""Seeded synthetic meshes and nodal fields.

This module is the one place that both the product path and the oracle take
their inputs from.  It builds meshes (a jittered unit cube of HEX08 cells, the
same cube split into TET04, PEN06 or PYR05 cells, or a hybrid of all four),
random renumberings, Dirichlet node lists and the nodal fields (velocity,
density, viscosity, species).  It holds
none of the finite-element arithmetic: no shape function, quadrature rule,
Jacobian, elemental matrix or solver lives here.

The paper's test case is a swirl burner on a 64 M-cell mixed tet/pyramid/hex
mesh (Section 5.1) with a flamelet database; neither is available, so these
synthetic cubes stand in for it.  Recipes:

* geometry: unit cube, n cells per side, h = 1/n.  Nodes are jittered by an
  i.i.d. uniform offset in [-j*h, +j*h] per coordinate; nodes on the boundary
  move only tangentially (faces stay planar, corners stay put), so the domain
  stays exactly [0,1]^3.
* HEX08 node order: 0:(-,-,-) 1:(+,-,-) 2:(+,+,-) 3:(-,+,-) 4:(-,-,+)
  5:(+,-,+) 6:(+,+,+) 7:(-,+,+).
* TET04: each cube split into six tetrahedra around the 0-6 diagonal,
  (0,1,2,6) (0,2,3,6) (0,3,7,6) (0,7,4,6) (0,4,5,6) (0,5,1,6), all positively
  oriented and conforming across cubes.
* PEN06: each cube split into two prisms along the 0-2 diagonal of its
  bottom face, (0,1,2|4,5,6) and (0,2,3|4,6,7) (bottom triangle, then the
  nodes above it); conforming across cubes.
* PYR05: each cube split into six pyramids, one per face, with a new apex
  node at the mean of the cube's eight corners; bases ordered
  counter-clockwise seen from the apex: (0,1,2,3) (4,7,6,5) (0,4,5,1)
  (3,2,6,7) (0,3,7,4) (1,5,6,2).  Centre nodes are numbered after the grid
  nodes, in cube order.
* HYBRID: slabs of cubes along x, i the cube's x index: prisms for
  i < n/4, hexahedra for n/4 <= i < n/2, one transition slab i = n/2 and
  Kuhn tetrahedra beyond.  A transition cube holds one pyramid on its x = 0
  face (the hexahedra's side) and ten tetrahedra that join its centre node
  to the halves of its five other faces, each face split along the Kuhn
  diagonal (its first and third base node above), so every interface
  conforms.  Connectivity is [E, 8] padded with -1 and `types` gives each
  element's node count (4, 5, 6 or 8).
* velocity: Taylor-Green u = sin2πx cos2πy cos2πz, v = -cos2πx sin2πy cos2πz,
  w = 0, plus i.i.d. N(0, 0.01^2) per component.
* density U[0.2, 1.2] i.i.d. per node; viscosity 1.8e-5 (air).
* flame-kernel temperature T = 300 + 1700 * (1 - tanh((r - 0.25)/0.03))/2
  around the cube centre; density p0/(R T), Sutherland viscosity.
* species Y_k ~ U[0,1], diffusivities D_k = 10^U(-6,-4).
* time step dt = 0.5 h / U0 with U0 = 1.

Random sub-streams come from numpy.random.SeedSequence(case_id).spawn(9) in
the fixed order: jitter, u-noise, rho, node permutation, element permutation,
Y, D, arrivals, sizes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import json
import math
import os
from typing import Optional

import numpy as np

HEX08 = 8
TET04 = 4
PEN06 = 6
PYR05 = 5
HYBRID = 0      # mixed element types, padded connectivity plus a type array

# Six positively oriented tetrahedra per hexahedron, local HEX08 node ids.
KUHN_TETS = np.array(
    [[0, 1, 2, 6], [0, 2, 3, 6], [0, 3, 7, 6], [0, 7, 4, 6], [0, 4, 5, 6], [0, 5, 1, 6]],
    dtype=np.int64,
)

PRISM_SPLIT = np.array([[0, 1, 2, 4, 5, 6], [0, 2, 3, 4, 6, 7]], dtype=np.int64)
PYRAMID_BASES = np.array([[0, 1, 2, 3], [4, 7, 6, 5], [0, 4, 5, 1], [3, 2, 6, 7], [0, 3, 7, 4],
                          [1, 5, 6, 2]], dtype=np.int64)

AIR_P0 = 101325.0        # Pa
AIR_R = 287.05           # J/(kg K)
SUTH_MU_REF = 1.716e-5   # Pa s
SUTH_T_REF = 273.15      # K
SUTH_S = 110.4           # K
MU_AIR = 1.8e-5

_STREAMS = ("jitter", "unoise", "rho", "nperm", "eperm", "Y", "D", "arrivals", "sizes")


def streams(case_id: int, sub=None) -> dict:
    """Named numpy Generators for a case (and optional sub-case id)."""
    key = [int(case_id)] if sub is None else [int(case_id), int(sub)]
    ss = np.random.SeedSequence(key)
    return {name: np.random.Generator(np.random.PCG64(s))
            for name, s in zip(_STREAMS, ss.spawn(len(_STREAMS)))}


@dataclass
class Case:
    """A mesh plus its nodal fields, all in the user's numbering.

    coords [N,3] float64; conn [E,nen] int32 ([E,8] padded with -1 for
    HYBRID, with types [E] the node counts); dirichlet int32 node ids;
    u [3,N]; rho [N]; mu [N]; Y [k,N]; D [k]; dt scalar.
    """
    elem_type: int
    n: int
    coords: np.ndarray
    conn: np.ndarray
    dirichlet: np.ndarray
    u: np.ndarray
    rho: np.ndarray
    mu: np.ndarray
    dt: float
    Y: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))
    D: np.ndarray = field(default_factory=lambda: np.zeros(0))
    name: str = ""
    types: Optional[np.ndarray] = None   # HYBRID: [E] uint8 node counts
    wall_nen: Optional[np.ndarray] = None    # wall faces: [F] uint8, 3 or 4 nodes
    wall_conn: Optional[np.ndarray] = None   # [F, 4] int32 node ids, -1 padded

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def nen(self) -> int:
        return int(self.conn.shape[1])


def node_id(n: int, i, j, k):
    return i + (n + 1) * (j + (n + 1) * k)


def cube_nodes(n: int, jitter: float = 0.0, rng=None) -> np.ndarray:
    """Nodes of an n^3 grid on [0,1]^3, id = i + (n+1)(j + (n+1)k).

    Jitter is uniform in [-jitter*h, jitter*h] per coordinate; a boundary node
    keeps the coordinate normal to each boundary face it lies on.
    """
    h = 1.0 / n
    g = np.arange(n + 1, dtype=np.float64) * h
    kk, jj, ii = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    idx = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    x = g[idx]
    if jitter > 0.0:
        if rng is None:
            raise ValueError("jitter needs an rng")
        d = rng.uniform(-jitter * h, jitter * h, size=x.shape)
        on_bnd = (idx == 0) | (idx == n)
        d[on_bnd] = 0.0
        x = x + d
    return np.ascontiguousarray(x)


def hex_conn(n: int) -> np.ndarray:
    """HEX08 connectivity of the n^3 grid, elements i-fastest."""
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = ii.ravel(), jj.ravel(), kk.ravel()
    corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
               (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    conn = np.stack([node_id(n, i + a, j + b, k + c) for a, b, c in corners], axis=1)
    return np.ascontiguousarray(conn.astype(np.int32))


def kuhn_split(hconn: np.ndarray) -> np.ndarray:
    """Split every HEX08 into six TET04 (hex order kept, tets consecutive)."""
    t = hconn[:, KUHN_TETS]                      # [E, 6, 4]
    return np.ascontiguousarray(t.reshape(-1, 4).astype(np.int32))


def prism_split(hconn: np.ndarray) -> np.ndarray:
    """Split every HEX08 into two PEN06 (hex order kept)."""
    return np.ascontiguousarray(hconn[:, PRISM_SPLIT].reshape(-1, 6).astype(np.int32))


def cube_centres(coords: np.ndarray, hconn: np.ndarray) -> np.ndarray:
    """Mean of each cube's eight corners."""
    return coords[hconn].mean(axis=1)


def pyramid_split(hconn: np.ndarray, centre_ids: np.ndarray) -> np.ndarray:
    """Split every HEX08 into six PYR05 around its centre node."""
    E = hconn.shape[0]
    base = hconn[:, PYRAMID_BASES]                       # [E, 6, 4]
    apex = np.broadcast_to(centre_ids[:, None, None], (E, 6, 1))
    return np.ascontiguousarray(np.concatenate([base, apex], axis=2).reshape(-1, 5).astype(np.int32))


def hybrid_mesh(n: int, coords: np.ndarray):
    """Slabs of prisms, hexahedra, pyramid-tet transition cubes and Kuhn
    tetrahedra along x (see the module docstring).  Returns the coordinates
    with the transition cubes' centre nodes appended, the [E, 8] connectivity
    padded with -1 and the per-element node counts."""
    if n < 4:
        raise ValueError("a hybrid cube needs n >= 4")
    hconn = hex_conn(n).astype(np.int64)
    ci = np.arange(hconn.shape[0]) % n                   # cube x index (cubes are i-fastest)
    i0, i1 = n // 4, n // 2
    trans = np.flatnonzero(ci == i1)
    cid = coords.shape[0] + np.arange(trans.size)
    coords = np.concatenate([coords, cube_centres(coords, hconn[trans])])
    # elements of each kind as [cubes, per cube, 8] blocks, merged in cube order
    # (within a cube: the order listed below)
    parts = []

    def add(cubes, rows, t):
        k = rows.shape[1]
        pad = np.full((cubes.size, k, 8), -1, dtype=np.int32)
        pad[:, :, :rows.shape[2]] = rows
        key = (cubes[:, None] * 16 + np.arange(k)[None, :]).ravel()
        parts.append((key, pad.reshape(-1, 8), np.full(key.size, t, np.uint8)))

    c = np.flatnonzero(ci < i0)
    add(c, hconn[c][:, PRISM_SPLIT], PEN06)
    c = np.flatnonzero((ci >= i0) & (ci < i1))
    add(c, hconn[c][:, None, :], HEX08)
    c = np.flatnonzero(ci > i1)
    add(c, hconn[c][:, KUHN_TETS], TET04)
    h = hconn[trans]
    rows = [np.concatenate([h[:, PYRAMID_BASES[4]], cid[:, None]], axis=1)[:, None, :]]
    for f in (0, 1, 2, 3, 5):
        b = h[:, PYRAMID_BASES[f]]
        for tri in ((0, 1, 2), (0, 2, 3)):
            rows.append(np.concatenate([b[:, list(tri)], cid[:, None]], axis=1)[:, None, :])
    tets = np.concatenate(rows[1:], axis=1)                 # [cubes, 10, 4]
    key = np.concatenate([trans[:, None] * 16, trans[:, None] * 16 + 1 + np.arange(10)[None, :]], axis=1)
    conn_t = np.full((trans.size, 11, 8), -1, np.int32)
    conn_t[:, 0, :5] = rows[0][:, 0, :]
    conn_t[:, 1:, :4] = tets
    typ_t = np.full((trans.size, 11), TET04, np.uint8)
    typ_t[:, 0] = PYR05
    parts.append((key.ravel(), conn_t.reshape(-1, 8), typ_t.ravel()))
    key = np.concatenate([q[0] for q in parts])
    order = np.argsort(key, kind="stable")
    conn = np.concatenate([q[1] for q in parts])[order]
    types = np.concatenate([q[2] for q in parts])[order]
    return np.ascontiguousarray(coords), np.ascontiguousarray(conn), np.ascontiguousarray(types)


def wall_faces_z0(n: int, elem_type: int):
    """Element faces on the z = 0 plane (the wall of the wall-model tests),
    node ids of the unshuffled cube: a quadrilateral (0,1,2,3) where the
    cell's bottom is a HEX08 face or a PYR05 base, else the two triangles
    (0,1,2) and (0,2,3) along the cell's 0-2 diagonal (prism bottoms, Kuhn and
    transition tetrahedra).  Returns (nen [F] uint8, conn [F, 4] int32)."""
    hconn = hex_conn(n)[: n * n]                          # cells with k = 0
    ci = np.arange(n * n) % n
    if elem_type in (HEX08, PYR05):
        quad = np.ones(n * n, bool)
    elif elem_type == HYBRID:
        quad = (ci >= n // 4) & (ci < n // 2)
    else:
        quad = np.zeros(n * n, bool)
    nen, conn = [], []
    for c in range(n * n):
        h = hconn[c]
        if quad[c]:
            nen.append(4)
            conn.append([h[0], h[1], h[2], h[3]])
        else:
            nen += [3, 3]
            conn += [[h[0], h[1], h[2], -1], [h[0], h[2], h[3], -1]]
    return np.array(nen, np.uint8), np.array(conn, np.int32)


def boundary_nodes(n: int) -> np.ndarray:
    kk, jj, ii = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    m = (ii == 0) | (ii == n) | (jj == 0) | (jj == n) | (kk == 0) | (kk == n)
    return np.flatnonzero(m.ravel()).astype(np.int32)


def permute(coords, conn, dirichlet, node_fields, rng_nodes, rng_elems, types=None, faces=None):
    """Random renumbering: new id of old node i is pn[i]; elements shuffled.

    node_fields: list of arrays whose LAST axis is the node axis.  Padding
    entries (-1) of the connectivity stay -1; `types` follows the elements;
    `faces` (a face connectivity, -1 padded) is renumbered, not reordered.
    """
    N = coords.shape[0]
    E = conn.shape[0]
    pn = rng_nodes.permutation(N)
    pe = rng_elems.permutation(E)
    inv = np.empty(N, dtype=np.int64)
    inv[pn] = np.arange(N)
    coords2 = np.ascontiguousarray(coords[inv])
    c = conn[pe]
    conn2 = np.ascontiguousarray(np.where(c >= 0, pn[np.maximum(c, 0)], -1).astype(np.int32))
    dir2 = np.sort(pn[dirichlet]).astype(np.int32)
    f2 = [np.ascontiguousarray(f[..., inv]) for f in node_fields]
    faces2 = None if faces is None else np.ascontiguousarray(
        np.where(faces >= 0, pn[np.maximum(faces, 0)], -1).astype(np.int32))
    if types is None and faces is None:
        return coords2, conn2, dir2, f2
    return coords2, conn2, dir2, f2, None if types is None else np.ascontiguousarray(types[pe]), faces2


def taylor_green(coords, rng=None, noise=0.01) -> np.ndarray:
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    tp = 2.0 * math.pi
    u = np.stack([np.sin(tp * x) * np.cos(tp * y) * np.cos(tp * z),
                  -np.cos(tp * x) * np.sin(tp * y) * np.cos(tp * z),
                  np.zeros_like(x)])
    if noise > 0.0:
        u = u + rng.normal(0.0, noise, size=u.shape)
    return np.ascontiguousarray(u)


def flame_temperature(coords) -> np.ndarray:
    r = np.linalg.norm(coords - 0.5, axis=1)
    return 300.0 + 1700.0 * 0.5 * (1.0 - np.tanh((r - 0.25) / 0.03))


def ideal_gas_density(T) -> np.ndarray:
    return AIR_P0 / (AIR_R * T)


def sutherland(T) -> np.ndarray:
    return SUTH_MU_REF * (T / SUTH_T_REF) ** 1.5 * (SUTH_T_REF + SUTH_S) / (T + SUTH_S)


def time_step(n: int, u0: float = 1.0) -> float:
    return 0.5 * (1.0 / n) / u0


def make_case(n: int, elem_type: int = HEX08, jitter: float = 0.10, case_id: int = 0,
              sub=None, shuffle: bool = False, temperature: bool = False,
              n_scalars: int = 0, noise: float = 0.01, name: str = "", walls: bool = False) -> Case:
    """Build one synthetic case (see the module docstring for the recipe)."""
    rs = streams(case_id, sub)
    coords = cube_nodes(n, jitter, rs["jitter"])
    hconn = hex_conn(n)
    types = None
    if elem_type == HEX08:
        conn = hconn
    elif elem_type == TET04:
        conn = kuhn_split(hconn)
    elif elem_type == PEN06:
        conn = prism_split(hconn)
    elif elem_type == PYR05:
        cid = coords.shape[0] + np.arange(hconn.shape[0])
        coords = np.ascontiguousarray(np.concatenate([coords, cube_centres(coords, hconn)]))
        conn = pyramid_split(hconn, cid)
    elif elem_type == HYBRID:
        coords, conn, types = hybrid_mesh(n, coords)
    else:
        raise ValueError(f"unknown element type {elem_type}")
    dirichlet = boundary_nodes(n)
    wnen, wconn = wall_faces_z0(n, elem_type) if walls else (None, None)
    N = coords.shape[0]
    u = taylor_green(coords, rs["unoise"], noise)
    if temperature:
        T = flame_temperature(coords)
        rho = ideal_gas_density(T)
        mu = sutherland(T)
    else:
        rho = rs["rho"].uniform(0.2, 1.2, size=N)
        mu = np.full(N, MU_AIR)
    Y = rs["Y"].uniform(0.0, 1.0, size=(n_scalars, N)) if n_scalars else np.zeros((0, N))
    D = 10.0 ** rs["D"].uniform(-6.0, -4.0, size=n_scalars) if n_scalars else np.zeros(0)
    if shuffle:
        out = permute(coords, conn, dirichlet, [u, rho, mu, Y], rs["nperm"], rs["eperm"], types, wconn)
        coords, conn, dirichlet, (u, rho, mu, Y) = out[:4]
        if types is not None:
            types = out[4]
        if wconn is not None:
            wconn = out[5]
    return Case(elem_type, n, coords, conn.astype(np.int32), dirichlet, u, rho, mu,
                time_step(n), Y, D, name, types, wnen, wconn)


# --- the five workloads -----------------------------------------------------
# Their parameters live in configs/cfg0..cfg4.json (name, mesh, jitter, seed,
# numbering, fields, solve); the functions below build them.

_CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")
_TYPES = {"HEX08": HEX08, "TET04": TET04, "PEN06": PEN06, "PYR05": PYR05, "HYBRID": HYBRID}


def config(name: str) -> dict:
    """The parameters of workload `name` (cfg0 ... cfg4)."""
    with open(os.path.join(_CONFIG_DIR, name + ".json")) as fh:
        return json.load(fh)


def _from_config(name: str, n: Optional[int] = None) -> Case:
    c = config(name)
    n = c["n"] if n is None else n
    label = c["name"].replace(str(c["n"]) + "^3", f"{n}^3")
    return make_case(n, _TYPES[c["elem_type"]], c["jitter"], case_id=c["seed"], shuffle=c["shuffle"],
                     temperature=c["temperature"], n_scalars=c["n_scalars"], walls=c["walls"], name=label)


def cfg0() -> Case:
    """10^3 HEX08, jitter 10 %, Taylor-Green + noise, rho U[0.2,1.2]."""
    return _from_config("cfg0")


def cfg1(n: int = 128) -> Case:
    """128^3 HEX08, jitter 15 %, node and element ids shuffled; the z = 0
    faces are the wall of the wall model."""
    return _from_config("cfg1", n)


def cfg2(n: int = 128) -> Case:
    """128^3 cubes x 6 Kuhn TET04, jitter 10 %, flame-kernel T, shuffled."""
    return _from_config("cfg2", n)


def cfg4(n: int = 256) -> Case:
    """256^3 HEX08, jitter 15 %, plus 5 species and diffusivities."""
    return _from_config("cfg4", n)


def hybrid(n: int = 128) -> Case:
    """n^3 cubes as prism / hex / pyramid-tet transition / Kuhn-tet slabs
    (HYBRID), jitter 10 %, flame-kernel T, shuffled; 7.9 M elements and
    2.16 M nodes at n = 128."""
    return make_case(n, HYBRID, 0.10, case_id=5, shuffle=True, temperature=True, name=f"hybrid-{n}^3-flame")


def serving_stream(n_requests: int = 2000, qps: float = 1.0, lo: int = 8, hi: int = 96):
    """Arrival times (s) and cube sides of the serving workload (configs/cfg3.json)."""
    rs = streams(config("cfg3")["seed"])
    gaps = rs["arrivals"].exponential(1.0 / qps, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    sides = np.rint(np.exp(rs["sizes"].uniform(math.log(lo), math.log(hi), size=n_requests)))
    return t, sides.astype(np.int64)


def serving_case(req: int, n: int) -> Case:
    """Request `req` of the serving workload: a jittered HEX08 cube as cfg0."""
    c = config("cfg3")
    return make_case(int(n), _TYPES[c["elem_type"]], c["jitter"], case_id=c["seed"], sub=req,
                     name=f"req{req}-hex08-{n}^3")


def hex_pattern_nnz(n: int) -> int:
    return (3 * n + 1) ** 3


def kuhn_pattern_nnz(n: int) -> int:
    edges = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    return (n + 1) ** 3 + 2 * edges
