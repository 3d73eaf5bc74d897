"""Python access to the FP64 CPU oracle (feoracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.
It shares no code with the GPU path.  The shared object is built with plain
gcc and no FMA contraction (see build()).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "feoracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OP_MOMENTUM, OP_SCALAR, OP_POISSON = 0, 1, 2
OK, EINVAL, ENOMEM, EBADELEM, ENOCONV, EBREAKDOWN = 0, 1, 2, 4, 5, 6

_lib = None


def build() -> str:
    """Compile liboracle.so with gcc (serial, -ffp-contract=off), and the
    all-core timing build liboracle_omp.so (oracle/omp.py)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-std=c99", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    from . import omp
    omp.build()
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.or_pattern.restype = i64
        L.or_pattern.argtypes = [i32, i64, i64, P, P, P]
        L.or_pattern_typed.restype = i64
        L.or_pattern_typed.argtypes = [i32, P, i64, i64, P, P, P]
        L.or_assemble.restype = i32
        L.or_assemble.argtypes = [i32, i64, P, i64, P, i32, dbl, P, P, P, i32, P, P, P, P, P, P,
                                  C.POINTER(i64), C.POINTER(dbl)]
        L.or_assemble_typed.restype = i32
        L.or_assemble_typed.argtypes = [i32, P, i64, P, i64, P, i32, dbl, P, P, P, i32, P, P, P, P, P, P,
                                        C.POINTER(i64), C.POINTER(dbl)]
        L.or_assemble_block.restype = i32
        L.or_assemble_block.argtypes = [i32, P, i64, P, i64, P, i32, dbl, P, P, P, P, P, P, P,
                                        C.POINTER(i64), C.POINTER(dbl)]
        L.or_element_vectors.restype = i32
        L.or_element_vectors.argtypes = [i32, P, i64, P, i64, P, i32, i32, P, P, P, P, P, dbl, P,
                                         C.POINTER(i64), C.POINTER(dbl)]
        L.or_wall_utau.restype = dbl
        L.or_wall_utau.argtypes = [dbl, dbl, dbl]
        L.or_wall_traction.restype = i32
        L.or_wall_traction.argtypes = [i64, P, i64, P, P, P, P, P, dbl, P]
        L.or_dirichlet.restype = i32
        L.or_dirichlet.argtypes = [i64, P, P, P, P, i64, P, P]
        L.or_spmv.restype = None
        L.or_spmv.argtypes = [i64, P, P, P, P, P]
        L.or_dot.restype = dbl
        L.or_dot.argtypes = [i64, P, P]
        L.or_pcg.restype = i32
        L.or_pcg.argtypes = [i64, P, P, P, P, P, dbl, i32, P]
        for name in ("or_hex08_shape", "or_tet04_shape", "or_pen06_shape", "or_pyr05_shape"):
            getattr(L, name).restype = None
            getattr(L, name).argtypes = [P, P, P]
        for name in ("or_hex08_gauss", "or_tet04_gauss", "or_pen06_gauss", "or_pyr05_gauss"):
            getattr(L, name).restype = None
            getattr(L, name).argtypes = [P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# --- reference element -------------------------------------------------------

_NAMES = {8: "hex08", 6: "pen06", 5: "pyr05", 4: "tet04"}
_NGAUSS = {8: 8, 6: 6, 5: 8, 4: 4}


def shape(nen: int, xi):
    xi = _f64(xi)
    N = np.zeros(nen)
    dN = np.zeros((nen, 3))
    getattr(lib(), "or_%s_shape" % _NAMES[nen])(_p(xi), _p(N), _p(dN))
    return N, dN


def gauss(nen: int):
    ng = _NGAUSS[nen]
    pts = np.zeros((ng, 3))
    w = np.zeros(ng)
    getattr(lib(), "or_%s_gauss" % _NAMES[nen])(_p(pts), _p(w))
    return pts, w


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


# --- assembly ----------------------------------------------------------------

def pattern(conn, n_nodes: int, types=None):
    """CSR pattern; conn [E, stride], types [E] node counts (None: single type)."""
    conn = _i32(conn)
    types = _u8(types)
    S = conn.shape[1]
    rowptr = np.zeros(n_nodes + 1, dtype=np.int32)
    nnz = lib().or_pattern_typed(S, _p(types), n_nodes, conn.shape[0], _p(conn), _p(rowptr), None)
    if nnz < 0:
        raise ValueError("invalid connectivity")
    colidx = np.zeros(max(nnz, 1), dtype=np.int32)[:nnz]
    lib().or_pattern_typed(S, _p(types), n_nodes, conn.shape[0], _p(conn), _p(rowptr), _p(colidx))
    return rowptr, colidx


class AssembleError(RuntimeError):
    def __init__(self, status, bad_elem, min_det):
        super().__init__(f"oracle assembly failed: status {status}, element {bad_elem}, min detJ {min_det}")
        self.status, self.bad_elem, self.min_det = status, bad_elem, min_det


def assemble(coords, conn, op: int, dt: float, u=None, rho=None, mu=None, Y=None, D=None,
             pattern_=None, types=None):
    """Return (rowptr, colidx, values[n_mat, nnz], rhs[n_rhs, N]).

    conn [E, stride]; types [E] per-element node counts for a mixed mesh
    (None: every element has `stride` nodes)."""
    coords = _f64(coords)
    conn = _i32(conn)
    types = _u8(types)
    N = coords.shape[0]
    S = conn.shape[1]
    rowptr, colidx = pattern_ if pattern_ is not None else pattern(conn, N, types)
    nnz = int(rowptr[-1])
    ns = 0 if Y is None else int(np.asarray(Y).shape[0])
    n_mat = ns if op == OP_SCALAR else 1
    n_rhs = 3 if op == OP_MOMENTUM else (ns if op == OP_SCALAR else 1)
    u = _f64(u if u is not None else np.zeros((3, N)))
    rho = _f64(rho if rho is not None else np.ones(N))
    mu = _f64(mu if mu is not None else np.ones(N))
    Yp = _f64(Y) if ns else None
    Dp = _f64(D) if ns else None
    values = np.zeros((n_mat, nnz))
    rhs = np.zeros((n_rhs, N))
    bad = C.c_int64(-1)
    mdet = C.c_double(0.0)
    st = lib().or_assemble_typed(S, _p(types), N, _p(coords), conn.shape[0], _p(conn), op, dt, _p(u),
                                 _p(rho), _p(mu), ns, _p(Yp), _p(Dp), _p(rowptr), _p(colidx),
                                 _p(values), _p(rhs), C.byref(bad), C.byref(mdet))
    if st != OK:
        raise AssembleError(st, bad.value, mdet.value)
    return rowptr, colidx, values, rhs


FULL_STRESS, EMAC = 1, 2    # residual operator variants (bits of `form`)


def assemble_block(coords, conn, form: int, dt: float, u, rho, mu, pattern_=None, types=None):
    """Momentum operator with 3x3 blocks (full-stress viscous term with form
    bit FULL_STRESS, EMAC's (div u) term with EMAC; or_assemble_block).
    Returns (rowptr, colidx, values[nnz, 3, 3], rhs[3, N])."""
    coords = _f64(coords)
    conn = _i32(conn)
    types = _u8(types)
    N = coords.shape[0]
    rowptr, colidx = pattern_ if pattern_ is not None else pattern(conn, N, types)
    nnz = int(rowptr[-1])
    u, rho, mu = _f64(u), _f64(rho), _f64(mu)
    values = np.zeros((nnz, 3, 3))
    rhs = np.zeros((3, N))
    bad = C.c_int64(-1)
    mdet = C.c_double(0.0)
    st = lib().or_assemble_block(conn.shape[1], _p(types), N, _p(coords), conn.shape[0], _p(conn), int(form), dt,
                                 _p(u), _p(rho), _p(mu), _p(rowptr), _p(colidx), _p(values), _p(rhs),
                                 C.byref(bad), C.byref(mdet))
    if st != OK:
        raise AssembleError(st, bad.value, mdet.value)
    return rowptr, colidx, values, rhs


def _element_vectors(coords, conn, kind, u=None, rho=None, mu=None, p=None, types=None, form=0, Y=None, D=0.0):
    coords, conn, types = _f64(coords), _i32(conn), _u8(types)
    # contiguous copies held in locals: they must outlive the C call
    u, rho, mu, p, Y = [None if a is None else _f64(a) for a in (u, rho, mu, p, Y)]
    N = coords.shape[0]
    out = np.zeros(({0: 4, 1: 3, 2: 2}[kind], N))
    bad = C.c_int64(-1)
    mdet = C.c_double(0.0)
    st = lib().or_element_vectors(conn.shape[1], _p(types), N, _p(coords), conn.shape[0], _p(conn), kind, form,
                                  _p(u), _p(rho), _p(mu), _p(p), _p(Y), float(D), _p(out), C.byref(bad),
                                  C.byref(mdet))
    if st != OK:
        raise AssembleError(st, bad.value, mdet.value)
    return out


def residual(coords, conn, u, rho, mu, types=None, form=0):
    """Matrix-free momentum residual r[3, N] = -(C(u) + K_mu) u_i and the
    rho-weighted lumped mass m[N] (or_element_vectors kind 0); form: bits
    FULL_STRESS (viscous term 2 mu eps(u)) and EMAC (convective term of
    Eq. (1) at the Gauss points)."""
    out = _element_vectors(coords, conn, 0, u=u, rho=rho, mu=mu, types=types, form=form)
    return out[:3], out[3]


def scalar_residual(coords, conn, u, rho, Y, D, types=None):
    """Matrix-free scalar-transport residual r[N] = -(C(u) + K_{rho D}) Y and
    the rho-weighted lumped mass m[N] (or_element_vectors kind 2)."""
    out = _element_vectors(coords, conn, 2, u=u, rho=rho, types=types, Y=Y, D=D)
    return out[0], out[1]


def scalar_step(coords, conn, dirichlet_nodes, dt, u, rho, Y, D, types=None, rk=None):
    """One explicit Runge-Kutta step (SSP-RK3 by default) of M_L dY/dt =
    scalar_residual(Y), the scalar held at Dirichlet nodes; no solve
    (the heat and species equations of Section 2).  Returns Y_new[N]."""
    rk = SSP_RK3 if rk is None else rk
    free = np.ones(len(Y), bool)
    free[np.asarray(dirichlet_nodes)] = False
    y0 = np.array(Y, dtype=np.float64)
    ys = y0.copy()
    for a, b in rk:
        r, m = scalar_residual(coords, conn, u, rho, ys, D, types)
        ys = np.where(free, a * y0 + b * (ys + dt * r / m), y0)
    return ys


def gradient(coords, conn, p, types=None):
    """g[3, N]: g_j[a] = int N_a d p_h / d x_j (or_element_vectors kind 1)."""
    return _element_vectors(coords, conn, 1, p=p, types=types)


def wall_utau(U, nu, delta):
    """Friction velocity of the equilibrium wall law (Reichardt) at distance delta."""
    return lib().or_wall_utau(float(U), float(nu), float(delta))


def wall_traction(coords, face_nen, face_conn, u, rho, mu, delta):
    """Wall-model traction out[3, N] = sum over wall faces of int N_a t dS,
    t = -rho u_tau^2 u_t / |u_t| (or_wall_traction)."""
    coords, u, rho, mu = _f64(coords), _f64(u), _f64(rho), _f64(mu)
    nen, fc = _u8(face_nen), _i32(face_conn)
    N = coords.shape[0]
    out = np.zeros((3, N))
    st = lib().or_wall_traction(N, _p(coords), nen.shape[0], _p(nen), _p(fc), _p(u), _p(rho), _p(mu),
                                float(delta), _p(out))
    if st != OK:
        raise ValueError(f"oracle wall traction failed: {st}")
    return out


# Shu-Osher strong-stability-preserving third-order Runge-Kutta: stage s
# maps (u^n, u_s) to alpha_s u^n + beta_s (u_s + dt L(u_s)).
SSP_RK3 = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def rk_predictor(coords, conn, dirichlet_nodes, dt, u, rho, mu, types=None, rk=SSP_RK3, form=0, wall=None):
    """Explicit RK stages of M_L du/dt = R(u) (velocity held at Dirichlet
    nodes); wall = (face_nen, face_conn, delta) adds the wall-model traction
    to R.  Returns (u*, lumped mass m)."""
    free = np.ones(u.shape[1], bool)
    free[np.asarray(dirichlet_nodes)] = False
    u0 = np.array(u, dtype=np.float64)
    us = u0.copy()
    m = None
    for a, b in rk:
        r, m = residual(coords, conn, us, rho, mu, types, form)
        if wall is not None:
            r = r + wall_traction(coords, wall[0], wall[1], us, rho, mu, wall[2])
        nxt = a * u0 + b * (us + dt * r / m)
        us = np.where(free, nxt, u0)
    return us, m


def fractional_step(coords, conn, dirichlet_nodes, dt, u, rho, mu, L, rtol=1e-12, max_iter=20000, p0=None,
                    types=None, rk=SSP_RK3, form=0, wall=None):
    """One step of the fractional-step scheme around the assembly (Algorithm 1):
      1. momentum predictor, explicit RK (SSP-RK3) on M_L du/dt = R(u), with
         M_L the rho-weighted lumped mass and R the matrix-free residual; the
         velocity at Dirichlet nodes is held;
      2. pressure: (rowptr, colidx, values) = L, the Poisson matrix after the
         Dirichlet elimination; right-hand side (1/dt) int grad N . (rho u*),
         zero at Dirichlet rows; Jacobi-PCG from p0 (zero if None);
      3. correction u = u* - dt M_L^-1 G p at free nodes.
    Returns (u_new[3, N], p[N], cg_iterations)."""
    rp, ci, Lv = L
    dn = np.asarray(dirichlet_nodes)
    free = np.ones(u.shape[1], bool)
    free[dn] = False
    us, m = rk_predictor(coords, conn, dirichlet_nodes, dt, u, rho, mu, types, rk, form, wall)
    _, _, _, f = assemble(coords, conn, OP_POISSON, dt, us, rho, None, pattern_=(rp, ci), types=types)
    f = f[0]
    f[dn] = 0.0
    p, st, it, _, _ = pcg(rp, ci, Lv, f, x0=p0, rtol=rtol, max_iter=max_iter)
    if st != OK:
        raise RuntimeError(f"oracle pressure solve failed: {st}")
    g = gradient(coords, conn, p, types)
    un = np.where(free, us - dt * g / m, us)
    return un, p, it


def dirichlet(rowptr, colidx, values, rhs, dnodes, g=None):
    """Apply symmetric elimination in place (values [nnz], rhs [N])."""
    N = rowptr.shape[0] - 1
    dn = _i32(dnodes)
    gp = _f64(g) if g is not None else None
    assert values.flags.c_contiguous and rhs.flags.c_contiguous
    st = lib().or_dirichlet(N, _p(rowptr), _p(colidx), _p(values), _p(rhs), dn.shape[0], _p(dn), _p(gp))
    if st != OK:
        raise ValueError(f"oracle dirichlet failed: {st}")


def spmv(rowptr, colidx, values, x):
    N = rowptr.shape[0] - 1
    x = _f64(x)
    y = np.zeros(N)
    values = _f64(values)   # held until the call returns
    lib().or_spmv(N, _p(rowptr), _p(colidx), _p(values), _p(x), _p(y))
    return y


def dot(x, y):
    x, y = _f64(x), _f64(y)
    return lib().or_dot(x.shape[0], _p(x), _p(y))


def pcg(rowptr, colidx, values, b, x0=None, rtol=1e-10, max_iter=10000):
    """Jacobi-PCG; returns (x, status, iterations, rel_res, true_rel_res)."""
    N = rowptr.shape[0] - 1
    b = _f64(b)
    x = np.zeros(N) if x0 is None else _f64(x0).copy()
    info = np.zeros(3)
    values = _f64(values)
    st = lib().or_pcg(N, _p(rowptr), _p(colidx), _p(values), _p(b), _p(x), rtol, max_iter, _p(info))
    return x, st, int(info[0]), float(info[1]), float(info[2])


def time_call(fn, *a, **k):
    t0 = time.perf_counter()
    r = fn(*a, **k)
    return r, time.perf_counter() - t0
