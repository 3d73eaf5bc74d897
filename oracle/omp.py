"""The oracle on every host core (feoracle_omp.c), for the benchmark's CPU
baseline.

TEST INFRASTRUCTURE ONLY, like the rest of this package.  It runs the
serial oracle's element computation, Dirichlet elimination and PCG
recurrence, with the element loop in colour order (elements of one colour
in parallel, no two sharing a node) and the PCG kernels over rows in
parallel.  Parity tests use the serial oracle; tests/test_oracle_omp.py
checks this build against it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import OK, OP_SCALAR, OP_MOMENTUM, AssembleError, _f64, _i32, _p, _u8, pattern

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "feoracle_omp.c")
LIB = os.path.join(HERE, "liboracle_omp.so")
MAX_COLOURS = 64
_lib = None


def build() -> str:
    """gcc -O3 for a portable x86-64 level (the timing host may differ from
    the build host), OpenMP, no FMA contraction."""
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-std=gnu99", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.or_omp_threads.restype = i32
        L.or_omp_threads.argtypes = []
        L.or_omp_colour.restype = i32
        L.or_omp_colour.argtypes = [i32, P, i64, i64, P, P, P]
        L.or_omp_assemble.restype = i32
        L.or_omp_assemble.argtypes = [i32, P, i64, P, i64, P, i32, dbl, P, P, P, i32, P, P, P, P, i32, P, P, P, P,
                                      C.POINTER(i64), C.POINTER(dbl)]
        L.or_omp_dirichlet.restype = i32
        L.or_omp_dirichlet.argtypes = [i64, P, P, P, P, i64, P, P]
        L.or_omp_pcg.restype = i32
        L.or_omp_pcg.argtypes = [i64, P, P, P, P, P, dbl, i32, P]
        _lib = L
    return _lib


def threads() -> int:
    """Threads each parallel region uses (OMP_NUM_THREADS, else every core)."""
    return int(lib().or_omp_threads())


def colour(conn, n_nodes: int, types=None):
    """(n_colours, order, colour_ptr) of the greedy element colouring."""
    conn = _i32(conn)
    types = _u8(types)
    order = np.zeros(conn.shape[0], np.int32)
    ptr = np.zeros(MAX_COLOURS + 1, np.int32)
    nc = lib().or_omp_colour(conn.shape[1], _p(types), n_nodes, conn.shape[0], _p(conn), _p(order), _p(ptr))
    if nc < 0:
        raise RuntimeError("element colouring needs more than 64 colours")
    return nc, order, ptr[:nc + 1].copy()


def assemble(coords, conn, op: int, dt: float, u=None, rho=None, mu=None, Y=None, D=None, pattern_=None,
             types=None, colouring=None):
    """oracle.assemble on every core; colouring = colour(conn, N, types)."""
    coords = _f64(coords)
    conn = _i32(conn)
    types = _u8(types)
    N = coords.shape[0]
    rowptr, colidx = pattern_ if pattern_ is not None else pattern(conn, N, types)
    nc, order, ptr = colouring if colouring is not None else colour(conn, N, types)
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
    st = lib().or_omp_assemble(conn.shape[1], _p(types), N, _p(coords), conn.shape[0], _p(conn), op, dt, _p(u),
                               _p(rho), _p(mu), ns, _p(Yp), _p(Dp), _p(rowptr), _p(colidx), nc, _p(order),
                               _p(ptr), _p(values), _p(rhs), C.byref(bad), C.byref(mdet))
    if st != OK:
        raise AssembleError(st, bad.value, mdet.value)
    return rowptr, colidx, values, rhs


def dirichlet(rowptr, colidx, values, rhs, dnodes, g=None):
    N = rowptr.shape[0] - 1
    dn = _i32(dnodes)
    gp = _f64(g) if g is not None else None
    assert values.flags.c_contiguous and rhs.flags.c_contiguous
    st = lib().or_omp_dirichlet(N, _p(rowptr), _p(colidx), _p(values), _p(rhs), dn.shape[0], _p(dn), _p(gp))
    if st != OK:
        raise ValueError(f"oracle dirichlet failed: {st}")


def pcg(rowptr, colidx, values, b, x0=None, rtol=1e-10, max_iter=10000):
    """Returns (x, status, iterations, rel_res, true_rel_res) like oracle.pcg."""
    N = rowptr.shape[0] - 1
    b = _f64(b)
    x = np.zeros(N) if x0 is None else _f64(x0).copy()
    info = np.zeros(3)
    values = _f64(values)
    st = lib().or_omp_pcg(N, _p(rowptr), _p(colidx), _p(values), _p(b), _p(x), rtol, max_iter, _p(info))
    return x, st, int(info[0]), float(info[1]), float(info[2])
