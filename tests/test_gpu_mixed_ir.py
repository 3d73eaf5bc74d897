"""GPU tests of the mixed-precision pressure solve (FP32 Jacobi-PCG inside
FP64 iterative refinement, fe_cg_solve(FE_MIXED)) against the FP64 oracle.

Mixed mode is an approximation of the exact solve, so its reference is the
FP64 result: the oracle's Poisson system (assembly, Dirichlet elimination)
solved by the oracle's PCG to rtol 1e-13 and, on the small meshes, by a
dense direct solve.  Nothing below uses the library to judge the library:
the true residual of the returned x is recomputed on the host with the
oracle's SpMV on the oracle's matrix.

Stated bound (reading of "1e-8 relative error": a true FP64 relative
residual <= 1e-8): for an SPD matrix L with extreme eigenvalues lmin, lmax,
||x - x*|| = ||L^-1 r|| <= ||r|| / lmin and ||x*|| >= ||b|| / lmax, so

    ||x - x*|| / ||x*|| <= kappa_2(L) ||b - L x|| / ||b||,

with kappa_2 = lmax / lmin computed here from the oracle's matrix.  The
tests assert the residual bound, this solution bound against the oracle's
tight solve (whose own error obeys the same inequality), and print the
error per result.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import meshgen
import oracle
from tests.gpu_helpers import dev, host, make_mesh, rel

pytestmark = pytest.mark.gpu

POI = oracle.OP_POISSON


@pytest.fixture(scope="module")
def fe_ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_11541_amd as fe
    ctx = fe.Context(0)
    yield ctx
    torch.cuda.synchronize()


def _fe():
    import paper_2107_11541_amd as fe
    return fe


CASES = {
    "cfg0": lambda: meshgen.cfg0(),
    "hex16": lambda: meshgen.make_case(16, meshgen.HEX08, 0.15, case_id=61, shuffle=True),
    "hybrid6": lambda: meshgen.make_case(6, meshgen.HYBRID, 0.10, case_id=62, shuffle=True, temperature=True),
}


def oracle_system(c):
    rp, ci, L, f = oracle.assemble(c.coords, c.conn, POI, c.dt, c.u, c.rho, None, types=c.types)
    L, f = L[0].copy(), f[0].copy()
    oracle.dirichlet(rp, ci, L, f, c.dirichlet)
    return rp, ci, L, f


def kappa2(rp, ci, L):
    n = rp.shape[0] - 1
    A = sp.csr_matrix((L, ci, rp), shape=(n, n))
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    lmin = spla.eigsh(A, k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-6)[0]
    assert lmin > 0.0
    return float(lmax / lmin)


def host_true_residual(rp, ci, L, f, x):
    r = f - oracle.spmv(rp, ci, L, x)
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def gpu_solve(fe_ctx, c, rtol, precision):
    fe = _fe()
    import torch
    mesh = make_mesh(fe_ctx, c)
    u, rho = mesh.to_mesh(dev(c.u)), mesh.to_mesh(dev(c.rho))
    L, f, _ = fe.assemble(mesh, fe.POISSON, c.dt, u, rho)
    fe.apply_dirichlet(mesh, L, f)
    x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
    x, info = fe.cg_solve(mesh, L[0], f[0], x=x, rtol=rtol, max_iter=20000, precision=precision)
    xu = host(mesh.to_user(x))
    mesh.close()
    return xu, info


@pytest.mark.parametrize("name", sorted(CASES))
def test_mixed_ir_against_fp64_oracle(fe_ctx, name):
    fe = _fe()
    c = CASES[name]()
    rp, ci, L, f = oracle_system(c)
    kap = kappa2(rp, ci, L)
    xo, st, it_o, rr_o, tr_o = oracle.pcg(rp, ci, L, f, rtol=1e-13, max_iter=50000)
    assert st == oracle.OK
    res_o = host_true_residual(rp, ci, L, f, xo)
    for rtol in (1e-8, 1e-11):
        x, info = gpu_solve(fe_ctx, c, rtol, fe.MIXED)
        res = host_true_residual(rp, ci, L, f, x)
        err = rel(x, xo)
        bound = kap * (res + res_o) * 1.01 + 1e-15
        print(f"{name} N={c.n_nodes} kappa={kap:.1f} rtol={rtol:g}: inner its {info['iterations']}, "
              f"outer {info['outer_iterations']}, host residual {res:.3e} (library {info['true_rel_residual']:.3e}), "
              f"error vs FP64 oracle {err:.3e} <= bound {bound:.3e}", flush=True)
        assert info["status"] == 0
        assert info["outer_iterations"] >= 2          # the refinement ran: FP32 alone cannot reach it
        assert res <= rtol * 1.0001                    # R14, checked on the host
        assert abs(res - info["true_rel_residual"]) <= 1e-3 * res + 1e-16
        assert err <= bound
    # the tight mixed solve reaches the FP64 solution to the stated 1e-8
    assert err <= 1e-8, err


def test_mixed_ir_matches_dense_solve(fe_ctx):
    """cfg0 (1331 unknowns): against numpy's dense LU on the oracle's matrix."""
    fe = _fe()
    c = meshgen.cfg0()
    rp, ci, L, f = oracle_system(c)
    n = c.n_nodes
    A = np.zeros((n, n))
    A[np.repeat(np.arange(n), np.diff(rp)), ci] = L
    xd = np.linalg.solve(A, f)
    x, info = gpu_solve(fe_ctx, c, 1e-11, fe.MIXED)
    err = rel(x, xd)
    print("cfg0 mixed vs dense", err, info, flush=True)
    assert err <= 1e-8


def test_fractional_step_mixed_against_oracle(fe_ctx):
    """The whole fractional step with its pressure solved in mixed precision
    against the oracle's FP64 step: the pressure obeys the solve's bound, the
    corrected velocity follows from it."""
    fe = _fe()
    import torch
    c = meshgen.make_case(6, meshgen.HYBRID, 0.12, case_id=63, shuffle=True, temperature=True)
    c.mu = np.random.default_rng(63).uniform(1e-3, 3e-3, c.n_nodes)
    dt = 0.05
    mesh = make_mesh(fe_ctx, c)
    u, rho, mu = mesh.to_mesh(dev(c.u)), mesh.to_mesh(dev(c.rho)), mesh.to_mesh(dev(c.mu))
    Lg, fg, _ = fe.assemble(mesh, fe.POISSON, dt, u, rho)
    fe.apply_dirichlet(mesh, Lg, fg)
    p = torch.zeros(c.n_nodes, dtype=torch.float64, device="cuda")
    info = fe.fractional_step(mesh, dt, rho, mu, Lg[0].contiguous(), u, p, rtol=1e-10, max_iter=5000,
                              precision=fe.MIXED)
    rp, ci, Lo, fo = oracle.assemble(c.coords, c.conn, POI, dt, c.u, c.rho, None, types=c.types)
    Lo = Lo[0].copy()
    fo = fo[0].copy()
    oracle.dirichlet(rp, ci, Lo, fo, c.dirichlet)
    un, pn, it = oracle.fractional_step(c.coords, c.conn, c.dirichlet, dt, c.u, c.rho, c.mu, (rp, ci, Lo),
                                        rtol=1e-13, types=c.types)
    kap = kappa2(rp, ci, Lo)
    pu = np.empty(c.n_nodes)
    pu[mesh.node_perm] = host(p)
    uu = np.empty((3, c.n_nodes))
    uu[:, mesh.node_perm] = host(u)
    ep, eu = rel(pu, pn), rel(uu, un)
    # the correction is linear in p: once the oracle's step is corrected by
    # -dt M_L^-1 G (p_gpu - p_oracle) at the free nodes, the velocities must
    # agree to FP64 rounding
    _, mass = oracle.residual(c.coords, c.conn, c.u, c.rho, c.mu, c.types)
    free = np.ones(c.n_nodes, bool)
    free[c.dirichlet] = False
    du = np.where(free, -dt * oracle.gradient(c.coords, c.conn, pu - pn, c.types) / mass, 0.0)
    eu_c = rel(uu, un + du)
    print(f"mixed step: cg {info}, kappa {kap:.1f}, pressure error {ep:.3e}, velocity error {eu:.3e}, "
          f"after the pressure difference {eu_c:.3e}", flush=True)
    assert info["cg_true_rel_residual"] <= 1e-10
    # the predictor is FP64 and agrees to ~1e-12, so does the pressure
    # system's right-hand side, and the solve adds at most kappa * residual
    assert ep <= kap * (1e-10 + 1e-12) * 1.01
    assert eu_c <= 1e-11
    mesh.close()
