"""GPU tests of how a Jacobi-PCG solve stops (Algorithm 1, last step).

The third step of iteration k applies x += alpha_k p_k in every work-group
and, when ||r_{k+1}|| <= rtol ||b||, records the stop for the following
launches.  A stop found in that same launch must not keep any of its
work-groups from applying the x update, however late they are scheduled:
a solve that converges after k iterations must give bitwise the x of a
solve told to run exactly k iterations (the same arithmetic on the same
data), on a one-system launch and on the serving runtime's batched launches,
whose work-groups outnumber what the GPU holds at once.
"""
import numpy as np
import pytest

import meshgen
import oracle
from tests.gpu_helpers import dev, host, rel

pytestmark = pytest.mark.gpu

HEX = meshgen.HEX08


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


def _poisson(fe, mesh, c):
    u, rho = mesh.to_mesh(dev(c.u)), mesh.to_mesh(dev(c.rho))
    L, f, _ = fe.assemble(mesh, fe.POISSON, c.dt, u, rho)
    fe.apply_dirichlet(mesh, L, f)
    return L[0].contiguous(), f[0].contiguous()


@pytest.mark.parametrize("n,rtol", [(64, 1e-6), (24, 1e-9)])
def test_converged_solve_equals_fixed_iteration_solve(fe_ctx, n, rtol):
    fe = _fe()
    import torch
    c = meshgen.make_case(n, HEX, 0.15, case_id=70 + n, shuffle=True)
    print(f"hex {n}^3 N={c.n_nodes} rtol={rtol}", flush=True)
    mesh = fe.Mesh(fe_ctx, HEX, c.coords, c.conn, c.dirichlet)
    L, f = _poisson(fe, mesh, c)
    outs = {}
    for label, profiled in (("graph", False), ("eager", True)):
        fe_ctx.profile(profiled)
        x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
        x, info = fe.cg_solve(mesh, L, f, x=x, rtol=rtol, max_iter=20000)
        assert info["status"] == 0 and info["rel_residual"] <= rtol
        it = info["iterations"]
        xf = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
        xf, infof = fe.cg_solve(mesh, L, f, x=xf, rtol=0.0, max_iter=it)
        assert infof["iterations"] == it
        print(label, "iterations", it, "max |x - x_fixed|", float((x - xf).abs().max()), flush=True)
        assert torch.equal(x, xf), label
        outs[label] = (host(x), it)
    fe_ctx.profile(False)
    assert outs["graph"][1] == outs["eager"][1]
    assert np.array_equal(outs["graph"][0], outs["eager"][0])
    if n <= 24:
        # the oracle's PCG, stopped after the same number of iterations: the
        # same recurrence, iterates equal to rounding
        rp, ci, Lo, fo = oracle.assemble(c.coords, c.conn, oracle.OP_POISSON, c.dt, c.u, c.rho, None)
        Lo, fo = Lo[0].copy(), fo[0].copy()
        oracle.dirichlet(rp, ci, Lo, fo, c.dirichlet)
        xo, st, ito, rro, tro = oracle.pcg(rp, ci, Lo, fo, rtol=0.0, max_iter=outs["graph"][1])
        xu = np.empty(c.n_nodes)
        xu[mesh.node_perm] = outs["graph"][0]
        print("vs oracle after", ito, "iterations:", rel(xu, xo), flush=True)
        assert rel(xu, xo) <= 1e-10
    mesh.close()


def test_served_batch_beyond_residency_equals_plain_api(fe_ctx):
    """Six 56^3..64^3 requests in one server: their batched update launches
    carry ~3000 work-groups of 256 threads, more than the 2048 a 256-CU GPU
    holds at once.  Each served x must be bitwise the plain API's solve
    with the general SpMV (fe_cg_solve_noalloc)."""
    fe = _fe()
    import torch
    sides = (64, 56, 60, 64, 58, 62)
    cases = [meshgen.make_case(n, HEX, 0.10, case_id=3, sub=900 + i, shuffle=True, name=f"big-{i}-{n}")
             for i, n in enumerate(sides)]
    srv = fe.Server(fe_ctx, hbm_budget=8 << 30, max_slots=8, host_threads=6)
    tickets = [srv.submit(HEX, c.coords, c.conn, c.dirichlet, c.dt, c.u, c.rho, c.mu, rtol=1e-8, max_iter=20000)
               for c in cases]
    served = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print("served", [(r["status"], r["iterations"]) for r in served], "stats", st, flush=True)
    assert st["mean_batch"] > 1.0
    for c, r in zip(cases, served):
        assert r["status"] == 0, r["message"]
        mesh = fe.Mesh(fe_ctx, HEX, c.coords, c.conn, c.dirichlet, coloured=True)   # the served form
        L, f = _poisson(fe, mesh, c)
        x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
        x, info = fe.cg_solve_noalloc(mesh, L, f, x=x, rtol=1e-8, max_iter=20000)
        xu = host(mesh.to_user(x))
        mesh.close()
        print(c.name, "served", r["iterations"], "plain", info["iterations"], flush=True)
        assert r["iterations"] == info["iterations"]
        assert np.array_equal(r["x"], xu)
        assert r["true_rel_residual"] <= 1e-8
