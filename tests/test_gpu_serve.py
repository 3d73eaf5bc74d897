"""GPU tests of the serving runtime (fe_serve_*): continuous batching of
momentum + Poisson assembly, Dirichlet elimination and the Jacobi-PCG
pressure solve over many independent meshes.

A served request must give what the same request gives alone: bitwise the
same solution and iteration count, because its work-group counts and
summation orders do not depend on the other requests in a batch, and
bitwise what the plain API's general-SpMV solve (fe_cg_solve_noalloc)
gives for the same system.  Against
the FP64 oracle: the momentum right-hand side to 1e-12 and the pressure
solution to the CG bound (both solved to rtol 1e-10).
"""
import numpy as np
import pytest

import meshgen
import oracle

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
    ctx.close()


def _fe():
    import paper_2107_11541_amd as fe
    return fe


def _case(n, req, jitter=0.10):
    return meshgen.make_case(n, HEX, jitter, case_id=3, sub=req, shuffle=True, name=f"serve-{req}-{n}")


def _submit(srv, case, rtol=1e-10, max_iter=5000, want_mom_rhs=False):
    return srv.submit(HEX, case.coords, case.conn, case.dirichlet, case.dt, case.u, case.rho, case.mu,
                      rtol=rtol, max_iter=max_iter, want_mom_rhs=want_mom_rhs)


def _oracle_solution(case, rtol):
    rp, ci, L, f = oracle.assemble(case.coords, case.conn, oracle.OP_POISSON, case.dt, case.u, case.rho, None)
    L, f = L[0].copy(), f[0].copy()
    oracle.dirichlet(rp, ci, L, f, case.dirichlet)
    x, st, it, rr, tr = oracle.pcg(rp, ci, L, f, rtol=rtol)
    return x, it


def test_served_requests_match_oracle(fe_ctx):
    fe = _fe()
    srv = fe.Server(fe_ctx, hbm_budget=1 << 30, max_slots=4, host_threads=2)
    cases = [_case(n, 100 + i) for i, n in enumerate((3, 5, 8, 6))]
    tickets = [_submit(srv, c, want_mom_rhs=True) for c in cases]
    for c, t in zip(cases, tickets):
        r = srv.wait(t)
        print(c.name, r["status_name"], r["iterations"], r["true_rel_residual"], flush=True)
        assert r["status"] == 0, r["message"]
        assert r["true_rel_residual"] <= 2e-10
        xo, it = _oracle_solution(c, 1e-10)
        err = np.linalg.norm(r["x"] - xo) / np.linalg.norm(xo)
        assert err <= 1e-8, err
        assert abs(r["iterations"] - it) <= max(2, 0.1 * it)
        _, _, _, Bo = oracle.assemble(c.coords, c.conn, oracle.OP_MOMENTUM, c.dt, c.u, c.rho, c.mu)
        rerr = np.linalg.norm(r["mom_rhs"] - Bo) / np.linalg.norm(Bo)
        assert rerr <= 1e-12, rerr
    srv.close()


def test_served_alone_equals_served_in_a_mix(fe_ctx):
    fe = _fe()
    probe = _case(7, 200)
    srv = fe.Server(fe_ctx, hbm_budget=1 << 30, max_slots=1, host_threads=1)
    alone = srv.wait(_submit(srv, probe))
    srv.close()
    srv = fe.Server(fe_ctx, hbm_budget=1 << 30, max_slots=8, host_threads=4)
    rng = np.random.default_rng(5)
    others = [_case(int(n), 300 + i) for i, n in enumerate(rng.integers(3, 11, size=12))]
    tk = [_submit(srv, c) for c in others[:6]]
    tp = _submit(srv, probe)
    tk += [_submit(srv, c) for c in others[6:]]
    mixed = srv.wait(tp)
    rest = [srv.wait(t) for t in tk]
    st = srv.stats()
    srv.close()
    print("alone", alone["iterations"], "mixed", mixed["iterations"], "stats", st, flush=True)
    assert alone["status"] == 0 and mixed["status"] == 0
    assert all(r["status"] == 0 for r in rest)
    assert mixed["iterations"] == alone["iterations"]
    assert np.array_equal(mixed["x"], alone["x"])
    assert mixed["true_rel_residual"] == alone["true_rel_residual"]
    assert st["completed"] == 13
    assert st["mean_batch"] > 1.0


def test_served_equals_plain_api(fe_ctx):
    """The batched kernels and the one-system PCG with the general SpMV
    (fe_cg_solve_noalloc) give bitwise the same x; fe_cg_solve, which runs
    the symmetric SpMV on this matrix, agrees to rounding."""
    fe = _fe()
    import torch
    from tests.gpu_helpers import dev, host
    from tests.gpu_helpers import rel
    case = _case(9, 400)
    srv = fe.Server(fe_ctx, hbm_budget=1 << 30, max_slots=2, host_threads=1)
    served = srv.wait(_submit(srv, case, rtol=1e-9))
    srv.close()
    mesh = fe.Mesh(fe_ctx, HEX, case.coords, case.conn, case.dirichlet, coloured=True)
    u, rho = mesh.to_mesh(dev(case.u)), mesh.to_mesh(dev(case.rho))
    L, f, _ = fe.assemble(mesh, fe.POISSON, case.dt, u, rho)
    fe.apply_dirichlet(mesh, L, f)
    x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
    x, info = fe.cg_solve_noalloc(mesh, L[0], f[0], x=x, rtol=1e-9, max_iter=5000)
    xu = host(mesh.to_user(x))
    xs, infos = fe.cg_solve(mesh, L[0], f[0], rtol=1e-9, max_iter=5000)
    xsu = host(mesh.to_user(xs))
    mesh.close()
    assert served["iterations"] == info["iterations"]
    assert np.array_equal(served["x"], xu)
    assert infos["symmetric_spmv"] and not info["symmetric_spmv"]
    assert abs(infos["iterations"] - info["iterations"]) <= 2
    assert rel(xsu, xu) <= 1e-7


def test_bad_element_fails_only_its_request(fe_ctx):
    fe = _fe()
    good = _case(5, 500)
    bad = meshgen.make_case(4, HEX, 0.0, case_id=43, shuffle=True)
    c = bad.conn[17]
    X = bad.coords.copy()
    X[[c[0], c[6]]] = X[[c[6], c[0]]]
    bad.coords = X
    srv = fe.Server(fe_ctx, hbm_budget=1 << 30, max_slots=4, host_threads=2)
    tb = _submit(srv, bad)
    tg = _submit(srv, good)
    rb, rg = srv.wait(tb), srv.wait(tg)
    srv.close()
    assert rb["status"] == 4, rb
    assert rb["first_bad_elem"] >= 0
    assert rg["status"] == 0 and rg["true_rel_residual"] <= 2e-10


def test_budget_and_iteration_limits(fe_ctx):
    fe = _fe()
    srv = fe.Server(fe_ctx, hbm_budget=2 << 20, max_slots=2, host_threads=1)
    r = srv.wait(_submit(srv, _case(20, 600)))
    assert r["status"] == 2, r          # FE_ENOMEM: larger than the whole arena
    srv.close()
    srv = fe.Server(fe_ctx, hbm_budget=256 << 20, max_slots=2, host_threads=1)
    r = srv.wait(_submit(srv, _case(6, 601), rtol=1e-12, max_iter=3))
    assert r["status"] == 5 and r["iterations"] == 3, r     # FE_ENOCONV, x still written
    assert np.isfinite(r["x"]).all() and np.abs(r["x"]).max() > 0
    r = srv.wait(_submit(srv, _case(6, 601), rtol=1e-12, max_iter=0))
    assert r["status"] == 5 and r["iterations"] == 0, r
    srv.close()


def test_many_requests_small_arena(fe_ctx):
    """More requests than slots and an arena that holds only a few at once:
    admission waits for space, and every request still completes."""
    fe = _fe()
    rng = np.random.default_rng(11)
    cases = [_case(int(n), 700 + i) for i, n in enumerate(rng.integers(3, 15, size=30))]
    srv = fe.Server(fe_ctx, hbm_budget=48 << 20, max_slots=6, host_threads=4)
    tickets = [_submit(srv, c, rtol=1e-8) for c in cases]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print("stats", st, flush=True)
    assert all(r["status"] == 0 for r in res), [r["message"] for r in res if r["status"]]
    assert all(r["true_rel_residual"] <= 1.5e-8 for r in res)
    assert st["completed"] == 30


def test_hybrid_and_prism_requests_in_a_mix(fe_ctx):
    """Hybrid (all four types) and prism meshes served in one batch with
    hexahedral ones: each equals the plain API's general-SpMV solve
    (fe_cg_solve_noalloc) on the same mesh bitwise and the oracle's pressure
    to the CG bound."""
    fe = _fe()
    import torch
    from tests.gpu_helpers import dev, host, make_mesh
    hyb = meshgen.make_case(6, meshgen.HYBRID, 0.1, case_id=3, sub=700, shuffle=True)
    pen = meshgen.make_case(5, meshgen.PEN06, 0.1, case_id=3, sub=701, shuffle=True)
    hexes = [_case(n, 702 + i) for i, n in enumerate((4, 7))]
    srv = fe.Server(fe_ctx, hbm_budget=1 << 30, max_slots=4, host_threads=2)
    t_h = srv.submit(fe.HYBRID, hyb.coords, hyb.conn, hyb.dirichlet, hyb.dt, hyb.u, hyb.rho, hyb.mu,
                     rtol=1e-10, max_iter=5000, types=hyb.types)
    t_p = srv.submit(fe.PEN06, pen.coords, pen.conn, pen.dirichlet, pen.dt, pen.u, pen.rho, pen.mu,
                     rtol=1e-10, max_iter=5000)
    t_x = [_submit(srv, c) for c in hexes]
    res = {"hyb": srv.wait(t_h), "pen": srv.wait(t_p)}
    for t in t_x:
        assert srv.wait(t)["status"] == 0
    srv.close()
    for key, case in (("hyb", hyb), ("pen", pen)):
        r = res[key]
        assert r["status"] == 0, (key, r["message"])
        mesh = make_mesh(fe_ctx, case, coloured=True)   # the served form
        u, rho = mesh.to_mesh(dev(case.u)), mesh.to_mesh(dev(case.rho))
        L, f, _ = fe.assemble(mesh, fe.POISSON, case.dt, u, rho)
        fe.apply_dirichlet(mesh, L, f)
        x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
        x, info = fe.cg_solve_noalloc(mesh, L[0], f[0], x=x, rtol=1e-10, max_iter=5000)
        xu = host(mesh.to_user(x))
        mesh.close()
        assert r["iterations"] == info["iterations"]
        assert np.array_equal(r["x"], xu), key
        rp, ci, Lo, fo = oracle.assemble(case.coords, case.conn, oracle.OP_POISSON, case.dt, case.u, case.rho,
                                         None, types=case.types)
        Lo, fo = Lo[0].copy(), fo[0].copy()
        oracle.dirichlet(rp, ci, Lo, fo, case.dirichlet)
        xo, st, it, _, _ = oracle.pcg(rp, ci, Lo, fo, rtol=1e-10)
        assert np.linalg.norm(r["x"] - xo) <= 1e-8 * np.linalg.norm(xo)
