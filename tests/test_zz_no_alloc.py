"""GPU tests of fe_cg_solve_noalloc, the allocation-free form of the FP64
Jacobi-PCG solve (Algorithm 1, last step): its work vectors live in the
library's fixed device area instead of buffers allocated on the mesh.

Two calls in a row on one device share that area; the second, on a smaller
system, must not see anything the first left behind.  Each call is compared
with fe_cg_solve(FE_FP64) on the same system.  On these symmetric matrices
fe_cg_solve runs the symmetric SpMV and the allocation-free form the general
one, so the two agree to rounding: fixed-count iterates to 1e-10 (the bound
of the PCG iterates against the oracle's), converged solutions to the CG
bound.  On a matrix that is not symmetric both run the general SpMV and
agree bitwise.  The solutions are also checked against the FP64 oracle's
solve to the CG bound.
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


def _system(fe, ctx, c):
    mesh = fe.Mesh(ctx, HEX, c.coords, c.conn, c.dirichlet)
    u, rho = mesh.to_mesh(dev(c.u)), mesh.to_mesh(dev(c.rho))
    L, f, _ = fe.assemble(mesh, fe.POISSON, c.dt, u, rho)
    fe.apply_dirichlet(mesh, L, f)
    return mesh, L[0].contiguous(), f[0].contiguous()


def _oracle_solution(c):
    rp, ci, Lo, fo = oracle.assemble(c.coords, c.conn, oracle.OP_POISSON, c.dt, c.u, c.rho, None)
    Lo, fo = Lo[0].copy(), fo[0].copy()
    oracle.dirichlet(rp, ci, Lo, fo, c.dirichlet)
    xo, st, it, rr, tr = oracle.pcg(rp, ci, Lo, fo, rtol=1e-13, max_iter=20000)
    return xo


@pytest.mark.parametrize("rtol,max_iter", [(1e-10, 20000), (0.0, 37)])
def test_noalloc_equals_cg_solve_on_two_calls_in_a_row(fe_ctx, rtol, max_iter):
    import torch
    import paper_2107_11541_amd as fe
    cases = [meshgen.make_case(24, HEX, 0.15, case_id=301, shuffle=True),
             meshgen.make_case(10, HEX, 0.10, case_id=302, shuffle=True)]   # second call: smaller
    for c in cases:
        print(f"hex {c.n}^3 N={c.n_nodes} rtol={rtol} max_iter={max_iter}", flush=True)
        mesh, L, f = _system(fe, fe_ctx, c)
        x0 = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
        x_na, info_na = fe.cg_solve_noalloc(mesh, L, f, x=x0.clone(), rtol=rtol, max_iter=max_iter)
        x_ref, info_ref = fe.cg_solve(mesh, L, f, x=x0.clone(), rtol=rtol, max_iter=max_iter)
        torch.cuda.synchronize()
        assert info_na["status"] == 0
        assert info_ref["symmetric_spmv"] and not info_na["symmetric_spmv"]
        if rtol == 0.0:
            assert info_na["iterations"] == info_ref["iterations"] == max_iter
            assert rel(host(x_na), host(x_ref)) <= 1e-10
            assert abs(info_na["rel_residual"] - info_ref["rel_residual"]) <= 1e-8 * info_ref["rel_residual"]
        else:
            assert abs(info_na["iterations"] - info_ref["iterations"]) <= 2
            assert info_ref["true_rel_residual"] <= 2 * rtol
            assert rel(host(x_na), host(x_ref)) <= 1e-7
        if rtol > 0.0:
            # against the oracle's FP64 solve, in user numbering
            xo = _oracle_solution(c)
            xu = host(mesh.to_user(x_na))
            assert info_na["true_rel_residual"] <= 2 * rtol
            assert rel(xu, xo) <= 1e-7
        mesh.close()


def test_noalloc_bitwise_equals_cg_solve_on_a_nonsymmetric_matrix(fe_ctx):
    """The off-diagonal entries of one row scaled by 1 + 1e-9 (beyond the
    symmetric-pair check): fe_cg_solve runs the general SpMV, the same kernels with the same
    launch shapes as the allocation-free form, so x, the iteration count and
    the residuals agree bitwise."""
    import torch
    import paper_2107_11541_amd as fe
    c = meshgen.make_case(12, HEX, 0.15, case_id=303, shuffle=True)
    mesh, L, f = _system(fe, fe_ctx, c)
    rp, ci = mesh.pattern_host()
    rows = np.repeat(np.arange(mesh.n_nodes), np.diff(rp))
    # the off-diagonal entries of the row holding the off-diagonal entry of
    # largest magnitude (Dirichlet rows hold zeros), not their transposes
    q = int(np.argmax(np.where(ci != rows, np.abs(host(L)), 0.0)))
    r = rows[q]
    off = torch.tensor([p for p in range(rp[r], rp[r + 1]) if ci[p] != r], dtype=torch.int64, device=L.device)
    L[off] *= 1.0 + 1e-9
    for rtol, max_iter in ((1e-10, 20000), (0.0, 37)):
        x_na, info_na = fe.cg_solve_noalloc(mesh, L, f, rtol=rtol, max_iter=max_iter)
        x_ref, info_ref = fe.cg_solve(mesh, L, f, rtol=rtol, max_iter=max_iter)
        torch.cuda.synchronize()
        assert not info_ref["symmetric_spmv"] and not info_na["symmetric_spmv"]
        assert info_na["iterations"] == info_ref["iterations"]
        assert info_na["rel_residual"] == info_ref["rel_residual"]
        assert info_na["true_rel_residual"] == info_ref["true_rel_residual"]
        assert torch.equal(x_na, x_ref)
    mesh.close()


def test_noalloc_nonzero_initial_guess(fe_ctx):
    import torch
    import paper_2107_11541_amd as fe
    c = meshgen.make_case(12, HEX, 0.10, case_id=303, shuffle=True)
    mesh, L, f = _system(fe, fe_ctx, c)
    g = torch.Generator().manual_seed(5)
    x0 = torch.rand(mesh.n_nodes, generator=g, dtype=torch.float64).cuda()
    x_na, i_na = fe.cg_solve_noalloc(mesh, L, f, x=x0.clone(), rtol=1e-9, max_iter=5000)
    x_ref, i_ref = fe.cg_solve(mesh, L, f, x=x0.clone(), rtol=1e-9, max_iter=5000)
    assert i_ref["symmetric_spmv"] and not i_na["symmetric_spmv"]
    assert abs(i_na["iterations"] - i_ref["iterations"]) <= 2
    assert i_na["true_rel_residual"] <= 2e-9 and i_ref["true_rel_residual"] <= 2e-9
    assert rel(host(x_na), host(x_ref)) <= 1e-6
    mesh.close()


def test_noalloc_rejects_sizes_beyond_the_area(fe_ctx):
    import torch
    import paper_2107_11541_amd as fe
    c = meshgen.make_case(4, HEX, 0.10, case_id=304, shuffle=True)
    mesh, L, f = _system(fe, fe_ctx, c)
    x = torch.zeros(mesh.n_nodes, dtype=torch.float64, device="cuda")
    # 4 doubles of per-iteration scalars per iteration: 3 M iterations need
    # more than the 64 MiB area
    with pytest.raises(fe.FeError) as ei:
        fe.cg_solve_noalloc(mesh, L, f, x=x, rtol=1e-8, max_iter=3_000_000)
    assert ei.value.status == 2   # FE_ENOMEM
    assert "fixed area" in str(ei.value)
    # the area is still usable afterwards
    x, info = fe.cg_solve_noalloc(mesh, L, f, x=x, rtol=1e-10, max_iter=1000)
    assert info["status"] == 0 and info["true_rel_residual"] <= 2e-10
    mesh.close()
