/* oracle_check.c -- runs the oracle (oracle/feoracle.c) under
 * AddressSanitizer / UndefinedBehaviorSanitizer: pattern, every assembly
 * operator, the block operator, element vectors, Dirichlet elimination and
 * PCG on small HEX08, TET04 and mixed meshes.  Test infrastructure: built and
 * run by tests/test_sanitizers_cpu.py. */
#include "../../oracle/feoracle.c"
#include "meshes.h"

int main(void)
{
    int fails = 0;
    for (int kind = 0; kind < 3; ++kind) {
        SanMesh m = san_cube(3, kind);
        const int64_t N = m.n_nodes, E = m.n_elems;
        int32_t *rowptr = malloc(sizeof(int32_t) * (size_t)(N + 1));
        const int64_t nnz = or_pattern_typed(m.stride, m.types, N, E, m.conn, rowptr, NULL);
        int32_t *colidx = malloc(sizeof(int32_t) * (size_t)nnz);
        or_pattern_typed(m.stride, m.types, N, E, m.conn, rowptr, colidx);
        double *u = malloc(sizeof(double) * 3 * (size_t)N), *rho = malloc(sizeof(double) * (size_t)N);
        double *mu = malloc(sizeof(double) * (size_t)N), *Y = malloc(sizeof(double) * 2 * (size_t)N);
        for (int64_t i = 0; i < 3 * N; ++i) u[i] = san_uniform() - 0.5;
        for (int64_t i = 0; i < N; ++i) {
            rho[i] = 0.2 + san_uniform();
            mu[i] = 1e-3;
            Y[i] = san_uniform();
            Y[N + i] = san_uniform();
        }
        const double D[2] = {1e-5, 1e-4};
        double *vals = malloc(sizeof(double) * 9 * (size_t)nnz), *rhs = malloc(sizeof(double) * 9 * (size_t)N);
        int64_t bad;
        double mdet;
        for (int op = 0; op < 3; ++op) {
            const int st = or_assemble_typed(m.stride, m.types, N, m.coords, E, m.conn, op, 0.05, u, rho, mu, 2, Y, D,
                                             rowptr, colidx, vals, rhs, &bad, &mdet);
            fails += st != 0;
        }
        for (int form = 0; form < 4; ++form)
            fails += or_assemble_block(m.stride, m.types, N, m.coords, E, m.conn, form, 0.05, u, rho, mu, rowptr,
                                       colidx, vals, rhs, &bad, &mdet) != 0;
        fails += or_element_vectors(m.stride, m.types, N, m.coords, E, m.conn, 0, 3, u, rho, mu, NULL, NULL, 0.0,
                                    rhs, &bad, &mdet) != 0;
        /* Poisson system, all boundary-free nodes left free: Dirichlet on node 0 and the last node */
        fails += or_assemble_typed(m.stride, m.types, N, m.coords, E, m.conn, 2, 0.05, u, rho, mu, 0, NULL, NULL,
                                   rowptr, colidx, vals, rhs, &bad, &mdet) != 0;
        const int32_t dn[2] = {0, (int32_t)(N - 1)};
        fails += or_dirichlet(N, rowptr, colidx, vals, rhs, 2, dn, NULL) != 0;
        double *x = calloc((size_t)N, sizeof(double)), info[3];
        const int st = or_pcg(N, rowptr, colidx, vals, rhs, x, 1e-10, 10000, info);
        fails += st != 0;
        free(x);
        free(vals);
        free(rhs);
        free(u);
        free(rho);
        free(mu);
        free(Y);
        free(rowptr);
        free(colidx);
        san_free(&m);
    }
    printf("oracle_check: %d failures\n", fails);
    return fails ? 1 : 0;
}
