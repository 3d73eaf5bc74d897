/*
 * feoracle_omp.c -- the oracle of feoracle.c run on every host core, for
 * timing only.
 *
 * TEST INFRASTRUCTURE ONLY, like feoracle.c: the benchmark's CPU-baseline
 * leg times it; parity tests use the serial build.  It includes feoracle.c
 * and reuses its element computation (element_terms, element_scatter), its
 * Dirichlet elimination and its PCG recurrence step by step; what changes
 * is the order of the element loop and the threads:
 *
 *  - elements are greedily coloured so that no two elements of one colour
 *    share a node; colours run one after the other, the elements of a colour
 *    in parallel (each CSR row receives the contributions of one colour from
 *    one element, so there is no race and, for a fixed colouring, the sums
 *    are deterministic);
 *  - the PCG's SpMV and vector updates run in parallel over rows, and its
 *    dot products add fixed per-thread partial sums in thread order.
 *
 * Build: gcc -O3 -march=x86-64-v3 -fopenmp -ffp-contract=off -fPIC -shared.
 */
#include <omp.h>

#include "feoracle.c"

int or_omp_threads(void) { return omp_get_max_threads(); }

/*
 * Greedy colouring of the elements: element e (in order) takes the smallest
 * colour that none of the elements sharing one of its nodes already has.
 * order[n_elems] receives the elements by colour (element order within a
 * colour), colour_ptr[n_colours + 1] the colour boundaries (sized
 * OR_OMP_MAX_COLOURS + 1).  Returns the number of colours, or -1 if more
 * than OR_OMP_MAX_COLOURS are needed or memory runs out.
 */
#define OR_OMP_MAX_COLOURS 64
int or_omp_colour(int stride, const uint8_t *types, int64_t n_nodes, int64_t n_elems, const int32_t *conn,
                  int32_t *order, int32_t *colour_ptr)
{
    uint64_t *used = calloc((size_t)n_nodes, sizeof(uint64_t));
    int8_t *col = malloc((size_t)n_elems);
    if (!used || !col) {
        free(used);
        free(col);
        return -1;
    }
    int nc = 0;
    int64_t count[OR_OMP_MAX_COLOURS] = {0};
    for (int64_t e = 0; e < n_elems; ++e) {
        const int nen = elem_nen(stride, types, e);
        const int32_t *c = conn + e * stride;
        uint64_t m = 0;
        for (int a = 0; a < nen; ++a) m |= used[c[a]];
        if (m == ~(uint64_t)0) {
            free(used);
            free(col);
            return -1;
        }
        int k = 0;
        while (m & ((uint64_t)1 << k)) ++k;
        col[e] = (int8_t)k;
        ++count[k];
        if (k + 1 > nc) nc = k + 1;
        for (int a = 0; a < nen; ++a) used[c[a]] |= (uint64_t)1 << k;
    }
    colour_ptr[0] = 0;
    for (int k = 0; k < nc; ++k) colour_ptr[k + 1] = colour_ptr[k] + (int32_t)count[k];
    int64_t fill[OR_OMP_MAX_COLOURS];
    for (int k = 0; k < nc; ++k) fill[k] = colour_ptr[k];
    for (int64_t e = 0; e < n_elems; ++e) order[fill[col[e]]++] = (int32_t)e;
    free(used);
    free(col);
    return nc;
}

/* or_assemble_typed with the colour-ordered parallel element loop. */
int or_omp_assemble(int stride, const uint8_t *types, int64_t n_nodes, const double *coords, int64_t n_elems,
                    const int32_t *conn, int op, double dt, const double *u, const double *rho, const double *mu,
                    int n_scalars, const double *Y, const double *D, const int32_t *rowptr,
                    const int32_t *colidx, int n_colours, const int32_t *order, const int32_t *colour_ptr,
                    double *values, double *rhs, int64_t *bad_elem, double *min_det)
{
    static RefSet R;
    ref_set(&R);
    AsmOp A;
    int st = asm_begin(&A, stride, types, n_nodes, coords, n_elems, conn, op, dt, u, rho, mu, n_scalars, Y, D,
                       rowptr, values, rhs);
    if (st != OR_OK) return st;
    double md = INFINITY;
    int64_t bad = INT64_MAX;
    int fail = 0;
    for (int k = 0; k < n_colours; ++k) {
#pragma omp parallel reduction(min : md, bad) reduction(| : fail)
        {
            double M[MAXN][MAXN], Cm[MAXN][MAXN], K[MAXS][MAXN][MAXN], B[MAXS][MAXN];
#pragma omp for schedule(static)
            for (int64_t q = colour_ptr[k]; q < colour_ptr[k + 1]; ++q) {
                const int64_t e = order[q];
                if (element_terms(&R, &A, e, M, Cm, K, B, &md) != OR_OK) {
                    if (e < bad) bad = e;
                    continue;
                }
                if (element_scatter(&A, e, rowptr, colidx, M, Cm, K, B, values, rhs) != OR_OK) fail = 1;
            }
        }
    }
    *min_det = md;
    *bad_elem = bad == INT64_MAX ? -1 : bad;
    if (fail) return OR_EINVAL;
    return bad == INT64_MAX ? OR_OK : OR_EBADELEM;
}

/* or_dirichlet with its row loops in parallel (every row is independent). */
int or_omp_dirichlet(int64_t n_nodes, const int32_t *rowptr, const int32_t *colidx, double *values, double *rhs,
                     int64_t n_dir, const int32_t *dnodes, const double *g)
{
    unsigned char *isd = calloc((size_t)n_nodes, 1);
    if (!isd) return OR_ENOMEM;
    for (int64_t k = 0; k < n_dir; ++k) {
        if (dnodes[k] < 0 || dnodes[k] >= n_nodes) {
            free(isd);
            return OR_EINVAL;
        }
        isd[dnodes[k]] = 1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_nodes; ++i) {
        if (isd[i]) {
            double diag = 0.0;
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                if (colidx[p] == i) diag = values[p];
                else values[p] = 0.0;
            }
            rhs[i] = diag * (g ? g[i] : 0.0);
        } else {
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                int32_t j = colidx[p];
                if (isd[j]) {
                    double gj = g ? g[j] : 0.0;
                    rhs[i] -= values[p] * gj;
                    values[p] = 0.0;
                }
            }
        }
    }
    free(isd);
    return OR_OK;
}

static void par_spmv(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *vals, const double *x,
                     double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s += vals[p] * x[colidx[p]];
        y[i] = s;
    }
}

/* x . y: each thread sums a fixed contiguous range, the partials are added
 * in thread order (deterministic for a given thread count). */
static double par_dot(int64_t n, const double *x, const double *y)
{
    double part[256] = {0};
    int nt = 1;
#pragma omp parallel
    {
        const int t = omp_get_thread_num();
#pragma omp single
        nt = omp_get_num_threads();
        const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += x[i] * y[i];
        if (t < 256) part[t] = s;
    }
    double s = 0.0;
    for (int t = 0; t < nt && t < 256; ++t) s += part[t];
    return s;
}

/* or_pcg's recurrence with its kernels in parallel. */
int or_omp_pcg(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *vals, const double *b,
               double *x, double rtol, int max_iter, double *info)
{
    if (omp_get_max_threads() > 256) omp_set_num_threads(256);
    double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    double *dinv = malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q || !dinv) return OR_ENOMEM;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (colidx[k] == i) d = vals[k];
        dinv[i] = 1.0 / d;
    }
    par_spmv(n, rowptr, colidx, vals, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - q[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double bnorm = sqrt(par_dot(n, b, b));
    double rho = par_dot(n, r, z);
    int status = OR_ENOCONV, it = 0;
    double rnorm = sqrt(par_dot(n, r, r));
    if (rtol > 0.0 && rnorm <= rtol * bnorm) status = OR_OK;
    while (status == OR_ENOCONV && it < max_iter) {
        par_spmv(n, rowptr, colidx, vals, p, q);
        double pq = par_dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = OR_EBREAKDOWN;
            break;
        }
        double alpha = rho / pq;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] += -alpha * q[i];
        }
        ++it;
        rnorm = sqrt(par_dot(n, r, r));
        if (rtol > 0.0 && rnorm <= rtol * bnorm) {
            status = OR_OK;
            break;
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rho1 = par_dot(n, r, z);
        double beta = rho1 / rho;
        rho = rho1;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (rtol <= 0.0 && status == OR_ENOCONV && it == max_iter) status = OR_OK;
    par_spmv(n, rowptr, colidx, vals, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
    info[0] = it;
    info[1] = bnorm > 0.0 ? rnorm / bnorm : rnorm;
    info[2] = bnorm > 0.0 ? sqrt(par_dot(n, q, q)) / bnorm : sqrt(par_dot(n, q, q));
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    return status;
}
