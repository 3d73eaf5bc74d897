/*
 * feoracle.c -- plain, serial FP64 reference of the finite-element hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.  Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction,
 * so every product and sum is rounded as written).
 *
 * What it computes (paper: Oyarzun, Mira, Houzeaux, "Performance assessment
 * of CUDA and OpenACC in large scale combustion simulations"):
 *
 *  - Element-by-element Galerkin assembly (Section 4.2, Listing 1: an outer
 *    loop over elements, an inner loop over Gauss points and node pairs that
 *    accumulates Ae(a,b) from shape functions N and the Jacobian weight).
 *    The operator is the momentum operator of Eq. (1) in a reduced form
 *    (the paper gives no discretisation): density-weighted mass / dt +
 *    Galerkin advective convection linearised about the nodal velocity +
 *    Laplacian-form viscous term (one scalar operator shared by the three
 *    components), and its right-hand side M_rho u / dt;
 *    a scalar-transport variant with coefficient rho*D_k; and the
 *    constant-coefficient pressure Laplacian assembled once before the time
 *    loop (Algorithm 1, first step).
 *  - Scatter of the elemental matrices into CSR (Section 4.2), in element
 *    order: A = sum_e P_e^T A_e P_e.
 *  - Symmetric Dirichlet elimination for the pressure system.
 *  - Jacobi-preconditioned conjugate gradients for the pressure equation
 *    (Algorithm 1, last step; Section 5.2 names its SpMV, AXPY and dot
 *    kernels).
 *
 * Reference elements (the paper's meshes mix tetrahedra, pyramids, prisms
 * and hexahedra, Sections 3 and 4.2; it gives no element formulation, so
 * these are the standard isoparametric ones):
 *  - HEX08 trilinear with the 2x2x2 Gauss rule at +-1/sqrt3 (weights 1, xi
 *    fastest);
 *  - TET04 linear with the 4-point rule at the barycentric permutations of
 *    (b,a,a,a), a = (5-sqrt5)/20, b = 1-3a, weights 1/24;
 *  - PEN06 (prism) linear-triangle x linear-line with the 3-point triangle
 *    rule x 2-point Gauss-Legendre (6 points);
 *  - PYR05 (pyramid) with the rational basis that is bilinear on the base
 *    and linear on the triangular faces, and the 8-point conical product
 *    rule (2x2 Gauss-Legendre in collapsed coordinates x 2-point
 *    Gauss-Jacobi for the weight (1-zeta)^2).
 * Jacobian J_ij = d x_i / d xi_j; grad N = J^-T grad_ref N.  A mesh may mix
 * types: the typed entry points take a padded connectivity of stride S and
 * one node count (4, 5, 6 or 8) per element.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2
#define OR_EBADELEM 4
#define OR_ENOCONV 5
#define OR_EBREAKDOWN 6

#define OP_MOMENTUM 0
#define OP_SCALAR 1
#define OP_POISSON 2

#define MAXN 8
#define MAXG 8
#define MAXS 8

/* ------------------------------------------------------------------ */
/* Reference elements                                                 */
/* ------------------------------------------------------------------ */

static const double HEX_CORNER[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

/* Trilinear shape functions N_a(xi) = 1/8 (1+xa xi)(1+ya eta)(1+za zeta)
 * and their reference gradients dN[a][j] = dN_a / dxi_j. */
void or_hex08_shape(const double *xi, double *N, double *dN)
{
    for (int a = 0; a < 8; ++a) {
        double sx = HEX_CORNER[a][0], sy = HEX_CORNER[a][1], sz = HEX_CORNER[a][2];
        double fx = 1.0 + sx * xi[0], fy = 1.0 + sy * xi[1], fz = 1.0 + sz * xi[2];
        N[a] = 0.125 * fx * fy * fz;
        dN[a * 3 + 0] = 0.125 * sx * fy * fz;
        dN[a * 3 + 1] = 0.125 * fx * sy * fz;
        dN[a * 3 + 2] = 0.125 * fx * fy * sz;
    }
}

/* 2x2x2 Gauss-Legendre points (xi fastest, then eta, then zeta), weight 1. */
void or_hex08_gauss(double *pts, double *w)
{
    double g = 1.0 / sqrt(3.0);
    int q = 0;
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i) {
                pts[q * 3 + 0] = i ? g : -g;
                pts[q * 3 + 1] = j ? g : -g;
                pts[q * 3 + 2] = k ? g : -g;
                w[q] = 1.0;
                ++q;
            }
}

/* Linear tetrahedron on (0,0,0),(1,0,0),(0,1,0),(0,0,1). */
void or_tet04_shape(const double *xi, double *N, double *dN)
{
    N[0] = 1.0 - xi[0] - xi[1] - xi[2];
    N[1] = xi[0];
    N[2] = xi[1];
    N[3] = xi[2];
    static const double g[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int a = 0; a < 4; ++a)
        for (int j = 0; j < 3; ++j) dN[a * 3 + j] = g[a][j];
}

/* Degree-2 four-point rule: point q has barycentric coordinate b at vertex q
 * and a at the other three; weights 1/24 (reference volume 1/6). */
void or_tet04_gauss(double *pts, double *w)
{
    double a = (5.0 - sqrt(5.0)) / 20.0;
    double b = 1.0 - 3.0 * a;
    for (int q = 0; q < 4; ++q) {
        /* (xi,eta,zeta) are the barycentric coordinates of vertices 1..3 */
        for (int j = 0; j < 3; ++j) pts[q * 3 + j] = (q == j + 1) ? b : a;
        w[q] = 1.0 / 24.0;
    }
}

/* Prism on the reference triangle (0,0),(1,0),(0,1) extruded over zeta in
 * [-1,1]: nodes 0-2 on the triangle at zeta = -1, nodes 3-5 above them at
 * zeta = +1.  N_a = L_i(xi,eta) (1 -+ zeta)/2 with the barycentric
 * L = (1-xi-eta, xi, eta). */
void or_pen06_shape(const double *xi, double *N, double *dN)
{
    const double L[3] = {1.0 - xi[0] - xi[1], xi[0], xi[1]};
    static const double dL[3][2] = {{-1, -1}, {1, 0}, {0, 1}};
    for (int h = 0; h < 2; ++h) {
        double s = h ? 1.0 : -1.0;
        double f = 0.5 * (1.0 + s * xi[2]);
        for (int i = 0; i < 3; ++i) {
            int a = 3 * h + i;
            N[a] = L[i] * f;
            dN[a * 3 + 0] = dL[i][0] * f;
            dN[a * 3 + 1] = dL[i][1] * f;
            dN[a * 3 + 2] = 0.5 * s * L[i];
        }
    }
}

/* Triangle points (1/6,1/6), (2/3,1/6), (1/6,2/3) with weight 1/6 each
 * (degree 2), times Gauss-Legendre +-1/sqrt3 in zeta; triangle point
 * fastest.  Reference volume 1. */
void or_pen06_gauss(double *pts, double *w)
{
    static const double tp[3][2] = {{1.0 / 6, 1.0 / 6}, {2.0 / 3, 1.0 / 6}, {1.0 / 6, 2.0 / 3}};
    double g = 1.0 / sqrt(3.0);
    int q = 0;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < 3; ++i) {
            pts[q * 3 + 0] = tp[i][0];
            pts[q * 3 + 1] = tp[i][1];
            pts[q * 3 + 2] = k ? g : -g;
            w[q] = 1.0 / 6.0;
            ++q;
        }
}

/* Pyramid with the square base [-1,1]^2 at zeta = 0 (nodes 0-3 at
 * (-1,-1), (1,-1), (1,1), (-1,1): counter-clockwise seen from the apex) and
 * the apex, node 4, at (0,0,1).  With m = 1 - zeta and (xa, ya) the base
 * node's corner, N_a = (m + xa xi)(m + ya eta) / (4 m) and N_4 = zeta:
 * bilinear on the base, linear on every triangular face, so it conforms with
 * HEX08 across the base and with TET04 across the sides.  Its derivatives
 * follow from the quotient rule; d/dzeta reduces to
 * (xa ya xi eta - m^2) / (4 m^2). */
void or_pyr05_shape(const double *xi, double *N, double *dN)
{
    static const double B[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
    double m = 1.0 - xi[2];
    for (int a = 0; a < 4; ++a) {
        double P = m + B[a][0] * xi[0], Q = m + B[a][1] * xi[1];
        N[a] = P * Q / (4.0 * m);
        dN[a * 3 + 0] = B[a][0] * Q / (4.0 * m);
        dN[a * 3 + 1] = B[a][1] * P / (4.0 * m);
        dN[a * 3 + 2] = (B[a][0] * B[a][1] * xi[0] * xi[1] - m * m) / (4.0 * m * m);
    }
    N[4] = xi[2];
    dN[12] = 0.0;
    dN[13] = 0.0;
    dN[14] = 1.0;
}

/* Conical product rule: (xi, eta) = (1 - zeta)(s, t) with s, t = +-1/sqrt3
 * (Gauss-Legendre, weights 1) and zeta at the 2-point Gauss-Jacobi nodes for
 * the weight (1-zeta)^2 on [0,1], the roots 1/3 -+ sqrt(10)/15 of
 * t^2 - 2t/3 + 1/15, with weights 1/6 +- sqrt(10)/48 (sum 1/3).  s fastest,
 * then t, then zeta.  Reference volume 4/3. */
void or_pyr05_gauss(double *pts, double *w)
{
    double g = 1.0 / sqrt(3.0), r = sqrt(10.0);
    const double zt[2] = {1.0 / 3.0 - r / 15.0, 1.0 / 3.0 + r / 15.0};
    const double zw[2] = {1.0 / 6.0 + r / 48.0, 1.0 / 6.0 - r / 48.0};
    int q = 0;
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i) {
                double m = 1.0 - zt[k];
                pts[q * 3 + 0] = (i ? g : -g) * m;
                pts[q * 3 + 1] = (j ? g : -g) * m;
                pts[q * 3 + 2] = zt[k];
                w[q] = zw[k];
                ++q;
            }
}

static int ref_element(int nen, double pts[MAXG][3], double w[MAXG],
                       double N[MAXG][MAXN], double dN[MAXG][MAXN][3])
{
    int ng;
    void (*shape)(const double *, double *, double *);
    if (nen == 8) {
        or_hex08_gauss(&pts[0][0], w);
        ng = 8;
        shape = or_hex08_shape;
    } else if (nen == 6) {
        or_pen06_gauss(&pts[0][0], w);
        ng = 6;
        shape = or_pen06_shape;
    } else if (nen == 5) {
        or_pyr05_gauss(&pts[0][0], w);
        ng = 8;
        shape = or_pyr05_shape;
    } else if (nen == 4) {
        or_tet04_gauss(&pts[0][0], w);
        ng = 4;
        shape = or_tet04_shape;
    } else {
        return -1;
    }
    for (int g = 0; g < ng; ++g) shape(pts[g], N[g], &dN[g][0][0]);
    return ng;
}

/* Node count of element e: the type array (4, 5, 6 or 8 per element) if
 * given, else the connectivity stride (a single-type mesh). */
static int elem_nen(int stride, const uint8_t *types, int64_t e)
{
    return types ? (int)types[e] : stride;
}

static int valid_nen(int nen, int stride)
{
    return (nen == 4 || nen == 5 || nen == 6 || nen == 8) && nen <= stride;
}

/* ------------------------------------------------------------------ */
/* CSR pattern: row i holds every node that shares an element with i,   */
/* columns sorted ascending.                                            */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Pass colidx == NULL to get nnz and rowptr; call again to fill colidx.
 * conn [n_elems][stride]; element e has elem_nen() nodes, the rest of its
 * slots are ignored.  Returns nnz, or -1 on an invalid connectivity entry or
 * element type. */
int64_t or_pattern_typed(int stride, const uint8_t *types, int64_t n_nodes, int64_t n_elems,
                         const int32_t *conn, int32_t *rowptr, int32_t *colidx)
{
    int64_t *cnt = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int64_t e = 0; e < n_elems; ++e) {
        int nen = elem_nen(stride, types, e);
        if (!valid_nen(nen, stride)) { free(cnt); return -1; }
        for (int a = 0; a < nen; ++a) {
            int32_t v = conn[e * stride + a];
            if (v < 0 || v >= n_nodes) { free(cnt); return -1; }
            cnt[v + 1]++;
        }
    }
    for (int64_t i = 0; i < n_nodes; ++i) cnt[i + 1] += cnt[i];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    int64_t *inc = malloc(sizeof(int64_t) * (size_t)(cnt[n_nodes] + 1));
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(n_nodes + 1));
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < elem_nen(stride, types, e); ++a) inc[fill[conn[e * stride + a]]++] = e;
    int32_t *buf = malloc(sizeof(int32_t) * 4096);
    size_t cap = 4096;
    int64_t nnz = 0;
    rowptr[0] = 0;
    for (int64_t i = 0; i < n_nodes; ++i) {
        size_t m = 0;
        for (int64_t k = cnt[i]; k < cnt[i + 1]; ++k) {
            int64_t e = inc[k];
            int nen = elem_nen(stride, types, e);
            if (m + (size_t)nen > cap) {
                cap *= 2;
                buf = realloc(buf, sizeof(int32_t) * cap);
            }
            for (int a = 0; a < nen; ++a) buf[m++] = conn[e * stride + a];
        }
        qsort(buf, m, sizeof(int32_t), cmp_i32);
        size_t u = 0;
        for (size_t k = 0; k < m; ++k)
            if (k == 0 || buf[k] != buf[k - 1]) buf[u++] = buf[k];
        if (colidx)
            for (size_t k = 0; k < u; ++k) colidx[nnz + (int64_t)k] = buf[k];
        nnz += (int64_t)u;
        rowptr[i + 1] = (int32_t)nnz;
    }
    free(buf);
    free(inc);
    free(fill);
    free(cnt);
    return nnz;
}

/* Single-type mesh: conn [n_elems][nen]. */
int64_t or_pattern(int nen, int64_t n_nodes, int64_t n_elems, const int32_t *conn,
                   int32_t *rowptr, int32_t *colidx)
{
    return or_pattern_typed(nen, NULL, n_nodes, n_elems, conn, rowptr, colidx);
}

static int64_t find_col(const int32_t *rowptr, const int32_t *colidx, int32_t i, int32_t j)
{
    int64_t lo = rowptr[i], hi = rowptr[i + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (colidx[mid] == j) return mid;
        if (colidx[mid] < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Assembly                                                            */
/* ------------------------------------------------------------------ */

/* Geometry at one Gauss point: J, det J, J^-1 and physical gradients. */
static double geometry(int nen, double X[MAXN][3], double dNr[MAXN][3], double dNx[MAXN][3])
{
    double J[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int a = 0; a < nen; ++a) s += X[a][i] * dNr[a][j];
            J[i][j] = s;
        }
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det > 0.0)) return det;
    double Ji[3][3]; /* inverse of J */
    Ji[0][0] = c00 / det;
    Ji[1][0] = c01 / det;
    Ji[2][0] = c02 / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    /* grad_x N_a = J^-T grad_xi N_a :  (grad N_a)_i = sum_j Ji[j][i] dNr[a][j] */
    for (int a = 0; a < nen; ++a)
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += Ji[j][i] * dNr[a][j];
            dNx[a][i] = s;
        }
    return det;
}

/*
 * Assemble one operator into a CSR pattern produced by or_pattern.
 *
 *   op = 0 MOMENTUM: values[1][nnz] = M/dt + C + K_mu ; rhs[3][N], b_i = M_rho u_i / dt
 *   op = 1 SCALAR  : values[k][nnz] = M/dt + C + K_{rho D_k} ; rhs[k][N] = M_rho Y_k / dt
 *   op = 2 POISSON : values[1][nnz] = L ; rhs[1][N], f_a = (1/dt) int grad N_a . (rho u)
 *
 * with, at each Gauss point, dV = w det J, rho_g, mu_g, u_g the nodal
 * interpolants, and
 *   M_ab = sum dV rho_g N_a N_b
 *   C_ab = sum dV rho_g N_a (u_g . grad N_b)
 *   K_ab = sum dV coef_g grad N_a . grad N_b.
 * Inputs: coords [N][3]; conn [E][stride], element e using its
 * first elem_nen() slots; u [3][N]; rho, mu [N];
 * Y [k][N]; D [k].  Outputs are overwritten.  Returns OR_EBADELEM (with the
 * first element index and the smallest det J) for det J <= 0.
 */
/* Reference tables of every element type, indexed by node count. */
typedef struct {
    double pts[MAXN + 1][MAXG][3], w[MAXN + 1][MAXG], N[MAXN + 1][MAXG][MAXN], dN[MAXN + 1][MAXG][MAXN][3];
    int ng[MAXN + 1];
} RefSet;

static void ref_set(RefSet *R)
{
    for (int t = 0; t <= MAXN; ++t) R->ng[t] = ref_element(t, R->pts[t], R->w[t], R->N[t], R->dN[t]);
}

/* Operator of one assembly call: fields and sizes. */
typedef struct {
    int stride;
    const uint8_t *types;
    int64_t n_nodes;
    const double *coords;
    const int32_t *conn;
    int op;
    double dt;
    const double *u, *rho, *mu, *Y, *D;
    int n_scalars, n_mat, n_rhs;
} AsmOp;

/* Elemental matrices and right-hand sides of element e: the Gauss loop
 * accumulating M, C, K (one per scalar) and B.  *min_det takes the
 * smallest det J met; returns OR_EBADELEM at the first det J <= 0. */
static int element_terms(const RefSet *R, const AsmOp *A, int64_t e, double M[MAXN][MAXN], double Cm[MAXN][MAXN],
                         double K[MAXS][MAXN][MAXN], double B[MAXS][MAXN], double *min_det)
{
    const int op = A->op, n_scalars = A->n_scalars;
    const int64_t n_nodes = A->n_nodes;
    const double dt = A->dt, *u = A->u, *rho = A->rho, *mu = A->mu, *Y = A->Y, *D = A->D;
    const int nen = elem_nen(A->stride, A->types, e), ng = R->ng[nen];
    const double (*Ng)[MAXN] = R->N[nen];
    const double (*dNr)[MAXN][3] = R->dN[nen];
    const double *wg = R->w[nen];
    const int32_t *c = A->conn + e * A->stride;
    double X[MAXN][3];
    for (int a = 0; a < nen; ++a)
        for (int i = 0; i < 3; ++i) X[a][i] = A->coords[(int64_t)c[a] * 3 + i];
    memset(M, 0, sizeof(double) * MAXN * MAXN);
    memset(Cm, 0, sizeof(double) * MAXN * MAXN);
    memset(K, 0, sizeof(double) * MAXS * MAXN * MAXN);
    memset(B, 0, sizeof(double) * MAXS * MAXN);

    for (int g = 0; g < ng; ++g) {
        double dNx[MAXN][3];
        double det = geometry(nen, X, (double (*)[3])dNr[g], dNx);
        if (det < *min_det) *min_det = det;
        if (!(det > 0.0)) return OR_EBADELEM;
        double dV = wg[g] * det;
        double rg = 0.0, mg = 0.0, ug[3] = {0.0, 0.0, 0.0}, yg[MAXS] = {0};
        for (int a = 0; a < nen; ++a) {
            double Na = Ng[g][a];
            rg += Na * rho[c[a]];
            if (op == OP_MOMENTUM) mg += Na * mu[c[a]];
            for (int i = 0; i < 3; ++i) ug[i] += Na * u[(int64_t)i * n_nodes + c[a]];
            if (op == OP_SCALAR)
                for (int k = 0; k < n_scalars; ++k) yg[k] += Na * Y[(int64_t)k * n_nodes + c[a]];
        }
        for (int a = 0; a < nen; ++a) {
            double Na = Ng[g][a];
            for (int b = 0; b < nen; ++b) {
                double Nb = Ng[g][b];
                double gg = dNx[a][0] * dNx[b][0] + dNx[a][1] * dNx[b][1] + dNx[a][2] * dNx[b][2];
                double ugb = ug[0] * dNx[b][0] + ug[1] * dNx[b][1] + ug[2] * dNx[b][2];
                if (op == OP_POISSON) {
                    K[0][a][b] += dV * gg;
                } else {
                    M[a][b] += dV * rg * Na * Nb;
                    Cm[a][b] += dV * rg * Na * ugb;
                    if (op == OP_MOMENTUM)
                        K[0][a][b] += dV * mg * gg;
                    else
                        for (int k = 0; k < n_scalars; ++k) K[k][a][b] += dV * (rg * D[k]) * gg;
                }
            }
            if (op == OP_MOMENTUM)
                for (int i = 0; i < 3; ++i) B[i][a] += dV * rg * Na * ug[i] / dt;
            else if (op == OP_SCALAR)
                for (int k = 0; k < n_scalars; ++k) B[k][a] += dV * rg * Na * yg[k] / dt;
            else
                B[0][a] += (1.0 / dt) * dV *
                           (dNx[a][0] * (rg * ug[0]) + dNx[a][1] * (rg * ug[1]) + dNx[a][2] * (rg * ug[2]));
        }
    }
    return OR_OK;
}

/* A_e = M/dt + C + K (momentum, scalar) or L (Poisson), and B, added into
 * the CSR rows and right-hand sides of element e's nodes. */
static int element_scatter(const AsmOp *A, int64_t e, const int32_t *rowptr, const int32_t *colidx,
                           double M[MAXN][MAXN], double Cm[MAXN][MAXN], double K[MAXS][MAXN][MAXN],
                           double B[MAXS][MAXN], double *values, double *rhs)
{
    const int nen = elem_nen(A->stride, A->types, e);
    const int32_t *c = A->conn + e * A->stride;
    const int64_t nnz = rowptr[A->n_nodes], n_nodes = A->n_nodes;
    for (int a = 0; a < nen; ++a) {
        for (int b = 0; b < nen; ++b) {
            int64_t pos = find_col(rowptr, colidx, c[a], c[b]);
            if (pos < 0) return OR_EINVAL;
            for (int k = 0; k < A->n_mat; ++k) {
                double v = (A->op == OP_POISSON) ? K[0][a][b] : (M[a][b] / A->dt + Cm[a][b] + K[k][a][b]);
                values[(int64_t)k * nnz + pos] += v;
            }
        }
        for (int k = 0; k < A->n_rhs; ++k) rhs[(int64_t)k * n_nodes + c[a]] += B[k][a];
    }
    return OR_OK;
}

/* Checks the arguments, fills *A and zeroes the outputs. */
static int asm_begin(AsmOp *A, int stride, const uint8_t *types, int64_t n_nodes, const double *coords,
                     int64_t n_elems, const int32_t *conn, int op, double dt, const double *u, const double *rho,
                     const double *mu, int n_scalars, const double *Y, const double *D, const int32_t *rowptr,
                     double *values, double *rhs)
{
    for (int64_t e = 0; e < n_elems; ++e)
        if (!valid_nen(elem_nen(stride, types, e), stride)) return OR_EINVAL;
    if (op == OP_SCALAR && (n_scalars < 1 || n_scalars > MAXS)) return OR_EINVAL;
    A->stride = stride;
    A->types = types;
    A->n_nodes = n_nodes;
    A->coords = coords;
    A->conn = conn;
    A->op = op;
    A->dt = dt;
    A->u = u;
    A->rho = rho;
    A->mu = mu;
    A->Y = Y;
    A->D = D;
    A->n_scalars = n_scalars;
    A->n_mat = (op == OP_SCALAR) ? n_scalars : 1;
    A->n_rhs = (op == OP_MOMENTUM) ? 3 : (op == OP_SCALAR ? n_scalars : 1);
    int64_t nnz = rowptr[n_nodes];
    memset(values, 0, sizeof(double) * (size_t)(nnz * A->n_mat));
    memset(rhs, 0, sizeof(double) * (size_t)(n_nodes * A->n_rhs));
    return OR_OK;
}

int or_assemble_typed(int stride, const uint8_t *types, int64_t n_nodes, const double *coords,
                      int64_t n_elems, const int32_t *conn, int op, double dt, const double *u,
                      const double *rho, const double *mu, int n_scalars, const double *Y,
                      const double *D, const int32_t *rowptr, const int32_t *colidx, double *values,
                      double *rhs, int64_t *bad_elem, double *min_det)
{
    static RefSet R;   /* large: kept off the stack */
    ref_set(&R);
    AsmOp A;
    int st = asm_begin(&A, stride, types, n_nodes, coords, n_elems, conn, op, dt, u, rho, mu, n_scalars, Y, D,
                       rowptr, values, rhs);
    if (st != OR_OK) return st;
    *bad_elem = -1;
    *min_det = INFINITY;
    int status = OR_OK;
    double M[MAXN][MAXN], Cm[MAXN][MAXN], K[MAXS][MAXN][MAXN], B[MAXS][MAXN];
    /* element order: the outer loop of Listing 1 */
    for (int64_t e = 0; e < n_elems; ++e) {
        if (element_terms(&R, &A, e, M, Cm, K, B, min_det) != OR_OK) {
            if (*bad_elem < 0) *bad_elem = e;
            status = OR_EBADELEM;
            continue;
        }
        if (element_scatter(&A, e, rowptr, colidx, M, Cm, K, B, values, rhs) != OR_OK) return OR_EINVAL;
    }
    return status;
}

/* Single-type mesh: conn [n_elems][nen]. */
int or_assemble(int nen, int64_t n_nodes, const double *coords, int64_t n_elems,
                const int32_t *conn, int op, double dt, const double *u, const double *rho,
                const double *mu, int n_scalars, const double *Y, const double *D,
                const int32_t *rowptr, const int32_t *colidx, double *values, double *rhs,
                int64_t *bad_elem, double *min_det)
{
    return or_assemble_typed(nen, NULL, n_nodes, coords, n_elems, conn, op, dt, u, rho, mu,
                             n_scalars, Y, D, rowptr, colidx, values, rhs, bad_elem, min_det);
}

/* ------------------------------------------------------------------ */
/* Momentum operator with the full-stress viscous term: 3x3 blocks     */
/* ------------------------------------------------------------------ */

/*
 * The implicit momentum operator of Eq. (1) with its viscous term in the
 * full-stress form -div(2 mu eps(u)) and, optionally, the EMAC convective
 * form, linearised about the nodal velocity a = u (Picard).  Testing
 * 2 mu eps(u) with N_a e_i couples the components: row (a, i), column
 * (b, k) of the block matrix is
 *
 *   delta_ik (M_ab / dt + C_ab + K_ab + E_ab) + T_ab[i][k],
 *
 *   M_ab = sum_g dV rho_g N_a N_b,   C_ab = sum_g dV rho_g N_a (a_g . grad N_b),
 *   K_ab = sum_g dV mu_g grad N_a . grad N_b            (Laplacian part),
 *   T_ab[i][k] = sum_g dV mu_g (d N_a / d x_k)(d N_b / d x_i)   (form bit 0),
 *   E_ab = sum_g dV rho_g (div a)_g N_a N_b                     (form bit 1:
 *          EMAC's (div u) u term at the Gauss point, with u frozen as a);
 *
 * T and E are left out when their bit is clear (form 0 is the scalar
 * momentum operator of or_assemble times the 3x3 identity).  values[nnz][3][3]
 * on the canonical scalar pattern (block (i, k) of entry p at p * 9 + 3i + k),
 * rhs[3][N] = M_rho u_i / dt as for or_assemble.  With b the rhs, b - A u is
 * the matrix-free residual of or_element_vectors (kind 0, same form).
 */
int or_assemble_block(int stride, const uint8_t *types, int64_t n_nodes, const double *coords, int64_t n_elems,
                      const int32_t *conn, int form, double dt, const double *u, const double *rho,
                      const double *mu, const int32_t *rowptr, const int32_t *colidx, double *values, double *rhs,
                      int64_t *bad_elem, double *min_det)
{
    static RefSet R;
    ref_set(&R);
    for (int64_t e = 0; e < n_elems; ++e)
        if (!valid_nen(elem_nen(stride, types, e), stride)) return OR_EINVAL;
    if (form & ~3) return OR_EINVAL;
    const int64_t nnz = rowptr[n_nodes];
    memset(values, 0, sizeof(double) * (size_t)(9 * nnz));
    memset(rhs, 0, sizeof(double) * (size_t)(3 * n_nodes));
    *bad_elem = -1;
    *min_det = INFINITY;
    int status = OR_OK;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int nen = elem_nen(stride, types, e), ng = R.ng[nen];
        const int32_t *c = conn + e * stride;
        double X[MAXN][3];
        for (int a = 0; a < nen; ++a)
            for (int i = 0; i < 3; ++i) X[a][i] = coords[(int64_t)c[a] * 3 + i];
        double S[MAXN][MAXN] = {{0}}, T[MAXN][MAXN][3][3] = {{{{0}}}}, B[3][MAXN] = {{0}};
        int bad = 0;
        for (int g = 0; g < ng && !bad; ++g) {
            double dNx[MAXN][3];
            double det = geometry(nen, X, R.dN[nen][g], dNx);
            if (det < *min_det) *min_det = det;
            if (!(det > 0.0)) {
                bad = 1;
                break;
            }
            const double dV = R.w[nen][g] * det;
            double rg = 0.0, mg = 0.0, ag[3] = {0.0, 0.0, 0.0}, diva = 0.0;
            for (int b = 0; b < nen; ++b) {
                const double Nb = R.N[nen][g][b];
                rg += Nb * rho[c[b]];
                mg += Nb * mu[c[b]];
                for (int i = 0; i < 3; ++i) {
                    const double ub = u[(int64_t)i * n_nodes + c[b]];
                    ag[i] += Nb * ub;
                    diva += dNx[b][i] * ub;
                }
            }
            for (int a = 0; a < nen; ++a) {
                const double Na = R.N[nen][g][a];
                for (int b = 0; b < nen; ++b) {
                    const double Nb = R.N[nen][g][b];
                    const double gg = dNx[a][0] * dNx[b][0] + dNx[a][1] * dNx[b][1] + dNx[a][2] * dNx[b][2];
                    const double agb = ag[0] * dNx[b][0] + ag[1] * dNx[b][1] + ag[2] * dNx[b][2];
                    /* M / dt + C + K (+ E) */
                    double s = dV * rg * Na * Nb / dt + dV * rg * Na * agb + dV * mg * gg;
                    if (form & 2) s += dV * rg * diva * Na * Nb;
                    S[a][b] += s;
                    if (form & 1)
                        for (int i = 0; i < 3; ++i)
                            for (int k = 0; k < 3; ++k) T[a][b][i][k] += dV * mg * dNx[a][k] * dNx[b][i];
                }
                for (int i = 0; i < 3; ++i) B[i][a] += dV * rg * Na * ag[i] / dt;
            }
        }
        if (bad) {
            if (*bad_elem < 0) *bad_elem = e;
            status = OR_EBADELEM;
            continue;
        }
        for (int a = 0; a < nen; ++a) {
            for (int b = 0; b < nen; ++b) {
                const int64_t pos = find_col(rowptr, colidx, c[a], c[b]);
                if (pos < 0) return OR_EINVAL;
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) values[pos * 9 + 3 * i + k] += (i == k ? S[a][b] : 0.0) + T[a][b][i][k];
            }
            for (int i = 0; i < 3; ++i) rhs[(int64_t)i * n_nodes + c[a]] += B[i][a];
        }
    }
    return status;
}

/* ------------------------------------------------------------------ */
/* Matrix-free element vectors for the explicit step (Algorithm 1)     */
/* ------------------------------------------------------------------ */

/*
 * Element loop that integrates nodal vectors instead of matrices (the
 * Runge-Kutta stages of Algorithm 1 assemble the momentum equations as
 * residuals; the paper gives no formulation, see the step below):
 *
 *   kind 0  residual: r_i[a] = - sum_g dV (rho_g N_a (u_g . grad u_i,g)
 *                                          + mu_g grad N_a . grad u_i,g)
 *           for i = 0..2 into out[0..2][N], and the rho-weighted lumped mass
 *           m[a] = sum_g dV rho_g N_a into out[3][N].  form selects the
 *           operator variants of Eq. (1): bit 0 the full-stress viscous term
 *           2 mu eps(u) tested with grad N_a, i.e. + mu_g (d u_j / d x_i)
 *           (d N_a / d x_j) on top of the Laplacian form; bit 1 the EMAC
 *           convective term 2 eps(u) u + (div u) u - grad(|u|^2)/2 evaluated
 *           at the Gauss point, which is (u . grad) u + (div u) u there, i.e.
 *           + rho_g N_a (div u_g) u_i,g on top of the advective form;
 *   kind 1  gradient: g_j[a] = sum_g dV N_a (grad p)_j,g into out[0..2][N];
 *   kind 2  scalar residual (the heat and species equations, advanced by
 *           the same Runge-Kutta stages without an algebraic solver,
 *           Section 2): r[a] = - sum_g dV rho_g (N_a (u_g . grad Y_g)
 *           + D grad N_a . grad Y_g) into out[0][N] and the lumped mass
 *           into out[1][N], for the scalar Y with diffusivity D;
 *
 * with u_g, grad u_i,g, rho_g, mu_g, grad p_g interpolated from the nodal
 * fields.  out is overwritten.  Same element types, connectivity convention
 * and bad-element report as or_assemble_typed.
 */
int or_element_vectors(int stride, const uint8_t *types, int64_t n_nodes, const double *coords,
                       int64_t n_elems, const int32_t *conn, int kind, int form, const double *u,
                       const double *rho, const double *mu, const double *p, const double *Y,
                       double D, double *out, int64_t *bad_elem, double *min_det)
{
    double pts[MAXN + 1][MAXG][3], w[MAXN + 1][MAXG], Nt[MAXN + 1][MAXG][MAXN],
        dNt[MAXN + 1][MAXG][MAXN][3];
    int ngt[MAXN + 1];
    for (int t = 0; t <= MAXN; ++t) ngt[t] = ref_element(t, pts[t], w[t], Nt[t], dNt[t]);
    if (kind < 0 || kind > 2) return OR_EINVAL;
    for (int64_t e = 0; e < n_elems; ++e)
        if (!valid_nen(elem_nen(stride, types, e), stride)) return OR_EINVAL;
    int nout = kind == 0 ? 4 : (kind == 1 ? 3 : 2);
    memset(out, 0, sizeof(double) * (size_t)(n_nodes * nout));
    *bad_elem = -1;
    *min_det = INFINITY;
    int status = OR_OK;
    for (int64_t e = 0; e < n_elems; ++e) {
        const int nen = elem_nen(stride, types, e), ng = ngt[nen];
        const int32_t *c = conn + e * stride;
        double X[MAXN][3];
        for (int a = 0; a < nen; ++a)
            for (int i = 0; i < 3; ++i) X[a][i] = coords[(int64_t)c[a] * 3 + i];
        double B[4][MAXN] = {{0}};
        int bad = 0;
        for (int g = 0; g < ng; ++g) {
            double dNx[MAXN][3];
            double det = geometry(nen, X, dNt[nen][g], dNx);
            if (det < *min_det) *min_det = det;
            if (!(det > 0.0)) {
                if (*bad_elem < 0) *bad_elem = e;
                status = OR_EBADELEM;
                bad = 1;
                break;
            }
            double dV = w[nen][g] * det;
            const double *Ng = Nt[nen][g];
            if (kind == 0) {
                double rg = 0.0, mg = 0.0, ug[3] = {0, 0, 0}, gu[3][3] = {{0}};
                for (int b = 0; b < nen; ++b) {
                    rg += Ng[b] * rho[c[b]];
                    mg += Ng[b] * mu[c[b]];
                    for (int i = 0; i < 3; ++i) {
                        double ub = u[(int64_t)i * n_nodes + c[b]];
                        ug[i] += Ng[b] * ub;
                        for (int j = 0; j < 3; ++j) gu[i][j] += dNx[b][j] * ub;   /* d u_i / d x_j */
                    }
                }
                double divu = gu[0][0] + gu[1][1] + gu[2][2];
                for (int a = 0; a < nen; ++a) {
                    for (int i = 0; i < 3; ++i) {
                        double adv = ug[0] * gu[i][0] + ug[1] * gu[i][1] + ug[2] * gu[i][2];
                        double vis = dNx[a][0] * gu[i][0] + dNx[a][1] * gu[i][1] + dNx[a][2] * gu[i][2];
                        if (form & 1) /* + (grad u)^T part of 2 eps(u) */
                            vis += dNx[a][0] * gu[0][i] + dNx[a][1] * gu[1][i] + dNx[a][2] * gu[2][i];
                        if (form & 2) /* EMAC: + (div u) u */
                            adv += divu * ug[i];
                        B[i][a] -= dV * (rg * Ng[a] * adv + mg * vis);
                    }
                    B[3][a] += dV * rg * Ng[a];
                }
            } else if (kind == 1) {
                double gp[3] = {0, 0, 0};
                for (int b = 0; b < nen; ++b)
                    for (int j = 0; j < 3; ++j) gp[j] += dNx[b][j] * p[c[b]];
                for (int a = 0; a < nen; ++a)
                    for (int j = 0; j < 3; ++j) B[j][a] += dV * Ng[a] * gp[j];
            } else {
                double rg = 0.0, ug[3] = {0, 0, 0}, gy[3] = {0, 0, 0};
                for (int b = 0; b < nen; ++b) {
                    rg += Ng[b] * rho[c[b]];
                    for (int i = 0; i < 3; ++i) {
                        ug[i] += Ng[b] * u[(int64_t)i * n_nodes + c[b]];
                        gy[i] += dNx[b][i] * Y[c[b]];
                    }
                }
                double adv = ug[0] * gy[0] + ug[1] * gy[1] + ug[2] * gy[2];
                for (int a = 0; a < nen; ++a) {
                    double dif = dNx[a][0] * gy[0] + dNx[a][1] * gy[1] + dNx[a][2] * gy[2];
                    B[0][a] -= dV * rg * (Ng[a] * adv + D * dif);
                    B[1][a] += dV * rg * Ng[a];
                }
            }
        }
        if (bad) continue;
        for (int a = 0; a < nen; ++a)
            for (int k = 0; k < nout; ++k) out[(int64_t)k * n_nodes + c[a]] += B[k][a];
    }
    return status;
}

/* ------------------------------------------------------------------ */
/* Boundary assembly: equilibrium wall model (Algorithm 1)             */
/* ------------------------------------------------------------------ */

#define WALL_KAPPA 0.41
#define WALL_NEWTON 16

/* Reichardt's law of the wall u+ (y+) and its derivative. */
static double reichardt(double yp, double *dudy)
{
    double e1 = exp(-yp / 11.0), e3 = exp(-yp / 3.0);
    *dudy = 1.0 / (1.0 + WALL_KAPPA * yp) + 7.8 * (e1 / 11.0 - e3 / 11.0 + yp * e3 / 33.0);
    return log(1.0 + WALL_KAPPA * yp) / WALL_KAPPA + 7.8 * (1.0 - e1 - yp / 11.0 * e3);
}

/* Friction velocity u_tau from U = u_tau u+(delta u_tau / nu): Newton on
 * g(u_tau) = u_tau u+(delta u_tau / nu) - U from the laminar guess
 * sqrt(nu U / delta), a fixed number of steps. */
double or_wall_utau(double U, double nu, double delta)
{
    if (!(U > 0.0)) return 0.0;
    double ut = sqrt(nu * U / delta);
    for (int k = 0; k < WALL_NEWTON; ++k) {
        double yp = delta * ut / nu, d;
        double up = reichardt(yp, &d);
        double g = ut * up - U;
        double dg = up + yp * d;
        ut -= g / dg;
        if (ut <= 0.0) ut = 1e-300;
    }
    return ut;
}

/*
 * Wall-model traction on wall faces (the boundary assembly of Algorithm 1;
 * the paper names it but gives no law, so the equilibrium law above is used):
 * at each face Gauss point the velocity u_h is interpolated from the face's
 * nodes, its tangential part u_t = u_h - (u_h . n) n gives U = |u_t|, rho
 * and mu are interpolated, u_tau solves the law at distance delta, and the
 * traction t = -rho u_tau^2 u_t / U is integrated:
 *   out_i[a] = sum_faces sum_g w_g |dx/dxi x dx/deta| N_a t_i.
 * Faces: face_nen[f] = 3 (triangle, reference (0,0),(1,0),(0,1), the
 * 3-point rule (1/6,1/6),(2/3,1/6),(1/6,2/3), weights 1/6) or 4
 * (quadrilateral [-1,1]^2, nodes counter-clockwise, 2x2 Gauss); face_conn
 * [F][4].  out [3][N] is overwritten.
 */
int or_wall_traction(int64_t n_nodes, const double *coords, int64_t n_faces, const uint8_t *face_nen,
                     const int32_t *face_conn, const double *u, const double *rho, const double *mu,
                     double delta, double *out)
{
    if (!(delta > 0.0)) return OR_EINVAL;
    memset(out, 0, sizeof(double) * (size_t)(3 * n_nodes));
    const double g = 1.0 / sqrt(3.0);
    for (int64_t f = 0; f < n_faces; ++f) {
        int nn = face_nen[f];
        if (nn != 3 && nn != 4) return OR_EINVAL;
        const int32_t *c = face_conn + 4 * f;
        for (int a = 0; a < nn; ++a)
            if (c[a] < 0 || c[a] >= n_nodes) return OR_EINVAL;
        int ng = nn == 3 ? 3 : 4;
        for (int q = 0; q < ng; ++q) {
            double N[4], dNs[4], dNt[4], w;
            if (nn == 3) {
                static const double tp[3][2] = {{1.0 / 6, 1.0 / 6}, {2.0 / 3, 1.0 / 6}, {1.0 / 6, 2.0 / 3}};
                double s = tp[q][0], t = tp[q][1];
                N[0] = 1.0 - s - t; N[1] = s; N[2] = t;
                dNs[0] = -1.0; dNs[1] = 1.0; dNs[2] = 0.0;
                dNt[0] = -1.0; dNt[1] = 0.0; dNt[2] = 1.0;
                w = 1.0 / 6.0;
            } else {
                static const double cs[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
                double s = (q & 1) ? g : -g, t = (q & 2) ? g : -g;
                for (int a = 0; a < 4; ++a) {
                    N[a] = 0.25 * (1.0 + cs[a][0] * s) * (1.0 + cs[a][1] * t);
                    dNs[a] = 0.25 * cs[a][0] * (1.0 + cs[a][1] * t);
                    dNt[a] = 0.25 * cs[a][1] * (1.0 + cs[a][0] * s);
                }
                w = 1.0;
            }
            double xs[3] = {0, 0, 0}, xt[3] = {0, 0, 0}, ug[3] = {0, 0, 0}, rg = 0.0, mg = 0.0;
            for (int a = 0; a < nn; ++a) {
                for (int i = 0; i < 3; ++i) {
                    xs[i] += dNs[a] * coords[(int64_t)c[a] * 3 + i];
                    xt[i] += dNt[a] * coords[(int64_t)c[a] * 3 + i];
                    ug[i] += N[a] * u[(int64_t)i * n_nodes + c[a]];
                }
                rg += N[a] * rho[c[a]];
                mg += N[a] * mu[c[a]];
            }
            double nv[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2],
                            xs[0] * xt[1] - xs[1] * xt[0]};
            double area = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            if (!(area > 0.0)) return OR_EBADELEM;
            double un = (ug[0] * nv[0] + ug[1] * nv[1] + ug[2] * nv[2]) / (area * area);
            double ut[3] = {ug[0] - un * nv[0], ug[1] - un * nv[1], ug[2] - un * nv[2]};
            double U = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
            if (!(U > 0.0)) continue;
            double tau = or_wall_utau(U, mg / rg, delta);
            double fac = -w * area * rg * tau * tau / U;
            for (int a = 0; a < nn; ++a)
                for (int i = 0; i < 3; ++i) out[(int64_t)i * n_nodes + c[a]] += fac * N[a] * ut[i];
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Dirichlet elimination (symmetric)                                   */
/* ------------------------------------------------------------------ */

/* For a free row i: f_i -= sum_{j in D} L_ij g_j and L_ij = 0 for j in D.
 * For a Dirichlet row i: off-diagonals = 0, diagonal kept, f_i = L_ii g_i.
 * g == NULL means g = 0. */
int or_dirichlet(int64_t n_nodes, const int32_t *rowptr, const int32_t *colidx, double *values,
                 double *rhs, int64_t n_dir, const int32_t *dnodes, const double *g)
{
    unsigned char *isd = calloc((size_t)n_nodes, 1);
    if (!isd) return OR_ENOMEM;
    for (int64_t k = 0; k < n_dir; ++k) {
        if (dnodes[k] < 0 || dnodes[k] >= n_nodes) { free(isd); return OR_EINVAL; }
        isd[dnodes[k]] = 1;
    }
    for (int64_t i = 0; i < n_nodes; ++i) {
        if (isd[i]) continue;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int32_t j = colidx[p];
            if (isd[j]) {
                double gj = g ? g[j] : 0.0;
                rhs[i] -= values[p] * gj;
                values[p] = 0.0;
            }
        }
    }
    for (int64_t i = 0; i < n_nodes; ++i) {
        if (!isd[i]) continue;
        double diag = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            if (colidx[p] == i) diag = values[p];
            else values[p] = 0.0;
        }
        rhs[i] = diag * (g ? g[i] : 0.0);
    }
    free(isd);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Solver kernels and Jacobi-PCG                                       */
/* ------------------------------------------------------------------ */

void or_spmv(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *vals,
             const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s += vals[p] * x[colidx[p]];
        y[i] = s;
    }
}

double or_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

void or_axpy(int64_t n, double a, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) y[i] += a * x[i];
}

/*
 * Jacobi-preconditioned CG on an SPD CSR matrix.
 * x holds x0 on entry and the iterate on return.  Stop when
 * ||r_k||_2 <= rtol ||b||_2 (recursive residual).  rtol <= 0 runs exactly
 * max_iter iterations.  info[0] = iterations, info[1] = ||r||/||b||
 * (recursive), info[2] = ||b - A x||/||b|| recomputed.
 * Returns OR_OK, OR_ENOCONV or OR_EBREAKDOWN (p.Ap <= 0 or not finite).
 */
int or_pcg(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *vals,
           const double *b, double *x, double rtol, int max_iter, double *info)
{
    double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    double *dinv = malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q || !dinv) return OR_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (colidx[k] == i) d = vals[k];
        dinv[i] = 1.0 / d;
    }
    or_spmv(n, rowptr, colidx, vals, x, q);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    double bnorm = sqrt(or_dot(n, b, b));
    for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = or_dot(n, r, z);
    int status = OR_ENOCONV, it = 0;
    double rnorm = sqrt(or_dot(n, r, r));
    if (rtol > 0.0 && rnorm <= rtol * bnorm) status = OR_OK;
    while (status == OR_ENOCONV && it < max_iter) {
        or_spmv(n, rowptr, colidx, vals, p, q);
        double pq = or_dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = OR_EBREAKDOWN; break; }
        double alpha = rho / pq;
        or_axpy(n, alpha, p, x);
        or_axpy(n, -alpha, q, r);
        ++it;
        rnorm = sqrt(or_dot(n, r, r));
        if (rtol > 0.0 && rnorm <= rtol * bnorm) { status = OR_OK; break; }
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rho1 = or_dot(n, r, z);
        double beta = rho1 / rho;
        rho = rho1;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (rtol <= 0.0 && status == OR_ENOCONV && it == max_iter) status = OR_OK;
    or_spmv(n, rowptr, colidx, vals, x, q);
    for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
    info[0] = it;
    info[1] = bnorm > 0.0 ? rnorm / bnorm : rnorm;
    info[2] = bnorm > 0.0 ? sqrt(or_dot(n, q, q)) / bnorm : sqrt(or_dot(n, q, q));
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}
