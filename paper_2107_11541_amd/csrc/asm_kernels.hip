// asm_kernels.hip -- element-by-element assembly into CSR on gfx950.
//
// Section 4.2 / Listing 1 of the paper: an outer loop over elements and an
// inner loop over Gauss points and node pairs accumulating the elemental
// matrix from shape functions and the Jacobian weight, then a scatter into
// CSR.  Section 4.3 packs elements so that a SIMD unit processes several at
// once.  gfx950 form:
//
//   * one work-group = one block of <= 64 spatially compact elements of one
//     type; a TET04, PYR05 or PEN06 element is one lane, a HEX08 element two
//     lanes in two waves (4 matrix rows each), which keeps a wave under 256
//     registers so that two blocks share each SIMD and hide each other's
//     memory latency;
//   * the block's nodal fields are staged in LDS (structure of arrays, so that
//     lanes reading different nodes hit different banks);
//   * the CSR rows the block touches live in an LDS image, initialised from
//     HBM (or zero for the first block to touch a row), accumulated with
//     conflict-free ds_add_f64 in a fixed (phase, a, b) order, and written
//     back once -- one coalesced read-modify-write per touched row instead of
//     one per element entry;
//   * blocks of one colour share no node, so a launch per (colour, element
//     type) needs no atomics in HBM; the launch order fixes the summation
//     order, so the result is bitwise reproducible.
//
// Precision: FP64, or (mixed) FP32 Gauss-point products and elemental sums
// with the Jacobian, det J, J^-1 and the CSR accumulation in FP64.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "internal.h"
#include "plan.h"

namespace feasm {
namespace {

constexpr int OP_MOM = FE_OP_MOMENTUM, OP_SCA = FE_OP_SCALAR, OP_POI = FE_OP_POISSON;
// element-vector passes of the explicit step (no matrix): residual + lumped
// mass, pressure gradient, divergence right-hand side
constexpr int OP_RES = kOpResidual, OP_GRD = kOpGradient, OP_DIV = kOpDivergence, OP_SRS = kOpScalarResidual;

// Trilinear hexahedron, 2x2x2 Gauss rule (points xi fastest, weights 1).
struct Hex {
    static constexpr int NEN = 8, NG = 8;
    static constexpr double kG = 0.57735026918962576451;   // 1/sqrt(3)
    __host__ __device__ static constexpr int sx(int a) { return ((a & 3) == 1 || (a & 3) == 2) ? 1 : -1; }
    __host__ __device__ static constexpr int sy(int a) { return (a & 3) >= 2 ? 1 : -1; }
    __host__ __device__ static constexpr int sz(int a) { return a >= 4 ? 1 : -1; }
    __host__ __device__ static constexpr double gp(int g, int d) { return ((g >> d) & 1) ? kG : -kG; }
    __host__ __device__ static constexpr double w(int) { return 1.0; }
    __host__ __device__ static constexpr double N(int g, int a)
    {
        return 0.125 * (1.0 + sx(a) * gp(g, 0)) * (1.0 + sy(a) * gp(g, 1)) * (1.0 + sz(a) * gp(g, 2));
    }
    static constexpr bool kRolled = true, kSparse = false;
    __host__ __device__ static constexpr double dN(int g, int a, int j)
    {
        return j == 0 ? 0.125 * sx(a) * (1.0 + sy(a) * gp(g, 1)) * (1.0 + sz(a) * gp(g, 2))
             : j == 1 ? 0.125 * sy(a) * (1.0 + sx(a) * gp(g, 0)) * (1.0 + sz(a) * gp(g, 2))
                      : 0.125 * sz(a) * (1.0 + sx(a) * gp(g, 0)) * (1.0 + sy(a) * gp(g, 1));
    }
};

// Shape-function values and reference gradients at the Gauss points of an
// element type, for the rolled Gauss loop (read from constant memory).
template <class EL> struct RefTables {
    double N[EL::NG][EL::NEN];        // N[g][a]
    double dN[EL::NG][EL::NEN][3];    // dN[g][a][j]
};

template <class EL> constexpr RefTables<EL> make_tables()
{
    RefTables<EL> t{};
    for (int g = 0; g < EL::NG; ++g)
        for (int a = 0; a < EL::NEN; ++a) {
            t.N[g][a] = EL::N(g, a);
            for (int j = 0; j < 3; ++j) t.dN[g][a][j] = EL::dN(g, a, j);
        }
    return t;
}

__constant__ RefTables<Hex> kHexTab = make_tables<Hex>();

// Linear tetrahedron, 4-point degree-2 rule (weights 1/24).
struct Tet {
    static constexpr int NEN = 4, NG = 4;
    static constexpr bool kRolled = false, kSparse = true;
    __device__ static constexpr double Nv(int g, int a) { return N(g, a); }
    __device__ static constexpr double dNv(int g, int a, int j) { return dN(g, a, j); }
    static constexpr double kA = 0.13819660112501051518;   // (5 - sqrt5)/20
    static constexpr double kB = 0.58541019662496845446;   // 1 - 3a
    __host__ __device__ static constexpr double w(int) { return 1.0 / 24.0; }
    __host__ __device__ static constexpr double N(int g, int a) { return a == g ? kB : kA; }
    __host__ __device__ static constexpr double dN(int, int a, int j) { return a == 0 ? -1.0 : (a == j + 1 ? 1.0 : 0.0); }
};

// Linear prism: triangle (0,0),(1,0),(0,1) x zeta in [-1,1], nodes 0-2 at
// zeta = -1 and 3-5 above them; N_a = L_i (1 -+ zeta)/2 with the barycentric
// L = (1-xi-eta, xi, eta).  Rule: the degree-2 triangle points (1/6,1/6),
// (2/3,1/6), (1/6,2/3) x Gauss-Legendre +-1/sqrt3 (point g: triangle point
// g % 3, zeta side g / 3), weights 1/6.
struct Pen {
    static constexpr int NEN = 6, NG = 6;
    static constexpr bool kRolled = true, kSparse = false;
    static constexpr double kG = 0.57735026918962576451;
    __host__ __device__ static constexpr double px(int g) { return g % 3 == 1 ? 2.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr double py(int g) { return g % 3 == 2 ? 2.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr double pz(int g) { return g >= 3 ? kG : -kG; }
    __host__ __device__ static constexpr double bary(int i, int g)
    {
        return i == 0 ? 1.0 - px(g) - py(g) : i == 1 ? px(g) : py(g);
    }
    __host__ __device__ static constexpr double side(int a) { return a >= 3 ? 1.0 : -1.0; }
    __host__ __device__ static constexpr double w(int) { return 1.0 / 6.0; }
    __host__ __device__ static constexpr double N(int g, int a)
    {
        return bary(a % 3, g) * 0.5 * (1.0 + side(a) * pz(g));
    }
    __host__ __device__ static constexpr double dN(int g, int a, int j)
    {
        // d bary / d xi = (-1, 1, 0), d bary / d eta = (-1, 0, 1)
        return j == 2 ? 0.5 * side(a) * bary(a % 3, g)
                      : (a % 3 == 0 ? -1.0 : (a % 3 == j + 1 ? 1.0 : 0.0)) * 0.5 * (1.0 + side(a) * pz(g));
    }
};

// Pyramid on the base [-1,1]^2 at zeta = 0 (nodes 0-3 at (-,-), (+,-), (+,+),
// (-,+)) with the apex, node 4, at (0,0,1).  Rational basis, m = 1 - zeta:
// N_a = (m + sx xi)(m + sy eta) / (4m), N_4 = zeta.  Rule: conical product,
// (xi, eta) = m (+-1/sqrt3, +-1/sqrt3) and zeta at the 2-point Gauss-Jacobi
// nodes for the weight (1-zeta)^2 on [0,1], 1/3 -+ sqrt10/15, with weights
// 1/6 +- sqrt10/48 (point g: xi side bit 0, eta side bit 1, zeta node bit 2).
struct Pyr {
    static constexpr int NEN = 5, NG = 8;
    static constexpr bool kRolled = true, kSparse = false;
    static constexpr double kG = 0.57735026918962576451;    // 1/sqrt(3)
    static constexpr double kR = 3.16227766016837933200;    // sqrt(10)
    __host__ __device__ static constexpr double pz(int g) { return (g & 4) ? 1.0 / 3.0 + kR / 15.0 : 1.0 / 3.0 - kR / 15.0; }
    __host__ __device__ static constexpr double pm(int g) { return 1.0 - pz(g); }
    __host__ __device__ static constexpr double px(int g) { return ((g & 1) ? kG : -kG) * pm(g); }
    __host__ __device__ static constexpr double py(int g) { return ((g & 2) ? kG : -kG) * pm(g); }
    __host__ __device__ static constexpr double sx(int a) { return (a == 1 || a == 2) ? 1.0 : -1.0; }
    __host__ __device__ static constexpr double sy(int a) { return a >= 2 ? 1.0 : -1.0; }
    __host__ __device__ static constexpr double w(int g) { return (g & 4) ? 1.0 / 6.0 - kR / 48.0 : 1.0 / 6.0 + kR / 48.0; }
    __host__ __device__ static constexpr double N(int g, int a)
    {
        return a == 4 ? pz(g) : (pm(g) + sx(a) * px(g)) * (pm(g) + sy(a) * py(g)) / (4.0 * pm(g));
    }
    __host__ __device__ static constexpr double dN(int g, int a, int j)
    {
        return a == 4 ? (j == 2 ? 1.0 : 0.0)
             : j == 0 ? sx(a) * (pm(g) + sy(a) * py(g)) / (4.0 * pm(g))
             : j == 1 ? sy(a) * (pm(g) + sx(a) * px(g)) / (4.0 * pm(g))
                      : (sx(a) * sy(a) * px(g) * py(g) - pm(g) * pm(g)) / (4.0 * pm(g) * pm(g));
    }
};

__constant__ RefTables<Pen> kPenTab = make_tables<Pen>();
__constant__ RefTables<Pyr> kPyrTab = make_tables<Pyr>();

struct KArgs {
    const double *X;
    const int32_t *blk_elem_ptr, *blk_node_ptr, *blk_nodes, *blk_rdesc, *blk_rowstart, *color_blk;
    const uint8_t *blk_nphase, *elem_off, *elem_phase;
    const uint16_t *elem_lnode;
    int64_t N, E;
    int off_stride;           // bytes of elem_off per element
    int form;                 // residual pass: FE_FORM_* operator variants
    const double *u, *rho, *mu, *Y, *p;
    double dt, Dk;
    double *values, *rhs;
    double *blk_mindet;       // [nblk] per-block smallest det J
    long long *blk_bad;       // [nblk] per-block first bad element (mesh index) or -1
    int blk_offset;
};

template <int OP> struct OpTraits;
template <> struct OpTraits<FE_OP_MOMENTUM> { static constexpr int NF = 8, NRHS = 3; };
template <> struct OpTraits<FE_OP_SCALAR> { static constexpr int NF = 8, NRHS = 1; };
template <> struct OpTraits<FE_OP_POISSON> { static constexpr int NF = 7, NRHS = 1; };
template <> struct OpTraits<kOpResidual> { static constexpr int NF = 8, NRHS = 4; };    // r_x, r_y, r_z, lumped mass
template <> struct OpTraits<kOpGradient> { static constexpr int NF = 4, NRHS = 3; };    // x, y, z, p
template <> struct OpTraits<kOpDivergence> { static constexpr int NF = 7, NRHS = 1; };
template <> struct OpTraits<kOpScalarResidual> { static constexpr int NF = 8, NRHS = 2; };   // r, lumped mass

// Waves per element block: a HEX08 element's 8 rows are split between two
// waves (4 rows each) so that a wave needs <= 256 registers and two blocks'
// waves share each SIMD; a TET04 element stays on one lane.
template <class EL> struct Split { static constexpr int W = EL::NEN == 8 ? 2 : 1; };

__device__ inline void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <class EL> __device__ inline double RefN(int g, int a);
template <class EL> __device__ inline double RefdN(int g, int a, int j);
template <> __device__ inline double RefN<Hex>(int g, int a) { return kHexTab.N[g][a]; }
template <> __device__ inline double RefdN<Hex>(int g, int a, int j) { return kHexTab.dN[g][a][j]; }
template <> __device__ inline double RefN<Tet>(int g, int a) { return Tet::N(g, a); }
template <> __device__ inline double RefdN<Tet>(int g, int a, int j) { return Tet::dN(g, a, j); }
template <> __device__ inline double RefN<Pen>(int g, int a) { return kPenTab.N[g][a]; }
template <> __device__ inline double RefdN<Pen>(int g, int a, int j) { return kPenTab.dN[g][a][j]; }
template <> __device__ inline double RefN<Pyr>(int g, int a) { return kPyrTab.N[g][a]; }
template <> __device__ inline double RefdN<Pyr>(int g, int a, int j) { return kPyrTab.dN[g][a][j]; }

// One Gauss point for rows [a0, a0 + RA) of the elemental matrix.
// Geometry in FP64 (from the LDS-staged nodal data), products in Q.
//   MOM/SCA: A_ab += N_a s_b + wk grad N_a . grad N_b,
//            s_b = rho dV (N_b / dt + u . grad N_b), wk = mu dV or rho D dV;
//            B_a += rho dV / dt N_a f, f = u (MOM) or Y (SCA).
//   POI    : A_ab += dV grad N_a . grad N_b,
//            B_a += dV / dt grad N_a . (rho u).
// Geometry of one element kept in registers for the Gauss loop: HEX08 the
// trilinear coefficients c1..c7 of x(xi), the other types the node coordinates.
template <class EL> struct Geo { double v[EL::NEN == 8 ? 7 : EL::NEN][3]; };

template <class EL>
__device__ __forceinline__ void load_geo(const double *nd, int T, const int (&ln)[EL::NEN], Geo<EL> &G)
{
    constexpr int NEN = EL::NEN;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double x[NEN];
#pragma unroll
        for (int a = 0; a < NEN; ++a) x[a] = nd[i * T + ln[a]];
        if (NEN == 8) {
#pragma unroll
            for (int m = 1; m < 8; ++m) {
                double sum = 0.0;
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    const int sx = Hex::sx(a), sy = Hex::sy(a), sz = Hex::sz(a);
                    const int sgn = m == 1 ? sx : m == 2 ? sy : m == 3 ? sz : m == 4 ? sx * sy
                                  : m == 5 ? sy * sz : m == 6 ? sx * sz : sx * sy * sz;
                    sum = sgn > 0 ? sum + x[a] : sum - x[a];
                }
                G.v[m - 1][i] = 0.125 * sum;
            }
        } else {
#pragma unroll
            for (int a = 0; a < NEN; ++a) G.v[a][i] = x[a];
        }
    }
}

// Jacobian of the map at Gauss point g, its determinant (returned) and inverse.
template <class EL>
__device__ __forceinline__ double jacobian_inverse(int g, const Geo<EL> &GE, double (&Ji)[3][3])
{
    constexpr int NEN = EL::NEN;
    const auto &geo = GE.v;
    double J[3][3];
    if (NEN == 8) {
        // x(xi) = c0 + c1 xi + c2 eta + c3 zeta + c4 xi eta + c5 eta zeta + c6 xi zeta
        //         + c7 xi eta zeta (geo[m-1] = c_m): each Jacobian column is 3 FMAs.
        const double xi = (g & 1) ? Hex::kG : -Hex::kG;
        const double et = (g & 2) ? Hex::kG : -Hex::kG;
        const double ze = (g & 4) ? Hex::kG : -Hex::kG;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            J[i][0] = geo[0][i] + et * geo[3][i] + ze * geo[5][i] + (et * ze) * geo[6][i];
            J[i][1] = geo[1][i] + xi * geo[3][i] + ze * geo[4][i] + (xi * ze) * geo[6][i];
            J[i][2] = geo[2][i] + et * geo[4][i] + xi * geo[5][i] + (xi * et) * geo[6][i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < NEN; ++a) {
                    const double d = RefdN<EL>(g, a, j);
                    if (!EL::kSparse || d != 0.0) s += geo[a][i] * d;
                }
                J[i][j] = s;
            }
    }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = 1.0 / det;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    return det;
}

// One Gauss point of an element-vector pass for rows [A0, A0 + RA), FP64,
// from the physical gradients dN and dV = w det J:
//   OP_RES: B_i[a] -= dV (rho N_a (u . grad u_i) + mu grad N_a . grad u_i), i < 3,
//           B_3[a] += dV rho N_a (lumped mass); form FE_FORM_FULL_STRESS adds
//           mu (d u_j / d x_i)(d N_a / d x_j) (the viscous term 2 mu eps(u)),
//           FE_FORM_EMAC adds rho N_a (div u) u_i (Eq. (1)'s convective form
//           at the Gauss point);
//   OP_GRD: B_j[a] += dV N_a (grad p)_j;
//   OP_DIV: B_0[a] += dV / dt grad N_a . (rho u);
//   OP_SRS: B_0[a] -= dV rho (N_a (u . grad Y) + D grad N_a . grad Y),
//           B_1[a] += dV rho N_a (Y in slot 7, D = Dk).
// Fields in LDS: x, y, z, then u_x, u_y, u_z, rho, mu (OP_GRD: p in slot 3).
template <class EL, int OP, int RA, int A0>
__device__ __forceinline__ void element_vector_point(int g, const double *nd, int T, const int (&ln)[EL::NEN],
                                                     const double (&dN)[EL::NEN][3], double dV,
                                                     double (&B)[OpTraits<OP>::NRHS][RA], double inv_dt,
                                                     int form, double Dk)
{
    constexpr int NEN = EL::NEN;
    if constexpr (OP == OP_SRS) {
        double rg = 0.0, ug[3] = {0.0, 0.0, 0.0}, gy[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            const double Nb = RefN<EL>(g, b), yb = nd[7 * T + ln[b]];
            rg += Nb * nd[6 * T + ln[b]];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ug[i] += Nb * nd[(3 + i) * T + ln[b]];
                gy[i] += dN[b][i] * yb;
            }
        }
        const double adv = ug[0] * gy[0] + ug[1] * gy[1] + ug[2] * gy[2], w = dV * rg;
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const int a = A0 + r;
            const double Na = RefN<EL>(g, a);
            const double dif = dN[a][0] * gy[0] + dN[a][1] * gy[1] + dN[a][2] * gy[2];
            B[0][r] -= w * (Na * adv + Dk * dif);
            B[1][r] += w * Na;
        }
    } else if constexpr (OP == OP_GRD) {
        double gp[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            const double pb = nd[3 * T + ln[b]];
#pragma unroll
            for (int j = 0; j < 3; ++j) gp[j] += dN[b][j] * pb;
        }
#pragma unroll
        for (int r = 0; r < RA; ++r) {
            const double wn = dV * RefN<EL>(g, A0 + r);
#pragma unroll
            for (int j = 0; j < 3; ++j) B[j][r] += wn * gp[j];
        }
    } else {
        double rg = 0.0, mg = 0.0, ug[3] = {0.0, 0.0, 0.0}, gu[3][3] = {};
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            const double Nb = RefN<EL>(g, b);
            rg += Nb * nd[6 * T + ln[b]];
            if (OP == OP_RES) mg += Nb * nd[7 * T + ln[b]];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double ub = nd[(3 + i) * T + ln[b]];
                ug[i] += Nb * ub;
                if (OP == OP_RES) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) gu[i][j] += dN[b][j] * ub;   // d u_i / d x_j
                }
            }
        }
        if constexpr (OP == OP_RES) {
            const bool full = (form & FE_FORM_FULL_STRESS) != 0, emac = (form & FE_FORM_EMAC) != 0;
            const double divu = gu[0][0] + gu[1][1] + gu[2][2];
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const int a = A0 + r;
                const double wr = dV * rg * RefN<EL>(g, a), wm = dV * mg;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    double adv = ug[0] * gu[i][0] + ug[1] * gu[i][1] + ug[2] * gu[i][2];
                    double vis = dN[a][0] * gu[i][0] + dN[a][1] * gu[i][1] + dN[a][2] * gu[i][2];
                    if (full) vis += dN[a][0] * gu[0][i] + dN[a][1] * gu[1][i] + dN[a][2] * gu[2][i];
                    if (emac) adv += divu * ug[i];
                    B[i][r] -= wr * adv + wm * vis;
                }
                B[3][r] += wr;
            }
        } else {
            const double f0 = rg * ug[0], f1 = rg * ug[1], f2 = rg * ug[2], w = dV * inv_dt;
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const int a = A0 + r;
                B[0][r] += w * (dN[a][0] * f0 + dN[a][1] * f1 + dN[a][2] * f2);
            }
        }
    }
}

template <class EL, int OP, class Q, int RA, int A0, class FT>
__device__ __forceinline__ void gauss_point(int g, const Geo<EL> &GE, const double *nd, const FT *nf, int T,
                                            const int (&ln)[EL::NEN],
                                            Q (&A)[RA][EL::NEN], Q (&B)[OpTraits<OP>::NRHS][RA], double &mindet,
                                            double inv_dt, double Dk, int form)
{
    constexpr int NEN = EL::NEN;
    double Ji[3][3];
    const double det = jacobian_inverse<EL>(g, GE, Ji);
    mindet = fmin(mindet, det);
    // physical gradients grad N_a = J^-T grad_ref N_a (all nodes: needed for columns)
    Q dN[NEN][3];
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double d = RefdN<EL>(g, a, j);
                if (!EL::kSparse || d != 0.0) s += Ji[j][i] * d;
            }
            dN[a][i] = Q(s);
        }
    if constexpr (OP >= OP_RES) {
        element_vector_point<EL, OP, RA, A0>(g, nd, T, ln, dN, EL::w(g) * det, B, inv_dt, form, Dk);
    } else {
        // nf: the fields after x, y, z (u_x, u_y, u_z, rho, mu / Y), interpolated
        // in their staged precision FT
        FT rg = 0, fg = 0, ug0 = 0, ug1 = 0, ug2 = 0;
#pragma unroll
        for (int a = 0; a < NEN; ++a) {
            const FT Na = FT(RefN<EL>(g, a));
            rg += Na * nf[3 * T + ln[a]];
            ug0 += Na * nf[0 * T + ln[a]];
            ug1 += Na * nf[1 * T + ln[a]];
            ug2 += Na * nf[2 * T + ln[a]];
            if (OP != OP_POI) fg += Na * nf[4 * T + ln[a]];
        }
        const double dV = EL::w(g) * det;
        if (OP == OP_POI) {
            const Q qdV = Q(dV), qi = Q(inv_dt);
            const Q f0 = Q(rg * ug0), f1 = Q(rg * ug1), f2 = Q(rg * ug2);
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const int a = A0 + r;
                const Q G0 = qdV * dN[a][0], G1 = qdV * dN[a][1], G2 = qdV * dN[a][2];
#pragma unroll
                for (int b = 0; b < NEN; ++b) A[r][b] += G0 * dN[b][0] + G1 * dN[b][1] + G2 * dN[b][2];
                B[0][r] += qi * (G0 * f0 + G1 * f1 + G2 * f2);
            }
        } else {
            const Q w1 = Q(dV) * Q(rg);
            const Q wk = (OP == OP_MOM) ? Q(dV) * Q(fg) : Q(dV) * (Q(rg) * Q(Dk));   // fg = mu (MOM) or Y (SCA)
            const Q qi = Q(inv_dt);
            const Q qu0 = Q(ug0), qu1 = Q(ug1), qu2 = Q(ug2);
            Q s[NEN];
#pragma unroll
            for (int b = 0; b < NEN; ++b)
                s[b] = w1 * (Q(RefN<EL>(g, b)) * qi + (qu0 * dN[b][0] + qu1 * dN[b][1] + qu2 * dN[b][2]));
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const int a = A0 + r;
                const Q Na = Q(RefN<EL>(g, a));
                const Q G0 = wk * dN[a][0], G1 = wk * dN[a][1], G2 = wk * dN[a][2];
#pragma unroll
                for (int b = 0; b < NEN; ++b) A[r][b] += Na * s[b] + (G0 * dN[b][0] + G1 * dN[b][1] + G2 * dN[b][2]);
                const Q wn = w1 * Na * qi;
                if (OP == OP_MOM) {
                    B[0][r] += wn * qu0;
                    B[1][r] += wn * qu1;
                    B[2][r] += wn * qu2;
                } else {
                    B[0][r] += wn * Q(fg);
                }
            }
        }
    }
}

// All Gauss points of one element for rows [A0, A0 + RA).  ln is taken by
// value: the loop makes its copy opaque at every point so that the nodal
// field reads are re-issued from LDS instead of being hoisted into registers.
template <class EL> struct Rows { int v[EL::NEN]; };

template <class EL, int OP, class Q, int RA, int A0, class FT = double>
__device__ __forceinline__ void gauss_loop(const Geo<EL> &GE, const double *nd, const FT *nf, int T, Rows<EL> rows,
                                           Q (&A)[RA][EL::NEN], Q (&B)[OpTraits<OP>::NRHS][RA], double &mindet,
                                           double inv_dt, double Dk, int form)
{
    constexpr int NEN = EL::NEN, NG = EL::NG;
    int ln[NEN];
#pragma unroll
    for (int a = 0; a < NEN; ++a) ln[a] = rows.v[a];
    if (EL::kRolled) {
#pragma unroll 1
        for (int g = 0; g < NG; ++g) {
#pragma unroll
            for (int a = 0; a < NEN; ++a) asm volatile("" : "+v"(ln[a]));
            gauss_point<EL, OP, Q, RA, A0, FT>(g, GE, nd, nf, T, ln, A, B, mindet, inv_dt, Dk, form);
        }
    } else {
#pragma unroll
        for (int g = 0; g < NG; ++g)
            gauss_point<EL, OP, Q, RA, A0, FT>(g, GE, nd, nf, T, ln, A, B, mindet, inv_dt, Dk, form);
    }
}

// One work-group = one block of <= 64 elements = W waves.  Lane l computes
// rows [a0, a0 + RA) of element l mod 64 with a0 = (l / 64) * RA.
// The block body of every assembly and element-vector pass: block
// color_blk[blk_offset + wg] of the launch.  FORM >= 0 fixes the residual
// pass's operator variants at compile time; -1 reads them from the arguments.
template <class EL, int OP, class Q, int FORM>
__device__ __forceinline__ void assemble_block(const KArgs &k, int wg)
{
    constexpr int NEN = EL::NEN, NG = EL::NG, W = Split<EL>::W, RA = NEN / W, NT = 64 * W;
    constexpr int NF = OpTraits<OP>::NF, NRHS = OpTraits<OP>::NRHS;
    constexpr bool VEC = OP >= OP_RES;       // element-vector pass: no row image
    extern __shared__ double lds[];

    const int blk = k.color_blk[k.blk_offset + wg];
    const int e0 = k.blk_elem_ptr[blk], ne = k.blk_elem_ptr[blk + 1] - e0;
    const int n0 = k.blk_node_ptr[blk], T = k.blk_node_ptr[blk + 1] - n0;
    const int tid = threadIdx.x;
    const int el = tid & 63, wv = tid >> 6, a0 = wv * RA;
    const int64_t N = k.N;

    double *nd = lds;                        // [NF][T] nodal fields
    double *rimg = nd + NF * T;              // [NRHS][T] rhs image
    int *rdesc = (int *)(rimg + NRHS * T);   // [T] row descriptors
    double *img = (double *)(rdesc + T + (T & 1));   // 8-byte aligned row image (matrix passes)

    // Element data that depends only on the block: issue these loads first.
    const bool act = el < ne;
    const int e = e0 + (act ? el : 0);
    int ln[NEN];
#pragma unroll
    for (int a = 0; a < NEN; ++a) ln[a] = k.elem_lnode[(int64_t)a * k.E + e];
    // in-row offsets of this lane's rows: a multiple of 4 bytes from a 4-byte
    // boundary (off_stride is a multiple of 4, a0 * NEN is 0 or 32), padded
    // to whole words inside the element's slot
    constexpr int kOffWords = (RA * NEN + 3) / 4;
    uint32_t offw[kOffWords];
    if constexpr (!VEC) {
        const uint32_t *op = (const uint32_t *)(k.elem_off + (int64_t)e * k.off_stride + a0 * NEN);
#pragma unroll
        for (int q = 0; q < kOffWords; ++q) offw[q] = op[q];
    }
    const int ph = act ? (int)k.elem_phase[e] : -1;

    // 1. stage, one touched row per lane: nodal fields, rhs and the row's
    //    previous partial sums (zero for the first writer) into LDS.  Two
    //    dependent load rounds: the block's row tables, then fields + values.
    constexpr int kRowBatch = 32;   // columns loaded per batch (rows are <= 255)
    for (int t = tid; t < T; t += NT) {
        const int g = k.blk_nodes[n0 + t];
        const int rd = k.blk_rdesc[n0 + t];
        const int r0 = VEC ? 0 : k.blk_rowstart[n0 + t];   // matrix passes: the row in CSR
        const int len = VEC ? 0 : (rd >> 16) & 0xff, base = rd & 0xffff;
        const bool first = rd < 0;
        double f[NF + NRHS];
        f[0] = k.X[g];
        f[1] = k.X[N + g];
        f[2] = k.X[2 * N + g];
        if constexpr (OP == OP_GRD) {
            f[3] = k.p[g];
        } else {
            f[3] = k.u[g];
            f[4] = k.u[N + g];
            f[5] = k.u[2 * N + g];
            f[6] = k.rho[g];
            if (OP == OP_MOM || OP == OP_RES) f[7] = k.mu[g];
            if (OP == OP_SCA || OP == OP_SRS) f[7] = k.Y[g];
        }
#pragma unroll
        for (int r = 0; r < NRHS; ++r) f[NF + r] = first ? 0.0 : k.rhs[r * N + g];
        // matrix passes: the row's previous values, loaded before the LDS
        // writes below so that the loads overlap them
        double v[kRowBatch];
        if constexpr (!VEC) {
#pragma unroll
            for (int q = 0; q < kRowBatch; ++q) v[q] = (!first && q < len) ? k.values[r0 + q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NF; ++q) nd[q * T + t] = f[q];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) rimg[r * T + t] = f[NF + r];
        rdesc[t] = rd;
        if constexpr (!VEC) {
#pragma unroll
            for (int q = 0; q < kRowBatch; ++q)
                if (q < len) img[base + q] = v[q];
            for (int q = kRowBatch; q < len; ++q) img[base + q] = first ? 0.0 : k.values[r0 + q];
        }
    }
    __syncthreads();

    // 3. elemental matrix rows of this lane
    Q A[RA][NEN];
    Q B[NRHS][RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) {
#pragma unroll
        for (int b = 0; b < NEN; ++b) A[r][b] = Q(0);
#pragma unroll
        for (int q = 0; q < NRHS; ++q) B[q][r] = Q(0);
    }
    double mindet = __builtin_huge_val();
    const double inv_dt = 1.0 / k.dt;
    Geo<EL> GE;
    load_geo<EL>(nd, T, ln, GE);
    // the row range is a compile-time constant in each branch (wave-uniform)
    {
        Rows<EL> rows;
#pragma unroll
        for (int a = 0; a < NEN; ++a) rows.v[a] = ln[a];
        const int form = FORM >= 0 ? FORM : k.form;
        if (W == 1 || wv == 0)
            gauss_loop<EL, OP, Q, RA, 0>(GE, nd, nd + 3 * T, T, rows, A, B, mindet, inv_dt, k.Dk, form);
        else
            gauss_loop<EL, OP, Q, RA, (RA % NEN)>(GE, nd, nd + 3 * T, T, rows, A, B, mindet, inv_dt, k.Dk, form);
    }
    // this lane's rows of the element, selected without dynamic indexing
    int lr[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) {
        // arithmetic blend (a select of two loads would become one load at a
        // computed address and push ln[] to scratch)
        const int hi = (W == 1) ? 0 : wv;
        lr[r] = ln[r] + hi * (ln[(RA + r) % NEN] - ln[r]);
    }

    // 4. scatter into the LDS images: wave by wave, then phase by phase, then
    //    in (a, b) order -- no two lanes of one instruction hit one address.
    int base[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) base[r] = VEC ? 0 : rdesc[lr[r]] & 0xffff;
    const int nph = k.blk_nphase[blk];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (wv == w) {
            for (int p = 0; p < nph; ++p) {
                if (ph == p) {
#pragma unroll
                    for (int r = 0; r < RA; ++r) {
                        if constexpr (!VEC) {
#pragma unroll
                            for (int b = 0; b < NEN; ++b) {
                                const int idx = r * NEN + b;
                                const int off = (offw[idx >> 2] >> (8 * (idx & 3))) & 0xff;
                                lds_add(&img[base[r] + off], (double)A[r][b]);
                            }
                        }
#pragma unroll
                        for (int q = 0; q < NRHS; ++q) lds_add(&rimg[q * T + lr[r]], (double)B[q][r]);
                    }
                }
            }
        }
        if (W > 1) __syncthreads();
    }

    // status: per-block smallest det J and first non-positive element
    if (wv == 0) {
        double md = act ? mindet : __builtin_huge_val();
        long long bad = (act && !(mindet > 0.0)) ? (long long)e : (long long)0x7fffffffffffffffLL;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            md = fmin(md, __shfl_xor(md, o));
            const long long ob = __shfl_xor(bad, o);
            bad = ob < bad ? ob : bad;
        }
        if (el == 0) {
            k.blk_mindet[blk] = md;
            k.blk_bad[blk] = bad == 0x7fffffffffffffffLL ? -1 : bad;
        }
    }
    __syncthreads();

    // 5. write back, one touched row per lane (LDS reads batched ahead of the
    //    stores)
    for (int t = tid; t < T && !VEC; t += NT) {
        const int rd = rdesc[t];
        const int64_t r0 = k.blk_rowstart[n0 + t];
        const int len = (rd >> 16) & 0xff, base = rd & 0xffff;
        double v[kRowBatch];
#pragma unroll
        for (int q = 0; q < kRowBatch; ++q)
            if (q < len) v[q] = img[base + q];
#pragma unroll
        for (int q = 0; q < kRowBatch; ++q)
            if (q < len) k.values[r0 + q] = v[q];
        for (int q = kRowBatch; q < len; ++q) k.values[r0 + q] = img[base + q];
    }
    for (int t = tid; t < T; t += NT) {
        const int g = k.blk_nodes[n0 + t];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) k.rhs[r * N + g] = rimg[r * T + t];
    }
}

template <class EL, int OP, class Q>
__global__ void __launch_bounds__(64 * Split<EL>::W, 2) k_assemble(KArgs k)
{
    assemble_block<EL, OP, Q, -1>(k, blockIdx.x);
}

// Batched coloured assembly (the serving runtime): one launch runs the same
// (colour, type) launch of several meshes.  Work-group w belongs to entry j
// with wgs[j] <= w < wgs[j + 1] (a handful of entries: a linear scan); the
// entry's kernel arguments are ks[slot[j]], its blocks color_blk[first[j] +
// w - wgs[j]].  Each block runs the code of k_assemble, so a mesh's results
// do not depend on what shares the launch.
struct AsmBatch {
    int n;
    int slot[kMaxBatch];
    int first[kMaxBatch];
    int wgs[kMaxBatch + 1];
};
static_assert(sizeof(KArgs) <= kKArgsBytes, "the device table's slot size");

template <class EL, int OP>
__global__ void __launch_bounds__(64 * Split<EL>::W, 2) k_bat_assemble(const KArgs *__restrict__ ks, AsmBatch B)
{
    int j = 0;
    while (j + 1 < B.n && (int)blockIdx.x >= B.wgs[j + 1]) ++j;
    // read in place (its blk_offset is 0): a copy would hold every field live
    const KArgs &k = *(const KArgs *)((const char *)ks + (size_t)B.slot[j] * kKArgsBytes);
    assemble_block<EL, OP, double, -1>(k, B.first[j] + (int)blockIdx.x - B.wgs[j]);
}

// The momentum residual pass with its operator variants (FE_FORM_* bits)
// fixed at compile time.
template <class EL, int FORM>
__global__ void __launch_bounds__(64 * Split<EL>::W, 2) k_residual(KArgs k)
{
    assemble_block<EL, OP_RES, double, FORM>(k, blockIdx.x);
}

// ---- owner assembly of the matrix operators ---------------------------------
// One work-group owns a group of consecutive CSR rows and computes every
// element contribution to them, so each row is written once and never read
// back, in a single launch (no colours).  Steps:
//   1. stage the group's touched nodes' fields in LDS (owned rows first);
//      zero the owned rows' image and right-hand sides;
//   2. one task per lane: the Gauss loop of rows [0, RA) of its element,
//      presented in the task's node order (a HEX08 element rotated so that
//      the rows the group owns lie on its first face);
//   3. phase by phase (a barrier between phases), add the owned rows of the
//      tasks of that phase into LDS: the tasks of one phase hold distinct
//      owned rows, so no two lanes add to one address and the order of the
//      sums is fixed by the plan.  Wave-private form (PRIV, element types
//      whose nodes lie in many elements): each wave adds into its own copy
//      of the rows, phases within the wave, no barriers; the copies are
//      then summed in wave order;
//   4. write the rows (contiguous in CSR) and right-hand sides once.
struct OArgs {
    const double *X;
    const int32_t *rowptr;
    const int4 *groups;
    const int32_t *node_ptr, *nodes, *elem;
    const uint8_t *nphase, *off, *phase;
    const uint16_t *ln;
    int ln_stride, off_stride;
    int64_t N;
    const double *u, *rho, *mu, *Y;
    double dt, Dk;
    double *values, *rhs;
    double *g_mindet;
    long long *g_bad;
};

template <class EL> struct OwnRows { static constexpr int RA = EL::NEN == 8 ? 4 : EL::NEN; };

// Work-groups are dispatched round-robin over MI355X's 8 XCDs (work-group b
// on XCD b % 8), each with its own L2.  xcd_item maps work-group b of a
// G-group launch to item i so that every XCD takes one contiguous range of
// items (a bijection of [0, G)).  Consecutive owner groups cover neighbouring
// rows and share halo nodes, so their cache lines of the nodal fields are then
// fetched once into that XCD's L2 instead of once into each of several.
constexpr int kAsmXcds = 8;
__device__ inline int xcd_item(int b, int G)
{
    const int q = G / kAsmXcds, rem = G % kAsmXcds, x = b % kAsmXcds, slot = b / kAsmXcds;
    return x * q + (x < rem ? x : rem) + slot;
}

template <class EL, int OP, class Q, bool PRIV>
__global__ void __launch_bounds__(kOwnTasks, 2) k_own(OArgs k)
{
    constexpr int NEN = EL::NEN, RA = OwnRows<EL>::RA;
    constexpr int NF = OpTraits<OP>::NF, NRHS = OpTraits<OP>::NRHS;
    extern __shared__ double lds[];
    const int gi = xcd_item(blockIdx.x, gridDim.x);   // this work-group's group
    const int4 gd = k.groups[gi];   // first task, tasks, first row, rows
    const int tid = threadIdx.x;
    const int r0 = gd.z, nr = gd.w;
    const int n0 = k.node_ptr[gi], T = k.node_ptr[gi + 1] - n0;
    const int64_t v0 = k.rowptr[r0];
    const int L = (int)(k.rowptr[r0 + nr] - v0);
    const int64_t N = k.N;
    constexpr int NC = PRIV ? kOwnTasks / 64 : 1;   // copies of the rows
    // Fields of the touched nodes: x, y, z in FP64 (the geometry is FP64 in
    // both modes), the others in the quadrature's precision (the mixed mode
    // interpolates them in FP32, which halves their LDS traffic).
    using FT = Q;
    double *nd = lds;                   // [3][T] coordinates
    FT *nf = (FT *)(nd + 3 * T);        // [NF - 3][T] u_x, u_y, u_z, rho, mu / Y
    double *img0 = nd + 3 * T + ((NF - 3) * T * (int)sizeof(FT) + 7) / 8;   // [NC][L] the owned rows
    double *rimg0 = img0 + NC * L;  // [NC][NRHS][nr] their right-hand sides
    double *img = img0 + (PRIV ? (tid >> 6) * L : 0);                 // this wave's copy
    double *rimg = rimg0 + (PRIV ? (tid >> 6) * NRHS * nr : 0);

    // task data first: its loads overlap the staging below
    const bool live = tid < gd.y;
    const int64_t t = gd.x + (live ? tid : 0);
    int ln[NEN];
    {
        const uint16_t *lp = k.ln + t * k.ln_stride;
#pragma unroll
        for (int a = 0; a < NEN; ++a) ln[a] = lp[a];
    }
    constexpr int kOffWords = (RA * NEN + 3) / 4;
    uint32_t offw[kOffWords];
    {
        const uint32_t *op = (const uint32_t *)(k.off + t * k.off_stride);
#pragma unroll
        for (int q = 0; q < kOffWords; ++q) offw[q] = op[q];
    }
    const int ph = live ? (int)k.phase[t] : -1;
    const int64_t elem = k.elem[t];

    // 1. stage
    for (int q = tid; q < T; q += kOwnTasks) {
        const int g = k.nodes[n0 + q];
        double f[NF];
        f[0] = k.X[g];
        f[1] = k.X[N + g];
        f[2] = k.X[2 * N + g];
        f[3] = k.u[g];
        f[4] = k.u[N + g];
        f[5] = k.u[2 * N + g];
        f[6] = k.rho[g];
        if constexpr (NF > 7) f[7] = OP == OP_MOM ? k.mu[g] : k.Y[g];
#pragma unroll
        for (int c = 0; c < 3; ++c) nd[c * T + q] = f[c];
#pragma unroll
        for (int c = 3; c < NF; ++c) nf[(c - 3) * T + q] = FT(f[c]);
    }
    for (int q = tid; q < NC * L; q += kOwnTasks) img0[q] = 0.0;
    for (int q = tid; q < NC * NRHS * nr; q += kOwnTasks) rimg0[q] = 0.0;
    __syncthreads();

    // 2. this lane's rows
    Q A[RA][NEN];
    Q B[NRHS][RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) {
#pragma unroll
        for (int b = 0; b < NEN; ++b) A[r][b] = Q(0);
#pragma unroll
        for (int q = 0; q < NRHS; ++q) B[q][r] = Q(0);
    }
    double mindet = __builtin_huge_val();
    if (live) {
        Geo<EL> GE;
        load_geo<EL>(nd, T, ln, GE);
        Rows<EL> rows;
#pragma unroll
        for (int a = 0; a < NEN; ++a) rows.v[a] = ln[a];
        gauss_loop<EL, OP, Q, RA, 0, FT>(GE, nd, nf, T, rows, A, B, mindet, 1.0 / k.dt, k.Dk, 0);
    }
    int base[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) base[r] = ln[r] < nr ? (int)(k.rowptr[r0 + ln[r]] - v0) : -1;

    // 3. phases
    const int nph = k.nphase[gi];
    for (int p = 0; p < nph; ++p) {
        if (ph == p) {
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                if (base[r] < 0) continue;   // a row another group owns
#pragma unroll
                for (int b = 0; b < NEN; ++b) {
                    const int idx = r * NEN + b;
                    const int o = (offw[idx >> 2] >> (8 * (idx & 3))) & 0xff;
                    lds_add(&img[base[r] + o], (double)A[r][b]);
                }
#pragma unroll
                for (int q = 0; q < NRHS; ++q) lds_add(&rimg[q * nr + ln[r]], (double)B[q][r]);
            }
        }
        if (!PRIV) __syncthreads();
    }
    if (PRIV) __syncthreads();

    // 4. write the owned rows and right-hand sides once (the wave copies
    //    summed in wave order)
    for (int q = tid; q < L; q += kOwnTasks) {
        double v = img0[q];
#pragma unroll
        for (int c = 1; c < NC; ++c) v += img0[c * L + q];
        k.values[v0 + q] = v;
    }
    for (int q = tid; q < NRHS * nr; q += kOwnTasks) {
        const int c = q / nr, i = q - c * nr;
        double v = rimg0[q];
#pragma unroll
        for (int w = 1; w < NC; ++w) v += rimg0[w * NRHS * nr + q];
        k.rhs[c * N + r0 + i] = v;
    }
    // status: the group's smallest det J and first element with det J <= 0
    __shared__ double smd[kOwnTasks / 64];
    __shared__ long long sbad[kOwnTasks / 64];
    double md = live ? mindet : __builtin_huge_val();
    long long bad = (live && !(mindet > 0.0)) ? (long long)elem : (long long)0x7fffffffffffffffLL;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        md = fmin(md, __shfl_xor(md, o));
        const long long ob = __shfl_xor(bad, o);
        bad = ob < bad ? ob : bad;
    }
    if ((tid & 63) == 0) {
        smd[tid >> 6] = md;
        sbad[tid >> 6] = bad;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int w = 1; w < kOwnTasks / 64; ++w) {
            md = fmin(md, smd[w]);
            bad = sbad[w] < bad ? sbad[w] : bad;
        }
        k.g_mindet[gi] = md;
        k.g_bad[gi] = bad == 0x7fffffffffffffffLL ? -1 : bad;
    }
}

// HEX08 accumulates into one copy of the group's rows, the other types
// wave-privately (the planner's choice, OwnerPlan::wave_private).
template <class EL, int OP>
void launch_own_op(const OArgs &k, int64_t G, size_t lds, bool mixed, hipStream_t s)
{
    constexpr bool PRIV = EL::NEN != 8;
    if (mixed) hipLaunchKernelGGL((k_own<EL, OP, float, PRIV>), dim3((unsigned)G), dim3(kOwnTasks), lds, s, k);
    else hipLaunchKernelGGL((k_own<EL, OP, double, PRIV>), dim3((unsigned)G), dim3(kOwnTasks), lds, s, k);
}

template <class EL>
void launch_own(const OArgs &k, int op, int64_t G, size_t lds, bool mixed, hipStream_t s)
{
    switch (op) {
    case OP_MOM: launch_own_op<EL, OP_MOM>(k, G, lds, mixed, s); break;
    case OP_SCA: launch_own_op<EL, OP_SCA>(k, G, lds, mixed, s); break;
    default: launch_own_op<EL, OP_POI>(k, G, lds, mixed, s); break;
    }
}

// Reduce the per-block status into (min det, first bad mesh element): one
// group of 1024 threads, four independent loads in flight per thread.
constexpr int kStatusThreads = 1024;
__global__ void __launch_bounds__(kStatusThreads) k_asm_status(const double *mindet, const long long *bad, int64_t n,
                                                               AsmStatus *out)
{
    __shared__ double sd[kStatusThreads];
    __shared__ long long sb[kStatusThreads];
    double md = __builtin_huge_val();
    long long b = 0x7fffffffffffffffLL;
    const int64_t t = threadIdx.x;
    for (int64_t i = t; i < n; i += 4 * kStatusThreads) {
        double m4[4];
        long long b4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ii = i + u * kStatusThreads;
            m4[u] = ii < n ? mindet[ii] : __builtin_huge_val();
            b4[u] = ii < n ? bad[ii] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            md = fmin(md, m4[u]);
            if (b4[u] >= 0 && b4[u] < b) b = b4[u];
        }
    }
    sd[t] = md;
    sb[t] = b;
    __syncthreads();
    for (int s = kStatusThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            sd[t] = fmin(sd[t], sd[t + s]);
            if (sb[t + s] < sb[t]) sb[t] = sb[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        double d = sd[0];
        unsigned long long u;
        __builtin_memcpy(&u, &d, 8);
        out->min_det_key = u;
        out->first_bad = sb[0] == 0x7fffffffffffffffLL ? -1 : sb[0];
    }
}

template <class EL, int OP, class Q>
void launch_one(const AsmLaunch &L, KArgs k, hipStream_t s)
{
    k.blk_offset = L.first;
    hipLaunchKernelGGL((k_assemble<EL, OP, Q>), dim3(L.count), dim3(64 * Split<EL>::W), L.lds[OP], s, k);
}

template <class EL, int FORM>
void launch_residual(const AsmLaunch &L, KArgs k, hipStream_t s)
{
    k.blk_offset = L.first;
    hipLaunchKernelGGL((k_residual<EL, FORM>), dim3(L.count), dim3(64 * Split<EL>::W), L.lds[OP_RES], s, k);
}

template <class EL>
void launch_type(const AsmLaunch &L, const KArgs &k, int op, bool mixed, hipStream_t s)
{
    switch (op) {
    case OP_MOM: mixed ? launch_one<EL, OP_MOM, float>(L, k, s) : launch_one<EL, OP_MOM, double>(L, k, s); break;
    case OP_SCA: mixed ? launch_one<EL, OP_SCA, float>(L, k, s) : launch_one<EL, OP_SCA, double>(L, k, s); break;
    case OP_POI: mixed ? launch_one<EL, OP_POI, float>(L, k, s) : launch_one<EL, OP_POI, double>(L, k, s); break;
    // element-vector passes are FP64 only
    case OP_RES:
        switch (k.form) {
        case 0: launch_residual<EL, 0>(L, k, s); break;
        case 1: launch_residual<EL, 1>(L, k, s); break;
        case 2: launch_residual<EL, 2>(L, k, s); break;
        default: launch_residual<EL, 3>(L, k, s); break;
        }
        break;
    case OP_GRD: launch_one<EL, OP_GRD, double>(L, k, s); break;
    case OP_SRS: launch_one<EL, OP_SRS, double>(L, k, s); break;
    default: launch_one<EL, OP_DIV, double>(L, k, s); break;
    }
}

// ---- momentum operator with the full-stress viscous term: 3x3 blocks ------
// Eq. (1)'s viscous term -div(2 mu eps(u)) tested with N_a e_i couples the
// velocity components.  Row (a, i), column (b, k) of the element matrix:
//   delta_ik (M_ab / dt + C_ab + K_ab [+ E_ab]) [+ T_ab[i][k]],
//   T_ab[i][k] = sum_g dV mu_g (dN_a / dx_k)(dN_b / dx_i)   (FE_FORM_FULL_STRESS),
//   E_ab = sum_g dV rho_g (div u)_g N_a N_b                  (FE_FORM_EMAC),
// with M, C, K those of the scalar momentum operator.  Row-owner form: one
// lane per (element, row) task, one wavefront per group of whole rows, the
// rows' block values accumulated in LDS in phase order (a row's tasks in
// element order) and written to HBM once, contiguously.
struct BArgs {
    const double *X;
    const int32_t *conn;
    const uint8_t *etype;
    int stride;
    const int32_t *rowptr;
    const int32_t *task_elem;
    const uint16_t *task_meta;
    const uint8_t *task_cols;
    const int4 *wdesc;
    int64_t N;
    const double *u, *rho, *mu;
    double inv_dt;
    double *values, *rhs;
    double *w_mindet;
    long long *w_bad;
};

// Element e's block row a: S[b] (the scalar part, times the identity) and
// T[b][3i + k] (the full-stress coupling), and the right-hand side B[i].
template <class EL, int FORM>
__device__ __forceinline__ void block_row(const BArgs &k, int64_t e, int a, double (&S)[8], double (&T)[8][9],
                                          double (&B)[3], double &mindet)
{
    constexpr int NEN = EL::NEN, NG = EL::NG;
    constexpr bool FULL = (FORM & FE_FORM_FULL_STRESS) != 0, EMAC = (FORM & FE_FORM_EMAC) != 0;
    const int64_t N = k.N;
    int c[NEN];
#pragma unroll
    for (int b = 0; b < NEN; ++b) c[b] = k.conn[e * k.stride + b];
    double xl[3 * NEN], ul[3][NEN], rl[NEN], ml[NEN];
#pragma unroll
    for (int b = 0; b < NEN; ++b) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            xl[i * NEN + b] = k.X[i * N + c[b]];
            ul[i][b] = k.u[i * N + c[b]];
        }
        rl[b] = k.rho[c[b]];
        ml[b] = k.mu[c[b]];
    }
    int ln[NEN];
#pragma unroll
    for (int b = 0; b < NEN; ++b) ln[b] = b;
    Geo<EL> GE;
    load_geo<EL>(xl, NEN, ln, GE);
#pragma unroll 1
    for (int g = 0; g < NG; ++g) {
        double Ji[3][3];
        const double det = jacobian_inverse<EL>(g, GE, Ji);
        mindet = fmin(mindet, det);
        double dN[NEN][3];
#pragma unroll
        for (int b = 0; b < NEN; ++b)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < 3; ++j) s += Ji[j][i] * RefdN<EL>(g, b, j);
                dN[b][i] = s;
            }
        // the task's own row a (a runtime index: read from the tables, not
        // from the register array)
        double dNa[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) s += Ji[j][i] * RefdN<EL>(g, a, j);
            dNa[i] = s;
        }
        const double Na = RefN<EL>(g, a);
        const double dV = EL::w(g) * det;
        double rg = 0.0, mg = 0.0, ag[3] = {0.0, 0.0, 0.0}, diva = 0.0;
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            const double Nb = RefN<EL>(g, b);
            rg += Nb * rl[b];
            mg += Nb * ml[b];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ag[i] += Nb * ul[i][b];
                if (EMAC) diva += dN[b][i] * ul[i][b];
            }
        }
        const double w1 = dV * rg, wm = dV * mg, wa = w1 * Na;
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            const double Nb = RefN<EL>(g, b);
            const double gg = dNa[0] * dN[b][0] + dNa[1] * dN[b][1] + dNa[2] * dN[b][2];
            const double agb = ag[0] * dN[b][0] + ag[1] * dN[b][1] + ag[2] * dN[b][2];
            double sv = wa * (Nb * k.inv_dt + agb) + wm * gg;
            if (EMAC) sv += wa * diva * Nb;
            S[b] += sv;
            if (FULL) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) T[b][3 * i + kk] += wm * dNa[kk] * dN[b][i];
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) B[i] += wa * ag[i] * k.inv_dt;
    }
}

template <int FORM>
__global__ void __launch_bounds__(64) k_block(BArgs k)
{
    extern __shared__ double lds[];
    const int wi = xcd_item(blockIdx.x, gridDim.x);   // this wave's row range
    const int4 wd = k.wdesc[wi];   // first task, tasks, first row, rows
    const int lane = threadIdx.x;
    const int r0 = wd.z, nr = wd.w;
    const int64_t v0 = k.rowptr[r0];
    const int nimg = 9 * (int)(k.rowptr[r0 + nr] - v0);
    double *img = lds;            // [nimg] block values of the wave's rows
    double *rimg = lds + nimg;    // [3][64] their right-hand sides
    for (int j = lane; j < nimg; j += 64) img[j] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) rimg[i * 64 + lane] = 0.0;

    const bool live = lane < wd.y;
    const int64_t t = wd.x + (live ? lane : 0);
    const int64_t e = k.task_elem[t];
    const int meta = k.task_meta[t];
    const int a = meta & 15, ph = live ? (meta >> 4) : -1;
    const int nen = k.etype ? (int)k.etype[e] : k.stride;
    const uint64_t cols = *(const uint64_t *)(k.task_cols + 8 * t);
    const int row = k.conn[e * k.stride + a];
    const int ro = (int)(k.rowptr[row] - v0), rl = row - r0;
    double S[8], T[8][9], B[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        S[b] = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) T[b][q] = 0.0;
    }
    double mindet = __builtin_huge_val();
    if (live) {
        switch (nen) {
        case 8: block_row<Hex, FORM>(k, e, a, S, T, B, mindet); break;
        case 6: block_row<Pen, FORM>(k, e, a, S, T, B, mindet); break;
        case 5: block_row<Pyr, FORM>(k, e, a, S, T, B, mindet); break;
        default: block_row<Tet, FORM>(k, e, a, S, T, B, mindet); break;
        }
    }
    __syncthreads();
    // phases: a row's tasks one after the other in element order; the tasks
    // of one phase hold distinct rows, so no two lanes add to one address
    int nph = ph + 1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nph = max(nph, __shfl_xor(nph, o));
    for (int p = 0; p < nph; ++p) {
        if (ph == p) {
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                if (b < nen) {
                    double *dst = img + 9 * (ro + (int)((cols >> (8 * b)) & 0xff));
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int kk = 0; kk < 3; ++kk)
                            lds_add(dst + 3 * i + kk, (i == kk ? S[b] : 0.0) + T[b][3 * i + kk]);
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) lds_add(&rimg[i * 64 + rl], B[i]);
        }
    }
    __syncthreads();
    // each value and right-hand side entry written once, contiguously
    double *vout = k.values + 9 * v0;
    for (int j = lane; j < nimg; j += 64) vout[j] = img[j];
    if (lane < nr) {
#pragma unroll
        for (int i = 0; i < 3; ++i) k.rhs[i * k.N + r0 + lane] = rimg[i * 64 + lane];
    }
    // status: the wave's smallest det J and first element with det J <= 0
    double md = live ? mindet : __builtin_huge_val();
    long long bad = (live && !(mindet > 0.0)) ? (long long)e : (long long)0x7fffffffffffffffLL;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        md = fmin(md, __shfl_xor(md, o));
        const long long ob = __shfl_xor(bad, o);
        bad = ob < bad ? ob : bad;
    }
    if (lane == 0) {
        k.w_mindet[wi] = md;
        k.w_bad[wi] = bad == 0x7fffffffffffffffLL ? -1 : bad;
    }
}

// ---- boundary assembly: equilibrium wall model ---------------------------
// The wall law (Reichardt, kappa = 0.41) at exchange distance delta: u_tau
// from U = u_tau u+(delta u_tau / nu) by a fixed number of Newton steps from
// the laminar guess sqrt(nu U / delta); traction -rho u_tau^2 u_t / |u_t|
// with u_t the tangential part of the interpolated velocity.
constexpr double kWallKappa = 0.41;
constexpr int kWallNewton = 16;

__device__ double wall_utau(double U, double nu, double delta)
{
    if (!(U > 0.0)) return 0.0;
    double ut = sqrt(nu * U / delta);
    for (int k = 0; k < kWallNewton; ++k) {
        const double yp = delta * ut / nu;
        const double e1 = exp(-yp / 11.0), e3 = exp(-yp / 3.0);
        const double up = log(1.0 + kWallKappa * yp) / kWallKappa + 7.8 * (1.0 - e1 - yp / 11.0 * e3);
        const double du = 1.0 / (1.0 + kWallKappa * yp) + 7.8 * (e1 / 11.0 - e3 / 11.0 + yp * e3 / 33.0);
        ut -= (ut * up - U) / (up + yp * du);
        if (ut <= 0.0) ut = 1e-300;
    }
    return ut;
}

// Four lanes per face, one per Gauss point (3-point rule on triangles: the
// fourth lane adds nothing; 2x2 Gauss on quadrilaterals): each lane forms
// its point's w |x_s x x_t| N_a t, the quad of lanes sums them in the fixed
// order (q0 + q1) + (q2 + q3) and its first lane writes the face's part.
__global__ void __launch_bounds__(64) k_wall_faces(int64_t F, const uint8_t *fnen, const int32_t *fconn,
                                                   const double *X, int64_t N, const double *u, const double *rho,
                                                   const double *mu, double delta, double *part)
{
    const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t f = t >> 2;
    const int q = (int)(t & 3);
    const bool live = f < F;                  // whole quads are live or not (64 = 16 quads)
    const int64_t fs = live ? f : 0;
    const int nn = fnen[fs];
    int c[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) c[a] = fconn[4 * fs + a];
    double P[4][3] = {};
    const double g = 0.57735026918962576451;
    if (live && !(nn == 3 && q == 3)) {
        double Nq[4], ds[4], dt[4], w;
        if (nn == 3) {
            const double s = q == 1 ? 2.0 / 3.0 : 1.0 / 6.0, tt = q == 2 ? 2.0 / 3.0 : 1.0 / 6.0;
            Nq[0] = 1.0 - s - tt; Nq[1] = s; Nq[2] = tt; Nq[3] = 0.0;
            ds[0] = -1.0; ds[1] = 1.0; ds[2] = 0.0; ds[3] = 0.0;
            dt[0] = -1.0; dt[1] = 0.0; dt[2] = 1.0; dt[3] = 0.0;
            w = 1.0 / 6.0;
        } else {
            const double s = (q & 1) ? g : -g, tt = (q & 2) ? g : -g;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double cx = (a == 1 || a == 2) ? 1.0 : -1.0, cy = a >= 2 ? 1.0 : -1.0;
                Nq[a] = 0.25 * (1.0 + cx * s) * (1.0 + cy * tt);
                ds[a] = 0.25 * cx * (1.0 + cy * tt);
                dt[a] = 0.25 * cy * (1.0 + cx * s);
            }
            w = 1.0;
        }
        double xs[3] = {}, xt[3] = {}, ug[3] = {}, rg = 0.0, mg = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if (a >= nn) break;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double xi = X[i * N + c[a]];
                xs[i] += ds[a] * xi;
                xt[i] += dt[a] * xi;
                ug[i] += Nq[a] * u[i * N + c[a]];
            }
            rg += Nq[a] * rho[c[a]];
            mg += Nq[a] * mu[c[a]];
        }
        const double nv[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2],
                              xs[0] * xt[1] - xs[1] * xt[0]};
        const double a2 = nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2];
        if (a2 > 0.0) {
            const double area = sqrt(a2);
            const double un = (ug[0] * nv[0] + ug[1] * nv[1] + ug[2] * nv[2]) / a2;
            const double ut[3] = {ug[0] - un * nv[0], ug[1] - un * nv[1], ug[2] - un * nv[2]};
            const double U = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
            if (U > 0.0) {
                const double tau = wall_utau(U, mg / rg, delta);
                const double fac = -w * area * rg * tau * tau / U;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int i = 0; i < 3; ++i) P[a][i] = fac * Nq[a] * ut[i];
            }
        }
    }
    // (q0 + q1) + (q2 + q3): xor 1 pairs q0/q1 and q2/q3, xor 2 then adds the pairs
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double v = P[a][i];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            P[a][i] = v;
        }
    if (live && q == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) part[(4 * f + a) * 3 + i] = P[a][i];
    }
}

// One thread per wall node: its face entries summed in their fixed order.
__global__ void __launch_bounds__(256) k_wall_gather(int64_t W, const int32_t *nodes, const int32_t *ptr,
                                                     const int32_t *ent, const double *part, int64_t N, double *out)
{
    const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (w >= W) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int32_t k = ptr[w]; k < ptr[w + 1]; ++k) {
        const double *p = part + (int64_t)ent[k] * 3;
        s0 += p[0];
        s1 += p[1];
        s2 += p[2];
    }
    const int64_t i = nodes[w];
    out[i] += s0;
    out[N + i] += s1;
    out[2 * N + i] += s2;
}

__global__ void __launch_bounds__(256) k_zero(int64_t n, double *x)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] = 0.0;
}

}  // namespace

hipError_t launch_wall_traction(const DevMesh &m, const DevWall &w, const double *u, const double *rho,
                                const double *mu, double *out, bool zero_first, hipStream_t s)
{
    if (zero_first) {
        const int64_t n = 3 * m.N;
        const int64_t nb = std::min<int64_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(k_zero, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(256), 0, s, n, out);
    }
    if (w.F == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_wall_faces, dim3((unsigned)((4 * w.F + 63) / 64)), dim3(64), 0, s, w.F, w.nen, w.conn, m.X,
                       m.N, u, rho, mu, w.delta, w.part);
    hipLaunchKernelGGL(k_wall_gather, dim3((unsigned)((w.W + 255) / 256)), dim3(256), 0, s, w.W, w.nodes, w.ptr,
                       w.ent, w.part, m.N, out);
    return hipGetLastError();
}

namespace {

// The coloured kernels' arguments for one operator pass.
KArgs make_kargs(const AsmArgs &a)
{
    const DevMesh &m = *a.m;
    KArgs k{};
    k.X = m.X;
    k.blk_elem_ptr = m.blk_elem_ptr;
    k.blk_node_ptr = m.blk_node_ptr;
    k.blk_nodes = m.blk_nodes;
    k.blk_rdesc = m.blk_rdesc;
    k.blk_rowstart = m.blk_rowstart;
    k.color_blk = m.color_blk;
    k.blk_nphase = m.blk_nphase;
    k.elem_off = m.elem_off;
    k.elem_phase = m.elem_phase;
    k.elem_lnode = m.elem_lnode;
    k.N = m.N;
    k.E = m.E;
    k.u = a.u;
    k.rho = a.rho;
    k.mu = a.mu;
    k.Y = a.Y;
    k.p = a.p;
    k.dt = a.dt;
    k.Dk = a.Dk;
    k.values = a.values;
    k.rhs = a.rhs;
    // status scratch lives right after the AsmStatus word: per-block (or,
    // owner assembly, per-group) smallest det J, then first bad element, each
    // sized for the larger of the two counts
    const int64_t nstat = std::max<int64_t>(m.nblk, m.own_G);
    k.blk_mindet = (double *)(a.status + 1);
    k.blk_bad = (long long *)(k.blk_mindet + nstat);
    k.off_stride = m.off_stride;
    k.form = a.form;
    return k;
}

template <class EL>
void launch_bat(int op, const AsmBatch &B, const KArgs *ks, size_t lds, hipStream_t s)
{
    if (op == OP_MOM)
        hipLaunchKernelGGL((k_bat_assemble<EL, OP_MOM>), dim3(B.wgs[B.n]), dim3(64 * Split<EL>::W), lds, s, ks, B);
    else
        hipLaunchKernelGGL((k_bat_assemble<EL, OP_POI>), dim3(B.wgs[B.n]), dim3(64 * Split<EL>::W), lds, s, ks, B);
}

}  // namespace

void fill_kargs(const AsmArgs &a, void *out)
{
    const KArgs k = make_kargs(a);
    memset(out, 0, kKArgsBytes);
    memcpy(out, &k, sizeof(KArgs));
}

hipError_t launch_assemble_batch(const AsmArgs *a, const int *slot, int n, const void *kargs_d, hipStream_t s)
{
    if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
    const int op = a[0].op;
    if (op != OP_MOM && op != OP_POI) return hipErrorInvalidValue;
    size_t nl = 0;
    for (int i = 0; i < n; ++i) {
        if (a[i].op != op || a[i].m->own_G > 0) return hipErrorInvalidValue;
        nl = std::max(nl, a[i].m->launches.size());
    }
    const KArgs *ks = (const KArgs *)kargs_d;
    // launch li of every mesh, one launch per element type; launch li + 1
    // after it, so each mesh keeps its own colour order
    for (size_t li = 0; li < nl; ++li) {
        for (int nen : {8, 6, 5, 4}) {
            AsmBatch B{};
            size_t lds = 0;
            for (int i = 0; i < n; ++i) {
                const std::vector<AsmLaunch> &Ls = a[i].m->launches;
                if (li >= Ls.size() || Ls[li].nen != nen || Ls[li].count == 0) continue;
                B.slot[B.n] = slot[i];
                B.first[B.n] = Ls[li].first;
                B.wgs[B.n + 1] = B.wgs[B.n] + Ls[li].count;
                lds = std::max(lds, Ls[li].lds[op]);
                ++B.n;
            }
            if (B.n == 0) continue;
            switch (nen) {
            case 8: launch_bat<Hex>(op, B, ks, lds, s); break;
            case 6: launch_bat<Pen>(op, B, ks, lds, s); break;
            case 5: launch_bat<Pyr>(op, B, ks, lds, s); break;
            default: launch_bat<Tet>(op, B, ks, lds, s); break;
            }
            const hipError_t err = hipGetLastError();
            if (err != hipSuccess) return err;
        }
    }
    // each mesh's status word from its per-block scratch (as launch_assemble)
    for (int i = 0; i < n; ++i) {
        const KArgs k = make_kargs(a[i]);
        hipLaunchKernelGGL(k_asm_status, dim3(1), dim3(kStatusThreads), 0, s, k.blk_mindet, k.blk_bad, a[i].m->nblk,
                           a[i].status_out ? a[i].status_out : a[i].status);
    }
    return hipGetLastError();
}

hipError_t launch_assemble(const AsmArgs &a, bool mixed, hipStream_t s)
{
    const DevMesh &m = *a.m;
    if (a.op < 0 || a.op >= kNumOps) return hipErrorInvalidValue;
    KArgs k = make_kargs(a);
    if (a.op < OP_RES && m.own_G > 0) {
        // matrix operators of a single-type mesh: the owner assembly, one launch
        OArgs o{};
        o.X = m.X;
        o.rowptr = m.rowptr;
        o.groups = m.own_groups;
        o.node_ptr = m.own_node_ptr;
        o.nodes = m.own_nodes;
        o.elem = m.own_elem;
        o.nphase = m.own_nphase;
        o.ln = m.own_ln;
        o.off = m.own_off;
        o.phase = m.own_phase;
        o.ln_stride = m.own_ln_stride;
        o.off_stride = m.own_off_stride;
        o.N = m.N;
        o.u = a.u;
        o.rho = a.rho;
        o.mu = a.mu;
        o.Y = a.Y;
        o.dt = a.dt;
        o.Dk = a.Dk;
        o.values = a.values;
        o.rhs = a.rhs;
        o.g_mindet = k.blk_mindet;
        o.g_bad = k.blk_bad;
        const int nf = a.op == OP_POI ? 7 : 8, nrhs = a.op == OP_MOM ? 3 : 1;
        const int copies = m.own_priv ? kOwnTasks / 64 : 1;
        if ((m.own_priv != 0) != (m.nen != 8)) return hipErrorInvalidValue;   // plan and kernel disagree
        // x, y, z in FP64, the other fields in the quadrature's precision
        const size_t fb = mixed ? sizeof(float) : sizeof(double);
        const size_t fields = 3 * (size_t)m.own_max_nodes + ((nf - 3) * (size_t)m.own_max_nodes * fb + 7) / 8;
        const size_t lds = (fields + (size_t)copies * (m.own_max_img + nrhs * m.own_max_rows)) * sizeof(double);
        switch (m.nen) {
        case 8: launch_own<Hex>(o, a.op, m.own_G, lds, mixed, s); break;
        case 6: launch_own<Pen>(o, a.op, m.own_G, lds, mixed, s); break;
        case 5: launch_own<Pyr>(o, a.op, m.own_G, lds, mixed, s); break;
        case 4: launch_own<Tet>(o, a.op, m.own_G, lds, mixed, s); break;
        default: return hipErrorInvalidValue;
        }
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_asm_status, dim3(1), dim3(kStatusThreads), 0, s, k.blk_mindet, k.blk_bad, m.own_G,
                           a.status_out ? a.status_out : a.status);
        return hipGetLastError();
    }
    // one launch per (colour, element type), in the planned order
    for (const AsmLaunch &L : m.launches) {
        if (L.count == 0) continue;
        switch (L.nen) {
        case 8: launch_type<Hex>(L, k, a.op, mixed, s); break;
        case 6: launch_type<Pen>(L, k, a.op, mixed, s); break;
        case 5: launch_type<Pyr>(L, k, a.op, mixed, s); break;
        case 4: launch_type<Tet>(L, k, a.op, mixed, s); break;
        default: return hipErrorInvalidValue;
        }
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(k_asm_status, dim3(1), dim3(kStatusThreads), 0, s, k.blk_mindet, k.blk_bad, m.nblk,
                       a.status_out ? a.status_out : a.status);
    return hipGetLastError();
}

hipError_t launch_assemble_block(const DevMesh &m, const DevRowPlan &r, int form, double dt, const double *u,
                                 const double *rho, const double *mu, double *values, double *rhs,
                                 AsmStatus *status, hipStream_t s)
{
    if (r.n_waves <= 0) return hipErrorInvalidValue;
    BArgs k{};
    k.X = m.X;
    k.conn = r.conn;
    k.etype = r.etype;
    k.stride = r.stride;
    k.rowptr = m.rowptr;
    k.task_elem = r.task_elem;
    k.task_meta = r.task_meta;
    k.task_cols = r.task_cols;
    k.wdesc = r.wdesc;
    k.N = m.N;
    k.u = u;
    k.rho = rho;
    k.mu = mu;
    k.inv_dt = 1.0 / dt;
    k.values = values;
    k.rhs = rhs;
    k.w_mindet = r.w_mindet;
    k.w_bad = r.w_bad;
    const size_t lds = (size_t)(r.max_img + 3 * 64) * sizeof(double);
    const dim3 grid((unsigned)r.n_waves), blk(64);
    switch (form) {
    case 0: hipLaunchKernelGGL(k_block<0>, grid, blk, lds, s, k); break;
    case 1: hipLaunchKernelGGL(k_block<1>, grid, blk, lds, s, k); break;
    case 2: hipLaunchKernelGGL(k_block<2>, grid, blk, lds, s, k); break;
    default: hipLaunchKernelGGL(k_block<3>, grid, blk, lds, s, k); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_asm_status, dim3(1), dim3(kStatusThreads), 0, s, r.w_mindet, r.w_bad, r.n_waves, status);
    return hipGetLastError();
}

}  // namespace feasm
