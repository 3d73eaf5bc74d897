// asm_kernels.hip -- element-by-element assembly into CSR on gfx950.
//
// Section 4.2 / Listing 1 of the paper: an outer loop over elements and an
// inner loop over Gauss points and node pairs accumulating the elemental
// matrix from shape functions and the Jacobian weight, then a scatter into
// CSR.  Section 4.3 packs elements so that a SIMD unit processes several at
// once.  gfx950 form:
//
//   * one work-group = one wavefront = one block of <= 64 spatially compact
//     elements; one lane computes one element (Gauss loop fully unrolled,
//     reference-element tables folded to constants);
//   * the block's nodal fields are staged in LDS (structure of arrays, so that
//     lanes reading different nodes hit different banks);
//   * the CSR rows the block touches live in an LDS image, initialised from
//     HBM (or zero for the first block to touch a row), accumulated with
//     conflict-free ds_add_f64 in a fixed (phase, a, b) order, and written
//     back once -- one coalesced read-modify-write per touched row instead of
//     one per element entry;
//   * blocks of one colour share no node, so a launch per colour needs no
//     atomics in HBM; the colour order fixes the summation order, so the
//     result is bitwise reproducible.
//
// Precision: FP64, or (mixed) FP32 Gauss-point products and elemental sums
// with the Jacobian, det J, J^-1 and the CSR accumulation in FP64.
#include "internal.h"

namespace feasm {
namespace {

constexpr int OP_MOM = FE_OP_MOMENTUM, OP_SCA = FE_OP_SCALAR, OP_POI = FE_OP_POISSON;

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

struct HexTables {
    double N[8][8];        // N[g][a]
    double dN[8][8][3];    // dN[g][a][j]
};

constexpr HexTables make_hex_tables()
{
    HexTables t{};
    for (int g = 0; g < 8; ++g)
        for (int a = 0; a < 8; ++a) {
            t.N[g][a] = Hex::N(g, a);
            for (int j = 0; j < 3; ++j) t.dN[g][a][j] = Hex::dN(g, a, j);
        }
    return t;
}

__constant__ HexTables kHexTab = make_hex_tables();

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

struct KArgs {
    const double *X;
    const int32_t *rowptr, *blk_elem_ptr, *blk_node_ptr, *blk_nodes, *blk_lbase, *color_blk;
    const uint8_t *blk_nphase, *elem_off, *elem_phase;
    const uint16_t *elem_lnode;
    int64_t N, E;
    const double *u, *rho, *mu, *Y;
    double dt, Dk;
    double *values, *rhs;
    double *blk_mindet;       // [nblk] per-block smallest det J
    long long *blk_bad;       // [nblk] per-block first bad element (mesh index) or -1
    int blk_offset, gshift;
};

template <int OP> struct OpTraits;
template <> struct OpTraits<FE_OP_MOMENTUM> { static constexpr int NF = 8, NRHS = 3; };
template <> struct OpTraits<FE_OP_SCALAR> { static constexpr int NF = 8, NRHS = 1; };
template <> struct OpTraits<FE_OP_POISSON> { static constexpr int NF = 7, NRHS = 1; };

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

// One Gauss point: geometry in FP64, quadrature products in Q.
//   MOM/SCA: A_ab += N_a s_b + wk grad N_a . grad N_b,
//            s_b = rho dV (N_b / dt + u . grad N_b), wk = mu dV or rho D dV;
//            rho dV / dt is stored in cgs for the rhs pass.
//   POI    : A_ab += dV grad N_a . grad N_b (upper triangle),
//            B_a += dV / dt grad N_a . (rho u).
template <class EL, int OP, class Q>
__device__ __forceinline__ void gauss_point(int g, const double *nd, int T, const int (&ln)[EL::NEN],
                                            Q (&A)[EL::NEN][EL::NEN], Q (&B)[OpTraits<OP>::NRHS][EL::NEN],
                                            double &mindet, double *cgs, double inv_dt, double Dk)
{
    constexpr int NEN = EL::NEN;
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
        const double xa = nd[0 * T + ln[a]], ya = nd[1 * T + ln[a]], za = nd[2 * T + ln[a]];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double d = RefdN<EL>(g, a, j);
            if (!EL::kSparse || d != 0.0) {
                J[0][j] += xa * d;
                J[1][j] += ya * d;
                J[2][j] += za * d;
            }
        }
    }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    mindet = fmin(mindet, det);
    const double id = 1.0 / det;
    double Ji[3][3];
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    // physical gradients grad N_a = J^-T grad_ref N_a
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
    double rg = 0.0, fg = 0.0, ug0 = 0.0, ug1 = 0.0, ug2 = 0.0;
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
        const double Na = RefN<EL>(g, a);
        rg += Na * nd[6 * T + ln[a]];
        ug0 += Na * nd[3 * T + ln[a]];
        ug1 += Na * nd[4 * T + ln[a]];
        ug2 += Na * nd[5 * T + ln[a]];
        if (OP == OP_MOM) fg += Na * nd[7 * T + ln[a]];
    }
    const double dV = EL::w(g) * det;
    if (OP == OP_POI) {
        const Q qdV = Q(dV), qi = Q(inv_dt);
        const Q f0 = Q(rg * ug0), f1 = Q(rg * ug1), f2 = Q(rg * ug2);
#pragma unroll
        for (int a = 0; a < NEN; ++a) {
#pragma unroll
            for (int b = a; b < NEN; ++b)
                A[a][b] += qdV * (dN[a][0] * dN[b][0] + dN[a][1] * dN[b][1] + dN[a][2] * dN[b][2]);
            B[0][a] += qdV * qi * (dN[a][0] * f0 + dN[a][1] * f1 + dN[a][2] * f2);
        }
    } else {
        const Q w1 = Q(dV) * Q(rg);
        const Q wk = (OP == OP_MOM) ? Q(dV) * Q(fg) : Q(dV) * (Q(rg) * Q(Dk));
        const Q qi = Q(inv_dt);
        cgs[g * 64 + threadIdx.x] = dV * rg * inv_dt;
        const Q qu0 = Q(ug0), qu1 = Q(ug1), qu2 = Q(ug2);
        Q s[NEN];
#pragma unroll
        for (int b = 0; b < NEN; ++b)
            s[b] = w1 * (Q(RefN<EL>(g, b)) * qi + (qu0 * dN[b][0] + qu1 * dN[b][1] + qu2 * dN[b][2]));
#pragma unroll
        for (int a = 0; a < NEN; ++a) {
            const Q Na = Q(RefN<EL>(g, a));
            const Q G0 = wk * dN[a][0], G1 = wk * dN[a][1], G2 = wk * dN[a][2];
#pragma unroll
            for (int b = 0; b < NEN; ++b) A[a][b] += Na * s[b] + (G0 * dN[b][0] + G1 * dN[b][1] + G2 * dN[b][2]);
        }
    }
}

template <class EL, int OP, class Q>
__global__ void __launch_bounds__(64) k_assemble(KArgs k)
{
    constexpr int NEN = EL::NEN, NG = EL::NG;
    constexpr int NF = OpTraits<OP>::NF, NRHS = OpTraits<OP>::NRHS;
    extern __shared__ double lds[];

    const int blk = k.color_blk[k.blk_offset + blockIdx.x];
    const int e0 = k.blk_elem_ptr[blk], ne = k.blk_elem_ptr[blk + 1] - e0;
    const int n0 = k.blk_node_ptr[blk], T = k.blk_node_ptr[blk + 1] - n0;
    const int lane = threadIdx.x;
    const int64_t N = k.N;

    double *nd = lds;                        // [NF][T] nodal fields
    double *rimg = nd + NF * T;              // [NRHS][T] rhs image
    double *cgs = rimg + NRHS * T;           // [NG][64] rho dV / dt per lane
    int *lbs = (int *)(cgs + NG * 64);       // [T] image base | first flag
    int *rs = lbs + T;                       // [T] CSR row start
    int *rl = rs + T;                        // [T] CSR row length
    double *img = (double *)(rl + T + ((3 * T) & 1));   // 8-byte aligned

    // 1. stage nodal fields, row descriptors and the rhs image
    for (int t = lane; t < T; t += 64) {
        const int g = k.blk_nodes[n0 + t];
        nd[0 * T + t] = k.X[g];
        nd[1 * T + t] = k.X[N + g];
        nd[2 * T + t] = k.X[2 * N + g];
        nd[3 * T + t] = k.u[g];
        nd[4 * T + t] = k.u[N + g];
        nd[5 * T + t] = k.u[2 * N + g];
        nd[6 * T + t] = k.rho[g];
        if (OP == OP_MOM) nd[7 * T + t] = k.mu[g];
        if (OP == OP_SCA) nd[7 * T + t] = k.Y[g];
        const int lb = k.blk_lbase[n0 + t];
        const int r0 = k.rowptr[g];
        lbs[t] = lb;
        rs[t] = r0;
        rl[t] = k.rowptr[g + 1] - r0;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) rimg[r * T + t] = lb < 0 ? 0.0 : k.rhs[r * N + g];
    }
    __syncthreads();
    // 2. row image: previous partial sums, or zero for the first writer
    {
        const int G = 1 << k.gshift, sub = lane & (G - 1);
        for (int t = lane >> k.gshift; t < T; t += 64 >> k.gshift) {
            const int lb = lbs[t], base = lb & 0x7fffffff, r0 = rs[t], len = rl[t];
            if (lb < 0) {
                for (int q = sub; q < len; q += G) img[base + q] = 0.0;
            } else {
                for (int q = sub; q < len; q += G) img[base + q] = k.values[r0 + q];
            }
        }
    }
    __syncthreads();

    // 3. elemental matrix, one element per lane
    const bool act = lane < ne;
    const int e = e0 + (act ? lane : 0);
    int ln[NEN];
#pragma unroll
    for (int a = 0; a < NEN; ++a) ln[a] = k.elem_lnode[(int64_t)a * k.E + e];

    Q A[NEN][NEN];
    Q B[NRHS][NEN];
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
#pragma unroll
        for (int b = 0; b < NEN; ++b) A[a][b] = Q(0);
#pragma unroll
        for (int r = 0; r < NRHS; ++r) B[r][a] = Q(0);
    }
    double mindet = __builtin_huge_val();
    const double inv_dt = 1.0 / k.dt;
    if (EL::kRolled) {
#pragma unroll 1
        for (int g = 0; g < NG; ++g) {
            // opaque row indices: the nodal reads stay inside the loop
#pragma unroll
            for (int a = 0; a < NEN; ++a) asm volatile("" : "+v"(ln[a]));
            gauss_point<EL, OP, Q>(g, nd, T, ln, A, B, mindet, cgs, inv_dt, k.Dk);
        }
    } else {
#pragma unroll
        for (int g = 0; g < NG; ++g) gauss_point<EL, OP, Q>(g, nd, T, ln, A, B, mindet, cgs, inv_dt, k.Dk);
    }
    if (OP == OP_POI) {
#pragma unroll
        for (int a = 0; a < NEN; ++a)
#pragma unroll
            for (int b = 0; b < a; ++b) A[a][b] = A[b][a];
    }

    // 4. scatter into the LDS images, phase by phase (fixed order, no conflicts)
    int base[NEN];
#pragma unroll
    for (int a = 0; a < NEN; ++a) base[a] = lbs[ln[a]] & 0x7fffffff;
    uint32_t offw[NEN * NEN / 4];
    {
        const uint4 *op = (const uint4 *)(k.elem_off + (int64_t)e * (NEN * NEN));
#pragma unroll
        for (int q = 0; q < NEN * NEN / 16; ++q) {
            const uint4 v = op[q];
            offw[4 * q + 0] = v.x;
            offw[4 * q + 1] = v.y;
            offw[4 * q + 2] = v.z;
            offw[4 * q + 3] = v.w;
        }
    }
    const int ph = act ? (int)k.elem_phase[e] : -1;
    const int nph = k.blk_nphase[blk];
    for (int p = 0; p < nph; ++p) {
        if (ph == p) {
#pragma unroll
            for (int a = 0; a < NEN; ++a) {
#pragma unroll
                for (int b = 0; b < NEN; ++b) {
                    const int idx = a * NEN + b;
                    const int off = (offw[idx >> 2] >> (8 * (idx & 3))) & 0xff;
                    lds_add(&img[base[a] + off], (double)A[a][b]);
                }
                if (OP == OP_POI) lds_add(&rimg[ln[a]], (double)B[0][a]);
            }
        }
    }
    if (OP != OP_POI) {
        // rhs b_a = sum_g (rho dV / dt)_g N_a(g) f_g, f = u (MOM) or Y (SCA)
        auto rhs_point = [&](int g) {
            double f[NRHS];
#pragma unroll
            for (int r = 0; r < NRHS; ++r) f[r] = 0.0;
#pragma unroll
            for (int a = 0; a < NEN; ++a) {
                const double Na = RefN<EL>(g, a);
#pragma unroll
                for (int r = 0; r < NRHS; ++r) f[r] += Na * nd[(OP == OP_MOM ? 3 + r : 7) * T + ln[a]];
            }
            const Q c = Q(cgs[g * 64 + lane]);
#pragma unroll
            for (int a = 0; a < NEN; ++a) {
                const Q cn = c * Q(RefN<EL>(g, a));
#pragma unroll
                for (int r = 0; r < NRHS; ++r) B[r][a] += cn * Q(f[r]);
            }
        };
        if (EL::kRolled) {
#pragma unroll 1
            for (int g = 0; g < NG; ++g) {
#pragma unroll
                for (int a = 0; a < NEN; ++a) asm volatile("" : "+v"(ln[a]));
                rhs_point(g);
            }
        } else {
#pragma unroll
            for (int g = 0; g < NG; ++g) rhs_point(g);
        }
        for (int p = 0; p < nph; ++p) {
            if (ph == p) {
#pragma unroll
                for (int a = 0; a < NEN; ++a)
#pragma unroll
                    for (int r = 0; r < NRHS; ++r) lds_add(&rimg[r * T + ln[a]], (double)B[r][a]);
            }
        }
    }

    // status: per-block smallest det J and first non-positive element
    {
        double md = act ? mindet : __builtin_huge_val();
        long long bad = (act && !(mindet > 0.0)) ? (long long)e : (long long)0x7fffffffffffffffLL;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            md = fmin(md, __shfl_xor(md, o));
            const long long ob = __shfl_xor(bad, o);
            bad = ob < bad ? ob : bad;
        }
        if (lane == 0) {
            k.blk_mindet[blk] = md;
            k.blk_bad[blk] = bad == 0x7fffffffffffffffLL ? -1 : bad;
        }
    }
    __syncthreads();

    // 5. write the touched rows and rhs entries back
    {
        const int G = 1 << k.gshift, sub = lane & (G - 1);
        for (int t = lane >> k.gshift; t < T; t += 64 >> k.gshift) {
            const int base_t = lbs[t] & 0x7fffffff, r0 = rs[t], len = rl[t];
            for (int q = sub; q < len; q += G) k.values[r0 + q] = img[base_t + q];
        }
    }
    for (int t = lane; t < T; t += 64) {
        const int g = k.blk_nodes[n0 + t];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) k.rhs[r * N + g] = rimg[r * T + t];
    }
}

// Reduce the per-block status into (min det, first bad mesh element).
__global__ void __launch_bounds__(256) k_asm_status(const double *mindet, const long long *bad, int64_t n,
                                                    AsmStatus *out)
{
    __shared__ double sd[256];
    __shared__ long long sb[256];
    double md = __builtin_huge_val();
    long long b = 0x7fffffffffffffffLL;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        md = fmin(md, mindet[i]);
        const long long v = bad[i];
        if (v >= 0 && v < b) b = v;
    }
    sd[threadIdx.x] = md;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sd[threadIdx.x] = fmin(sd[threadIdx.x], sd[threadIdx.x + s]);
            if (sb[threadIdx.x + s] < sb[threadIdx.x]) sb[threadIdx.x] = sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double d = sd[0];
        unsigned long long u;
        __builtin_memcpy(&u, &d, 8);
        out->min_det_key = u;
        out->first_bad = sb[0] == 0x7fffffffffffffffLL ? -1 : sb[0];
    }
}

template <class EL, int OP, class Q>
hipError_t run(const AsmArgs &a, const KArgs &k0, hipStream_t s)
{
    const DevMesh &m = *a.m;
    constexpr int NF = OpTraits<OP>::NF, NRHS = OpTraits<OP>::NRHS;
    const size_t lds = (size_t)(NF + NRHS) * m.max_T * 8 + (size_t)EL::NG * 64 * 8 + (size_t)m.max_T * 12 + 8 +
                       (size_t)m.max_L * 8;
    KArgs k = k0;
    for (int c = 0; c < m.n_colors; ++c) {
        const int nb = m.color_ptr[c + 1] - m.color_ptr[c];
        if (nb == 0) continue;
        k.blk_offset = m.color_ptr[c];
        hipLaunchKernelGGL((k_assemble<EL, OP, Q>), dim3(nb), dim3(64), lds, s, k);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_assemble(const AsmArgs &a, bool mixed, hipStream_t s)
{
    const DevMesh &m = *a.m;
    KArgs k{};
    k.X = m.X;
    k.rowptr = m.rowptr;
    k.blk_elem_ptr = m.blk_elem_ptr;
    k.blk_node_ptr = m.blk_node_ptr;
    k.blk_nodes = m.blk_nodes;
    k.blk_lbase = m.blk_lbase;
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
    k.dt = a.dt;
    k.Dk = a.Dk;
    k.values = a.values;
    k.rhs = a.rhs;
    // status scratch lives right after the AsmStatus word
    k.blk_mindet = (double *)(a.status + 1);
    k.blk_bad = (long long *)(k.blk_mindet + m.nblk);
    int gs = 0;
    while ((1 << gs) < m.max_row && gs < 6) ++gs;
    k.gshift = gs;
    hipError_t err;
    const bool hex = m.nen == 8;
#define FE_RUN(EL, OPV)                                                                     \
    err = mixed ? run<EL, OPV, float>(a, k, s) : run<EL, OPV, double>(a, k, s)
    if (hex) {
        if (a.op == OP_MOM) FE_RUN(Hex, OP_MOM);
        else if (a.op == OP_SCA) FE_RUN(Hex, OP_SCA);
        else FE_RUN(Hex, OP_POI);
    } else {
        if (a.op == OP_MOM) FE_RUN(Tet, OP_MOM);
        else if (a.op == OP_SCA) FE_RUN(Tet, OP_SCA);
        else FE_RUN(Tet, OP_POI);
    }
#undef FE_RUN
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_asm_status, dim3(1), dim3(256), 0, s, k.blk_mindet, k.blk_bad, m.nblk, a.status);
    return hipGetLastError();
}

}  // namespace feasm
