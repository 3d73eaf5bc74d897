// solver_kernels.hip -- memory-bound kernels of the Jacobi-PCG pressure solve.
//
// Section 5.2 of the paper: the algebraic solver is vector operations (AXPY,
// dot; no memory reuse) plus a CSR SpMV with indirect accesses.  gfx950 form:
//
//   * vector kernels use a fixed grid of at most 512 work-groups of 256
//     threads, each thread walking a fixed strided subset, so every reduction
//     has a fixed order and results are bitwise reproducible;
//   * SpMV streams row blocks whose nonzeros are contiguous (fixed at
//     upload) on five work-groups per CU: 16-byte loads of values and one-byte
//     indices into each block's column set, the products formed in LDS, four
//     threads per row adding them in a fixed order;
//   * one PCG iteration is three launches: SpMV fused with p.Ap; the r, z
//     update fused with r.z and r.r; the x and p updates with the stop test.
//     (Forming z + beta p inside the SpMV gather was measured slower: two
//     gathered vectors cost more than the separate streaming update.)
//     Instead of a separate
//     single-work-group reduction kernel, every work-group of the consuming
//     kernel re-reduces the <= 2048 partial sums itself in the same fixed
//     order (<= 16 KB of L2 reads), so all work-groups hold bitwise the same
//     alpha / beta without a grid-wide barrier;
//   * CG scalars stay on the device; the host polls a flag word.
#include "internal.h"
#include "plan.h"

namespace feasm {

int stream_blocks(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    // at most two groups per CU of a 256-CU device: the CG vector updates on
    // 2.1 M rows took 37.4 us per iteration with 512 groups, 39.1 with 384,
    // 40.2 with 640, 43.1 with 1024 and 43.0 with 2048
    if (b > 512) b = 512;
    return (int)b;
}

namespace {

constexpr int kTB = 256;
template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };
// Partial-sum buffer layout (doubles): SpMV p.q partials, then r.z, r.r, b.b.
constexpr int kMaxParts = 2048;
constexpr int kPartPQ = 0, kPartRZ = 2048, kPartRR = 4096, kPartBB = 6144;

// Work-group sum with a fixed pattern: wave butterfly, then waves in order.
__device__ inline double wg_sum(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Every work-group computes the same total of part[0..nb) in the same order.
__device__ inline double reduce_parts(const double *part, int nb, double *sh)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kTB) v += part[i];
    return wg_sum(v, sh);
}

__device__ inline int load_flag(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The stop word flags[0]: 0 while the solve runs; once it stops, the number
// of iterations completed when the stop was decided, plus one (1 = converged
// at set-up).  It is read once per work-group so that every thread of the
// group takes the same branch (another group may store it meanwhile).
__device__ inline int wg_stop_word(const int32_t *flags)
{
    __shared__ int f;
    if (threadIdx.x == 0) f = load_flag(flags);
    __syncthreads();
    return f;
}

// Nothing in the SpMV launch stores the stop word, and a store in the x/r/z
// update launch is a breakdown that every group of it detects itself, so for
// those two any stop counts.
__device__ inline bool wg_done(const int32_t *flags) { return wg_stop_word(flags) != 0; }

// The p update of iteration k: a stop decided before it (word <= k + 1)
// ends it, but not the convergence found in this same launch (word k + 2,
// stored by group 0 while the other groups may not have started): every
// group finds that convergence from the same reduced r.r and must still
// apply x += alpha_k p_k.
__device__ inline bool wg_stopped_before(const int32_t *flags, int k)
{
    const int f = wg_stop_word(flags);
    return f != 0 && f <= k + 1;
}

__device__ inline void store_flag(int32_t *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// CSR-stream SpMV: a work-group takes a row block whose nonzeros are
// contiguous (<= kSpmvBlockNnz - 3 of them, <= kStreamRows rows, <=
// kSpmvBlockCols distinct columns), streams its values with coalesced loads,
// and lets kTPR threads per row add the products (thread j takes entries j,
// j+kTPR, ..., then a fixed shuffle combines the four).  Row blocks are fixed
// at upload: the summation order, and the result, do not depend on the grid.
//
// The upload stores, per block b, desc[b] = {first row, first nonzero,
// local-index segment, column-set offset}, the in-block row offsets
// roff[first row + b + i] = rowptr[r0 + i] - rowptr[r0] (i = 0..rows,
// uint16), the block's column set (its distinct columns) and one local index
// per entry into that set, so every load of a block depends only on its
// descriptor.
//
// Loads (VEC): the block is read through a window that starts at its first
// nonzero rounded down to a multiple of 4; thread t owns window entries
// 4t..4t+3 and reads their 4 local indices with one 4-byte load and their
// values with 16-byte loads (entries outside the block are weighted 0), and
// column t of the set.  Thread t gathers that column's vector entry once;
// the values, local indices and gathered entries go to LDS, and the row
// threads form each product there, rounded on its own (as a stored product
// would be).  FP64 values belong to the caller and are never read past
// nnz - 1: a pair that would cross the end is re-based to the last full
// pair and the final entry comes from one uniform load.  When the caller's
// value array is not 16-byte aligned, the scalar form (one entry per thread
// and pass, stride 256, plain column indices, products in registers) is
// used instead; both forms give bitwise the same y.
// The next block's loads are issued before the current block's products are
// formed, and both paths of the loop's last pass issue the same loads, so
// the stream never waits behind the gathers.
// xget(c) supplies the gathered vector entry of column c; wget(i) a per-row
// weight read before the row sums (so its latency overlaps them); yput(i, y,
// w) stores row i and returns its contribution to this work-group's sum.
constexpr int kStreamNnz = kSpmvBlockNnz, kTPR = 4, kStreamRows = kSpmvBlockRows, kPer = kStreamNnz / 256;
static_assert(kPer == 4, "one 4-entry chunk per thread");
static_assert(kStreamRows * kTPR == 256, "four threads per row in a 256-thread group");
static_assert(kStreamRows < 256, "the row index of a block's rows must fit the thread count");
constexpr int kXcds = 8;   // MI355X: 8 accelerator complex dies, one L2 each

typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Entries e..e+3 (e a multiple of 4) of a value array of n entries; NT:
// nontemporal loads (a template argument: a run-time choice between two
// loads of one address lets the compiler merge them and drop the hint).
template <bool NT>
__device__ inline void load_quad(const double *__restrict__ v, int64_t e, int64_t last_even, double last,
                                 double out[4])
{
    const int64_t a = e < last_even ? e : last_even;
    const int64_t b = e + 2 < last_even ? e + 2 : last_even;
    v2d pa, pb;
    if constexpr (NT) {
        pa = __builtin_nontemporal_load((const v2d *)(v + a));
        pb = __builtin_nontemporal_load((const v2d *)(v + b));
    } else {
        pa = *(const v2d *)(v + a);
        pb = *(const v2d *)(v + b);
    }
    out[0] = a == e ? pa.x : last;
    out[1] = pa.y;   // a != e only when entry e+1 is past the end (weighted 0)
    out[2] = b == e + 2 ? pb.x : last;
    out[3] = pb.y;
}
// The FP32 copy is the library's own, padded by 4: no re-basing needed.
template <bool NT>
__device__ inline void load_quad(const float *__restrict__ v, int64_t e, int64_t, float, float out[4])
{
    v4f q;
    if constexpr (NT) q = __builtin_nontemporal_load((const v4f *)(v + e));
    else q = *(const v4f *)(v + e);
    out[0] = q.x;
    out[1] = q.y;
    out[2] = q.z;
    out[3] = q.w;
}

// a * b rounded on its own (never contracted into a fused multiply-add), as
// a product stored and summed later would be
template <class T>
__device__ inline T mul_rn(T a, T b)
{
#pragma clang fp contract(off)
    return a * b;
}

// wg / G: this group's index and the number of groups working on the matrix
// (G a multiple of kXcds, and wg % kXcds the group's XCD).  nnz: entries of
// vals (the 16-byte path needs nnz >= 4).
// done_flags (may be null): a solve's flag word; a group returns right
// after issuing its first block's loads when the solve has already stopped
// (checked there so that the check's latency overlaps those loads).
// Row blocks reduced per work-group pass.  A pass has a fixed cost (the
// column-set gathers, two barriers, the LDS round trip) and FP32 blocks carry
// half the value bytes of FP64 ones, so the FP32 form reduces two blocks per
// pass (256^3 mixed-precision solve 0.448 -> 0.398 s); two per pass were
// slower for FP64 (128^3 SpMV 132.3 -> 139.0 us).  A group's blocks enter its
// partial sum in the same order either way.
template <class T> struct SpmvPass { static constexpr int BPI = 1; };
template <> struct SpmvPass<float> { static constexpr int BPI = 2; };

template <class T, bool VEC, bool NT, class XF, class WF, class YF>
__device__ inline double spmv_stream(const SpmvMap &sm, const int4 *__restrict__ desc, const T *__restrict__ vals,
                                     int wg, int G, XF xget, WF wget, YF yput,
                                     const int32_t *done_flags = nullptr)
{
    constexpr int BPI = SpmvPass<T>::BPI;
    const uint16_t *__restrict__ roff = sm.roff;
    const int64_t nrb = sm.nrb, nnz = sm.nnz;
    const int tid = threadIdx.x;
    double acc = 0.0;
    // XCD-aware walk: work-groups are dispatched round-robin over the XCDs,
    // so group w runs on XCD w % kXcds.  Each XCD's groups stream one
    // contiguous share of the row blocks, which keeps that share's slice of
    // the gathered vector in the XCD's own L2.
    const int ngrp = G / kXcds;                  // groups per XCD
    const int xcd = wg % kXcds, slot = wg / kXcds;
    const int64_t share = (nrb + kXcds - 1) / kXcds;
    const int64_t lo = (int64_t)xcd * share, hi = lo + share < nrb ? lo + share : nrb;
    int64_t blk = lo + slot;
    if (blk >= hi) return acc;                    // uniform over the group
    const int64_t last_even = (nnz - 2) & ~(int64_t)1;
    const T last = VEC ? vals[nnz - 1] : T(0);
    // A pass reduces BPI blocks of the group (blk + u * ngrp, u < BPI) with
    // one pair of barriers; a slot past the group's share holds a copy of
    // the first block's loads and no rows.
    __shared__ T prod[BPI][kStreamNnz];          // VEC: masked values; else products
    __shared__ int rps[BPI][kStreamRows + 1];    // row starts in the window
    __shared__ T xs[BPI][kSpmvBlockCols];        // VEC: the gathered column set
    __shared__ uint32_t lw[BPI][kSpmvBlockNnz / 4];   // VEC: local indices
    uint32_t li[BPI];   // VEC: local indices of this thread's 4 window entries
    int cc[BPI];        // VEC: this thread's column of the set
    int c[BPI][kPer];   // one-entry form: column indices
    T v[BPI][kPer];
    int r0[BPI], nrows[BPI], nz[BPI], ro[BPI], shift[BPI];
    bool live[BPI];
    // fetch(u, b, d0, d1, real): issue the loads of block b into slot u, whose
    // descriptor pair (d0, d1) = (desc[b], desc[b + 1]) was read beforehand;
    // with real == false only one chunk is touched (the loop's last pass
    // issues the same loads on both paths, so the wait counts of the gathers
    // do not depend on the branch).
    auto fetch = [&](int u, int64_t b, const int4 d0, const int4 d1, bool real) {
        r0[u] = d0.x;
        nrows[u] = d1.x - d0.x;
        nz[u] = d1.y - d0.y;
        live[u] = real;
        if (VEC) {
            const int64_t a0 = (int64_t)d0.y & ~(int64_t)3;
            shift[u] = d0.y - (int)a0;
            const int chunks = real ? (shift[u] + nz[u] + 3) / 4 : 1;
            const int t = tid < chunks ? tid : chunks - 1;
            li[u] = *(const uint32_t *)(sm.lidx + (int64_t)d0.z * 16 + 4 * t);
            const int ncol = d1.w - d0.w;
            cc[u] = sm.cols[d0.w + (tid < ncol ? tid : ncol - 1)];
            load_quad<NT>(vals, a0 + 4 * (int64_t)t, last_even, last, v[u]);
        } else {
            const int32_t *__restrict__ colidx = sm.colidx;
            const int64_t p0 = d0.y;
            shift[u] = 0;
            const int span = real ? nz[u] : 1;
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int kk = tid + 256 * j;
                const int64_t idx = p0 + (kk < span ? kk : span - 1);
                c[u][j] = colidx[idx];
                v[u][j] = vals[idx];
            }
        }
        ro[u] = roff[(int64_t)r0[u] + b + (tid < nrows[u] ? tid : nrows[u])];
    };
    auto pos = [&](int j) { return VEC ? 4 * tid + j : tid + 256 * j; };
    {
        int4 d0[BPI], d1[BPI];
        int64_t fb[BPI];
        bool ok[BPI];
#pragma unroll
        for (int u = 0; u < BPI; ++u) {
            const int64_t b = blk + (int64_t)u * ngrp;
            ok[u] = b < hi;
            fb[u] = ok[u] ? b : blk;
            d0[u] = desc[fb[u]];
            d1[u] = desc[fb[u] + 1];
        }
#pragma unroll
        for (int u = 0; u < BPI; ++u) fetch(u, fb[u], d0[u], d1[u], ok[u]);
    }
    if (done_flags && wg_done(done_flags)) return acc;
    const int row = tid / kTPR, sub = tid % kTPR;
    for (;;) {
        int cr0[BPI], cn[BPI], cnz[BPI], csh[BPI];
#pragma unroll
        for (int u = 0; u < BPI; ++u) {
            cr0[u] = r0[u];
            cn[u] = live[u] ? nrows[u] : 0;
            cnz[u] = nz[u];
            csh[u] = shift[u];
            if (tid <= cn[u]) rps[u][tid] = ro[u] + csh[u];
        }
        // the next pass's descriptors are read before the gathers are issued,
        // so that waiting for them never waits for the gathers
        const int64_t next = blk + (int64_t)BPI * ngrp;
        const bool more = next < hi;
        int4 n0[BPI], n1[BPI];
        int64_t nb[BPI];
        bool nok[BPI];
#pragma unroll
        for (int u = 0; u < BPI; ++u) {
            const int64_t b = next + (int64_t)u * ngrp;
            nok[u] = more && b < hi;
            nb[u] = nok[u] ? b : blk;
            n0[u] = desc[nb[u]];
            n1[u] = desc[nb[u] + 1];
        }
        T xv[BPI][kPer], vv[BPI][kPer], xc[BPI], wrow[BPI];
        uint32_t cli[BPI];
#pragma unroll
        for (int u = 0; u < BPI; ++u) {
            cli[u] = li[u];
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                if (!VEC) xv[u][j] = xget(c[u][j]);
                const int w = pos(j);
                vv[u][j] = (w >= csh[u] && w < csh[u] + cnz[u]) ? v[u][j] : T(0);
            }
            xc[u] = VEC ? xget(cc[u]) : T(0);
            wrow[u] = wget(cr0[u] + (row < nrows[u] ? row : nrows[u] - 1));
        }
#pragma unroll
        for (int u = 0; u < BPI; ++u) fetch(u, nb[u], n0[u], n1[u], nok[u]);
        // keep every load of the next pass ahead of the first wait on the gathers
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < BPI; ++u) {
            if (VEC) {
                // masked values, local indices and the gathered column set to
                // LDS; the row threads form the products
#pragma unroll
                for (int j = 0; j < kPer; ++j) prod[u][pos(j)] = vv[u][j];
                lw[u][tid] = cli[u];
                xs[u][tid] = xc[u];
            } else {
#pragma unroll
                for (int j = 0; j < kPer; ++j) prod[u][pos(j)] = vv[u][j] * xv[u][j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < BPI; ++u) {
            // entry q's product: a rounded product, never fused with the sum
            auto term = [&](int q) {
                if (VEC) return mul_rn(prod[u][q], xs[u][(lw[u][q >> 2] >> (8 * (q & 3))) & 0xffu]);
                return prod[u][q];
            };
            // two interleaved partial sums per thread: entries sub, sub + 8,
            // ... and sub + 4, sub + 12, ... (a fixed order)
            T s = T(0), s1 = T(0);
            if (row < cn[u]) {
                const int q1 = rps[u][row + 1];
                int q = rps[u][row] + sub;
                for (; q + kTPR < q1; q += 2 * kTPR) {
                    s += term(q);
                    s1 += term(q + kTPR);
                }
                if (q < q1) s += term(q);
            }
            s += s1;
            s += __shfl_xor(s, 1, kTPR);
            s += __shfl_xor(s, 2, kTPR);
            if (sub == 0 && row < cn[u]) acc += yput(cr0[u] + row, s, wrow[u]);
        }
        if (!more) break;
        __syncthreads();
        blk = next;
    }
    return acc;
}

template <class T, bool VEC>
__global__ void __launch_bounds__(kTB) k_spmv(SpmvMap sm, const int4 *__restrict__ desc, const T *__restrict__ vals,
                                              const T *__restrict__ x, T *__restrict__ y)
{
    spmv_stream<T, VEC, false>(
        sm, desc, vals, blockIdx.x, gridDim.x, [&](int col) { return x[col]; }, [&](int) { return T(0); },
        [&](int row, T val, T) {
            y[row] = val;
            return 0.0;
        });
}

// The 16-byte form needs the value array 16-byte aligned and nnz >= 4.
template <class T>
inline bool spmv_vec_ok(const T *vals, int64_t nnz)
{
    return ((uintptr_t)vals & 15) == 0 && nnz >= 4;
}

// Work-groups of the stream SpMV: five per CU (fewer than can be
// co-resident: on the 128^3 HEX08 Poisson matrix the column-set kernel took
// 130.6 us with 5 groups per CU, 134.8 with 4 or 6, 137.1 with 8, 141.8 with
// 3, and 137.8 / 140.6 with 4.5 / 5.5 (an uneven count per CU); more
// concurrent streams per CU contend in the memory system without hiding more
// latency), at most kMaxParts, at most one per row block.  Fixed per device,
// so reductions over the per-group partials keep a fixed order.
constexpr int kSpmvGroupsPerCU = 5;
int g_spmv_resident = 0;

int spmv_blocks(int64_t nrb)
{
    int cap = g_spmv_resident > 0 ? g_spmv_resident : kMaxParts;
    if (cap > kMaxParts) cap = kMaxParts;
    int64_t g = nrb < cap ? nrb : cap;
    g = (g + kXcds - 1) / kXcds * kXcds;    // a multiple of the XCD count
    return (int)(g < kXcds ? kXcds : g);
}

template <class T>
hipError_t spmv_dispatch(const DevMesh &m, hipStream_t s, const T *v, const T *x, T *y)
{
    const SpmvMap sm = spmv_map(m, sizeof(T));
    if (spmv_vec_ok(v, m.nnz))
        hipLaunchKernelGGL((k_spmv<T, true>), dim3(spmv_blocks(m.spmv_nrb)), dim3(kTB), 0, s, sm,
                           (const int4 *)m.spmv_desc, v, x, y);
    else
        hipLaunchKernelGGL((k_spmv<T, false>), dim3(spmv_blocks(m.spmv_nrb)), dim3(kTB), 0, s, sm,
                           (const int4 *)m.spmv_desc, v, x, y);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kTB) k_dot_part(int64_t n, const double *x, const double *y, double *part)
{
    __shared__ double sh[4];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) v += x[i] * y[i];
    v = wg_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void __launch_bounds__(kTB) k_reduce_final(const double *part, int nb, int nvec, double *out)
{
    __shared__ double sh[4];
    for (int q = 0; q < nvec; ++q) {
        const double v = reduce_parts(part + (int64_t)q * nb, nb, sh);
        if (threadIdx.x == 0) out[q] = v;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kTB) k_axpy(int64_t n, double a, const double *x, double *y)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) y[i] += a * x[i];
}

// Explicit-step vector updates ([3][n] velocity rows, mass m[n], Dirichlet
// flags): one Runge-Kutta stage u = alpha u0 + beta (u + dt r / m) at free
// nodes, u = u0 at Dirichlet nodes (u may alias neither u0 nor r); the
// velocity correction u -= dt g / m at free nodes; and f = 0 at Dirichlet rows.
template <int NC>
__global__ void __launch_bounds__(kTB) k_rk_stage(int64_t n, double alpha, double beta, double dt, const double *u0,
                                                  const double *r, const double *m, const uint8_t *is_dir, double *u)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        const bool fixed = is_dir[i] != 0;
        const double h = dt / m[i];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int64_t j = c * n + i;
            u[j] = fixed ? u0[j] : alpha * u0[j] + beta * (u[j] + h * r[j]);
        }
    }
}

__global__ void __launch_bounds__(kTB) k_correct(int64_t n, double dt, const double *g, const double *m,
                                                 const uint8_t *is_dir, double *u)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        if (is_dir[i]) continue;
        const double h = dt / m[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) u[c * n + i] -= h * g[c * n + i];
    }
}

__global__ void __launch_bounds__(kTB) k_zero_fixed(int64_t n, const uint8_t *is_dir, double *f)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        if (is_dir[i]) f[i] = 0.0;
}

// Symmetric Dirichlet elimination on the affected rows, G lanes per row.
template <int G>
__global__ void __launch_bounds__(kTB) k_dirichlet(const int32_t *rowptr, const int32_t *colidx, const int32_t *rows,
                                                   int64_t nrows, const uint8_t *is_dir, double *vals, double *rhs,
                                                   const double *g)
{
    const int sub = threadIdx.x & (G - 1);
    const int64_t stride = (int64_t)gridDim.x * (kTB / G);
    for (int64_t q = (int64_t)blockIdx.x * (kTB / G) + threadIdx.x / G; q < nrows; q += stride) {
        const int i = rows[q];
        const int p0 = rowptr[i], p1 = rowptr[i + 1];
        double s = 0.0;
        if (is_dir[i]) {
            for (int p = p0 + sub; p < p1; p += G) {
                if (colidx[p] == i) s += vals[p];
                else vals[p] = 0.0;
            }
        } else {
            for (int p = p0 + sub; p < p1; p += G) {
                const int j = colidx[p];
                if (is_dir[j]) {
                    if (g) s += vals[p] * g[j];
                    vals[p] = 0.0;
                }
            }
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (sub == 0) {
            if (is_dir[i]) rhs[i] = s * (g ? g[i] : 0.0);
            else rhs[i] -= s;
        }
    }
}

__global__ void __launch_bounds__(kTB) k_permute(int64_t n, int ncomp, const int32_t *perm, const double *in,
                                                 double *out, int gather)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        const int64_t j = perm[i];
        for (int c = 0; c < ncomp; ++c) {
            if (gather) out[c * n + i] = in[c * n + j];
            else out[c * n + j] = in[c * n + i];
        }
    }
}

// ---- PCG ---------------------------------------------------------------------
// hist[k*4 + 0..3] = rz_k, rr_k, pq_k, alpha_k ;  flags = {stop word (wg_stop_word), status, iters,
// iteration counter}
// part layout: [0] p.q, [1] r.z, [2] r.r, [3] b.b  (each nb doubles)

template <class T>
__global__ void __launch_bounds__(kTB) k_dinv(int64_t n, const int32_t *diagpos, const T *vals, T *dinv)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        dinv[i] = T(1) / vals[diagpos[i]];
}

template <class T>
__global__ void __launch_bounds__(kTB) k_cg_init(int64_t n, const T *b, const T *q, T *x, T *r, T *z, T *p,
                                                 const T *dinv, double *part, int nb, int x_zero)
{
    __shared__ double sh[4];
    double rz = 0.0, rr = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        const T bi = b[i];
        T ri;
        if (x_zero) {
            x[i] = T(0);
            ri = bi;
        } else {
            ri = bi - q[i];
        }
        const T zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        p[i] = zi;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
        bb += (double)bi * (double)bi;
    }
    rz = wg_sum(rz, sh);
    rr = wg_sum(rr, sh);
    bb = wg_sum(bb, sh);
    if (threadIdx.x == 0) {
        part[kPartRZ + blockIdx.x] = rz;
        part[kPartRR + blockIdx.x] = rr;
        part[kPartBB + blockIdx.x] = bb;
    }
}

__global__ void __launch_bounds__(kTB) k_cg_init_fin(const double *part, int nb, double rtol, double *hist,
                                                     double *scal, int32_t *flags)
{
    __shared__ double sh[4];
    const double rz = reduce_parts(part + kPartRZ, nb, sh);
    const double rr = reduce_parts(part + kPartRR, nb, sh);
    const double bb = reduce_parts(part + kPartBB, nb, sh);
    if (threadIdx.x == 0) {
        hist[0] = rz;
        hist[1] = rr;
        scal[0] = bb;
        const double thr2 = rtol > 0.0 ? rtol * rtol * bb : -1.0;
        scal[1] = thr2;
        flags[0] = (rr <= thr2) ? 1 : 0;   // stop word: converged with 0 iterations
        flags[1] = FE_OK;
        flags[2] = 0;
        flags[3] = -1;   // iteration counter: each SpMV launch advances it
    }
}

// One PCG iteration is three steps over one system; each is written for a
// work-group wg of G groups, so that the same code runs as a launch of its
// own (wg = blockIdx.x) or as one system's share of a batched launch that
// advances many systems at once.  A system's result depends only on its own
// G, never on what else shares the launch.

// Iteration k, first step: q = A p and the partial p . q.
template <class T, bool VEC, bool NT>
__device__ inline void cg_spmv_pq_step(const SpmvMap &sm, const int4 *__restrict__ desc, const T *__restrict__ vals,
                                       const T *__restrict__ p,
                                       T *__restrict__ q, double *__restrict__ part, const int32_t *flags, int wg,
                                       int G)
{
    __shared__ double sh[4];
    double acc = spmv_stream<T, VEC, NT>(
        sm, desc, vals, wg, G, [&](int c) { return p[c]; }, [&](int row) { return p[row]; },
        [&](int row, T val, T prow) {
            q[row] = val;
            return (double)prow * (double)val;
        },
        flags);
    acc = wg_sum(acc, sh);
    if (threadIdx.x == 0) part[kPartPQ + wg] = acc;
}

// Iteration k, second step: alpha = rz_k / (p . q); r -= alpha q;
// z = D^-1 r; partials of r.z and r.r.  (x += alpha p is left to the third
// step, which reads p anyway: the same arithmetic, one vector pass less.)
template <class T>
__device__ inline void cg_update_xr_step(int64_t n, int k, T *r, T *z, const T *q, const T *dinv, double *part,
                                         int nb_spmv, double *hist, int32_t *flags, int wg, int G)
{
    __shared__ double sh[4];
    // two entries per thread and item (16-byte accesses for FP64); each
    // item's operands are requested one item ahead, the first ones before
    // the scalar reduction, so that their latency overlaps it
    using T2 = typename Vec2<T>::type;
    const int64_t n2 = n / 2, stride = (int64_t)G * kTB;
    int64_t j = (int64_t)wg * kTB + threadIdx.x;
    T2 qv{}, dv{}, rv{};
    if (n2 > 0) {
        const int64_t j0 = j < n2 ? j : 0;
        qv = ((const T2 *)q)[j0];
        dv = ((const T2 *)dinv)[j0];
        rv = ((const T2 *)r)[j0];
    }
    if (wg_done(flags)) return;
    const double pq = reduce_parts(part + kPartPQ, nb_spmv, sh);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (wg == 0 && threadIdx.x == 0) {
            store_flag(flags + 1, FE_EBREAKDOWN);
            store_flag(flags + 2, k);
            store_flag(flags + 0, k + 1);   // k iterations completed
        }
        return;
    }
    const double alpha = hist[(int64_t)k * 4 + 0] / pq;
    const T a = T(alpha);
    double rz = 0.0, rr = 0.0;
    for (; j < n2; j += stride) {
        const int64_t jn = j + stride < n2 ? j + stride : j;
        const T2 nq = ((const T2 *)q)[jn], nd = ((const T2 *)dinv)[jn], nr = ((const T2 *)r)[jn];
        rv.x -= a * qv.x;
        rv.y -= a * qv.y;
        T2 zv;
        zv.x = dv.x * rv.x;
        zv.y = dv.y * rv.y;
        ((T2 *)r)[j] = rv;
        ((T2 *)z)[j] = zv;
        rz += (double)rv.x * (double)zv.x + (double)rv.y * (double)zv.y;
        rr += (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
        qv = nq;
        dv = nd;
        rv = nr;
    }
    if ((n & 1) && wg == 0 && threadIdx.x == 0) {
        const int64_t i = n - 1;
        const T ri = r[i] - a * q[i];
        const T zi = dinv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
    rz = wg_sum(rz, sh);
    rr = wg_sum(rr, sh);
    if (threadIdx.x == 0) {
        part[kPartRZ + wg] = rz;
        part[kPartRR + wg] = rr;
    }
    if (wg == 0 && threadIdx.x == 0) {
        hist[(int64_t)k * 4 + 2] = pq;
        hist[(int64_t)k * 4 + 3] = alpha;
    }
}

// Iteration k, third step: every work-group reduces the r.z and r.r
// partials (same order, same result); x += alpha_k p_k; then
// ||r||^2 <= rtol^2 ||b||^2 ends the solve, else beta = rz_{k+1} / rz_k and
// p = z + beta p.
template <class T>
__device__ inline void cg_update_p_step(int64_t n, int k, T *x, const T *z, T *p, double *part, int nb, double *hist,
                                        const double *scal, int32_t *flags, int wg, int G)
{
    __shared__ double sh[4];
    using T2 = typename Vec2<T>::type;
    const int64_t n2 = n / 2, stride = (int64_t)G * kTB;
    int64_t j = (int64_t)wg * kTB + threadIdx.x;
    T2 zv{}, pv{}, xv{};
    if (n2 > 0) {
        const int64_t j0 = j < n2 ? j : 0;
        zv = ((const T2 *)z)[j0];
        pv = ((const T2 *)p)[j0];
        xv = ((const T2 *)x)[j0];
    }
    if (wg_stopped_before(flags, k)) return;
    const double rz1 = reduce_parts(part + kPartRZ, nb, sh);
    const double rr = reduce_parts(part + kPartRR, nb, sh);
    const bool conv = rr <= scal[1];
    if (wg == 0 && threadIdx.x == 0) {
        hist[(int64_t)(k + 1) * 4 + 0] = rz1;
        hist[(int64_t)(k + 1) * 4 + 1] = rr;
        store_flag(flags + 2, k + 1);
        if (conv) store_flag(flags + 0, k + 2);   // k + 1 iterations completed
    }
    const T a = T(hist[(int64_t)k * 4 + 3]);
    const T beta = T(rz1 / hist[(int64_t)k * 4 + 0]);
    for (; j < n2; j += stride) {
        const int64_t jn = j + stride < n2 ? j + stride : j;
        const T2 nz = ((const T2 *)z)[jn], np = ((const T2 *)p)[jn], nx = ((const T2 *)x)[jn];
        xv.x += a * pv.x;
        xv.y += a * pv.y;
        ((T2 *)x)[j] = xv;
        if (!conv) {
            pv.x = zv.x + beta * pv.x;
            pv.y = zv.y + beta * pv.y;
            ((T2 *)p)[j] = pv;
        }
        zv = nz;
        pv = np;
        xv = nx;
    }
    if ((n & 1) && wg == 0 && threadIdx.x == 0) {
        x[n - 1] += a * p[n - 1];
        if (!conv) p[n - 1] = z[n - 1] + beta * p[n - 1];
    }
}

// The one-system kernels take the iteration index from the device
// (flags[3]): the SpMV launch of iteration k advances it from k - 1 to k,
// and the two updates, which run after it, read it.  No launch argument
// changes from one iteration to the next, so a run of iterations can be
// recorded once as a HIP graph and replayed.
template <class T, bool VEC, bool NT>
__global__ void __launch_bounds__(kTB) k_cg_spmv_pq(SpmvMap sm, const int4 *__restrict__ desc,
                                                    const T *__restrict__ vals, const T *__restrict__ p,
                                                    T *__restrict__ q, double *__restrict__ part, int32_t *flags)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) store_flag(flags + 3, load_flag(flags + 3) + 1);
    cg_spmv_pq_step<T, VEC, NT>(sm, desc, vals, p, q, part, flags, blockIdx.x, gridDim.x);
}

// The PCG's SpMV on its symmetric matrix: the CSR-stream form above on the
// row blocks of the symmetric map (SymMap in plan.h).  A block's window of
// packed values holds its stored entries only; each lower entry (i, j) with
// both rows in the block (a mirror) reads the stored (j, i) from LDS, so the
// value stream shrinks by the block-internal lower triangle (~20 % of the
// entries of a HEX08 Poisson matrix).  The set's first slots are the block's
// own rows, so a mirror names its column by its row offset.  Loads, the
// one-block-ahead prefetch and the fixed summation order follow spmv_stream:
// thread t owns window entries 4t..4t+3, column t of the set and mirror
// word t; the four threads of a row add its stored products and then its
// mirror products in two interleaved partial sums and a fixed shuffle.
// Returns this group's share of p . q.
template <bool NT>
__device__ inline double spmv_sym_stream(const SymSpmv &sm, int wg, int G, const double *__restrict__ p,
                                         double *__restrict__ q, const int32_t *done_flags)
{
    const int tid = threadIdx.x;
    double acc = 0.0;
    const int ngrp = G / kXcds;
    const int xcd = wg % kXcds, slot = wg / kXcds;
    const int64_t nrb = sm.nrb;
    const int64_t share = (nrb + kXcds - 1) / kXcds;
    const int64_t lo = (int64_t)xcd * share, hi = lo + share < nrb ? lo + share : nrb;
    int64_t blk = lo + slot;
    if (blk >= hi) return acc;                   // uniform over the group
    __shared__ double vs[kStreamNnz];            // the window's values, masked to the block
    __shared__ double xs[kSpmvBlockCols];        // the gathered column set
    __shared__ uint32_t lw[kStreamNnz / 4];      // set slots of the window entries
    __shared__ uint32_t mw[kSymMirrors / 2];     // mirror entries, two per word
    __shared__ uint32_t rps[kStreamRows + 1];    // row starts: stored | mirrors << 16
    uint32_t li, mword, ro;
    int cc, r0, nrows, nz, shift;
    double v[4];
    // fetch(b, d0, d1, real): issue block b's loads (descriptor pair read
    // beforehand); real == false touches one chunk only (see spmv_stream)
    auto fetch = [&](int64_t b, const int4 d0, const int4 d1, bool real) {
        r0 = d0.x;
        nrows = d1.x - d0.x;
        nz = d1.y - d0.y;
        const int64_t a0 = (int64_t)d0.y & ~(int64_t)3;
        shift = d0.y - (int)a0;
        const int chunks = real ? (shift + nz + 3) / 4 : 1;
        const int t = tid < chunks ? tid : chunks - 1;
        li = *(const uint32_t *)(sm.lidx + a0 + 4 * t);
        const v2d *pv = (const v2d *)(sm.vals + a0 + 4 * (int64_t)t);
        v2d pa, pb;
        if constexpr (NT) {
            pa = __builtin_nontemporal_load(pv);
            pb = __builtin_nontemporal_load(pv + 1);
        } else {
            pa = pv[0];
            pb = pv[1];
        }
        v[0] = pa.x;
        v[1] = pa.y;
        v[2] = pb.x;
        v[3] = pb.y;
        const int ncol = d1.w - d0.w;
        cc = sm.cols[d0.w + (tid < ncol ? tid : ncol - 1)];
        const int nmw = d1.z - d0.z;
        mword = sm.mir[d0.z + (tid < nmw ? tid : 0)];
        ro = sm.roff[(int64_t)r0 + b + (tid < nrows ? tid : nrows)];
    };
    fetch(blk, sm.desc[blk], sm.desc[blk + 1], true);
    if (done_flags && wg_done(done_flags)) return acc;
    const int row = tid / kTPR, sub = tid % kTPR;
    for (;;) {
        const int cr0 = r0, cn = nrows, cnz = nz, csh = shift;
        if (tid <= cn) rps[tid] = ro;
        const int64_t next = blk + ngrp;
        const bool more = next < hi;
        const int64_t nb = more ? next : blk;
        const int4 n0 = sm.desc[nb], n1 = sm.desc[nb + 1];
        double vv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int w = 4 * tid + j;
            vv[j] = (w >= csh && w < csh + cnz) ? v[j] : 0.0;
        }
        const uint32_t cli = li, cmw = mword;
        const double xc = p[cc];
        fetch(nb, n0, n1, more);
        // keep every load of the next block ahead of the first wait on the gathers
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) vs[4 * tid + j] = vv[j];
        lw[tid] = cli;
        xs[tid] = xc;
        mw[tid] = cmw;
        __syncthreads();
        auto term = [&](int e) { return mul_rn(vs[e], xs[(lw[e >> 2] >> (8 * (e & 3))) & 0xffu]); };
        auto mterm = [&](int m) {
            const uint32_t w = (mw[m >> 1] >> (16 * (m & 1))) & 0xffffu;
            return mul_rn(vs[w & 1023u], xs[w >> 10]);
        };
        double s = 0.0, s1 = 0.0;
        if (row < cn) {
            const uint32_t a = rps[row], e = rps[row + 1];
            const int q1 = csh + (int)(e & 0xffffu);
            int k = csh + (int)(a & 0xffffu) + sub;
            for (; k + kTPR < q1; k += 2 * kTPR) {
                s += term(k);
                s1 += term(k + kTPR);
            }
            if (k < q1) s += term(k);
            const int m1 = (int)(e >> 16);
            int m = (int)(a >> 16) + sub;
            for (; m + kTPR < m1; m += 2 * kTPR) {
                s += mterm(m);
                s1 += mterm(m + kTPR);
            }
            if (m < m1) s += mterm(m);
        }
        s += s1;
        s += __shfl_xor(s, 1, kTPR);
        s += __shfl_xor(s, 2, kTPR);
        if (sub == 0 && row < cn) {
            q[cr0 + row] = s;
            acc += xs[row] * s;   // p[first row + row]: the set's own-row slot
        }
        if (!more) break;
        __syncthreads();
        blk = next;
    }
    return acc;
}

// Iteration k, first step on the symmetric map: q = A p and the partial p . q
// (advances the iteration counter like k_cg_spmv_pq).
template <bool NT>
__global__ void __launch_bounds__(kTB) k_cg_spmv_sym(SymSpmv sm, const double *__restrict__ p,
                                                     double *__restrict__ q, double *__restrict__ part,
                                                     int32_t *flags)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) store_flag(flags + 3, load_flag(flags + 3) + 1);
    __shared__ double sh[4];
    double acc = spmv_sym_stream<NT>(sm, blockIdx.x, gridDim.x, p, q, flags);
    acc = wg_sum(acc, sh);
    if (threadIdx.x == 0) part[kPartPQ + blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kTB) k_set_i32(int32_t *p, int v)
{
    if (threadIdx.x == 0) store_flag(p, v);
}

// Packs a matrix for the symmetric SpMV: one work-group per row block, four
// threads per row as in the SpMV.  Each row's stored entries go to their
// window positions in LDS (its mirror run left out, mstart); after a barrier
// the window is copied to the packed array in one coalesced pass (rows hold
// ~22 stored entries: written row by row they would leave partial lines), and
// each mirror entry (i, j) compares its
// value with the stored (j, i) it replaces, on the scale of the larger of the
// two and sqrt|a_ii a_jj| (the bound of an off-diagonal entry of an SPD
// matrix, which keeps an entry summed to nearly zero from failing the check
// on rounding alone).
__global__ void __launch_bounds__(kTB) k_sym_pack(SymSpmv sm, const int32_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ diagpos,
                                                  const uint8_t *__restrict__ mstart,
                                                  const double *__restrict__ vals, double *__restrict__ packed,
                                                  int32_t *bad)
{
    __shared__ double win[kStreamNnz];
    const int tid = threadIdx.x, row = tid / kTPR, sub = tid % kTPR;
    const uint16_t *__restrict__ mir16 = (const uint16_t *)sm.mir;
    bool ok = true;
    for (int64_t b = blockIdx.x; b < sm.nrb; b += gridDim.x) {
        const int4 d0 = sm.desc[b], d1 = sm.desc[b + 1];
        const int r0 = d0.x, R = d1.x - d0.x, shift = d0.y & 3;
        const int ns = (int)(sm.roff[(int64_t)r0 + b + R] & 0xffffu);   // the block's stored entries
        int64_t p0 = 0;
        int ms = 0, ml = 0, mo = 0;
        if (row < R) {
            const uint32_t ro = sm.roff[(int64_t)r0 + b + row], ro1 = sm.roff[(int64_t)r0 + b + row + 1];
            const int so = (int)(ro & 0xffffu), len = rowptr[r0 + row + 1] - rowptr[r0 + row];
            mo = (int)(ro >> 16);
            ml = (int)(ro1 >> 16) - mo;
            ms = mstart[r0 + row];
            p0 = rowptr[r0 + row];
            for (int k = sub; k < len; k += kTPR) {
                if (k >= ms && k < ms + ml) continue;   // a mirror: checked below
                win[shift + so + (k < ms ? k : k - ml)] = vals[p0 + k];
            }
        }
        __syncthreads();
        for (int t = tid; t < ns; t += kTB) packed[(int64_t)d0.y + t] = win[shift + t];
        if (row < R) {
            for (int m = sub; m < ml; m += kTPR) {
                const double a = vals[p0 + ms + m];
                const uint32_t w = mir16[2 * (int64_t)d0.z + mo + m];
                const double t = win[w & 1023u];
                const double dd = sqrt(fabs(vals[diagpos[r0 + row]] * vals[diagpos[r0 + (int)(w >> 10)]]));
                const double mx = fmax(fmax(fabs(a), fabs(t)), dd);
                ok = ok && isfinite(a) && isfinite(t) && fabs(a - t) <= 0x1p-40 * mx;
            }
        }
        __syncthreads();
    }
    if (!ok) store_flag(bad, 1);
}

template <class T>
__global__ void __launch_bounds__(kTB) k_cg_update_xr(int64_t n, T *r, T *z, const T *q, const T *dinv, double *part,
                                                      int nb_spmv, double *hist, int32_t *flags)
{
    const int k = load_flag(flags + 3);
    cg_update_xr_step<T>(n, k, r, z, q, dinv, part, nb_spmv, hist, flags, blockIdx.x, gridDim.x);
}

template <class T>
__global__ void __launch_bounds__(kTB) k_cg_update_p(int64_t n, T *x, const T *z, T *p, double *part, int nb,
                                                     double *hist, const double *scal, int32_t *flags)
{
    const int k = load_flag(flags + 3);
    cg_update_p_step<T>(n, k, x, z, p, part, nb, hist, scal, flags, blockIdx.x, gridDim.x);
}

// ---- batched PCG: one launch per step for every system of a BatchList ----
// Work-group w belongs to the system j with start[j] <= w < start[j+1]
// (a handful of entries: a linear scan).
__device__ inline int batch_find(const int *start, int n, int w)
{
    int j = 0;
    while (j + 1 < n && w >= start[j + 1]) ++j;
    return j;
}

__global__ void __launch_bounds__(kTB) k_bat_spmv_pq(const BatchJob *__restrict__ jobs, BatchList L)
{
    const int j = batch_find(L.wgs, L.n, blockIdx.x);
    const BatchJob &b = jobs[L.slot[j]];
    const int wg = blockIdx.x - L.wgs[j], G = L.wgs[j + 1] - L.wgs[j];
    // the serving arena keeps every value array 256-byte aligned (and every
    // mesh has nnz >= 4): the 16-byte form only
    cg_spmv_pq_step<double, true, false>(b.sm, b.sm.desc, b.vals, b.p, b.q, b.part, b.flags, wg, G);
}

__global__ void __launch_bounds__(kTB) k_bat_update_xr(const BatchJob *__restrict__ jobs, BatchList L)
{
    const int j = batch_find(L.wgv, L.n, blockIdx.x);
    const BatchJob &b = jobs[L.slot[j]];
    cg_update_xr_step<double>(b.n, L.k[j], b.r, b.z, b.q, b.dinv, b.part, b.nb_spmv, b.hist, b.flags,
                              blockIdx.x - L.wgv[j], L.wgv[j + 1] - L.wgv[j]);
}

__global__ void __launch_bounds__(kTB) k_bat_update_p(const BatchJob *__restrict__ jobs, BatchList L)
{
    const int j = batch_find(L.wgv, L.n, blockIdx.x);
    const BatchJob &b = jobs[L.slot[j]];
    cg_update_p_step<double>(b.n, L.k[j], b.x, b.z, b.p, b.part, b.nb_vec, b.hist, b.scal, b.flags,
                             blockIdx.x - L.wgv[j], L.wgv[j + 1] - L.wgv[j]);
}

__global__ void __launch_bounds__(kTB) k_cast(int64_t n, const double *in, float *out)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        out[i] = (float)in[i];
}

__global__ void __launch_bounds__(kTB) k_scale_cast(int64_t n, double s, const double *in, float *out)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        out[i] = (float)(in[i] * s);
}

__global__ void __launch_bounds__(kTB) k_add_scaled(int64_t n, double s, const float *d, double *x)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        x[i] += s * (double)d[i];
}

// r = b - q (q = A x on entry in r), partials of r.r and b.b
__global__ void __launch_bounds__(kTB) k_resid(int64_t n, const double *b, double *r, double *part, int nb)
{
    __shared__ double sh[4];
    double rr = 0.0, bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        const double ri = b[i] - r[i];
        r[i] = ri;
        rr += ri * ri;
        bb += b[i] * b[i];
    }
    rr = wg_sum(rr, sh);
    bb = wg_sum(bb, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rr;
        part[nb + blockIdx.x] = bb;
    }
}

}  // namespace

hipError_t init_spmv_grid(int device)
{
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void *>(&k_cg_spmv_pq<double, true, true>), kTB, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    if (per_cu > kSpmvGroupsPerCU) per_cu = kSpmvGroupsPerCU;
    g_spmv_resident = per_cu * prop.multiProcessorCount;
    return hipSuccess;
}

hipError_t launch_sym_pack(const DevMesh &m, const SymSpmv &map, const uint8_t *mstart, const double *vals,
                           double *packed, int32_t *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(kTB), 0, s, bad, 0);
    if (map.nrb > 0) {
        const unsigned grid = (unsigned)(map.nrb < (1 << 20) ? map.nrb : (1 << 20));
        hipLaunchKernelGGL(k_sym_pack, dim3(grid), dim3(kTB), 0, s, map, m.rowptr, m.diagpos, mstart, vals, packed,
                           bad);
    }
    return hipGetLastError();
}

hipError_t launch_spmv(const DevMesh &m, const double *vals, const double *x, double *y, hipStream_t s)
{
    return spmv_dispatch<double>(m, s, vals, x, y);
}

hipError_t launch_dot(int64_t n, const double *x, const double *y, double *part, double *out, hipStream_t s)
{
    const int nb = stream_blocks(n);
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(kTB), 0, s, n, x, y, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kTB), 0, s, part, nb, 1, out);
    return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, dim3(stream_blocks(n)), dim3(kTB), 0, s, n, a, x, y);
    return hipGetLastError();
}

hipError_t launch_rk_stage(const DevMesh &m, double alpha, double beta, double dt, const double *u0,
                           const double *r, const double *mass, double *u, hipStream_t s, int ncomp)
{
    if (ncomp == 3)
        hipLaunchKernelGGL(k_rk_stage<3>, dim3(stream_blocks(m.N)), dim3(kTB), 0, s, m.N, alpha, beta, dt, u0, r,
                           mass, m.is_dir, u);
    else
        hipLaunchKernelGGL(k_rk_stage<1>, dim3(stream_blocks(m.N)), dim3(kTB), 0, s, m.N, alpha, beta, dt, u0, r,
                           mass, m.is_dir, u);
    return hipGetLastError();
}

hipError_t launch_correct(const DevMesh &m, double dt, const double *g, const double *mass, double *u, hipStream_t s)
{
    hipLaunchKernelGGL(k_correct, dim3(stream_blocks(m.N)), dim3(kTB), 0, s, m.N, dt, g, mass, m.is_dir, u);
    return hipGetLastError();
}

hipError_t launch_zero_fixed(const DevMesh &m, double *f, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_fixed, dim3(stream_blocks(m.N)), dim3(kTB), 0, s, m.N, m.is_dir, f);
    return hipGetLastError();
}

hipError_t launch_dirichlet(const DevMesh &m, double *vals, double *rhs, const double *g, hipStream_t s)
{
    if (m.n_dir_rows == 0) return hipSuccess;
    int G = 2;
    while (G < m.max_row && G < 64) G <<= 1;
    int64_t rows_per_wg = kTB / G;
    int64_t nb64 = (m.n_dir_rows + rows_per_wg - 1) / rows_per_wg;
    const int nb = (int)(nb64 > 4096 ? 4096 : nb64);
#define FE_DIR(GV)                                                                                       \
    hipLaunchKernelGGL((k_dirichlet<GV>), dim3(nb), dim3(kTB), 0, s, m.rowptr, m.colidx, m.dir_rows,       \
                       m.n_dir_rows, m.is_dir, vals, rhs, g)
    switch (G) {
    case 2: FE_DIR(2); break;
    case 4: FE_DIR(4); break;
    case 8: FE_DIR(8); break;
    case 16: FE_DIR(16); break;
    case 32: FE_DIR(32); break;
    default: FE_DIR(64); break;
    }
#undef FE_DIR
    return hipGetLastError();
}

hipError_t launch_permute(int64_t n, int ncomp, const int32_t *perm, const double *in, double *out, bool gather,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_permute, dim3(stream_blocks(n)), dim3(kTB), 0, s, n, ncomp, perm, in, out, gather ? 1 : 0);
    return hipGetLastError();
}

template <class T>
hipError_t cg_setup(const DevMesh &m, const T *vals, const T *b, T *x, CGWork &w, double rtol, hipStream_t s,
                    bool x_zero)
{
    const int64_t n = m.N;
    const int nb = stream_blocks(n);
    w.nb = nb;
    T *r = sizeof(T) == 8 ? (T *)w.r : (T *)w.r32;
    T *z = sizeof(T) == 8 ? (T *)w.z : (T *)w.z32;
    T *p = sizeof(T) == 8 ? (T *)w.p : (T *)w.p32;
    T *q = sizeof(T) == 8 ? (T *)w.q : (T *)w.q32;
    T *dinv = sizeof(T) == 8 ? (T *)w.dinv : (T *)w.dinv32;
    hipLaunchKernelGGL((k_dinv<T>), dim3((n + kTB - 1) / kTB), dim3(kTB), 0, s, n, m.diagpos, vals, dinv);
    if (!x_zero) {
        hipError_t e = spmv_dispatch<T>(m, s, vals, x, q);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_cg_init<T>), dim3(nb), dim3(kTB), 0, s, n, b, q, x, r, z, p, dinv, w.part, nb,
                       x_zero ? 1 : 0);
    hipLaunchKernelGGL(k_cg_init_fin, dim3(1), dim3(kTB), 0, s, w.part, nb, rtol, w.hist, w.hist + 4 * w.hist_cap,
                       w.flags);
    return hipGetLastError();
}

template <class T>
hipError_t cg_spmv_pq(const DevMesh &m, const T *vals, CGWork &w, int, hipStream_t s)
{
    const T *p = sizeof(T) == 8 ? (const T *)w.p : (const T *)w.p32;
    T *q = sizeof(T) == 8 ? (T *)w.q : (T *)w.q32;
    if constexpr (sizeof(T) == 8) {
        if (w.sym.vals) {
            const dim3 grid(spmv_blocks(w.sym.nrb)), block(kTB);
            if (w.sym.nt)
                hipLaunchKernelGGL((k_cg_spmv_sym<true>), grid, block, 0, s, w.sym, p, q, w.part, w.flags);
            else
                hipLaunchKernelGGL((k_cg_spmv_sym<false>), grid, block, 0, s, w.sym, p, q, w.part, w.flags);
            return hipGetLastError();
        }
    }
    const SpmvMap sm = spmv_map(m, sizeof(T));
    const dim3 grid(spmv_blocks(m.spmv_nrb)), block(kTB);
    const int4 *desc = (const int4 *)m.spmv_desc;
    if (!spmv_vec_ok(vals, m.nnz))
        hipLaunchKernelGGL((k_cg_spmv_pq<T, false, false>), grid, block, 0, s, sm, desc, vals, p, q, w.part, w.flags);
    else if (sm.nt)
        hipLaunchKernelGGL((k_cg_spmv_pq<T, true, true>), grid, block, 0, s, sm, desc, vals, p, q, w.part, w.flags);
    else
        hipLaunchKernelGGL((k_cg_spmv_pq<T, true, false>), grid, block, 0, s, sm, desc, vals, p, q, w.part, w.flags);
    return hipGetLastError();
}

template <class T>
hipError_t cg_updates(const DevMesh &m, T *x, CGWork &w, int k, hipStream_t s)
{
    const int64_t n = m.N;
    T *r = sizeof(T) == 8 ? (T *)w.r : (T *)w.r32;
    T *z = sizeof(T) == 8 ? (T *)w.z : (T *)w.z32;
    T *p = sizeof(T) == 8 ? (T *)w.p : (T *)w.p32;
    T *q = sizeof(T) == 8 ? (T *)w.q : (T *)w.q32;
    T *dinv = sizeof(T) == 8 ? (T *)w.dinv : (T *)w.dinv32;
    // the partial p . q sums of the SpMV launch that ran (one per work-group)
    const int nb_spmv = sizeof(T) == 8 && w.sym.vals ? spmv_blocks(w.sym.nrb) : spmv_blocks(m.spmv_nrb);
    hipLaunchKernelGGL((k_cg_update_xr<T>), dim3(w.nb), dim3(kTB), 0, s, n, r, z, (const T *)q, (const T *)dinv,
                       w.part, nb_spmv, w.hist, w.flags);
    hipLaunchKernelGGL((k_cg_update_p<T>), dim3(w.nb), dim3(kTB), 0, s, n, x, (const T *)z, p, w.part, w.nb, w.hist,
                       (const double *)(w.hist + 4 * w.hist_cap), w.flags);
    return hipGetLastError();
}

template hipError_t cg_setup<double>(const DevMesh &, const double *, const double *, double *, CGWork &, double,
                                     hipStream_t, bool);
template hipError_t cg_setup<float>(const DevMesh &, const float *, const float *, float *, CGWork &, double,
                                    hipStream_t, bool);
template hipError_t cg_spmv_pq<double>(const DevMesh &, const double *, CGWork &, int, hipStream_t);
template hipError_t cg_spmv_pq<float>(const DevMesh &, const float *, CGWork &, int, hipStream_t);
template hipError_t cg_updates<double>(const DevMesh &, double *, CGWork &, int, hipStream_t);
template hipError_t cg_updates<float>(const DevMesh &, float *, CGWork &, int, hipStream_t);

int cg_spmv_groups(const DevMesh &m) { return spmv_blocks(m.spmv_nrb); }

bool spmv_vec_capable(const double *vals, int64_t nnz) { return spmv_vec_ok(vals, nnz); }

hipError_t batch_iteration(const BatchJob *jobs, const BatchList &L, hipStream_t s)
{
    if (L.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bat_spmv_pq, dim3(L.wgs[L.n]), dim3(kTB), 0, s, jobs, L);
    hipLaunchKernelGGL(k_bat_update_xr, dim3(L.wgv[L.n]), dim3(kTB), 0, s, jobs, L);
    hipLaunchKernelGGL(k_bat_update_p, dim3(L.wgv[L.n]), dim3(kTB), 0, s, jobs, L);
    return hipGetLastError();
}

hipError_t cast_f64_f32(int64_t n, const double *in, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast, dim3(stream_blocks(n)), dim3(kTB), 0, s, n, in, out);
    return hipGetLastError();
}

hipError_t scale_f64_to_f32(int64_t n, double scale, const double *in, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_cast, dim3(stream_blocks(n)), dim3(kTB), 0, s, n, scale, in, out);
    return hipGetLastError();
}

hipError_t add_f32_to_f64(int64_t n, double scale, const float *d, double *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_scaled, dim3(stream_blocks(n)), dim3(kTB), 0, s, n, scale, d, x);
    return hipGetLastError();
}

hipError_t residual_f64(const DevMesh &m, const double *vals, const double *b, const double *x, double *r,
                        double *part, double *out_rr_bb, hipStream_t s)
{
    const int64_t n = m.N;
    const int nb = stream_blocks(n);
    launch_spmv(m, vals, x, r, s);
    hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kTB), 0, s, n, b, r, part, nb);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kTB), 0, s, part, nb, 2, out_rr_bb);
    return hipGetLastError();
}

}  // namespace feasm
