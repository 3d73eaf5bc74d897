// internal.h -- structures shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/feasm.h"

namespace feasm {

// Element-vector passes of the explicit step, numbered after the fe_operator
// values: residual -(C(u) + K_mu) u per component plus the rho-weighted
// lumped mass, pressure gradient int N grad p, divergence right-hand side
// (1/dt) int grad N . (rho u), scalar-transport residual -(C(u) + K_{rho D}) Y
// plus the lumped mass.
constexpr int kOpResidual = 3, kOpGradient = 4, kOpDivergence = 5, kOpScalarResidual = 6, kNumOps = 7;

// One assembly launch: the blocks color_blk[first, first + count), all of one
// colour and one element type (nen nodes); lds[op] = LDS bytes of its
// largest block for operator (or element-vector pass) op.
struct AsmLaunch {
    int nen, first, count;
    size_t lds[kNumOps];
};

// Device-resident mesh: geometry, CSR pattern and the block scatter plan.
struct DevMesh {
    int nen = 0;                        // connectivity stride: nodes of the largest element type
    int off_stride = 0;                 // bytes of elem_off per element
    int64_t N = 0, E = 0, nnz = 0, nblk = 0;
    int n_colors = 0, max_T = 0, max_L = 0, max_row = 0, max_phase = 0;
    std::vector<AsmLaunch> launches;    // host: launch order (colour-major, then type)

    double *X = nullptr;                // [3][N]
    int32_t *rowptr = nullptr, *colidx = nullptr, *diagpos = nullptr;
    int32_t *blk_elem_ptr = nullptr, *blk_node_ptr = nullptr, *blk_nodes = nullptr;
    int32_t *blk_rdesc = nullptr, *blk_rowstart = nullptr;   // per touched row
    uint8_t *blk_nphase = nullptr;
    uint16_t *elem_lnode = nullptr;     // [nen][E]
    uint8_t *elem_off = nullptr;        // [E][off_stride], row a of an n-node element at a * n
    uint8_t *elem_phase = nullptr;      // [E]
    int32_t *color_blk = nullptr;
    int32_t *node_perm = nullptr;       // mesh -> user
    int32_t *elem_perm = nullptr;       // mesh -> user
    uint8_t *is_dir = nullptr;          // [N]
    int32_t *dir_rows = nullptr;        // rows touched by the Dirichlet elimination
    int64_t n_dir = 0, n_dir_rows = 0;
    // SpMV row blocks (see kSpmvBlockRows): desc[b] = {first row, first
    // nonzero, local-index segment offset in 16-byte units, offset of the
    // block's column set in cols}, b = 0..nrb (the last is the end
    // sentinel); roff holds each block's row offsets relative to its first
    // nonzero, rows + 1 entries at roff[first row + b]; lidx and cols the
    // block-local column indices and column sets (see SpmvMap).
    // Owner plan of the matrix assembly (single-type meshes; own_G = 0
    // otherwise): groups {first task, tasks, first row, rows}, their touched
    // nodes (owned rows first), phases, and per task the element, the local
    // node of each (rotated) element node and the in-row column positions.
    int64_t own_G = 0, own_T = 0;
    int own_ra = 0, own_ln_stride = 0, own_off_stride = 0, own_priv = 0;
    int own_max_nodes = 0, own_max_img = 0, own_max_rows = 0;
    int4 *own_groups = nullptr;
    int32_t *own_node_ptr = nullptr, *own_nodes = nullptr, *own_elem = nullptr;
    uint8_t *own_nphase = nullptr, *own_off = nullptr, *own_phase = nullptr;
    uint16_t *own_ln = nullptr;
    int4 *spmv_desc = nullptr;
    uint16_t *spmv_roff = nullptr;
    uint8_t *spmv_lidx = nullptr;
    int32_t *spmv_cols = nullptr;
    int64_t spmv_nrb = 0;
};

// What the SpMV kernels read besides values and vectors.  Each row block has
// a column set: its distinct columns in first-touch order (<= kSpmvBlockCols of them,
// cols[desc[b].w .. desc[b + 1].w)), and one byte per entry that indexes it.
// The local indices cover the block's 4-aligned window (first nonzero
// rounded down to a multiple of 4, a multiple of 4 entries); window entries
// outside the block hold 0 (a valid index, weighted 0).  The gathered
// vector is read once per column of the set instead of once per entry.
struct SpmvMap {
    const int4 *desc;
    const uint16_t *roff;
    const uint8_t *lidx;
    const int32_t *cols;
    const int32_t *colidx;   // canonical CSR columns (the one-entry form)
    int64_t nrb, nnz;
    int nt;                  // the PCG's SpMV streams the values with nontemporal loads
};
// The PCG's six vectors stay in MI355X's 256 MiB memory-side cache between
// the launches of an iteration when they take at most 3/4 of it; the matrix
// values are then loaded nontemporally so that their stream does not evict
// them (128^3 HEX08: SpMV 131.8 -> 128.4 us, vector updates 39.6 -> 34.9 us).
// Past that size the nontemporal loads cost (256^3: 1.34 -> 1.43 ms per
// iteration) and plain loads are used.
constexpr int64_t kMallResidentBytes = (int64_t)192 << 20;
inline SpmvMap spmv_map(const DevMesh &m, int elem_bytes = 8)
{
    const int nt = 6 * (int64_t)elem_bytes * m.N <= kMallResidentBytes ? 1 : 0;
    return SpmvMap{m.spmv_desc, m.spmv_roff, m.spmv_lidx, m.spmv_cols, m.colidx, m.spmv_nrb, m.nnz, nt};
}

// The symmetric PCG SpMV (see SymMap in plan.h): the map's device arrays and
// the packed values it reads (vals == nullptr: the general SpMV runs).
struct SymSpmv {
    const int4 *desc = nullptr;
    const uint32_t *roff = nullptr;
    const uint8_t *lidx = nullptr;
    const uint32_t *mir = nullptr;
    const int32_t *cols = nullptr;
    const double *vals = nullptr;
    int64_t nrb = 0;
    int nt = 0;              // nontemporal value loads, as SpmvMap::nt
};
// Packs the FP64 values of the mesh pattern's entries for the symmetric SpMV
// map (mstart: its per-row mirror-run starts) and sets *bad to 1 when a
// mirror entry a_ij differs from the stored a_ji by more than 2^-40
// max(|a_ij|, |a_ji|, sqrt|a_ii a_jj|) (or either is not finite).  *bad is
// set to 0 first.
hipError_t launch_sym_pack(const DevMesh &m, const SymSpmv &map, const uint8_t *mstart, const double *vals,
                           double *packed, int32_t *bad, hipStream_t s);

// Wall faces of a mesh (boundary assembly of the wall model): face node
// counts and connectivity (mesh numbering, unused slots repeat slot 0), the
// wall nodes with, for each, its (face, slot) entries in ascending order,
// and the per-face partial sums [F][4][3].
struct DevWall {
    int64_t F = 0, W = 0;
    double delta = 0.0;
    uint8_t *nen = nullptr;
    int32_t *conn = nullptr;    // [F][4]
    int32_t *nodes = nullptr;   // [W]
    int32_t *ptr = nullptr;     // [W + 1]
    int32_t *ent = nullptr;     // face * 4 + slot
    double *part = nullptr;     // [F][4][3]
};
// Wall-model traction (asm_kernels.hip): out[3][N] += sum over faces of
// int N_a t dS at the wall nodes (zero elsewhere when zero_first).
hipError_t launch_wall_traction(const DevMesh &m, const DevWall &w, const double *u, const double *rho,
                                const double *mu, double *out, bool zero_first, hipStream_t s);

// Device status word of an assembly launch sequence.
struct AsmStatus {
    unsigned long long min_det_key;     // order-preserving key of the smallest det J
    long long first_bad;                // smallest mesh element index with det J <= 0
};

// Systems (serving slots) one batched launch may cover.
constexpr int kMaxBatch = 32;

struct AsmArgs {
    const DevMesh *m;
    int op;                  // fe_operator, or kOpResidual / kOpGradient / kOpDivergence
    double dt, Dk;
    const double *u, *rho, *mu, *Y;   // Y: the scalar of this pass
    const double *p;         // kOpGradient: the pressure
    int form;                // kOpResidual: FE_FORM_* operator variants
    double *values;          // operator's value array [nnz]
    double *rhs;             // first rhs row [N] (momentum: 3 rows of N; element-vector passes: their rows)
    AsmStatus *status;       // status word, followed by the per-block / per-group scratch
    AsmStatus *status_out = nullptr;   // where the reduced word goes instead of *status (null: *status)
};

// Launchers (asm_kernels.hip).
hipError_t launch_assemble(const AsmArgs &a, bool mixed, hipStream_t s);
// Batched coloured assembly of one operator (MOMENTUM or POISSON, FP64) over
// n meshes that carry the coloured plan only (the serving runtime): launch li
// of every mesh's (colour, type) list runs as one launch per element type,
// launch li + 1 after it, then each mesh's status word.  Request i's kernel
// arguments must sit in the device table kargs_d at slot[i] * kKArgsBytes,
// written from fill_kargs(a[i]) before the launches run.
constexpr size_t kKArgsBytes = 256;
void fill_kargs(const AsmArgs &a, void *out);   // out: kKArgsBytes bytes
hipError_t launch_assemble_batch(const AsmArgs *a, const int *slot, int n, const void *kargs_d, hipStream_t s);

// Device copy of the row-owner plan of the 3x3-block momentum operator
// (plan.h RowPlan), built on the first block assembly of a mesh.
struct DevRowPlan {
    int64_t n_tasks = 0, n_waves = 0, max_img = 0;
    int stride = 0;
    int32_t *conn = nullptr;       // [E][stride] mesh numbering
    uint8_t *etype = nullptr;      // [E] node counts, or null (every element has stride nodes)
    int32_t *task_elem = nullptr;
    uint16_t *task_meta = nullptr;
    uint8_t *task_cols = nullptr;  // [T][8]
    int4 *wdesc = nullptr;         // {first task, tasks, first row, rows}
    double *w_mindet = nullptr;    // [waves]
    long long *w_bad = nullptr;    // [waves]
};
// values[nnz][3][3], rhs[3][N]: the momentum operator with the form bits'
// terms (FE_FORM_FULL_STRESS, FE_FORM_EMAC) as 3x3 blocks; status word as
// for launch_assemble.
hipError_t launch_assemble_block(const DevMesh &m, const DevRowPlan &r, int form, double dt, const double *u,
                                 const double *rho, const double *mu, double *values, double *rhs,
                                 AsmStatus *status, hipStream_t s);

// Solver launchers (solver_kernels.hip).
struct CGWork {
    int64_t n = 0;
    int nb = 0;                          // work-groups of the streaming kernels
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *dinv = nullptr;
    double *part = nullptr;              // partial sums (kPartDoubles)
    double *hist = nullptr;              // [cap][4] per-iteration scalars
    int32_t *flags = nullptr;            // [4]: stop word (0 running, else completed iterations + 1), status,
                                         // iterations, iteration counter
    int hist_cap = 0;
    // mixed precision buffers
    float *v32 = nullptr, *r32 = nullptr, *z32 = nullptr, *p32 = nullptr, *q32 = nullptr, *x32 = nullptr,
          *dinv32 = nullptr;
    int64_t v32_cap = 0;
    double *d64 = nullptr;               // FP64 outer residual
    size_t bytes = 0;
    SymSpmv sym;                         // FP64 iterations: the symmetric SpMV when sym.vals is set
};

constexpr int kPartDoubles = 8192;
// SpMV row blocks (fixed at upload): <= kSpmvBlockRows rows,
// <= kSpmvBlockNnz - 3 nonzeros, contiguous in CSR (a block read through a
// 4-aligned window of kSpmvBlockNnz entries), and <= kSpmvBlockCols distinct
// columns (one-byte local indices).  The device column-index array is
// padded by kColPad zeros.
constexpr int kSpmvBlockRows = 64, kSpmvBlockNnz = 1024, kSpmvBlockCols = 256, kColPad = 4;
int stream_blocks(int64_t n);
// Sizes the SpMV grid for the device: five work-groups per CU, at most as many
// as are co-resident (context creation).
hipError_t init_spmv_grid(int device);
hipError_t launch_spmv(const DevMesh &m, const double *vals, const double *x, double *y, hipStream_t s);
hipError_t launch_dot(int64_t n, const double *x, const double *y, double *part, double *out, hipStream_t s);
hipError_t launch_axpy(int64_t n, double a, const double *x, double *y, hipStream_t s);
hipError_t launch_dirichlet(const DevMesh &m, double *vals, double *rhs, const double *g, hipStream_t s);
// Explicit-step updates on [3][N] velocity rows (k_rk_stage, k_correct) and
// zeroing a right-hand side at the Dirichlet nodes.
hipError_t launch_rk_stage(const DevMesh &m, double alpha, double beta, double dt, const double *u0,
                           const double *r, const double *mass, double *u, hipStream_t s, int ncomp = 3);
hipError_t launch_correct(const DevMesh &m, double dt, const double *g, const double *mass, double *u, hipStream_t s);
hipError_t launch_zero_fixed(const DevMesh &m, double *f, hipStream_t s);
hipError_t launch_permute(int64_t n, int ncomp, const int32_t *perm, const double *in, double *out, bool gather,
                          hipStream_t s);

// PCG building blocks (see solver_kernels.hip for the iteration scheme).
template <class T>
hipError_t cg_setup(const DevMesh &m, const T *vals, const T *b, T *x, CGWork &w, double rtol, hipStream_t s,
                    bool x_zero);
// One PCG iteration k = cg_spmv_pq (q = A p, partial p.q) + cg_updates (x, r,
// z with r.z and r.r, then the stop test and p = z + beta p).
template <class T>
hipError_t cg_spmv_pq(const DevMesh &m, const T *vals, CGWork &w, int k, hipStream_t s);
template <class T>
hipError_t cg_updates(const DevMesh &m, T *x, CGWork &w, int k, hipStream_t s);
hipError_t cast_f64_f32(int64_t n, const double *in, float *out, hipStream_t s);

// Batched FP64 PCG (serving): the device-resident description of one system
// and the per-launch list of systems advanced together.  The work-group
// counts are the ones a launch of its own would use (cg_spmv_groups and
// stream_blocks), so a system's iterates do not depend on its neighbours.
struct BatchJob {
    SpmvMap sm;
    const double *vals;
    int64_t n;
    double *x, *r, *z, *p, *q, *dinv, *part, *hist;
    const double *scal;
    int32_t *flags;
    int nb_spmv, nb_vec;
    int vec;                     // 16-byte SpMV loads (vals aligned, nnz >= 4)
};

struct BatchList {
    int n;                       // systems in this launch
    int slot[kMaxBatch];         // index into the BatchJob table
    int k[kMaxBatch];            // iteration index of each system
    int wgs[kMaxBatch + 1];      // SpMV work-group prefix
    int wgv[kMaxBatch + 1];      // vector-kernel work-group prefix
};
int cg_spmv_groups(const DevMesh &m);
bool spmv_vec_capable(const double *vals, int64_t nnz);
hipError_t batch_iteration(const BatchJob *jobs, const BatchList &L, hipStream_t s);
hipError_t residual_f64(const DevMesh &m, const double *vals, const double *b, const double *x, double *r,
                        double *part, double *out_rr_bb, hipStream_t s);
hipError_t add_f32_to_f64(int64_t n, double scale, const float *d, double *x, hipStream_t s);
hipError_t scale_f64_to_f32(int64_t n, double scale, const double *in, float *out, hipStream_t s);

}  // namespace feasm
