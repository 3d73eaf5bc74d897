// feasm.cpp -- C ABI entry points: context, mesh upload, assembly, PCG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/feasm.h"
#include "host.h"
#include "internal.h"
#include "plan.h"

using namespace feasm;

// Work area of fe_cg_solve_noalloc (one copy per device, held until the
// process ends; its device address is looked up per device in fe_ctx_create).
static __device__ __align__(256) char scratch[FE_NOALLOC_BYTES];

namespace feasm {

fe_status fail(fe_ctx_s *c, fe_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

// ---- device arena (first fit over one allocation) ---------------------------

DevArena::DevArena(char *base, size_t bytes) : base_(base), cap_(bytes & ~(size_t)255), free_total_(cap_)
{
    if (cap_) holes_.push_back({0, cap_});
}

void *DevArena::alloc(size_t bytes)
{
    const size_t b = round(bytes ? bytes : 1);
    for (size_t i = 0; i < holes_.size(); ++i) {
        if (holes_[i].second < b) continue;
        const size_t off = holes_[i].first;
        holes_[i].first += b;
        holes_[i].second -= b;
        if (holes_[i].second == 0) holes_.erase(holes_.begin() + (long)i);
        auto it = std::lower_bound(used_.begin(), used_.end(), std::make_pair(off, (size_t)0));
        used_.insert(it, {off, b});
        free_total_ -= b;
        return base_ + off;
    }
    return nullptr;
}

void DevArena::release(void *p)
{
    if (!p) return;
    const size_t off = (size_t)((char *)p - base_);
    auto it = std::lower_bound(used_.begin(), used_.end(), std::make_pair(off, (size_t)0));
    if (it == used_.end() || it->first != off) return;   // not ours
    const size_t b = it->second;
    used_.erase(it);
    free_total_ += b;
    auto h = std::lower_bound(holes_.begin(), holes_.end(), std::make_pair(off, (size_t)0));
    h = holes_.insert(h, {off, b});
    // merge with the next and the previous hole
    if (h + 1 != holes_.end() && h->first + h->second == (h + 1)->first) {
        h->second += (h + 1)->second;
        holes_.erase(h + 1);
    }
    if (h != holes_.begin() && (h - 1)->first + (h - 1)->second == h->first) {
        (h - 1)->second += h->second;
        holes_.erase(h);
    }
}

// ---- mesh image / device copy --------------------------------------------------

namespace {

// Visits every device array of a mesh: f(device pointer slot, host source or
// nullptr, bytes).  The one list drives both the byte count and the upload.
template <class F>
void for_each_array(MeshImage &I, DevMesh &d, AsmStatus **status, F f)
{
    Plan &P = I.P;
    auto v = [&](auto **dst, const auto &src) {
        f((void **)dst, (const void *)src.data(), src.size() * sizeof(src[0]));
    };
    v(&d.X, P.X);
    v(&d.rowptr, P.rowptr);
    v(&d.colidx, P.colidx);
    v(&d.diagpos, P.diagpos);
    v(&d.blk_elem_ptr, P.blk_elem_ptr);
    v(&d.blk_node_ptr, P.blk_node_ptr);
    v(&d.blk_nodes, P.blk_nodes);
    v(&d.blk_rdesc, P.blk_rdesc);
    v(&d.blk_rowstart, P.blk_rowstart);
    v(&d.blk_nphase, P.blk_nphase);
    v(&d.elem_lnode, P.elem_lnode);
    v(&d.elem_off, P.elem_off);
    v(&d.elem_phase, P.elem_phase);
    v(&d.color_blk, P.color_blk);
    v(&d.node_perm, P.node_perm);
    v(&d.elem_perm, P.elem_perm);
    if (!I.O.groups.empty()) {
        v(&d.own_groups, I.O.groups);
        v(&d.own_node_ptr, I.O.node_ptr);
        v(&d.own_nodes, I.O.nodes);
        v(&d.own_nphase, I.O.nphase);
        v(&d.own_elem, I.O.tk_elem);
        v(&d.own_ln, I.O.tk_ln);
        v(&d.own_off, I.O.tk_off);
        v(&d.own_phase, I.O.tk_phase);
    }
    v(&d.spmv_desc, I.spmv_desc);
    v(&d.spmv_roff, I.spmv_roff);
    v(&d.spmv_lidx, I.spmv_lidx);
    v(&d.spmv_cols, I.spmv_cols);
    v(&d.is_dir, I.is_dir);
    v(&d.dir_rows, I.dir_rows);
    f((void **)status, nullptr, sizeof(AsmStatus) + (size_t)std::max<int64_t>(d.nblk, d.own_G) * 16);
}

}  // namespace

size_t MeshImage::device_bytes() const
{
    MeshImage &I = const_cast<MeshImage &>(*this);
    DevMesh d = I.d;
    AsmStatus *st = nullptr;
    size_t total = 0;
    for_each_array(I, d, &st, [&](void **, const void *, size_t b) { total += DevArena::round(b ? b : 1); });
    return total;
}

void MeshImage::clear()
{
    P.clear();
    O = OwnerPlan();
    is_dir.clear();
    dir_rows.clear();
    spmv_desc.clear();
    spmv_roff.clear();
    spmv_lidx.clear();
    spmv_cols.clear();
    d = DevMesh();
}

// Per-chunk outputs of the SpMV row blocks (see mesh_prepare), kept per
// calling thread like the planner's other temporaries.
struct RowChunk {
    std::vector<int32_t> rb, cols, coff;   // per block: end row, end of its column set
    std::vector<int64_t> seg;              // per block: byte offset of its local indices
    std::vector<uint8_t> lidx;             // a multiple of 16 bytes
};
static thread_local std::vector<RowChunk> t_rowchunks;
static thread_local std::vector<std::vector<int32_t>> t_spmv_stamp, t_spmv_loc;   // per worker, [N]

int mesh_prepare(int stride, const uint8_t *types, int64_t n_nodes, const double *coords, int64_t n_elems,
                 const int32_t *conn, int64_t n_dirichlet, const int32_t *dirichlet_nodes, bool renumber,
                 MeshImage &I, std::string &err, bool owner_plan)
{
    if (n_dirichlet < 0 || (n_dirichlet > 0 && !dirichlet_nodes)) {
        err = "bad Dirichlet list";
        return FE_EINVAL;
    }
    Plan &P = I.P;
    int st = build_plan(stride, types, n_nodes, coords, n_elems, conn, renumber, P, err);
    if (st != FE_OK) return st;
    I.is_dir.assign(n_nodes, 0);
    for (int64_t k = 0; k < n_dirichlet; ++k) {
        int32_t v = dirichlet_nodes[k];
        if (v < 0 || v >= n_nodes) {
            err = "Dirichlet node " + std::to_string(v) + " out of range";
            return FE_EINVAL;
        }
        I.is_dir[P.node_iperm[v]] = 1;
    }
    int64_t ndir = 0;
    for (int64_t i = 0; i < n_nodes; ++i) ndir += I.is_dir[i] != 0;
    // rows that hold a Dirichlet node (its own row or a column), ascending
    {
        const int64_t nch = (n_nodes + kPlanRowChunk - 1) / kPlanRowChunk;
        std::vector<std::vector<int32_t>> part(nch);
        parallel_chunks(nch, [&](int64_t c) {
            const int64_t r0 = c * kPlanRowChunk, r1 = std::min<int64_t>(n_nodes, r0 + kPlanRowChunk);
            for (int64_t i = r0; i < r1; ++i) {
                bool hit = I.is_dir[i] != 0;
                for (int32_t p = P.rowptr[i]; !hit && p < P.rowptr[i + 1]; ++p) hit = I.is_dir[P.colidx[p]] != 0;
                if (hit) part[c].push_back((int32_t)i);
            }
        });
        I.dir_rows.clear();
        for (const auto &v : part) I.dir_rows.insert(I.dir_rows.end(), v.begin(), v.end());
    }
    DevMesh &d = I.d;
    d = DevMesh();
    d.nen = P.nen;
    d.off_stride = P.off_stride;
    d.N = P.N;
    d.E = P.E;
    d.nnz = P.nnz;
    d.nblk = P.n_blocks();
    d.n_colors = P.n_colors;
    d.max_T = P.max_T;
    d.max_L = P.max_L;
    d.max_row = P.max_row;
    d.max_phase = P.max_phase;
    d.n_dir = ndir;
    d.n_dir_rows = (int64_t)I.dir_rows.size();
    // SpMV row blocks: consecutive rows, <= kSpmvBlockRows rows (4 threads per
    // row in a 256-thread group), <= kSpmvBlockNnz - 3 nonzeros (a 4-aligned
    // window of kSpmvBlockNnz entries in LDS) and <= kSpmvBlockCols distinct
    // columns, none across a kPlanRowChunk boundary.  A single row always
    // fits (rows are <= 255 entries).
    // Each row chunk (in parallel) builds its blocks greedily, their column
    // sets (distinct columns in first-touch order, found through a small
    // open-addressing table) and the local indices; the chunks are then
    // concatenated.  The set order is free (a product is v * x[col] whatever
    // slot x[col] is staged in); first-touch order keeps it nearly ascending.
    const int64_t nrch = (P.N + kPlanRowChunk - 1) / kPlanRowChunk;
    std::vector<RowChunk> &rch = t_rowchunks;
    if ((int64_t)rch.size() < nrch) rch.resize(nrch);
    // a column is in the open block's set while stamp[v] == the block's id
    // (ids unique per worker), at slot loc[v]
    const int nw = parallel_workers(nrch);
    std::vector<std::vector<int32_t>> &stamps = t_spmv_stamp, &locs = t_spmv_loc;
    if ((int)stamps.size() < nw) stamps.resize(nw);
    if ((int)locs.size() < nw) locs.resize(nw);
    std::vector<char> ready(nw, 0);
    std::vector<int32_t> next_id(nw, 0);
    parallel_chunks_w(nrch, [&](int64_t c, int w) {
        RowChunk &C = rch[c];
        C.rb.clear();
        C.cols.clear();
        C.coff.clear();
        C.seg.clear();
        C.lidx.clear();
        const int64_t R0 = c * kPlanRowChunk, R1 = std::min<int64_t>(P.N, R0 + kPlanRowChunk);
        C.lidx.reserve((size_t)(P.rowptr[R1] - P.rowptr[R0]) + 16 * (size_t)((R1 - R0) / 16 + 1));
        std::vector<int32_t> &stamp = stamps[w], &loc = locs[w];
        if (!ready[w]) {
            stamp.assign((size_t)P.N, -1);
            loc.resize((size_t)P.N);
            ready[w] = 1;
        }
        for (int64_t r = R0; r < R1;) {
            const int32_t bid = next_id[w]++;
            const int32_t c0 = (int32_t)C.cols.size();
            const int64_t p0 = P.rowptr[r], a0 = p0 & ~(int64_t)3;
            const size_t s0 = C.lidx.size();   // 16-byte aligned
            C.lidx.resize(s0 + (size_t)(p0 - a0), 0);   // window entries before the block
            auto take = [&](int64_t row) {
                for (int32_t q = P.rowptr[row]; q < P.rowptr[row + 1]; ++q) {
                    const int32_t v = P.colidx[q];
                    if (stamp[v] != bid) {
                        stamp[v] = bid;
                        loc[v] = (int32_t)C.cols.size() - c0;
                        C.cols.push_back(v);
                    }
                    C.lidx.push_back((uint8_t)loc[v]);
                }
            };
            take(r);
            int64_t r1 = r + 1;
            while (r1 < R1 && r1 - r < kSpmvBlockRows && P.rowptr[r1 + 1] - P.rowptr[r] <= kSpmvBlockNnz - 3) {
                const size_t nc = C.cols.size(), nl = C.lidx.size();
                take(r1);
                if ((int64_t)C.cols.size() - c0 > kSpmvBlockCols) {   // row r1 opens the next block
                    for (size_t k = nc; k < C.cols.size(); ++k) stamp[C.cols[k]] = -1;
                    C.cols.resize(nc);
                    C.lidx.resize(nl);
                    break;
                }
                ++r1;
            }
            // pad the window to a multiple of 4 entries, the segment to 16 bytes
            const int64_t win = ((p0 & 3) + (P.rowptr[r1] - p0) + 3) & ~(int64_t)3;
            C.lidx.resize(s0 + (size_t)((win + 15) & ~(int64_t)15), 0);
            C.seg.push_back((int64_t)s0);
            C.coff.push_back((int32_t)C.cols.size());
            C.rb.push_back((int32_t)r1);
            r = r1;
        }
    });
    std::vector<int32_t> rb{0}, col_off{0};
    std::vector<int64_t> seg_off;   // byte offset of each block's local indices
    {
        size_t nl = 16, nc = 0, nb = 0;
        for (int64_t c = 0; c < nrch; ++c) {
            const RowChunk &C = rch[c];
            nl += C.lidx.size();
            nc += C.cols.size();
            nb += C.rb.size();
        }
        I.spmv_cols.clear();
        I.spmv_lidx.clear();
        I.spmv_cols.reserve(nc);
        I.spmv_lidx.reserve(nl);
        rb.reserve(nb + 1);
        col_off.reserve(nb + 1);
        seg_off.reserve(nb);
        for (int64_t c = 0; c < nrch; ++c) {
            const RowChunk &C = rch[c];
            const int64_t lb = (int64_t)I.spmv_lidx.size();
            const int32_t cb = (int32_t)I.spmv_cols.size();
            I.spmv_lidx.insert(I.spmv_lidx.end(), C.lidx.begin(), C.lidx.end());
            I.spmv_cols.insert(I.spmv_cols.end(), C.cols.begin(), C.cols.end());
            for (size_t k = 0; k < C.rb.size(); ++k) {
                rb.push_back(C.rb[k]);
                col_off.push_back(cb + C.coff[k]);
                seg_off.push_back(lb + C.seg[k]);
            }
        }
    }
    {
        size_t kept = 0;
        for (const RowChunk &C : rch)
            kept += C.lidx.capacity() + 4 * (C.rb.capacity() + C.cols.capacity() + C.coff.capacity()) +
                    8 * C.seg.capacity();
        for (const auto &v : stamps) kept += 4 * v.capacity();
        for (const auto &v : locs) kept += 4 * v.capacity();
        if (kept > kPlanScratchKeep) {
            rch = std::vector<RowChunk>();
            stamps = std::vector<std::vector<int32_t>>();
            locs = std::vector<std::vector<int32_t>>();
        }
    }
    I.spmv_lidx.resize(I.spmv_lidx.size() + 16, 0);
    d.spmv_nrb = (int64_t)rb.size() - 1;
    I.spmv_desc.assign((size_t)d.spmv_nrb + 1, int4{0, 0, 0, 0});
    I.spmv_roff.assign((size_t)(P.N + d.spmv_nrb), 0);
    parallel_chunks((d.spmv_nrb + 4095) / 4096, [&](int64_t c) {
        for (int64_t b = c * 4096; b < std::min<int64_t>(d.spmv_nrb, (c + 1) * 4096); ++b) {
            I.spmv_desc[b] = int4{rb[b], P.rowptr[rb[b]], (int32_t)(seg_off[b] / 16), col_off[b]};
            for (int32_t i = rb[b]; i <= rb[b + 1]; ++i)
                I.spmv_roff[(size_t)(rb[b] + b + (i - rb[b]))] = (uint16_t)(P.rowptr[i] - P.rowptr[rb[b]]);
        }
    });
    I.spmv_desc[d.spmv_nrb] = int4{(int32_t)P.N, (int32_t)P.nnz, (int32_t)((I.spmv_lidx.size() - 16) / 16),
                                   col_off[d.spmv_nrb]};
    // the SpMV reads column indices in aligned groups of 4: pad the device copy
    P.colidx.resize((size_t)P.nnz + kColPad, 0);
    // assembly launches and their LDS per operator: [fields NF][rhs NRHS]
    // doubles per row, one int descriptor per row (+ alignment), then the row
    // image, for the launch's largest block
    // (the element-vector passes stage no row image)
    const int nf[kNumOps] = {8, 8, 7, 8, 4, 7, 8}, nr[kNumOps] = {3, 1, 1, 4, 3, 1, 2};
    d.launches.clear();
    for (const AsmSeg &g : P.segs) {
        AsmLaunch L{g.nen, g.first, g.count, {0, 0, 0, 0, 0, 0, 0}};
        for (int q = g.first; q < g.first + g.count; ++q) {
            const int32_t b = P.color_blk[q];
            const int64_t T = P.blk_node_ptr[b + 1] - P.blk_node_ptr[b];
            const int64_t nl = P.blk_img[b];
            for (int op = 0; op < kNumOps; ++op) {
                size_t by = (size_t)(nf[op] + nr[op]) * T * 8 + (size_t)T * 4 + 8 + (op < 3 ? (size_t)nl * 8 : 0);
                L.lds[op] = std::max(L.lds[op], by);
            }
        }
        d.launches.push_back(L);
    }
    // the owner plan of the matrix assembly (meshes of one element type)
    I.O = OwnerPlan();
    if (owner_plan && P.etype.empty()) {
        st = build_owner_plan(P, I.O, err);
        if (st != FE_OK) return st;
        const OwnerPlan &O = I.O;
        d.own_G = (int64_t)O.groups.size();
        d.own_T = (int64_t)O.tk_elem.size();
        d.own_ra = O.ra;
        d.own_priv = O.wave_private ? 1 : 0;
        d.own_ln_stride = O.ln_stride;
        d.own_off_stride = O.off_stride;
        d.own_max_nodes = O.max_nodes;
        d.own_max_img = O.max_img;
        d.own_max_rows = O.max_rows;
    }
    return FE_OK;
}

fe_status mesh_alloc(fe_mesh_s *m, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (m->arena) {
        *p = m->arena->alloc(bytes);
        if (!*p) return fail(m->ctx, FE_ENOMEM, "arena: no room for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess)
            return fail(m->ctx, FE_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    m->allocs.push_back(*p);
    m->bytes += m->arena ? DevArena::round(bytes) : bytes;
    return FE_OK;
}

static void mesh_free_ptr(fe_mesh_s *m, void *p)
{
    if (!p) return;
    auto it = std::find(m->allocs.begin(), m->allocs.end(), p);
    if (it != m->allocs.end()) m->allocs.erase(it);
    if (m->arena) m->arena->release(p);
    else (void)hipFree(p);
}

void mesh_release(fe_mesh_s *m)
{
    for (auto &g : m->graph) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = fe_mesh_s::PcgGraph();
    }
    for (void *p : m->allocs) {
        if (m->arena) m->arena->release(p);
        else (void)hipFree(p);
    }
    m->allocs.clear();
    m->cg = CGWork();
    m->sym = fe_mesh_s::SymState();
    m->step_work = nullptr;
    m->scalar_work = nullptr;
    m->wall = DevWall();
    m->rowplan = DevRowPlan();
}

fe_status mesh_commit(fe_mesh_s *m, MeshImage &I, hipStream_t stream)
{
    m->dm = I.d;
    fe_status s = FE_OK;
    for_each_array(I, m->dm, &m->status, [&](void **dst, const void *src, size_t bytes) {
        if (s != FE_OK) return;
        s = mesh_alloc(m, dst, bytes);
        if (s == FE_OK && src && bytes) {
            hipError_t e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) s = fail(m->ctx, FE_EDEVICE, "mesh upload copy: %s", hipGetErrorString(e));
        }
    });
    return s;
}

size_t cg_bytes(int64_t n, int max_iter)
{
    const int cap = std::max(max_iter + 2, 256);
    return 6 * DevArena::round((size_t)n * sizeof(double)) + DevArena::round(kPartDoubles * sizeof(double)) +
           DevArena::round(4 * sizeof(int32_t)) + DevArena::round((4 * (size_t)cap + 4) * sizeof(double));
}

fe_status ensure_cg(fe_mesh_s *m, int max_iter, bool mixed)
{
    CGWork &w = m->cg;
    const int64_t n = m->dm.N;
    fe_status s;
    if (!w.r) {
        size_t vb = (size_t)n * sizeof(double);
        double **v[] = {&w.r, &w.z, &w.p, &w.q, &w.dinv, &w.d64};
        for (double **pp : v) {
            if ((s = mesh_alloc(m, (void **)pp, vb)) != FE_OK) return s;
            w.bytes += vb;
        }
        if ((s = mesh_alloc(m, (void **)&w.part, kPartDoubles * sizeof(double))) != FE_OK) return s;
        if ((s = mesh_alloc(m, (void **)&w.flags, 4 * sizeof(int32_t))) != FE_OK) return s;
        w.n = n;
    }
    if (w.hist_cap < max_iter + 2) {
        mesh_free_ptr(m, w.hist);
        w.hist = nullptr;
        w.hist_cap = std::max(max_iter + 2, 256);
        if ((s = mesh_alloc(m, (void **)&w.hist, (4 * (size_t)w.hist_cap + 4) * sizeof(double))) != FE_OK)
            return s;
    }
    if (mixed && !w.r32) {
        size_t vb = (size_t)n * sizeof(float);
        float **v[] = {&w.r32, &w.z32, &w.p32, &w.q32, &w.x32, &w.dinv32};
        for (float **pp : v) {
            if ((s = mesh_alloc(m, (void **)pp, vb)) != FE_OK) return s;
            w.bytes += vb;
        }
    }
    if (mixed && w.v32_cap < m->dm.nnz) {
        mesh_free_ptr(m, w.v32);
        w.v32 = nullptr;
        // padded like the column indices (the SpMV reads groups of 4)
        if ((s = mesh_alloc(m, (void **)&w.v32, ((size_t)m->dm.nnz + kColPad) * sizeof(float))) != FE_OK) return s;
        w.v32_cap = m->dm.nnz;
        w.bytes += (size_t)m->dm.nnz * sizeof(float);
    }
    return FE_OK;
}

fe_status assemble_queue(fe_mesh_s *m, const fe_fields *f, fe_precision prec, double *values, double *rhs,
                         hipStream_t stream)
{
    fe_ctx_s *c = m->ctx;
    const DevMesh &d = m->dm;
    AsmArgs a{};
    a.m = &d;
    a.op = f->op;
    a.dt = f->dt;
    a.u = f->u;
    a.rho = f->rho;
    a.mu = f->mu;
    a.status = m->status;
    const int passes = f->op == FE_OP_SCALAR ? f->n_scalars : 1;
    for (int k = 0; k < passes; ++k) {
        a.values = values + (int64_t)k * d.nnz;
        a.rhs = rhs + (int64_t)k * d.N;
        if (f->op == FE_OP_SCALAR) {
            a.Y = f->Y + (int64_t)k * d.N;
            a.Dk = f->D[k];
        }
        HIPCALL(c, launch_assemble(a, prec == FE_MIXED, stream));
    }
    return FE_OK;
}

}  // namespace feasm

namespace {

hipEvent_t prof_event(fe_ctx_s *c, int slot)
{
    ProfSlot &p = c->prof[slot];
    if (p.used == p.ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p.ev.push_back(e);
    }
    return p.ev[p.used++];
}

struct ProfScope {
    fe_ctx_s *c;
    int slot;
    ProfScope(fe_ctx_s *c_, int s_) : c(c_), slot(s_)
    {
        if (c->profiling) {
            hipEvent_t e = prof_event(c, slot);
            if (e) (void)hipEventRecord(e, c->stream);   // a failed bracket only loses a timing
        }
    }
    ~ProfScope()
    {
        if (c->profiling) {
            hipEvent_t e = prof_event(c, slot);
            if (e) (void)hipEventRecord(e, c->stream);
        }
    }
};

fe_status sync(fe_ctx_s *c)
{
    HIPCALL(c, hipStreamSynchronize(c->stream));
    return FE_OK;
}

// Reads the status word of the assembly launches queued last (synchronises)
// and reports the first element with det J <= 0 by its user id.
// Interprets a status word read back to the host.
static fe_status check_asm_status(fe_mesh_s *m, const AsmStatus *hs, fe_asm_info *info)
{
    fe_ctx_s *c = m->ctx;
    double md;
    memcpy(&md, &hs->min_det_key, 8);
    long long bad = hs->first_bad;
    if (bad >= (long long)m->elem_perm.size())
        return fail(c, FE_EDEVICE, "assembly status names element %lld of %zu", bad, m->elem_perm.size());
    if (info) {
        info->min_detJ = md;
        info->first_bad_elem = bad >= 0 ? m->elem_perm[bad] : -1;
    }
    if (bad >= 0) return fail(c, FE_EBADELEM, "det J <= 0 in element %d (user id)", m->elem_perm[bad]);
    return FE_OK;
}

fe_status read_asm_status(fe_mesh_s *m, fe_asm_info *info)
{
    fe_ctx_s *c = m->ctx;
    AsmStatus *hs = (AsmStatus *)c->host;
    HIPCALL(c, hipMemcpyAsync(hs, m->status, sizeof(AsmStatus), hipMemcpyDeviceToHost, c->stream));
    fe_status s = sync(c);
    if (s != FE_OK) return s;
    return check_asm_status(m, hs, info);
}

// Queues one element-vector pass (kOpResidual, kOpGradient, kOpDivergence)
// writing its rows of N to out, and checks its status word; with defer set,
// the status word goes to *defer (device memory) unread, for the caller to
// read back with the others of a sequence (one synchronisation).
fe_status element_vectors(fe_mesh_s *m, int op, double dt, const double *u, const double *rho, const double *mu,
                          const double *p, double *out, int form = 0, const double *Y = nullptr, double D = 0.0,
                          AsmStatus *defer = nullptr)
{
    fe_ctx_s *c = m->ctx;
    AsmArgs a{};
    a.m = &m->dm;
    a.op = op;
    a.dt = dt;
    a.u = u;
    a.rho = rho;
    a.mu = mu;
    a.p = p;
    a.Y = Y;
    a.Dk = D;
    a.form = form;
    a.rhs = out;
    a.status = m->status;
    a.status_out = defer;
    {
        ProfScope ps(c, 4);
        HIPCALL(c, launch_assemble(a, false, c->stream));
    }
    return defer ? FE_OK : read_asm_status(m, nullptr);
}

// Iterations recorded per PCG graph.  A graph replays them with no launch
// argument depending on the iteration (the kernels keep the iteration index
// on the device), so one recording serves every run of the same system.
constexpr int kGraphIters = 8;

template <class T>
fe_status pcg_graph_launch(fe_mesh_s *m, const T *vals, T *x)
{
    fe_ctx_s *c = m->ctx;
    fe_mesh_s::PcgGraph &g = m->graph[sizeof(T) == 4 ? 1 : 0];
    const void *sym = sizeof(T) == 8 ? (const void *)m->cg.sym.vals : nullptr;
    if (!(g.exec && g.vals == vals && g.x == x && g.hist == m->cg.hist && g.sym == sym)) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = fe_mesh_s::PcgGraph();
        hipGraph_t graph = nullptr;
        HIPCALL(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < kGraphIters && e == hipSuccess; ++i) {
            e = cg_spmv_pq<T>(m->dm, vals, m->cg, 0, c->cap_stream);
            if (e == hipSuccess) e = cg_updates<T>(m->dm, x, m->cg, 0, c->cap_stream);
        }
        const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g = fe_mesh_s::PcgGraph();
            return fail(c, FE_EDEVICE, "recording the PCG graph: %s", hipGetErrorString(e));
        }
        g.vals = vals;
        g.x = x;
        g.hist = m->cg.hist;
        g.sym = sym;
    }
    HIPCALL(c, hipGraphLaunch(g.exec, c->stream));
    return FE_OK;
}

// Run FP64 or FP32 PCG iterations until the device flag says done or
// max_iter is reached.  Returns the flags word (done, status, iterations).
// Unless the context is profiling (which brackets single launches with
// events), runs of kGraphIters iterations go through a recorded graph; the
// stop flag is polled on a growing schedule as before.
// w: the mesh's work buffers (m->cg), or another set of the same sizes when
// recorded graphs are off (allow_graphs = false: every launch is eager).
template <class T>
fe_status run_pcg(fe_mesh_s *m, CGWork &w, const T *vals, const T *b, T *x, double rtol, int max_iter, bool x_zero,
                  int32_t flags_out[4], bool allow_graphs = true)
{
    fe_ctx_s *c = m->ctx;
    HIPCALL(c, cg_setup<T>(m->dm, vals, b, x, w, rtol, c->stream, x_zero));
    const bool graphs = allow_graphs && !c->profiling && c->cap_stream != nullptr;
    int k = 0;
    int next_poll = 8;
    int32_t *hf = (int32_t *)c->host;
    while (k < max_iter) {
        if (graphs && k + kGraphIters <= max_iter && (rtol <= 0.0 || k + kGraphIters <= next_poll)) {
            fe_status s = pcg_graph_launch<T>(m, vals, x);
            if (s != FE_OK) return s;
            k += kGraphIters;
        } else {
            {
                ProfScope ps(c, 0);
                HIPCALL(c, cg_spmv_pq<T>(m->dm, vals, w, k, c->stream));
            }
            {
                ProfScope ps(c, 2);
                HIPCALL(c, cg_updates<T>(m->dm, x, w, k, c->stream));
            }
            ++k;
        }
        if (rtol > 0.0 && (k == next_poll || k == max_iter)) {
            HIPCALL(c, hipMemcpyAsync(hf, w.flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            fe_status s = sync(c);
            if (s != FE_OK) return s;
            if (hf[0]) break;
            next_poll = k + std::max(8, k / 4);
            if (graphs) next_poll = (next_poll + kGraphIters - 1) / kGraphIters * kGraphIters;
        }
    }
    HIPCALL(c, hipMemcpyAsync(hf, w.flags, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    fe_status s = sync(c);
    if (s != FE_OK) return s;
    memcpy(flags_out, hf, 4 * sizeof(int32_t));
    return FE_OK;
}

// The symmetric SpMV map of the mesh's pattern, built on the host from the
// device pattern and uploaded on first use.  A pattern without one (not
// structurally symmetric), or a device without room for it, leaves state -1:
// the mesh's solves use the general SpMV.
static fe_status ensure_sym(fe_mesh_s *m)
{
    fe_mesh_s::SymState &Y = m->sym;
    if (Y.state != 0) return FE_OK;
    fe_ctx_s *c = m->ctx;
    const DevMesh &d = m->dm;
    std::vector<int32_t> rp(d.N + 1), ci(d.nnz);
    HIPCALL(c, hipMemcpy(rp.data(), d.rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCALL(c, hipMemcpy(ci.data(), d.colidx, ci.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    SymMap S;
    std::string err;
    if (build_sym_map(d.N, rp.data(), ci.data(), S, err) != 0) {
        Y.state = -1;
        return FE_OK;
    }
    fe_mesh_s::SymState N;
    fe_status s = FE_OK;
    auto up = [&](void **dst, const void *src, size_t bytes) {
        if (s != FE_OK) return;
        if ((s = mesh_alloc(m, dst, bytes)) != FE_OK) return;
        const hipError_t e = src && bytes ? hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice)
                                          : hipMemset(*dst, 0, bytes);
        if (e != hipSuccess) s = fail(c, FE_EDEVICE, "symmetric SpMV map upload: %s", hipGetErrorString(e));
    };
    void *desc = nullptr, *roff = nullptr, *lidx = nullptr, *mir = nullptr, *cols = nullptr, *vals = nullptr;
    up(&desc, S.desc.data(), S.desc.size() * sizeof(int32_t));
    up(&roff, S.roff.data(), S.roff.size() * sizeof(uint32_t));
    up(&lidx, S.lidx.data(), S.lidx.size());
    up(&mir, S.mir.data(), S.mir.size() * sizeof(uint32_t));
    up(&cols, S.cols.data(), std::max<size_t>(S.cols.size(), 1) * sizeof(int32_t));
    up((void **)&N.mstart, S.mstart.data(), std::max<size_t>(S.mstart.size(), 1));
    up(&vals, nullptr, ((size_t)S.n_packed + 4) * sizeof(double));   // zeros: the padding stays 0
    up((void **)&N.bad, nullptr, sizeof(int32_t));
    if (s != FE_OK) {
        void *ps[] = {desc, roff, lidx, mir, cols, N.mstart, vals, N.bad};
        for (void *q : ps) mesh_free_ptr(m, q);
        if (s != FE_ENOMEM) return s;
        Y.state = -1;   // no room for the map: this mesh's solves use the general SpMV
        return FE_OK;
    }
    N.map.desc = (const int4 *)desc;
    N.map.roff = (const uint32_t *)roff;
    N.map.lidx = (const uint8_t *)lidx;
    N.map.mir = (const uint32_t *)mir;
    N.map.cols = (const int32_t *)cols;
    N.map.vals = (const double *)vals;
    N.map.nrb = S.nrb;
    N.map.nt = spmv_map(d).nt;
    N.n_packed = S.n_packed;
    N.state = 1;
    Y = N;
    return FE_OK;
}

// Chooses the SpMV of an FP64 solve of `values` on w: the symmetric one when
// the mesh has its map and every mirrored pair of values agrees (see
// launch_sym_pack; the packed copy then holds the stored entry of each
// pair), else the general one.  Synchronises the stream.
static fe_status select_sym(fe_mesh_s *m, CGWork &w, const double *values)
{
    fe_ctx_s *c = m->ctx;
    w.sym = SymSpmv();
    fe_status s = ensure_sym(m);
    if (s != FE_OK || m->sym.state != 1) return s;
    fe_mesh_s::SymState &Y = m->sym;
    HIPCALL(c, launch_sym_pack(m->dm, Y.map, Y.mstart, values, const_cast<double *>(Y.map.vals), Y.bad, c->stream));
    int32_t *hf = (int32_t *)c->host;
    HIPCALL(c, hipMemcpyAsync(hf, Y.bad, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    if ((s = sync(c)) != FE_OK) return s;
    if (hf[0] == 0) w.sym = Y.map;
    return FE_OK;
}

// FP64 Jacobi-PCG on the work buffers w: fills the iteration count and the
// recursive residual of inf, and the outcome of the solve in result
// (FE_OK, FE_ENOCONV or FE_EBREAKDOWN).  use_sym: run the symmetric SpMV
// when the matrix allows it (select_sym), else the general one.
fe_status pcg_fp64(fe_mesh_s *m, CGWork &w, const double *values, const double *rhs, double *x, double rtol,
                   int max_iter, bool allow_graphs, fe_cg_info &inf, fe_status &result, bool use_sym)
{
    fe_ctx_s *c = m->ctx;
    int32_t fl[4];
    fe_status s = use_sym ? select_sym(m, w, values) : FE_OK;
    if (s != FE_OK) return s;
    s = run_pcg<double>(m, w, values, rhs, x, rtol, max_iter, false, fl, allow_graphs);
    inf.symmetric_spmv = w.sym.vals ? 1 : 0;
    w.sym = SymSpmv();
    if (s != FE_OK) return s;
    const int it = fl[2];
    double hv[2];
    HIPCALL(c, hipMemcpy(hv, w.hist + 4 * (size_t)it, 2 * sizeof(double), hipMemcpyDeviceToHost));
    double bb;
    HIPCALL(c, hipMemcpy(&bb, w.hist + 4 * (size_t)w.hist_cap, sizeof(double), hipMemcpyDeviceToHost));
    inf.iterations = it;
    inf.outer_iterations = 1;
    inf.rel_residual = bb > 0 ? std::sqrt(hv[1] / bb) : std::sqrt(hv[1]);
    if (fl[1] == FE_EBREAKDOWN) result = FE_EBREAKDOWN;
    else if (rtol > 0.0 && !fl[0]) result = FE_ENOCONV;
    return FE_OK;
}

// The true residual ||b - A x|| / ||b|| in FP64 (w.d64 and w.part as work),
// then the solve's status and info.
fe_status pcg_finish(fe_mesh_s *m, CGWork &w, const double *values, const double *rhs, const double *x, int max_iter,
                     fe_cg_info &inf, fe_status result, fe_cg_info *info)
{
    fe_ctx_s *c = m->ctx;
    HIPCALL(c, residual_f64(m->dm, values, rhs, x, w.d64, w.part, c->scratch + 2048, c->stream));
    HIPCALL(c, hipMemcpyAsync(c->host, c->scratch + 2048, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    fe_status s = sync(c);
    if (s != FE_OK) return s;
    inf.true_rel_residual = c->host[1] > 0 ? std::sqrt(c->host[0] / c->host[1]) : std::sqrt(c->host[0]);
    if (info) *info = inf;
    if (result == FE_EBREAKDOWN) return fail(c, FE_EBREAKDOWN, "CG breakdown (p.Ap <= 0 or non-finite)");
    if (result == FE_ENOCONV) return fail(c, FE_ENOCONV, "CG did not reach rtol in %d iterations", max_iter);
    return FE_OK;
}

// ---- allocation-free PCG: work buffers in a fixed device area -----------------
// The area is one file-scope device array.  In host code its name stands for
// the host-side shadow, not a device address: the device address of each
// device's copy is looked up once per device (fe_ctx_create) and kept in
// g_scratch_dev; only that pointer is passed to kernels.
constexpr size_t kNoAllocBytes = FE_NOALLOC_BYTES;
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kNoAllocMaxDevices] = {};

// Looks up this device's copy of the area (the device must be current).
hipError_t noalloc_init(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = (char *)p;
    return hipSuccess;
}

// Carves the PCG work buffers for n unknowns and max_iter iterations out of
// the area at base: r, z, p, q, dinv, d64, the partial sums, the stop word
// and the per-iteration scalars.  Returns the bytes used (base may be null
// to only count them).
size_t noalloc_layout(char *base, int64_t n, int max_iter, CGWork &w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += DevArena::round(bytes);
        return p;
    };
    w = CGWork();
    w.n = n;
    double **v[] = {&w.r, &w.z, &w.p, &w.q, &w.dinv, &w.d64};
    for (double **pp : v) *pp = (double *)take((size_t)n * sizeof(double));
    w.part = (double *)take(kPartDoubles * sizeof(double));
    w.flags = (int32_t *)take(4 * sizeof(int32_t));
    w.hist_cap = std::max(max_iter + 2, 256);
    w.hist = (double *)take((4 * (size_t)w.hist_cap + 4) * sizeof(double));
    return off;
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" {

fe_status fe_ctx_create(int device, void *hip_stream, fe_ctx *out)
{
    if (!out) return FE_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FE_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return FE_EDEVICE;
    if (init_spmv_grid(device) != hipSuccess) return FE_EDEVICE;
    if (noalloc_init(device) != hipSuccess) return FE_EDEVICE;
    auto *c = new fe_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipMalloc((void **)&c->scratch, (2048 + 64) * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&c->host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        if (c->scratch) (void)hipFree(c->scratch);
        delete c;
        return FE_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) c->cap_stream = nullptr;
    *out = c;
    return FE_OK;
}

void fe_ctx_destroy(fe_ctx c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->scratch) (void)hipFree(c->scratch);
    if (c->host) (void)hipHostFree(c->host);
    while (!c->meshes.empty()) fe_mesh_free(c->meshes.back());
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &p : c->prof)
        for (auto e : p.ev) (void)hipEventDestroy(e);
    delete c;
}

const char *fe_ctx_last_error(fe_ctx c) { return c ? c->err.c_str() : "null context"; }

fe_status fe_ctx_set_stream(fe_ctx c, void *hip_stream)
{
    if (!c) return FE_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return FE_OK;
}

static fe_status mesh_upload(fe_ctx c, int stride, const uint8_t *types, int64_t n_nodes, const double *coords,
                             int64_t n_elems, const int32_t *conn, int64_t n_dirichlet,
                             const int32_t *dirichlet_nodes, uint32_t flags, fe_mesh *out)
{
    if (!c || !out) return FE_EINVAL;
    *out = nullptr;
    RoctxRange rr("fe_mesh_upload");
    HIPCALL(c, hipSetDevice(c->device));
    auto img = std::make_unique<MeshImage>();
    std::string err;
    int st = mesh_prepare(stride, types, n_nodes, coords, n_elems, conn, n_dirichlet, dirichlet_nodes,
                          (flags & FE_UPLOAD_RENUMBER) != 0, *img, err, (flags & FE_UPLOAD_COLOURED) == 0);
    if (st != FE_OK) return fail(c, (fe_status)st, "%s", err.c_str());
    auto *m = new fe_mesh_s();
    m->ctx = c;
    fe_status s = mesh_commit(m, *img, c->stream);
    if (s == FE_OK && hipStreamSynchronize(c->stream) != hipSuccess) s = fail(c, FE_EDEVICE, "upload sync failed");
    if (s != FE_OK) {
        (void)hipStreamSynchronize(c->stream);
        mesh_release(m);
        delete m;
        return s;
    }
    m->node_perm = std::move(img->P.node_perm);
    m->elem_perm = std::move(img->P.elem_perm);
    m->conn_m = std::move(img->P.conn);
    m->etype_m = std::move(img->P.etype);
    m->stride_m = img->P.nen;
    if (flags & FE_UPLOAD_GENERAL_SPMV) m->sym.state = -1;   // never build the symmetric map
    c->meshes.push_back(m);
    *out = m;
    return FE_OK;
}

fe_status fe_mesh_upload(fe_ctx c, fe_elem_type type, int64_t n_nodes, const double *coords, int64_t n_elems,
                         const int32_t *conn, int64_t n_dirichlet, const int32_t *dirichlet_nodes, uint32_t flags,
                         fe_mesh *out)
{
    return mesh_upload(c, (int)type, nullptr, n_nodes, coords, n_elems, conn, n_dirichlet, dirichlet_nodes, flags,
                       out);
}

fe_status fe_mesh_upload_mixed(fe_ctx c, int64_t n_nodes, const double *coords, int64_t n_elems,
                               const uint8_t *elem_types, const int32_t *conn, int64_t n_dirichlet,
                               const int32_t *dirichlet_nodes, uint32_t flags, fe_mesh *out)
{
    if (!elem_types) return c ? fail(c, FE_EINVAL, "elem_types is NULL") : FE_EINVAL;
    return mesh_upload(c, 8, elem_types, n_nodes, coords, n_elems, conn, n_dirichlet, dirichlet_nodes, flags,
                       out);
}

fe_status fe_mesh_info(fe_mesh m, fe_mesh_desc *o)
{
    if (!m || !o) return FE_EINVAL;
    const DevMesh &d = m->dm;
    o->nen = d.nen;
    o->n_nodes = d.N;
    o->n_elems = d.E;
    o->nnz = d.nnz;
    o->rowptr = d.rowptr;
    o->colidx = d.colidx;
    o->n_blocks = d.nblk;
    o->n_colors = d.n_colors;
    o->max_row = d.max_row;
    o->n_dirichlet = d.n_dir;
    o->device_bytes = m->bytes + m->cg.bytes;
    return FE_OK;
}

fe_status fe_mesh_perm(fe_mesh m, int32_t *node_perm, int32_t *elem_perm)
{
    if (!m) return FE_EINVAL;
    if (node_perm) memcpy(node_perm, m->node_perm.data(), m->node_perm.size() * sizeof(int32_t));
    if (elem_perm) memcpy(elem_perm, m->elem_perm.data(), m->elem_perm.size() * sizeof(int32_t));
    return FE_OK;
}

fe_status fe_mesh_pattern_host(fe_mesh m, int32_t *rowptr, int32_t *colidx)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (rowptr)
        HIPCALL(c, hipMemcpyAsync(rowptr, m->dm.rowptr, (m->dm.N + 1) * sizeof(int32_t), hipMemcpyDeviceToHost,
                                  c->stream));
    if (colidx)
        HIPCALL(c, hipMemcpyAsync(colidx, m->dm.colidx, m->dm.nnz * sizeof(int32_t), hipMemcpyDeviceToHost,
                                  c->stream));
    return sync(c);
}

fe_status fe_mesh_to_mesh_order(fe_mesh m, const double *in, double *out, int32_t ncomp)
{
    if (!m || !in || !out || ncomp < 1 || in == out) return m ? fail(m->ctx, FE_EINVAL, "bad permute args") : FE_EINVAL;
    HIPCALL(m->ctx, launch_permute(m->dm.N, ncomp, m->dm.node_perm, in, out, true, m->ctx->stream));
    return FE_OK;
}

fe_status fe_mesh_to_user_order(fe_mesh m, const double *in, double *out, int32_t ncomp)
{
    if (!m || !in || !out || ncomp < 1 || in == out) return m ? fail(m->ctx, FE_EINVAL, "bad permute args") : FE_EINVAL;
    HIPCALL(m->ctx, launch_permute(m->dm.N, ncomp, m->dm.node_perm, in, out, false, m->ctx->stream));
    return FE_OK;
}

void fe_mesh_free(fe_mesh m)
{
    if (!m) return;
    auto &v = m->ctx->meshes;
    v.erase(std::remove(v.begin(), v.end(), m), v.end());
    (void)hipStreamSynchronize(m->ctx->stream);
    mesh_release(m);
    delete m;
}

fe_status fe_assemble(fe_mesh m, const fe_fields *f, fe_precision prec, double *values, double *rhs,
                      fe_asm_info *info)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (!f || !values || !rhs) return fail(c, FE_EINVAL, "null fields/values/rhs");
    if (prec != FE_FP64 && prec != FE_MIXED) return fail(c, FE_EINVAL, "bad precision %d", (int)prec);
    if (!(f->dt > 0.0) || !std::isfinite(f->dt)) return fail(c, FE_EINVAL, "dt must be > 0");
    if (!f->u || !f->rho) return fail(c, FE_EINVAL, "u and rho are required");
    if (f->op == FE_OP_MOMENTUM && !f->mu) return fail(c, FE_EINVAL, "MOMENTUM needs mu");
    if (f->op == FE_OP_SCALAR && (f->n_scalars < 1 || f->n_scalars > 8 || !f->Y || !f->D))
        return fail(c, FE_EINVAL, "SCALAR needs 1..8 scalars, Y and D");
    if (f->op != FE_OP_MOMENTUM && f->op != FE_OP_SCALAR && f->op != FE_OP_POISSON)
        return fail(c, FE_EINVAL, "bad operator %d", (int)f->op);
    RoctxRange rr("fe_assemble");
    HIPCALL(c, hipSetDevice(c->device));
    {
        ProfScope ps(c, 1);
        fe_status s = assemble_queue(m, f, prec, values, rhs, c->stream);
        if (s != FE_OK) return s;
    }
    return read_asm_status(m, info);
}

// Builds and uploads the row-owner plan of the block operator (first use).
static fe_status ensure_rowplan(fe_mesh_s *m)
{
    fe_ctx_s *c = m->ctx;
    DevRowPlan &D = m->rowplan;
    if (D.n_waves > 0) return FE_OK;
    if (m->conn_m.empty()) return fail(c, FE_EINVAL, "the mesh keeps no connectivity for the block operator");
    const DevMesh &d = m->dm;
    std::vector<int32_t> rp(d.N + 1), ci(d.nnz);
    HIPCALL(c, hipMemcpy(rp.data(), d.rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCALL(c, hipMemcpy(ci.data(), d.colidx, ci.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    RowPlan R;
    std::string err;
    const uint8_t *et = m->etype_m.empty() ? nullptr : m->etype_m.data();
    int st = build_row_plan(m->stride_m, et, d.N, d.E, m->conn_m.data(), rp.data(), ci.data(), R, err);
    if (st != FE_OK) return fail(c, (fe_status)st, "%s", err.c_str());
    DevRowPlan P;
    P.n_tasks = R.n_tasks;
    P.n_waves = (int64_t)R.wdesc.size();
    P.max_img = R.max_img;
    P.stride = m->stride_m;
    fe_status s = FE_OK;
    auto up = [&](void **dst, const void *src, size_t bytes) {
        if (s != FE_OK) return;
        if ((s = mesh_alloc(m, dst, bytes)) != FE_OK) return;
        if (src && bytes) {
            const hipError_t e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) s = fail(c, FE_EDEVICE, "block plan upload: %s", hipGetErrorString(e));
        }
    };
    up((void **)&P.conn, m->conn_m.data(), m->conn_m.size() * sizeof(int32_t));
    if (et) up((void **)&P.etype, et, m->etype_m.size());
    up((void **)&P.task_elem, R.task_elem.data(), R.task_elem.size() * sizeof(int32_t));
    up((void **)&P.task_meta, R.task_meta.data(), R.task_meta.size() * sizeof(uint16_t));
    up((void **)&P.task_cols, R.task_cols.data(), R.task_cols.size());
    up((void **)&P.wdesc, R.wdesc.data(), R.wdesc.size() * sizeof(RowWave));
    up((void **)&P.w_mindet, nullptr, (size_t)P.n_waves * sizeof(double));
    up((void **)&P.w_bad, nullptr, (size_t)P.n_waves * sizeof(long long));
    if (s != FE_OK) {
        void *ps[] = {P.conn, P.etype, P.task_elem, P.task_meta, P.task_cols, P.wdesc, P.w_mindet, P.w_bad};
        for (void *q : ps) mesh_free_ptr(m, q);
        return s;
    }
    D = P;
    return FE_OK;
}

fe_status fe_assemble_block(fe_mesh m, uint32_t form, double dt, const double *u, const double *rho,
                            const double *mu, double *values, double *rhs, fe_asm_info *info)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (!u || !rho || !mu || !values || !rhs) return fail(c, FE_EINVAL, "null u/rho/mu/values/rhs");
    if (form & ~(uint32_t)(FE_FORM_FULL_STRESS | FE_FORM_EMAC))
        return fail(c, FE_EINVAL, "unknown form bits 0x%x", form);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, FE_EINVAL, "dt must be > 0");
    RoctxRange rr("fe_assemble_block");
    HIPCALL(c, hipSetDevice(c->device));
    fe_status s = ensure_rowplan(m);
    if (s != FE_OK) return s;
    {
        ProfScope ps(c, 1);
        HIPCALL(c, launch_assemble_block(m->dm, m->rowplan, (int)form, dt, u, rho, mu, values, rhs, m->status,
                                         c->stream));
    }
    return read_asm_status(m, info);
}

fe_status fe_apply_dirichlet(fe_mesh m, double *values, double *rhs, const double *g)
{
    if (!m) return FE_EINVAL;
    if (!values || !rhs) return fail(m->ctx, FE_EINVAL, "null values/rhs");
    RoctxRange rr("fe_apply_dirichlet");
    ProfScope ps(m->ctx, 3);
    HIPCALL(m->ctx, launch_dirichlet(m->dm, values, rhs, g, m->ctx->stream));
    return FE_OK;
}

fe_status fe_spmv(fe_mesh m, const double *values, const double *x, double *y)
{
    if (!m) return FE_EINVAL;
    if (!values || !x || !y || x == y) return fail(m->ctx, FE_EINVAL, "bad spmv args");
    HIPCALL(m->ctx, launch_spmv(m->dm, values, x, y, m->ctx->stream));
    return FE_OK;
}

fe_status fe_dot(fe_ctx c, int64_t n, const double *x, const double *y, double *out)
{
    if (!c) return FE_EINVAL;
    if (n < 0 || !out || (n > 0 && (!x || !y))) return fail(c, FE_EINVAL, "bad dot args");
    if (n == 0) {
        *out = 0.0;
        return FE_OK;
    }
    HIPCALL(c, launch_dot(n, x, y, c->scratch, c->scratch + 2048, c->stream));
    HIPCALL(c, hipMemcpyAsync(c->host, c->scratch + 2048, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    fe_status s = sync(c);
    if (s != FE_OK) return s;
    *out = c->host[0];
    return FE_OK;
}

fe_status fe_axpy(fe_ctx c, int64_t n, double a, const double *x, double *y)
{
    if (!c) return FE_EINVAL;
    if (n < 0 || (n > 0 && (!x || !y))) return fail(c, FE_EINVAL, "bad axpy args");
    if (n == 0) return FE_OK;
    HIPCALL(c, launch_axpy(n, a, x, y, c->stream));
    return FE_OK;
}

fe_status fe_cg_solve(fe_mesh m, const double *values, const double *rhs, double *x, double rtol, int32_t max_iter,
                      fe_precision prec, fe_cg_info *info)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (!values || !rhs || !x) return fail(c, FE_EINVAL, "null values/rhs/x");
    if (max_iter < 0) return fail(c, FE_EINVAL, "max_iter < 0");
    if (prec != FE_FP64 && prec != FE_MIXED) return fail(c, FE_EINVAL, "bad precision");
    if (!std::isfinite(rtol)) return fail(c, FE_EINVAL, "rtol not finite");
    RoctxRange rr(prec == FE_MIXED ? "fe_cg_solve(mixed)" : "fe_cg_solve");
    HIPCALL(c, hipSetDevice(c->device));
    fe_status s = ensure_cg(m, max_iter, prec == FE_MIXED);
    if (s != FE_OK) return s;
    CGWork &w = m->cg;
    const DevMesh &d = m->dm;
    fe_cg_info inf{};
    fe_status result = FE_OK;
    if (prec == FE_FP64) {
        if ((s = pcg_fp64(m, w, values, rhs, x, rtol, max_iter, true, inf, result, true)) != FE_OK) return s;
    } else {
        HIPCALL(c, cast_f64_f32(d.nnz, values, w.v32, c->stream));
        int used = 0, outer = 0;
        double rel = 0.0;
        result = FE_ENOCONV;
        for (outer = 0; outer < 64; ++outer) {
            HIPCALL(c, residual_f64(d, values, rhs, x, w.d64, w.part, c->scratch + 2048, c->stream));
            HIPCALL(c, hipMemcpyAsync(c->host, c->scratch + 2048, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                      c->stream));
            if ((s = sync(c)) != FE_OK) return s;
            const double rr = c->host[0], bb = c->host[1];
            rel = bb > 0 ? std::sqrt(rr / bb) : std::sqrt(rr);
            if (!std::isfinite(rel)) {
                result = FE_EBREAKDOWN;
                break;
            }
            if (rtol > 0.0 ? rel <= rtol : used >= max_iter) {
                result = FE_OK;
                break;
            }
            if (used >= max_iter || rr == 0.0) break;
            const double rn = std::sqrt(rr);
            const double need = rtol > 0.0 ? rtol * std::sqrt(bb) / rn : 0.0;
            const double tol_in = std::max(0.5 * need, 1e-5);
            HIPCALL(c, scale_f64_to_f32(d.N, 1.0 / rn, w.d64, w.r32, c->stream));
            int32_t fl[4];
            s = run_pcg<float>(m, m->cg, w.v32, w.r32, w.x32, tol_in, max_iter - used, true, fl);
            if (s != FE_OK) return s;
            used += fl[2];
            HIPCALL(c, add_f32_to_f64(d.N, rn, w.x32, x, c->stream));
            if (fl[2] == 0) break;   // no progress possible (e.g. immediate breakdown)
        }
        inf.iterations = used;
        inf.outer_iterations = outer + (result == FE_OK ? 0 : 1);
        inf.rel_residual = rel;
    }
    return pcg_finish(m, w, values, rhs, x, max_iter, inf, result, info);
}

fe_status fe_cg_solve_noalloc(fe_mesh m, const double *values, const double *rhs, double *x, double rtol,
                              int32_t max_iter, fe_cg_info *info)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (!values || !rhs || !x) return fail(c, FE_EINVAL, "null values/rhs/x");
    if (max_iter < 0) return fail(c, FE_EINVAL, "max_iter < 0");
    if (!std::isfinite(rtol)) return fail(c, FE_EINVAL, "rtol not finite");
    RoctxRange rr("fe_cg_solve_noalloc");
    HIPCALL(c, hipSetDevice(c->device));
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (c->device >= 0 && c->device < kNoAllocMaxDevices) base = g_scratch_dev[c->device];
    }
    if (!base) return fail(c, FE_EDEVICE, "the fixed PCG work area of device %d was not set up", c->device);
    CGWork w;
    const size_t need = noalloc_layout(nullptr, m->dm.N, max_iter, w);
    if (need > kNoAllocBytes)
        return fail(c, FE_ENOMEM,
                    "fe_cg_solve_noalloc: %lld nodes and %d iterations need %zu bytes of work area, the fixed area "
                    "holds %zu (FE_NOALLOC_BYTES)",
                    (long long)m->dm.N, max_iter, need, kNoAllocBytes);
    noalloc_layout(base, m->dm.N, max_iter, w);
    fe_cg_info inf{};
    fe_status result = FE_OK;
    fe_status s = pcg_fp64(m, w, values, rhs, x, rtol, max_iter, false, inf, result, false);
    if (s != FE_OK) return s;
    return pcg_finish(m, w, values, rhs, x, max_iter, inf, result, info);
}

// ---- explicit step ----------------------------------------------------------

static bool valid_form(uint32_t form) { return (form & ~(uint32_t)(FE_FORM_FULL_STRESS | FE_FORM_EMAC)) == 0; }

fe_status fe_residual(fe_mesh m, const double *u, const double *rho, const double *mu, uint32_t form, double *out)
{
    if (!m) return FE_EINVAL;
    if (!u || !rho || !mu || !out) return fail(m->ctx, FE_EINVAL, "null u/rho/mu/out");
    if (!valid_form(form)) return fail(m->ctx, FE_EINVAL, "unknown form bits 0x%x", form);
    HIPCALL(m->ctx, hipSetDevice(m->ctx->device));
    return element_vectors(m, kOpResidual, 1.0, u, rho, mu, nullptr, out, (int)form);
}

fe_status fe_gradient(fe_mesh m, const double *p, double *g)
{
    if (!m) return FE_EINVAL;
    if (!p || !g) return fail(m->ctx, FE_EINVAL, "null p/g");
    HIPCALL(m->ctx, hipSetDevice(m->ctx->device));
    return element_vectors(m, kOpGradient, 1.0, nullptr, nullptr, nullptr, p, g);
}

fe_status fe_divergence(fe_mesh m, double dt, const double *u, const double *rho, double *f)
{
    if (!m) return FE_EINVAL;
    if (!u || !rho || !f) return fail(m->ctx, FE_EINVAL, "null u/rho/f");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(m->ctx, FE_EINVAL, "dt must be > 0");
    HIPCALL(m->ctx, hipSetDevice(m->ctx->device));
    return element_vectors(m, kOpDivergence, dt, u, rho, nullptr, nullptr, f);
}

fe_status fe_fractional_step(fe_mesh m, double dt, const double *rho, const double *mu, const double *L,
                             uint32_t form, double *u, double *p, double rtol, int32_t max_iter, fe_precision prec,
                             fe_step_info *info)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (!rho || !mu || !L || !u || !p) return fail(c, FE_EINVAL, "null rho/mu/L/u/p");
    if (!valid_form(form)) return fail(c, FE_EINVAL, "unknown form bits 0x%x", form);
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, FE_EINVAL, "dt must be > 0");
    if (!(rtol > 0.0) || max_iter < 1) return fail(c, FE_EINVAL, "need rtol > 0 and max_iter >= 1");
    RoctxRange rr("fe_fractional_step");
    HIPCALL(c, hipSetDevice(c->device));
    const DevMesh &d = m->dm;
    const int64_t N = d.N;
    fe_status s;
    // step_work: u0 [3][N], residual + mass [4][N], f [N], g [3][N], then the
    // status words of the step's 5 element-vector passes
    constexpr int kPasses = 5;
    const size_t work_doubles = 11 * (size_t)N + kPasses * sizeof(AsmStatus) / sizeof(double);
    if (!m->step_work && (s = mesh_alloc(m, (void **)&m->step_work, work_doubles * sizeof(double))) != FE_OK)
        return s;
    double *u0 = m->step_work, *res = u0 + 3 * N, *mass = res + 3 * N, *f = res + 4 * N, *g = f + N;
    AsmStatus *pass_status = (AsmStatus *)(g + 3 * N);
    // The passes' status words are read back once, at the end of the step (a
    // failed pass leaves undefined values behind it; the first failure in
    // program order is reported).  The pressure solve synchronises on its own.
    // 1. Runge-Kutta predictor (Shu-Osher SSP-RK3) on M_L du/dt = R(u)
    static const double kStage[3][2] = {{0.0, 1.0}, {0.75, 0.25}, {1.0 / 3.0, 2.0 / 3.0}};
    HIPCALL(c, hipMemcpyAsync(u0, u, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    int pass = 0;
    for (const auto &st : kStage) {
        if ((s = element_vectors(m, kOpResidual, dt, u, rho, mu, nullptr, res, (int)form, nullptr, 0.0,
                                 pass_status + pass++)) != FE_OK)
            return s;
        if (m->wall.F > 0) HIPCALL(c, launch_wall_traction(d, m->wall, u, rho, mu, res, false, c->stream));
        HIPCALL(c, launch_rk_stage(d, st[0], st[1], dt, u0, res, mass, u, c->stream));
    }
    // 2. pressure: L p = (1/dt) int grad N . (rho u*), zero at Dirichlet rows
    if ((s = element_vectors(m, kOpDivergence, dt, u, rho, nullptr, nullptr, f, 0, nullptr, 0.0,
                             pass_status + pass++)) != FE_OK)
        return s;
    HIPCALL(c, launch_zero_fixed(d, f, c->stream));
    fe_cg_info ci{};
    const fe_status cs = fe_cg_solve(m, L, f, p, rtol, max_iter, prec, &ci);
    if (info) {
        info->cg_iterations = ci.iterations;
        info->cg_true_rel_residual = ci.true_rel_residual;
    }
    // 3. correction u = u* - dt M_L^-1 G p
    if (cs == FE_OK) {
        if ((s = element_vectors(m, kOpGradient, dt, nullptr, nullptr, nullptr, p, g, 0, nullptr, 0.0,
                                 pass_status + pass++)) != FE_OK)
            return s;
        HIPCALL(c, launch_correct(d, dt, g, mass, u, c->stream));
    }
    AsmStatus *hs = (AsmStatus *)c->host;
    HIPCALL(c, hipMemcpyAsync(hs, pass_status, pass * sizeof(AsmStatus), hipMemcpyDeviceToHost, c->stream));
    if ((s = sync(c)) != FE_OK) return s;
    // program order: 3 predictor passes, the divergence, the solve, the gradient
    for (int q = 0; q < 4; ++q)
        if ((s = check_asm_status(m, hs + q, nullptr)) != FE_OK) return s;
    if (cs != FE_OK) return cs;
    return check_asm_status(m, hs + 4, nullptr);
}

fe_status fe_scalar_residual(fe_mesh m, const double *u, const double *rho, const double *Y, double D, double *out)
{
    if (!m) return FE_EINVAL;
    if (!u || !rho || !Y || !out) return fail(m->ctx, FE_EINVAL, "null u/rho/Y/out");
    if (!(D >= 0.0) || !std::isfinite(D)) return fail(m->ctx, FE_EINVAL, "D must be >= 0");
    HIPCALL(m->ctx, hipSetDevice(m->ctx->device));
    return element_vectors(m, kOpScalarResidual, 1.0, u, rho, nullptr, nullptr, out, 0, Y, D);
}

fe_status fe_scalar_step(fe_mesh m, double dt, const double *u, const double *rho, double D, double *Y)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (!u || !rho || !Y) return fail(c, FE_EINVAL, "null u/rho/Y");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, FE_EINVAL, "dt must be > 0");
    if (!(D >= 0.0) || !std::isfinite(D)) return fail(c, FE_EINVAL, "D must be >= 0");
    HIPCALL(c, hipSetDevice(c->device));
    const DevMesh &d = m->dm;
    const int64_t N = d.N;
    fe_status s;
    if (!m->scalar_work && (s = mesh_alloc(m, (void **)&m->scalar_work, 3 * (size_t)N * sizeof(double))) != FE_OK)
        return s;
    double *y0 = m->scalar_work, *res = y0 + N, *mass = res + N;
    static const double kStage[3][2] = {{0.0, 1.0}, {0.75, 0.25}, {1.0 / 3.0, 2.0 / 3.0}};
    HIPCALL(c, hipMemcpyAsync(y0, Y, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    for (const auto &st : kStage) {
        if ((s = element_vectors(m, kOpScalarResidual, dt, u, rho, nullptr, nullptr, res, 0, Y, D)) != FE_OK)
            return s;
        HIPCALL(c, launch_rk_stage(d, st[0], st[1], dt, y0, res, mass, Y, c->stream, 1));
    }
    return sync(c);
}

// ---- boundary assembly: wall model ------------------------------------------

fe_status fe_wall_faces(fe_mesh m, int64_t n_faces, const uint8_t *face_nen, const int32_t *face_conn,
                        double delta)
{
    if (!m) return FE_EINVAL;
    fe_ctx_s *c = m->ctx;
    if (n_faces < 0 || (n_faces > 0 && (!face_nen || !face_conn))) return fail(c, FE_EINVAL, "bad wall faces");
    if (n_faces > 0 && !(delta > 0.0 && std::isfinite(delta))) return fail(c, FE_EINVAL, "delta must be > 0");
    const int64_t N = m->dm.N;
    std::vector<int32_t> iperm(N);
    for (int64_t i = 0; i < N; ++i) iperm[m->node_perm[i]] = (int32_t)i;
    std::vector<int32_t> conn(4 * (size_t)n_faces);
    for (int64_t f = 0; f < n_faces; ++f) {
        const int nn = face_nen[f];
        if (nn != 3 && nn != 4) return fail(c, FE_EINVAL, "wall face %lld has %d nodes", (long long)f, nn);
        for (int a = 0; a < 4; ++a) {
            const int32_t v = face_conn[4 * f + (a < nn ? a : 0)];
            if (v < 0 || v >= N) return fail(c, FE_EINVAL, "wall face %lld: node out of range", (long long)f);
            conn[4 * f + a] = iperm[v];
        }
    }
    // wall nodes ascending; each node's (face, slot) entries by face index
    std::vector<int32_t> cnt(N + 1, 0);
    for (int64_t f = 0; f < n_faces; ++f)
        for (int a = 0; a < face_nen[f]; ++a) cnt[conn[4 * f + a] + 1]++;
    std::vector<int32_t> nodes, ptr{0};
    for (int64_t i = 0; i < N; ++i)
        if (cnt[i + 1]) {
            nodes.push_back((int32_t)i);
            ptr.push_back(ptr.back() + cnt[i + 1]);
        }
    std::vector<int32_t> first(N, -1);
    for (size_t w = 0; w < nodes.size(); ++w) first[nodes[w]] = ptr[w];
    std::vector<int32_t> ent(ptr.back());
    for (int64_t f = 0; f < n_faces; ++f)
        for (int a = 0; a < face_nen[f]; ++a) ent[first[conn[4 * f + a]]++] = (int32_t)(4 * f + a);
    HIPCALL(c, hipSetDevice(c->device));
    fe_status s = sync(c);   // work queued on the previous faces has finished
    if (s != FE_OK) return s;
    for (void *p : {(void *)m->wall.nen, (void *)m->wall.conn, (void *)m->wall.nodes, (void *)m->wall.ptr,
                    (void *)m->wall.ent, (void *)m->wall.part})
        mesh_free_ptr(m, p);
    m->wall = DevWall();
    if (n_faces == 0) return FE_OK;
    DevWall w;
    w.F = n_faces;
    w.W = (int64_t)nodes.size();
    w.delta = delta;
    auto up = [&](void **dst, const void *src, size_t bytes) -> fe_status {
        fe_status r = mesh_alloc(m, dst, bytes);
        if (r != FE_OK) return r;
        if (src) HIPCALL(c, hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, c->stream));
        return FE_OK;
    };
    if ((s = up((void **)&w.nen, face_nen, (size_t)n_faces)) != FE_OK ||
        (s = up((void **)&w.conn, conn.data(), conn.size() * 4)) != FE_OK ||
        (s = up((void **)&w.nodes, nodes.data(), nodes.size() * 4)) != FE_OK ||
        (s = up((void **)&w.ptr, ptr.data(), ptr.size() * 4)) != FE_OK ||
        (s = up((void **)&w.ent, ent.data(), ent.size() * 4)) != FE_OK ||
        (s = up((void **)&w.part, nullptr, 12 * (size_t)n_faces * sizeof(double))) != FE_OK) {
        (void)hipStreamSynchronize(c->stream);   // queued copies read the host vectors
        for (void *p : {(void *)w.nen, (void *)w.conn, (void *)w.nodes, (void *)w.ptr, (void *)w.ent, (void *)w.part})
            mesh_free_ptr(m, p);
        return s;
    }
    if ((s = sync(c)) != FE_OK) return s;   // the host vectors go out of scope
    m->wall = w;
    return FE_OK;
}

fe_status fe_wall_traction(fe_mesh m, const double *u, const double *rho, const double *mu, double *out)
{
    if (!m) return FE_EINVAL;
    if (!u || !rho || !mu || !out) return fail(m->ctx, FE_EINVAL, "null u/rho/mu/out");
    HIPCALL(m->ctx, hipSetDevice(m->ctx->device));
    {
        ProfScope ps(m->ctx, 4);
        HIPCALL(m->ctx, launch_wall_traction(m->dm, m->wall, u, rho, mu, out, true, m->ctx->stream));
    }
    return FE_OK;
}

// ---- profiling hooks (not part of the numerical API) -------------------------

fe_status fe_ctx_profile(fe_ctx c, int enable)
{
    if (!c) return FE_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    c->profiling = enable != 0;
    for (auto &p : c->prof) p.used = 0;
    return FE_OK;
}

fe_status fe_ctx_profile_read(fe_ctx c, int slot, int64_t *launches, double *total_ms)
{
    if (!c || slot < 0 || slot >= 5 || !launches || !total_ms) return FE_EINVAL;
    HIPCALL(c, hipStreamSynchronize(c->stream));
    ProfSlot &p = c->prof[slot];
    double tot = 0.0;
    for (size_t i = 0; i + 1 < p.used; i += 2) {
        float ms = 0.f;
        HIPCALL(c, hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
        tot += ms;
    }
    *launches = (int64_t)(p.used / 2);
    *total_ms = tot;
    return FE_OK;
}

// ---- host-only planner access -------------------------------------------------

struct fe_plan_s {
    Plan P;
    OwnerPlan O;   // single-type meshes
};

static thread_local std::string g_plan_err;

static fe_status plan_create(int stride, const uint8_t *types, int64_t n_nodes, const double *coords,
                             int64_t n_elems, const int32_t *conn, uint32_t flags, fe_plan *out)
{
    if (!out) return FE_EINVAL;
    *out = nullptr;
    auto *p = new fe_plan_s();
    std::string err;
    int st = build_plan(stride, types, n_nodes, coords, n_elems, conn, (flags & FE_UPLOAD_RENUMBER) != 0, p->P,
                        err);
    if (st == FE_OK && p->P.etype.empty()) st = build_owner_plan(p->P, p->O, err);
    if (st != FE_OK) {
        g_plan_err = err;
        delete p;
        return (fe_status)st;
    }
    *out = p;
    return FE_OK;
}

fe_status fe_plan_create(fe_elem_type type, int64_t n_nodes, const double *coords, int64_t n_elems,
                         const int32_t *conn, uint32_t flags, fe_plan *out)
{
    return plan_create((int)type, nullptr, n_nodes, coords, n_elems, conn, flags, out);
}

fe_status fe_plan_create_mixed(int64_t n_nodes, const double *coords, int64_t n_elems, const uint8_t *elem_types,
                               const int32_t *conn, uint32_t flags, fe_plan *out)
{
    if (!elem_types) return FE_EINVAL;
    return plan_create(8, elem_types, n_nodes, coords, n_elems, conn, flags, out);
}

fe_status fe_plan_info(fe_plan p, fe_plan_desc *o)
{
    if (!p || !o) return FE_EINVAL;
    const Plan &P = p->P;
    o->n_nodes = P.N;
    o->n_elems = P.E;
    o->nnz = P.nnz;
    o->n_blocks = P.n_blocks();
    o->n_colors = P.n_colors;
    o->max_row = P.max_row;
    o->max_block_nodes = P.max_T;
    o->max_block_slots = P.max_L;
    o->max_phases = P.max_phase;
    return FE_OK;
}

fe_status fe_plan_export(fe_plan p, int32_t *node_perm, int32_t *elem_perm, int32_t *rowptr, int32_t *colidx,
                         int32_t *block_elem_ptr, int32_t *block_color, int32_t *block_node_ptr, int32_t *block_nodes)
{
    if (!p) return FE_EINVAL;
    const Plan &P = p->P;
    auto cp = [](int32_t *dst, const std::vector<int32_t> &v) {
        if (dst && !v.empty()) memcpy(dst, v.data(), v.size() * sizeof(int32_t));
    };
    cp(node_perm, P.node_perm);
    cp(elem_perm, P.elem_perm);
    cp(rowptr, P.rowptr);
    cp(colidx, P.colidx);
    cp(block_elem_ptr, P.blk_elem_ptr);
    cp(block_color, P.blk_color);
    cp(block_node_ptr, P.blk_node_ptr);
    cp(block_nodes, P.blk_nodes);
    return FE_OK;
}

fe_status fe_plan_export_types(fe_plan p, uint8_t *elem_types, uint8_t *block_types, int32_t *launches,
                               int64_t *n_launches)
{
    if (!p) return FE_EINVAL;
    const Plan &P = p->P;
    if (elem_types)
        for (int64_t e = 0; e < P.E; ++e) elem_types[e] = P.etype.empty() ? (uint8_t)P.nen : P.etype[e];
    if (block_types && !P.blk_nen.empty()) memcpy(block_types, P.blk_nen.data(), P.blk_nen.size());
    if (launches)
        for (size_t q = 0; q < P.segs.size(); ++q) {
            launches[3 * q] = P.segs[q].nen;
            launches[3 * q + 1] = P.segs[q].first;
            launches[3 * q + 2] = P.segs[q].count;
        }
    if (n_launches) *n_launches = (int64_t)P.segs.size();
    return FE_OK;
}

fe_status fe_plan_export_color_blocks(fe_plan p, int32_t *color_blocks)
{
    if (!p || !color_blocks) return FE_EINVAL;
    const Plan &P = p->P;
    if (!P.color_blk.empty()) memcpy(color_blocks, P.color_blk.data(), P.color_blk.size() * sizeof(int32_t));
    return FE_OK;
}

fe_status fe_plan_owner_info(fe_plan p, int64_t *n_groups, int64_t *n_tasks, int32_t *rows_per_task,
                             int32_t *ln_stride, int32_t *off_stride, int32_t *wave_private)
{
    if (!p) return FE_EINVAL;
    const OwnerPlan &O = p->O;
    if (O.groups.empty()) return FE_EINVAL;
    if (n_groups) *n_groups = (int64_t)O.groups.size();
    if (n_tasks) *n_tasks = (int64_t)O.tk_elem.size();
    if (rows_per_task) *rows_per_task = O.ra;
    if (ln_stride) *ln_stride = O.ln_stride;
    if (off_stride) *off_stride = O.off_stride;
    if (wave_private) *wave_private = O.wave_private ? 1 : 0;
    return FE_OK;
}

fe_status fe_plan_export_owner(fe_plan p, int32_t *groups, int32_t *node_ptr, int32_t *nodes, uint8_t *nphase,
                               int32_t *task_elem, uint16_t *task_ln, uint8_t *task_off, uint8_t *task_phase)
{
    if (!p) return FE_EINVAL;
    const OwnerPlan &O = p->O;
    if (O.groups.empty()) return FE_EINVAL;
    auto cp = [](void *dst, const auto &v) {
        if (dst && !v.empty()) memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    cp(groups, O.groups);
    cp(node_ptr, O.node_ptr);
    cp(nodes, O.nodes);
    cp(nphase, O.nphase);
    cp(task_elem, O.tk_elem);
    cp(task_ln, O.tk_ln);
    cp(task_off, O.tk_off);
    cp(task_phase, O.tk_phase);
    return FE_OK;
}

void fe_plan_free(fe_plan p) { delete p; }

const char *fe_plan_last_error(void) { return g_plan_err.c_str(); }

fe_status fe_pack_layout(int64_t n_elems, int32_t vector_size, int64_t *packs, int64_t *padded)
{
    if (n_elems < 0 || vector_size < 1 || !packs || !padded) return FE_EINVAL;
    *packs = (n_elems + vector_size - 1) / vector_size;
    *padded = *packs * vector_size - n_elems;
    return FE_OK;
}

}  // extern "C"
