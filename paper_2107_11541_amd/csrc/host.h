// host.h -- host-side objects shared by the C ABI (feasm.cpp) and the serving
// runtime (serve.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/feasm.h"
#include "internal.h"
#include "plan.h"

namespace feasm {

// A region of device memory carved up by the serving runtime (first fit,
// 256-byte granules).  Meshes placed in an arena never call hipMalloc.
class DevArena {
  public:
    DevArena(char *base, size_t bytes);
    void *alloc(size_t bytes);        // nullptr when no hole is large enough
    void release(void *p);
    size_t free_bytes() const { return free_total_; }
    size_t capacity() const { return cap_; }
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }

  private:
    char *base_;
    size_t cap_, free_total_;
    std::vector<std::pair<size_t, size_t>> holes_;   // (offset, size), sorted by offset
    std::vector<std::pair<size_t, size_t>> used_;    // (offset, size), sorted by offset
};

// A roctx range over a scope: rocprofv3 --marker-trace shows the library's
// calls (upload, assembly, Dirichlet, solve, time step, serving stages) on
// the host timeline beside the kernels they launch.
struct RoctxRange {
    explicit RoctxRange(const char *name) { roctxRangePushA(name); }
    ~RoctxRange() { roctxRangePop(); }
    RoctxRange(const RoctxRange &) = delete;
    RoctxRange &operator=(const RoctxRange &) = delete;
};

struct ProfSlot {
    std::vector<hipEvent_t> ev;   // start/stop pairs
    size_t used = 0;
};

}  // namespace feasm

struct fe_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;   // private stream that PCG graphs are recorded on (never run on)
    std::string err;
    double *scratch = nullptr;    // 2048 partials + 64 results
    double *host = nullptr;       // pinned read-back area (64 doubles)
    bool profiling = false;
    std::vector<fe_mesh_s *> meshes;   // live meshes, freed by fe_ctx_destroy
    feasm::ProfSlot prof[5];      // 0 CG SpMV + p.q, 1 assembly (all colours), 2 CG vector updates, 3 Dirichlet,
                                  // 4 element-vector pass (explicit step)
};

struct fe_mesh_s {
    fe_ctx_s *ctx = nullptr;
    feasm::DevMesh dm;
    std::vector<int32_t> node_perm, elem_perm;
    std::vector<void *> allocs;
    size_t bytes = 0;
    feasm::AsmStatus *status = nullptr;  // + per-block scratch
    feasm::CGWork cg;
    double *step_work = nullptr;         // explicit step: u0 [3][N], residual + mass [4][N], f [N], g [3][N]
    feasm::DevWall wall;                 // wall faces of the wall model (F = 0: none)
    double *scalar_work = nullptr;       // explicit scalar step: Y0 [N], residual + mass [2][N]
    feasm::DevRowPlan rowplan;           // 3x3-block momentum operator (built on its first use)
    std::vector<int32_t> conn_m;         // [E][stride_m] connectivity, mesh numbering (block operator plan)
    std::vector<uint8_t> etype_m;        // [E] node counts (hybrid meshes), else empty
    int stride_m = 0;
    feasm::DevArena *arena = nullptr;    // device memory source (nullptr: hipMalloc)
    bool listed = true;                  // in ctx->meshes (freed with the context)
    // recorded PCG iterations (FP64, FP32), valid for the pointers they were
    // recorded with
    struct PcgGraph {
        hipGraphExec_t exec = nullptr;
        const void *vals = nullptr, *x = nullptr, *hist = nullptr, *sym = nullptr;
    } graph[2];
    // the symmetric PCG SpMV's map (built on the first FP64 solve; state 0:
    // not built, 1: built, -1: the pattern has none) and its packed values
    struct SymState {
        int state = 0;
        feasm::SymSpmv map;      // vals: the packed array
        uint8_t *mstart = nullptr;   // [n_nodes] per-row mirror-run starts
        int32_t *bad = nullptr;  // the symmetric-pair check word
        int64_t n_packed = 0;
    } sym;
};

namespace feasm {

fe_status fail(fe_ctx_s *c, fe_status s, const char *fmt, ...);

#define HIPCALL(ctx, expr)                                                                              \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail((ctx), FE_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Host image of a device mesh: the plan plus every array the device copy
// holds, built without touching the GPU (so planner threads can run it).
struct MeshImage {
    Plan P;
    OwnerPlan O;               // matrix assembly of a single-type mesh (no groups otherwise)
    std::vector<uint8_t> is_dir;
    std::vector<int32_t> dir_rows;
    std::vector<int4> spmv_desc;
    std::vector<uint16_t> spmv_roff;
    std::vector<uint8_t> spmv_lidx;
    std::vector<int32_t> spmv_cols;
    DevMesh d;                 // sizes filled, device pointers null
    // Device bytes of the mesh arrays (256-byte granules), without CG work.
    size_t device_bytes() const;
    // Empties the image for the next mesh, keeping its host arrays' capacity.
    void clear();
};

// Validates and plans a mesh on the host (no device calls).  0 or an
// fe_status code with a message in err.
// conn [n_elems][stride]; types as for build_plan (NULL: one type, stride nodes).
// owner_plan: build the owner plan of the HEX08 matrix assembly (the
// serving runtime, which assembles each mesh once, skips it: its host time
// exceeds the assembly time it saves there).
int mesh_prepare(int stride, const uint8_t *types, int64_t n_nodes, const double *coords, int64_t n_elems,
                 const int32_t *conn, int64_t n_dirichlet, const int32_t *dirichlet_nodes, bool renumber,
                 MeshImage &img, std::string &err, bool owner_plan = true);
// Allocates (from m->arena or hipMalloc) and queues the copies of img on
// `stream`.  img must stay alive until the copies have completed.
fe_status mesh_commit(fe_mesh_s *m, MeshImage &img, hipStream_t stream);
// Device memory of m (through the arena when it has one).
fe_status mesh_alloc(fe_mesh_s *m, void **p, size_t bytes);
void mesh_release(fe_mesh_s *m);
// Device bytes of the FP64 PCG work buffers for n unknowns and max_iter.
size_t cg_bytes(int64_t n, int max_iter);
fe_status ensure_cg(fe_mesh_s *m, int max_iter, bool mixed);
// Queues every assembly pass of one operator on `stream`; the status word
// stays on the device (m->status).
fe_status assemble_queue(fe_mesh_s *m, const fe_fields *f, fe_precision prec, double *values, double *rhs,
                         hipStream_t stream);

}  // namespace feasm
