// plan.h -- host-side mesh preprocessing for the block-LDS assembly.
//
// Section 4.3 of the paper groups elements by geometric type, renumbers them
// and packs them so that a SIMD/SIMT unit processes a pack at once.  The gfx950
// form of that idea built here:
//   * elements are reordered along a Morton curve of their centroids and nodes
//     renumbered by first touch, so that a block of consecutive elements is
//     spatially compact and touches few CSR rows;
//   * a block is at most one wavefront (64) of elements, cut early when the
//     LDS image of the rows it touches would exceed the budget, and at the
//     fixed element chunks the planner builds blocks in (kPlanElemChunk);
//   * blocks are coloured so that no two blocks of one colour share a node:
//     one launch per colour runs without write conflicts (no atomics);
//   * inside a block, elements are split into phases so that no two lanes of
//     one phase hold the same node at the same local position, which makes
//     every LDS accumulation instruction conflict-free and the summation
//     order fixed;
//   * for each touched row the first block (in launch order) that touches it
//     overwrites it, later blocks read-modify-write it.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace feasm {

// LDS budget of one assembly work-group (bytes).  The momentum kernel stages
// 8 fields per touched node, 3 RHS images, one int descriptor and the row image.
constexpr int kBlockElems = 64;
constexpr int kLdsBudget = 40 * 1024;
constexpr int kNodeFields = 8;
constexpr int kMaxRhs = 3;
constexpr int kMaxRow = 255;   // in-row offsets are stored as uint8
// The planner's parallel stages work on fixed chunks (elements for the
// assembly blocks, rows for the SpMV row blocks), so a plan does not depend
// on the number of host threads that built it.
constexpr int64_t kPlanElemChunk = 1 << 16;   // a multiple of kBlockElems
constexpr int64_t kPlanRowChunk = 1 << 15;
// Touched-row descriptor: image offset (bits 0-15) | row length (16-23) |
// first-writer flag (bit 31).
constexpr uint32_t kFirstBit = 0x80000000u;

// One assembly launch: blocks color_blk[first, first + count) of one colour
// and one element type (nen nodes per element).
struct AsmSeg {
    int nen, first, count;
};

// Position of an element type (by node count) in the order a mixed mesh
// groups them: HEX08, PEN06, PYR05, TET04.
inline int type_rank(int nen) { return nen == 8 ? 0 : nen == 6 ? 1 : nen == 5 ? 2 : 3; }

struct Plan {
    int nen = 0;          // connectivity stride: nodes of the largest element type
    int off_stride = 0;   // bytes of elem_off per element (nen * nen rounded up to 4)
    int64_t N = 0, E = 0, nnz = 0;
    std::vector<int32_t> node_perm;   // mesh index -> user node id
    std::vector<int32_t> node_iperm;  // user node id -> mesh index
    std::vector<int32_t> elem_perm;   // mesh element -> user element id
    std::vector<double> X;            // [3][N] coordinates, mesh numbering
    std::vector<int32_t> conn;        // [E][nen] mesh numbering, mesh order (short types padded)
    std::vector<uint8_t> etype;       // [E] nodes of each element (mesh order); empty: all nen
    std::vector<int32_t> rowptr, colidx, diagpos;
    int max_row = 0;

    // element blocks
    std::vector<int32_t> blk_elem_ptr;   // [nblk+1]
    std::vector<int32_t> blk_node_ptr;   // [nblk+1]
    std::vector<int32_t> blk_nodes;      // touched rows, ascending mesh ids
    std::vector<int32_t> blk_img;        // [nblk] entries of the touched rows (the block's row image)
    std::vector<int32_t> blk_rdesc;      // packed descriptor of each touched row (see kFirstBit)
    std::vector<int32_t> blk_rowstart;   // CSR start of each touched row
    std::vector<int32_t> blk_color;      // [nblk]
    std::vector<uint8_t> blk_nphase;     // [nblk]
    std::vector<uint16_t> elem_lnode;    // [nen][E] local row index of node a
    std::vector<uint8_t> elem_off;       // [E][off_stride]: offset of col b in row a at a * n_e + b
    std::vector<uint8_t> blk_nen;        // [nblk] element type of each block
    std::vector<uint8_t> elem_phase;     // [E]
    std::vector<int32_t> color_ptr;      // [ncolor+1]
    std::vector<int32_t> color_blk;      // blocks ordered by colour, then type (type_rank)
    std::vector<AsmSeg> segs;            // launch order: colour-major, one per type present
    int n_colors = 0, max_T = 0, max_L = 0, max_phase = 0;

    int64_t n_blocks() const { return (int64_t)blk_elem_ptr.size() - 1; }
    // Empties the plan but keeps its arrays' capacity, so that a plan object
    // reused for the next mesh (the serving runtime's planners) does not
    // fault its pages in again.
    void clear();
};

// conn [n_elems][stride]; types [n_elems] gives each element's node count
// (4, 5, 6 or 8, at most stride; the remaining slots are ignored) or is NULL
// for a mesh of one type with stride nodes.  Returns 0 on success, else an
// fe_status code with a message in err.
int build_plan(int stride, const uint8_t *types, int64_t n_nodes, const double *coords, int64_t n_elems,
               const int32_t *conn, bool renumber, Plan &P, std::string &err);

// Host memory of the planner's temporaries (per calling thread, kept between
// calls up to kPlanScratchKeep bytes so that a thread planning mesh after
// mesh reuses it; larger ones are released after the call).
constexpr size_t kPlanScratchKeep = (size_t)256 << 20;

// Runs f(c) for every c in [0, n) on up to host_threads() threads (chunks
// handed out in increasing order; f must only write chunk c's results).
void parallel_chunks(int64_t n, const std::function<void(int64_t)> &f);
// The same with the worker's index w in [0, parallel_workers(n)) passed as
// f(c, w), for per-worker scratch arrays.
int parallel_workers(int64_t n);
void parallel_chunks_w(int64_t n, const std::function<void(int64_t, int)> &f);

// Row-owner plan of the 3x3-block momentum operator (rowplan.cpp): tasks =
// (element, row) pairs ordered by row, then element; whole rows packed into
// waves of at most kRowTasksMax tasks and kRowImageDoubles block values.
constexpr int kRowTasksMax = 64;
constexpr int kRowImageDoubles = 3072;
struct RowWave {
    int32_t first_task, n_tasks, first_row, n_rows;
};
struct RowPlan {
    int64_t n_tasks = 0, max_img = 0;
    std::vector<int32_t> task_elem;    // [T] element (mesh order)
    std::vector<uint16_t> task_meta;   // [T] local row a (bits 0-3) | phase in the row (bits 4-15)
    std::vector<uint8_t> task_cols;    // [T][8] position of the element's node b in the row
    std::vector<RowWave> wdesc;        // [waves]
};
// conn [E][stride] and rowptr/colidx in mesh numbering; etype [E] node
// counts or NULL (every element has stride nodes).  0 or an fe_status code
// with a message in err (FE_EBADMESH: a node in more than kRowTasksMax
// elements).
int build_row_plan(int stride, const uint8_t *etype, int64_t N, int64_t E, const int32_t *conn,
                   const int32_t *rowptr, const int32_t *colidx, RowPlan &R, std::string &err);

// Owner plan of the matrix assembly (rowplan.cpp): the CSR rows are cut
// into groups of consecutive rows (mesh numbering, so spatially compact);
// one work-group owns a group, computes every element contribution to its
// rows and writes each row once.  A task is one lane's share: an element's
// rows that the group owns, at most 4 of them for HEX08 (the element is
// presented in a rotated node order that puts them on its first face; an
// element with owned nodes on no single face gives two tasks), every row of
// the element for the other types (rows the group does not own are
// dropped).  Tasks of one phase hold distinct owned rows (of the group, or,
// for wave-private accumulation, of the wave).
constexpr int kOwnTasks = 256;            // lanes of an owner work-group
constexpr int kOwnNodes = 1024;           // touched nodes of a group (uint16 local ids)
using OwnLn = uint16_t;                   // a task's group-local node index
constexpr int kOwnLdsBytes = 64 * 1024;   // LDS of a group for the momentum operator
struct OwnGroup {
    int32_t first_task, n_tasks, first_row, n_rows;
};
struct OwnerPlan {
    int ra = 0;                          // rows per task (4 for HEX08, else nodes per element)
    bool wave_private = false;           // each wave accumulates into its own copy of the group's rows
                                         // (phases per wave, no barriers; the copies are summed in wave
                                         // order); else one copy, phases over the group with barriers
    int ln_stride = 0, off_stride = 0;   // entries per task of tk_ln, bytes per task of tk_off
    int max_nodes = 0, max_img = 0, max_rows = 0, max_phase = 0;
    std::vector<OwnGroup> groups;
    std::vector<int32_t> node_ptr, nodes;   // per group: owned rows first, then the halo ascending
    std::vector<uint8_t> nphase;            // [groups]
    std::vector<int32_t> tk_elem;           // [T] mesh element
    std::vector<OwnLn> tk_ln;               // [T][ln_stride] local node of each (rotated) element node
    std::vector<uint8_t> tk_off;            // [T][off_stride] position of column b in row r (owned rows)
    std::vector<uint8_t> tk_phase;          // [T]
};
// Single-type meshes only (P.etype empty).  0 or an fe_status code with a
// message in err.
int build_owner_plan(const Plan &P, OwnerPlan &O, std::string &err);
// The node order of a HEX08 element seen from face f (0..5: -z, +z, -y, +y,
// -x, +x): kHexFaceRot[f][b] is the element's local node at the rotated
// element's node b; nodes 0-3 of the rotated element are face f.
extern const int kHexFaceRot[6][8];

// Row blocks of the symmetric PCG SpMV (Section 5.2's matrix-vector product
// on an SPD matrix).  A block is a run of consecutive rows r0..r1-1, built
// like the general SpMV's blocks.  Of each pair of entries (i, j), (j, i)
// with both rows in the block, only the upper one (j > i) is stored; the
// lower one is a mirror entry that reads the stored value.  Per block:
//   * <= kSymRows rows, <= kSymStored stored entries, <= kSymMirrors mirror
//     entries, <= kSymCols columns in its column set;
//   * the column set lists the block's own rows first (slot r - r0), then
//     its other columns in first-touch order;
//   * desc[4 b .. 4 b + 3] = {first row, first stored entry in the packed
//     value array, first mirror word, first column of the set}; b = nrb is
//     the end sentinel;
//   * roff[first row + b + i] (i = 0..rows) = offset of row i's stored
//     entries from the block's first | offset of its mirrors from the
//     block's first mirror << 16;
//   * lidx: one set slot per packed entry (parallel to the packed values);
//   * mir: two 16-bit mirror entries per word, each the window position of
//     the stored value (first stored entry's position modulo 4 plus its
//     index in the block; 10 bits) | the mirrored row minus the first row
//     << 10 (6 bits); a block's mirrors start at an even index;
//   * mstart[i]: the position in row i of its first mirror.  Rows are
//     sorted, so a row's mirrors (columns r0 .. i-1) are one run of its
//     entries; the packed position of entry k of row i is the block's first
//     stored entry + row i's stored offset + k, less the run's length when
//     k is past the run.
// Packed positions of stored entries follow CSR order with the mirrors left
// out; each row chunk (kPlanRowChunk rows) starts at a multiple of 4.
constexpr int kSymRows = 64, kSymStored = 1021, kSymMirrors = 512, kSymCols = 256;
struct SymMap {
    int64_t nrb = 0, n_packed = 0, n_mirror_words = 0;
    std::vector<int32_t> desc;    // [nrb + 1][4]
    std::vector<uint32_t> roff;   // [N + nrb]
    std::vector<uint8_t> lidx;    // [n_packed + 4]
    std::vector<uint32_t> mir;    // [n_mirror_words + 1]
    std::vector<int32_t> cols;
    std::vector<uint8_t> mstart;  // [N]
};
// 0, or FE_EBADMESH when the pattern is not structurally symmetric, a row is
// not sorted or does not fit a block (err says which).
int build_sym_map(int64_t N, const int32_t *rowptr, const int32_t *colidx, SymMap &S, std::string &err);

// Number of worker threads used by the host preprocessing.
int host_threads();
// Caps host_threads() for the calling thread (0: no cap); planner threads
// of the serving runtime plan one mesh each on a single thread.
void set_thread_budget(int n);

}  // namespace feasm
