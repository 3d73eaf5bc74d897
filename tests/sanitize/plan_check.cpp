// plan_check.cpp -- runs the host planner (csrc/plan.cpp, rowplan.cpp, symmap.cpp)
// under AddressSanitizer / UndefinedBehaviorSanitizer on small meshes of every
// kind, renumbered and not, and checks a few of its invariants.  Test
// infrastructure: built and run by tests/test_sanitizers_cpu.py.
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_2107_11541_amd/csrc/plan.h"
#include "meshes.h"

using namespace feasm;

static int fails = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                \
        }                                                           \
    } while (0)

// The symmetric SpMV map of a pattern: y = A x through the map, read the way
// the kernel reads it, equals the CSR product, for integer values and x
// (exact in double); every block within its limits.
static void check_sym_map(const Plan &P)
{
    SymMap S;
    std::string err;
    const int st = build_sym_map(P.N, P.rowptr.data(), P.colidx.data(), S, err);
    CHECK(st == 0);
    if (st != 0) {
        fprintf(stderr, "build_sym_map: %s\n", err.c_str());
        return;
    }
    auto aval = [&](int64_t i, int64_t j) {
        const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
        return (double)(1 + (lo * 7 + hi * 13) % 17);
    };
    std::vector<double> x((size_t)P.N), ycsr((size_t)P.N, 0.0), ysym((size_t)P.N, 0.0);
    for (int64_t i = 0; i < P.N; ++i) x[(size_t)i] = (double)(i % 11) - 5.0;
    for (int64_t i = 0; i < P.N; ++i)
        for (int32_t q = P.rowptr[i]; q < P.rowptr[i + 1]; ++q) ycsr[(size_t)i] += aval(i, P.colidx[q]) * x[P.colidx[q]];
    CHECK(S.lidx.size() == (size_t)S.n_packed + 4 && S.mstart.size() == (size_t)P.N);
    // the device pack, row by row: entry k of row i goes to the block's first
    // stored entry + the row's stored offset + k, less the mirror run's
    // length past the run; every mirror's window value is its transpose
    std::vector<double> packed((size_t)S.n_packed + 4, 0.0);
    std::vector<char> hit((size_t)S.n_packed + 4, 0);
    int64_t stored = 0;
    for (int64_t b = 0; b < S.nrb; ++b) {
        const int32_t *d0 = &S.desc[(size_t)b * 4], *d1 = d0 + 4;
        const int64_t r0 = d0[0], R = d1[0] - d0[0];
        for (int64_t i = 0; i < R; ++i) {
            const int64_t row = r0 + i, len = P.rowptr[row + 1] - P.rowptr[row];
            const uint32_t ro = S.roff[(size_t)(r0 + b + i)], ro1 = S.roff[(size_t)(r0 + b + i + 1)];
            const int64_t so = ro & 0xffffu, ml = (int64_t)(ro1 >> 16) - (int64_t)(ro >> 16), ms = S.mstart[(size_t)row];
            CHECK(ms + ml <= len && (int64_t)(ro1 & 0xffffu) - so == len - ml);
            for (int64_t k = 0; k < len; ++k) {
                const int32_t col = P.colidx[P.rowptr[row] + k];
                const bool mirror = k >= ms && k < ms + ml;
                CHECK(mirror == (col >= r0 && col < row));
                if (mirror) continue;
                const int64_t d = d0[1] + so + (k < ms ? k : k - ml);
                CHECK(d >= 0 && d < S.n_packed && !hit[(size_t)d]);
                hit[(size_t)d] = 1;
                packed[(size_t)d] = aval(row, col);
                ++stored;
            }
        }
    }
    for (int64_t b = 0; b < S.nrb; ++b) {
        const int32_t *d0 = &S.desc[(size_t)b * 4], *d1 = d0 + 4;
        const int64_t r0 = d0[0], R = d1[0] - d0[0], a0 = d0[1] & ~3, shift = d0[1] - a0, nz = d1[1] - d0[1];
        const int64_t nsetc = d1[3] - d0[3], nmw = d1[2] - d0[2];
        CHECK(R >= 1 && R <= kSymRows && shift + nz <= 1024 && nmw <= kSymMirrors / 2 && nsetc <= kSymCols);
        for (int64_t i = 0; i < R; ++i) CHECK(S.cols[(size_t)(d0[3] + i)] == (int32_t)(r0 + i));
        for (int64_t i = 0; i < R; ++i) {
            const uint32_t ro = S.roff[(size_t)(r0 + b + i)], ro1 = S.roff[(size_t)(r0 + b + i + 1)];
            double y = 0.0;
            for (uint32_t s = ro & 0xffffu; s < (ro1 & 0xffffu); ++s) {
                const int64_t pos = shift + s;
                CHECK(pos < 1024 && (int64_t)s < nz);
                const int slot = S.lidx[(size_t)(a0 + pos)];
                CHECK(slot < nsetc);
                y += packed[(size_t)(a0 + pos)] * x[S.cols[(size_t)(d0[3] + slot)]];
            }
            for (uint32_t m = ro >> 16; m < (ro1 >> 16); ++m) {
                CHECK((int64_t)m < 2 * nmw);
                const uint32_t w = (S.mir[(size_t)d0[2] + m / 2] >> (16 * (m & 1))) & 0xffffu;
                const int64_t pos = w & 1023u, ro_row = w >> 10;
                CHECK(pos >= shift && pos < shift + nz && ro_row < i);
                y += packed[(size_t)(a0 + pos)] * x[S.cols[(size_t)(d0[3] + ro_row)]];
            }
            ysym[(size_t)(r0 + i)] = y;
        }
    }
    CHECK(S.nrb == 0 || S.desc[(size_t)S.nrb * 4] == (int32_t)P.N);
    CHECK(ysym == ycsr);
    CHECK(stored <= P.nnz && (P.N == 0 || stored < P.nnz));
}

int main()
{
    for (int kind = 0; kind < 3; ++kind)
        for (int renumber = 0; renumber < 2; ++renumber)
            for (int n : {1, 3, 6}) {
                SanMesh m = san_cube(n, kind);
                Plan P;
                std::string err;
                const int st = build_plan(m.stride, m.types, m.n_nodes, m.coords, m.n_elems, m.conn, renumber != 0,
                                          P, err);
                CHECK(st == 0);
                if (st != 0) {
                    fprintf(stderr, "build_plan: %s\n", err.c_str());
                    san_free(&m);
                    continue;
                }
                CHECK(P.rowptr.size() == (size_t)m.n_nodes + 1);
                for (int64_t i = 0; i < m.n_nodes; ++i)
                    for (int32_t q = P.rowptr[i] + 1; q < P.rowptr[i + 1]; ++q) CHECK(P.colidx[q - 1] < P.colidx[q]);
                // the 3x3-block operator's row plan
                RowPlan R;
                CHECK(build_row_plan(P.nen, P.etype.empty() ? nullptr : P.etype.data(), P.N, P.E, P.conn.data(),
                                     P.rowptr.data(), P.colidx.data(), R, err) == 0);
                int64_t rows = 0;
                for (const RowWave &w : R.wdesc) rows += w.n_rows;
                CHECK(rows == m.n_nodes);
                // the owner plan (single-type meshes)
                if (P.etype.empty()) {
                    OwnerPlan O;
                    CHECK(build_owner_plan(P, O, err) == 0);
                    int64_t r = 0, t = 0;
                    for (const OwnGroup &g : O.groups) {
                        CHECK(g.first_row == r && g.first_task == t);
                        CHECK(g.n_tasks >= 1 && g.n_tasks <= kOwnTasks);
                        r += g.n_rows;
                        t += g.n_tasks;
                    }
                    CHECK(r == m.n_nodes && t == (int64_t)O.tk_elem.size());
                }
                check_sym_map(P);
                san_free(&m);
            }
    // a plan does not depend on the number of host threads that built it:
    // TET04 (kind 1) and mixed (kind 2) meshes of more than one element
    // chunk, built with 1 and with 4 threads
    for (int kind : {1, 2}) {
        SanMesh m = san_cube(kind == 1 ? 24 : 28, kind);
        CHECK(m.n_elems > kPlanElemChunk);
        Plan A, B;
        std::string err;
        set_thread_budget(1);
        const int sa = build_plan(m.stride, m.types, m.n_nodes, m.coords, m.n_elems, m.conn, true, A, err);
        set_thread_budget(4);
        const int sb = build_plan(m.stride, m.types, m.n_nodes, m.coords, m.n_elems, m.conn, true, B, err);
        set_thread_budget(0);
        CHECK(sa == 0 && sb == 0);
        CHECK(A.elem_perm == B.elem_perm && A.node_perm == B.node_perm);
        CHECK(A.rowptr == B.rowptr && A.colidx == B.colidx && A.diagpos == B.diagpos);
        CHECK(A.elem_off == B.elem_off && A.elem_lnode == B.elem_lnode && A.elem_phase == B.elem_phase);
        CHECK(A.blk_elem_ptr == B.blk_elem_ptr && A.blk_node_ptr == B.blk_node_ptr && A.blk_nodes == B.blk_nodes);
        CHECK(A.blk_img == B.blk_img && A.blk_color == B.blk_color && A.color_blk == B.color_blk);
        CHECK(A.blk_rdesc == B.blk_rdesc && A.blk_rowstart == B.blk_rowstart);
        // no block crosses an element chunk boundary
        for (size_t b = 0; b + 1 < A.blk_elem_ptr.size(); ++b)
            CHECK(A.blk_elem_ptr[b] / kPlanElemChunk == (A.blk_elem_ptr[b + 1] - 1) / kPlanElemChunk);
        san_free(&m);
    }
    // the symmetric SpMV map over more than one row chunk, built with 1 and
    // with 4 threads
    {
        SanMesh m = san_cube(32, 0);
        CHECK(m.n_nodes > kPlanRowChunk);
        Plan P;
        std::string err;
        CHECK(build_plan(m.stride, m.types, m.n_nodes, m.coords, m.n_elems, m.conn, true, P, err) == 0);
        check_sym_map(P);
        SymMap S1, S4;
        set_thread_budget(1);
        CHECK(build_sym_map(P.N, P.rowptr.data(), P.colidx.data(), S1, err) == 0);
        set_thread_budget(4);
        CHECK(build_sym_map(P.N, P.rowptr.data(), P.colidx.data(), S4, err) == 0);
        set_thread_budget(0);
        CHECK(S1.nrb == S4.nrb && S1.n_packed == S4.n_packed && S1.desc == S4.desc && S1.roff == S4.roff &&
              S1.lidx == S4.lidx && S1.mir == S4.mir && S1.cols == S4.cols && S1.mstart == S4.mstart);
        san_free(&m);
    }
    // a plan object reused for another mesh (the serving runtime's images)
    // equals a fresh one: larger hybrid mesh first, then a smaller TET04 one
    {
        SanMesh big = san_cube(6, 2), small = san_cube(3, 1);
        Plan reused, fresh;
        std::string err;
        CHECK(build_plan(big.stride, big.types, big.n_nodes, big.coords, big.n_elems, big.conn, true, reused, err) == 0);
        CHECK(build_plan(small.stride, small.types, small.n_nodes, small.coords, small.n_elems, small.conn, true, reused,
                         err) == 0);
        CHECK(build_plan(small.stride, small.types, small.n_nodes, small.coords, small.n_elems, small.conn, true, fresh,
                         err) == 0);
        CHECK(reused.nen == fresh.nen && reused.N == fresh.N && reused.E == fresh.E && reused.nnz == fresh.nnz);
        CHECK(reused.max_row == fresh.max_row && reused.n_colors == fresh.n_colors && reused.max_T == fresh.max_T &&
              reused.max_L == fresh.max_L && reused.max_phase == fresh.max_phase);
        CHECK(reused.elem_perm == fresh.elem_perm && reused.node_perm == fresh.node_perm &&
              reused.node_iperm == fresh.node_iperm && reused.conn == fresh.conn && reused.X == fresh.X);
        CHECK(reused.etype == fresh.etype && reused.rowptr == fresh.rowptr && reused.colidx == fresh.colidx);
        CHECK(reused.elem_off == fresh.elem_off && reused.elem_lnode == fresh.elem_lnode &&
              reused.elem_phase == fresh.elem_phase && reused.blk_nphase == fresh.blk_nphase);
        CHECK(reused.blk_elem_ptr == fresh.blk_elem_ptr && reused.blk_nodes == fresh.blk_nodes &&
              reused.blk_img == fresh.blk_img && reused.blk_rdesc == fresh.blk_rdesc &&
              reused.color_blk == fresh.color_blk && reused.segs.size() == fresh.segs.size());
        san_free(&big);
        san_free(&small);
    }
    printf("plan_check: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
