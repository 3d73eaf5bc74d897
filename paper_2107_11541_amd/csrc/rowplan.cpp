// rowplan.cpp -- host planning of the row-owner assembly (3x3-block momentum
// operator).
//
// The block operator's values are nine times the scalar operator's, so it is
// assembled with every CSR row written exactly once and never read back:
//   * a task is one (element, row) pair: element e's contribution to the
//     block row of one of its nodes;
//   * tasks are ordered by row (mesh numbering), and within a row by element;
//     the phase of a task is its position in its row's list;
//   * consecutive rows are packed into wavefronts: whole rows only, at most
//     64 tasks and kRowImageDoubles of block values per wave, so each wave
//     owns its rows outright (no other wave adds to them) and holds their
//     image in LDS.
#include <algorithm>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/feasm.h"
#include "plan.h"

namespace feasm {

namespace {

template <class F>
void chunks(int64_t n, F f)
{
    const int nt = n < 4096 ? 1 : host_threads();
    if (nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        const int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([=, &f] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

}  // namespace

int build_row_plan(int stride, const uint8_t *etype, int64_t N, int64_t E, const int32_t *conn,
                   const int32_t *rowptr, const int32_t *colidx, RowPlan &R, std::string &err)
{
    R = RowPlan();
    auto nen_of = [&](int64_t e) { return etype ? (int)etype[e] : stride; };
    // node -> element incidence, elements ascending
    std::vector<int32_t> inc_ptr(N + 1, 0);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nen_of(e); ++a) ++inc_ptr[conn[e * stride + a] + 1];
    for (int64_t i = 0; i < N; ++i) {
        if (inc_ptr[i + 1] > kRowTasksMax) {
            err = "node " + std::to_string(i) + " (mesh numbering) lies in " + std::to_string(inc_ptr[i + 1]) +
                  " elements; the block operator's row-owner assembly takes at most " +
                  std::to_string(kRowTasksMax);
            return FE_EBADMESH;
        }
        inc_ptr[i + 1] += inc_ptr[i];
    }
    const int64_t T = inc_ptr[N];
    std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    R.task_elem.resize(T);
    R.task_meta.resize(T);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nen_of(e); ++a) {
            const int32_t i = conn[e * stride + a];
            const int32_t t = fill[i]++;
            R.task_elem[t] = (int32_t)e;
            R.task_meta[t] = (uint16_t)(a | ((t - inc_ptr[i]) << 4));   // local row | phase
        }
    // columns of each task's element in its row
    R.task_cols.assign((size_t)T * 8, 0);
    bool missing = false;
    chunks(N, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const int32_t *c0 = colidx + rowptr[i], *c1 = colidx + rowptr[i + 1];
            for (int32_t t = inc_ptr[i]; t < inc_ptr[i + 1]; ++t) {
                const int64_t e = R.task_elem[t];
                for (int b = 0; b < nen_of(e); ++b) {
                    const int32_t j = conn[e * stride + b];
                    const int32_t *p = std::lower_bound(c0, c1, j);
                    if (p == c1 || *p != j) {
                        missing = true;
                        continue;
                    }
                    R.task_cols[(size_t)t * 8 + b] = (uint8_t)(p - c0);
                }
            }
        }
    });
    if (missing) {
        err = "the CSR pattern lacks an element's node pair";
        return FE_EBADMESH;
    }
    // whole rows into waves
    int64_t r = 0;
    while (r < N) {
        const int64_t r0 = r;
        int tasks = 0;
        while (r < N) {
            const int nt = inc_ptr[r + 1] - inc_ptr[r];
            const int64_t img = 9 * (int64_t)(rowptr[r + 1] - rowptr[r0]);
            if (r > r0 && (tasks + nt > kRowTasksMax || img > kRowImageDoubles || r - r0 >= kRowTasksMax)) break;
            tasks += nt;
            ++r;
        }
        R.wdesc.push_back({inc_ptr[r0], tasks, (int32_t)r0, (int32_t)(r - r0)});
        R.max_img = std::max<int64_t>(R.max_img, 9 * (int64_t)(rowptr[r] - rowptr[r0]));
    }
    R.n_tasks = T;
    return FE_OK;
}

}  // namespace feasm

namespace feasm {

// Proper rotations of the reference cube taking each face to the first one
// (z = -1): rotated node b is the original node kHexFaceRot[f][b].
const int kHexFaceRot[6][8] = {
    {0, 1, 2, 3, 4, 5, 6, 7},   // -z: identity
    {7, 6, 5, 4, 3, 2, 1, 0},   // +z: half turn about the x axis
    {4, 5, 1, 0, 7, 6, 2, 3},   // -y: quarter turn about x
    {3, 2, 6, 7, 0, 1, 5, 4},   // +y: quarter turn about x, the other way
    {4, 0, 3, 7, 5, 1, 2, 6},   // -x: quarter turn about y
    {1, 5, 6, 2, 0, 4, 7, 3},   // +x: quarter turn about y, the other way
};

namespace {

// Bit masks of the six faces' nodes.
uint8_t face_mask(int f)
{
    uint8_t m = 0;
    for (int b = 0; b < 4; ++b) m |= (uint8_t)(1u << kHexFaceRot[f][b]);
    return m;
}

}  // namespace

int build_owner_plan(const Plan &P, OwnerPlan &O, std::string &err)
{
    O = OwnerPlan();
    if (!P.etype.empty()) {
        err = "owner plan: one element type per mesh";
        return FE_EINVAL;
    }
    const int nen = P.nen;
    const int64_t N = P.N, E = P.E;
    const bool hex = nen == 8;
    O.ra = hex ? 4 : nen;
    // the other types' nodes lie in many elements (24 for a Kuhn
    // tetrahedron's), which would make as many barrier-separated phases:
    // their waves accumulate privately instead
    O.wave_private = !hex;
    const int copies = O.wave_private ? kOwnTasks / 64 : 1;
    O.ln_stride = nen;
    O.off_stride = (O.ra * nen + 3) & ~3;
    const int32_t *conn = P.conn.data();
    const int32_t *rowptr = P.rowptr.data(), *colidx = P.colidx.data();

    // tasks needed to cover a set of owned element nodes
    uint8_t fmask[6];
    for (int f = 0; f < 6; ++f) fmask[f] = face_mask(f);
    uint8_t cover[256];
    for (int m = 0; m < 256; ++m) {
        if (m == 0) cover[m] = 0;
        else if (!hex) cover[m] = 1;
        else {
            cover[m] = 2;
            for (int f = 0; f < 6; ++f)
                if ((m & ~fmask[f]) == 0) cover[m] = 1;
        }
    }
    // node -> (element, local index) incidence, elements ascending
    std::vector<int32_t> inc_ptr(N + 1, 0);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nen; ++a) ++inc_ptr[conn[e * nen + a] + 1];
    for (int64_t i = 0; i < N; ++i) inc_ptr[i + 1] += inc_ptr[i];
    std::vector<int32_t> inc(inc_ptr[N]);
    {
        std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nen; ++a) inc[fill[conn[e * nen + a]]++] = (int32_t)(e * 8 + a);
    }
    auto lds_bytes = [&](int64_t tn, int64_t img, int64_t nr) {
        return (kNodeFields * tn + copies * (img + kMaxRhs * nr)) * 8;
    };

    // 1. groups of consecutive rows: row r joins the open group unless the
    //    group's tasks, touched nodes or LDS would then exceed their limits
    std::vector<int32_t> estamp(E, -1), nstamp(N, -1);
    std::vector<int64_t> nmark(N, -1);
    std::vector<uint8_t> emask(E, 0);
    std::vector<int32_t> gstart(1, 0);   // first row of each group
    int32_t gid = 0;
    int64_t mark = 0;
    auto cost = [&](int64_t r, int64_t &dt, int64_t &dn) {
        dt = dn = 0;
        ++mark;
        for (int32_t q = inc_ptr[r]; q < inc_ptr[r + 1]; ++q) {
            const int32_t e = inc[q] >> 3, a = inc[q] & 7;
            const uint8_t old = estamp[e] == gid ? emask[e] : 0;
            dt += cover[old | (1u << a)] - cover[old];
            if (estamp[e] == gid) continue;
            for (int b = 0; b < nen; ++b) {
                const int32_t v = conn[(int64_t)e * nen + b];
                if (nstamp[v] != gid && nmark[v] != mark) {
                    nmark[v] = mark;
                    ++dn;
                }
            }
        }
    };
    auto commit = [&](int64_t r) {
        for (int32_t q = inc_ptr[r]; q < inc_ptr[r + 1]; ++q) {
            const int32_t e = inc[q] >> 3, a = inc[q] & 7;
            if (estamp[e] != gid) {
                estamp[e] = gid;
                emask[e] = 0;
                for (int b = 0; b < nen; ++b) nstamp[conn[(int64_t)e * nen + b]] = gid;
            }
            emask[e] |= (uint8_t)(1u << a);
        }
    };
    int64_t tasks = 0, tn = 0, img = 0, r0 = 0;
    for (int64_t r = 0; r < N; ++r) {
        int64_t dt, dn;
        cost(r, dt, dn);
        const int64_t len = rowptr[r + 1] - rowptr[r];
        auto over = [&](int64_t t_, int64_t n_, int64_t img_, int64_t nr_) {
            return t_ > kOwnTasks || n_ > kOwnNodes || nr_ > kOwnNodes || lds_bytes(n_, img_, nr_) > kOwnLdsBytes;
        };
        if (r > r0 && over(tasks + dt, tn + dn, img + len, r - r0 + 1)) {
            ++gid;
            gstart.push_back((int32_t)r);
            r0 = r;
            tasks = tn = img = 0;
            cost(r, dt, dn);
        }
        if (over(tasks + dt, tn + dn, img + len, r - r0 + 1)) {
            err = "node " + std::to_string(r) + " (mesh numbering): its elements exceed one owner group";
            return FE_EBADMESH;
        }
        commit(r);
        tasks += dt;
        tn += dn;
        img += len;
    }
    gstart.push_back((int32_t)N);
    const int64_t G = (int64_t)gstart.size() - 1;

    // 2. per group: node list, tasks, in-row offsets, phases.  Groups are
    //    independent; a first pass counts each group's nodes and tasks, a
    //    second writes them at their final places.
    std::vector<int32_t> gnodes(G), gtasks(G);
    std::vector<uint8_t> gbad(G, 0);
    const int nt = std::max(1, std::min<int>(host_threads(), (int)((G + 63) / 64)));
    auto run = [&](auto &&body) {
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t) th.emplace_back([&, t] { body(t); });
        for (auto &x : th) x.join();
    };
    // the elements of group g, ascending (est: per-thread stamps, [E])
    auto group_elems = [&](int64_t g, std::vector<int32_t> &elems, std::vector<int32_t> &est) {
        elems.clear();
        for (int32_t r = gstart[g]; r < gstart[g + 1]; ++r)
            for (int32_t q = inc_ptr[r]; q < inc_ptr[r + 1]; ++q) {
                const int32_t e = inc[q] >> 3;
                if (est[e] != (int32_t)g) {
                    est[e] = (int32_t)g;
                    elems.push_back(e);
                }
            }
        std::sort(elems.begin(), elems.end());
    };
    auto owned_mask = [&](int32_t e, int32_t a0, int32_t a1) {
        uint8_t m = 0;
        for (int b = 0; b < nen; ++b) {
            const int32_t v = conn[(int64_t)e * nen + b];
            if (v >= a0 && v < a1) m |= (uint8_t)(1u << b);
        }
        return m;
    };
    run([&](int t) {
        std::vector<int32_t> elems, est(E, -1), nst(N, -1);
        for (int64_t g = t; g < G; g += nt) {
            const int32_t a0 = gstart[g], a1 = gstart[g + 1];
            group_elems(g, elems, est);
            int32_t tasks_g = 0, nh = 0;
            for (int32_t e : elems) {
                tasks_g += cover[owned_mask(e, a0, a1)];
                for (int b = 0; b < nen; ++b) {
                    const int32_t v = conn[(int64_t)e * nen + b];
                    if ((v < a0 || v >= a1) && nst[v] != (int32_t)g) {
                        nst[v] = (int32_t)g;
                        ++nh;
                    }
                }
            }
            gnodes[g] = (a1 - a0) + nh;
            gtasks[g] = tasks_g;
        }
    });
    O.node_ptr.assign(G + 1, 0);
    O.groups.resize(G);
    int64_t T = 0;
    for (int64_t g = 0; g < G; ++g) {
        O.node_ptr[g + 1] = O.node_ptr[g] + gnodes[g];
        O.groups[g] = {(int32_t)T, gtasks[g], gstart[g], gstart[g + 1] - gstart[g]};
        T += gtasks[g];
    }
    O.nodes.resize(O.node_ptr[G]);
    O.nphase.assign(G, 0);
    O.tk_elem.resize(T);
    O.tk_ln.assign((size_t)T * O.ln_stride, 0);
    O.tk_off.assign((size_t)T * O.off_stride, 0);
    O.tk_phase.resize(T);
    std::vector<int32_t> gimg(G);
    run([&](int t) {
        std::vector<int32_t> lidx(N, -1);   // node -> local index in the current group
        std::vector<int32_t> elems, est(E, -1);
        std::vector<uint8_t> pos;             // [owned row][local node]: position in the row
        std::vector<uint64_t> used;
        struct Tk {
            int32_t e;
            uint8_t ph, off[36];
            OwnLn ln[8];
        };
        std::vector<Tk> tk;
        std::vector<int32_t> cnt, wcnt, wfill, wof;
        for (int64_t g = t; g < G; g += nt) {
            const int32_t a0 = gstart[g], a1 = gstart[g + 1], nr = a1 - a0;
            int32_t *gn = O.nodes.data() + O.node_ptr[g];
            const int32_t T_g = gnodes[g];
            group_elems(g, elems, est);
            for (int32_t r = a0; r < a1; ++r) gn[r - a0] = r;
            int32_t nh = nr;
            for (int32_t e : elems)
                for (int b = 0; b < nen; ++b) {
                    const int32_t v = conn[(int64_t)e * nen + b];
                    if ((v < a0 || v >= a1) && lidx[v] != -2) {
                        lidx[v] = -2;   // mark: collected once
                        gn[nh++] = v;
                    }
                }
            std::sort(gn + nr, gn + nh);
            if (nh != T_g || T_g > kOwnNodes) gbad[g] = 1;
            for (int32_t k = 0; k < nh; ++k) lidx[gn[k]] = k;
            // in-row position of every touched node for each owned row
            pos.assign((size_t)nr * T_g, 0xff);
            for (int32_t r = a0; r < a1; ++r)
                for (int32_t q = rowptr[r]; q < rowptr[r + 1]; ++q) {
                    const int32_t lc = lidx[colidx[q]];
                    if (lc < 0 || lc >= T_g) {
                        gbad[g] = 1;
                        continue;
                    }
                    pos[(size_t)(r - a0) * T_g + lc] = (uint8_t)(q - rowptr[r]);
                }
            gimg[g] = rowptr[a1] - rowptr[a0];
            used.assign(4 * (size_t)nr, 0);
            tk.clear();
            int nph = 0;
            auto add_task = [&](int32_t e, const int *rot) {
                Tk x{};
                x.e = e;
                for (int b = 0; b < nen; ++b) x.ln[b] = (OwnLn)lidx[conn[(int64_t)e * nen + (rot ? rot[b] : b)]];
                for (int r = 0; r < O.ra; ++r) {
                    if (x.ln[r] >= nr) continue;   // a row another group owns
                    const uint8_t *pr = pos.data() + (size_t)x.ln[r] * T_g;
                    for (int b = 0; b < nen; ++b) {
                        const uint8_t o = pr[x.ln[b]];
                        if (o == 0xff) gbad[g] = 1;
                        x.off[r * nen + b] = o;
                    }
                }
                tk.push_back(x);
            };
            // greedy phase: the smallest one none of the task's owned rows has
            // taken (among the tasks sharing its accumulation copy)
            auto take_phase = [&](Tk &x) {
                uint64_t m[4] = {0, 0, 0, 0};
                for (int r = 0; r < O.ra; ++r)
                    if (x.ln[r] < nr)
                        for (int w = 0; w < 4; ++w) m[w] |= used[4 * (size_t)x.ln[r] + w];
                int ph = 0;
                while (ph < 256 && ((m[ph >> 6] >> (ph & 63)) & 1)) ++ph;
                if (ph >= 256) {   // cannot happen: a group holds at most 256 tasks
                    gbad[g] = 1;
                    ph = 255;
                }
                for (int r = 0; r < O.ra; ++r)
                    if (x.ln[r] < nr) used[4 * (size_t)x.ln[r] + (ph >> 6)] |= 1ull << (ph & 63);
                x.ph = (uint8_t)ph;
                nph = std::max(nph, ph + 1);
            };
            for (int32_t e : elems) {
                const uint8_t m = owned_mask(e, a0, a1);
                if (!hex) {
                    add_task(e, nullptr);
                } else if (cover[m] == 1) {
                    int f = 0;
                    while ((m & ~fmask[f]) != 0) ++f;
                    add_task(e, kHexFaceRot[f]);
                } else {
                    add_task(e, kHexFaceRot[0]);
                    add_task(e, kHexFaceRot[1]);
                }
            }
            if ((int32_t)tk.size() != gtasks[g] || (int)tk.size() > kOwnTasks) gbad[g] = 1;
            if (O.wave_private) {
                // spread each row's tasks over the waves: a task goes to the
                // wave (with room) where its owned rows have the fewest tasks
                // yet, which bounds the phases each wave steps through
                const int nw = (int)((tk.size() + 63) / 64);
                wcnt.assign((size_t)nw * nr, 0);
                wfill.assign(nw, 0);
                wof.resize(tk.size());
                // every wave but the last holds exactly 64 tasks (a task's
                // wave is its lane / 64 in the kernel)
                auto cap = [&](int w) { return w < nw - 1 ? 64 : (int)tk.size() - 64 * (nw - 1); };
                for (size_t q = 0; q < tk.size(); ++q) {
                    int best = -1, bcost = 1 << 30;
                    for (int w = 0; w < nw; ++w) {
                        if (wfill[w] >= cap(w)) continue;
                        int c = 0;
                        for (int r = 0; r < O.ra; ++r)
                            if (tk[q].ln[r] < nr) c = std::max(c, wcnt[(size_t)w * nr + tk[q].ln[r]]);
                        if (c < bcost) {
                            bcost = c;
                            best = w;
                        }
                    }
                    wof[q] = best;
                    ++wfill[best];
                    for (int r = 0; r < O.ra; ++r)
                        if (tk[q].ln[r] < nr) ++wcnt[(size_t)best * nr + tk[q].ln[r]];
                }
                std::vector<Tk> by;   // tasks wave by wave, each wave in generation order
                for (int w = 0; w < nw; ++w) {
                    used.assign(4 * (size_t)nr, 0);
                    for (size_t q = 0; q < tk.size(); ++q)
                        if (wof[q] == w) {
                            take_phase(tk[q]);
                            by.push_back(tk[q]);
                        }
                }
                tk.swap(by);
            } else {
                for (Tk &x : tk) take_phase(x);
            }
            // tasks by phase, stably (a counting sort), over the group or,
            // wave-private, within each wave's 64: a wave then spans few
            // phases and skips the others' LDS additions
            const int64_t t0 = O.groups[g].first_task;
            const size_t span = O.wave_private ? 64 : tk.size() + 1;
            for (size_t w0 = 0; w0 < tk.size(); w0 += span) {
                const size_t w1 = std::min(tk.size(), w0 + span);
                cnt.assign(nph + 1, 0);
                for (size_t q = w0; q < w1; ++q) ++cnt[tk[q].ph + 1];
                for (int p = 0; p < nph; ++p) cnt[p + 1] += cnt[p];
                for (size_t q = w0; q < w1; ++q) {
                    const Tk &x = tk[q];
                    const int64_t d = t0 + (int64_t)w0 + cnt[x.ph]++;
                    if (d >= t0 + gtasks[g]) {
                        gbad[g] = 1;
                        continue;
                    }
                    O.tk_elem[d] = x.e;
                    O.tk_phase[d] = x.ph;
                    memcpy(&O.tk_ln[(size_t)d * O.ln_stride], x.ln, O.ln_stride * sizeof(OwnLn));
                    memcpy(&O.tk_off[(size_t)d * O.off_stride], x.off, O.off_stride);
                }
            }
            if (nph > 255) gbad[g] = 1;   // phase counts are stored in a byte
            O.nphase[g] = (uint8_t)nph;
            for (int32_t k = 0; k < nh; ++k) lidx[gn[k]] = -1;
        }
    });
    for (int64_t g = 0; g < G; ++g) {
        if (gbad[g]) {
            err = "owner plan: group " + std::to_string(g) + " exceeds its limits";
            return FE_EBADMESH;
        }
        O.max_nodes = std::max<int>(O.max_nodes, gnodes[g]);
        O.max_img = std::max(O.max_img, gimg[g]);
        O.max_rows = std::max<int>(O.max_rows, gstart[g + 1] - gstart[g]);
        O.max_phase = std::max<int>(O.max_phase, O.nphase[g]);
    }
    return FE_OK;
}

}  // namespace feasm
