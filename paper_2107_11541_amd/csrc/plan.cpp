// plan.cpp -- host preprocessing: renumbering, CSR pattern, blocks, colours.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "../../include/feasm.h"

namespace feasm {

static thread_local int t_thread_budget = 0;

void set_thread_budget(int n) { t_thread_budget = n; }

int host_threads()
{
    if (t_thread_budget > 0) return t_thread_budget;
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return (int)std::min(h, 16u);
}

// Run f(lo, hi) over [0, n) in contiguous chunks on host threads.
template <class F>
static void parallel_for(int64_t n, F f)
{
    int nt = host_threads();
    if (n < 4096 || nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([=, &f] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

static inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// Element order along a Morton curve of the centroids (ties: user order).
static void morton_order(int nen, int64_t N, const double *coords, int64_t E, const int32_t *conn,
                         std::vector<int32_t> &order)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], coords[i * 3 + d]);
            hi[d] = std::max(hi[d], coords[i * 3 + d]);
        }
    std::vector<uint64_t> key(E);
    parallel_for(E, [&](int64_t a, int64_t b) {
        for (int64_t e = a; e < b; ++e) {
            uint64_t k = 0;
            for (int d = 0; d < 3; ++d) {
                double c = 0.0;
                for (int j = 0; j < nen; ++j) c += coords[(int64_t)conn[e * nen + j] * 3 + d];
                c /= nen;
                double span = hi[d] - lo[d];
                double t = span > 0 ? (c - lo[d]) / span : 0.0;
                uint64_t q = (uint64_t)std::min(std::max(t * 2097151.0, 0.0), 2097151.0);
                k |= spread3(q) << d;
            }
            key[e] = k;
        }
    });
    order.resize(E);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
}

// CSR pattern in mesh numbering: row i = sorted unique nodes of the elements
// containing i.  Two passes (count, fill), parallel over rows.
static void build_pattern(Plan &P)
{
    const int nen = P.nen;
    const int64_t N = P.N, E = P.E;
    std::vector<int64_t> ip(N + 1, 0);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nen; ++a) ip[P.conn[e * nen + a] + 1]++;
    for (int64_t i = 0; i < N; ++i) ip[i + 1] += ip[i];
    std::vector<int32_t> inc(ip[N]);
    {
        std::vector<int64_t> fill(ip.begin(), ip.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nen; ++a) inc[fill[P.conn[e * nen + a]]++] = (int32_t)e;
    }
    std::vector<int32_t> len(N);
    auto row = [&](int64_t i, std::vector<int32_t> &buf) {
        buf.clear();
        for (int64_t k = ip[i]; k < ip[i + 1]; ++k) {
            const int32_t *c = &P.conn[(int64_t)inc[k] * nen];
            buf.insert(buf.end(), c, c + nen);
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    parallel_for(N, [&](int64_t a, int64_t b) {
        std::vector<int32_t> buf;
        for (int64_t i = a; i < b; ++i) {
            row(i, buf);
            len[i] = (int32_t)buf.size();
        }
    });
    P.rowptr.assign(N + 1, 0);
    int64_t s = 0;
    int mx = 0;
    for (int64_t i = 0; i < N; ++i) {
        P.rowptr[i] = (int32_t)s;
        s += len[i];
        mx = std::max(mx, len[i]);
    }
    P.rowptr[N] = (int32_t)s;
    P.nnz = s;
    P.max_row = mx;
    P.colidx.assign(s, 0);
    P.diagpos.assign(N, 0);
    parallel_for(N, [&](int64_t a, int64_t b) {
        std::vector<int32_t> buf;
        for (int64_t i = a; i < b; ++i) {
            row(i, buf);
            std::copy(buf.begin(), buf.end(), P.colidx.begin() + P.rowptr[i]);
            P.diagpos[i] = P.rowptr[i] + (int32_t)(std::lower_bound(buf.begin(), buf.end(), (int32_t)i) - buf.begin());
        }
    });
}

static inline int64_t slot_in_row(const Plan &P, int32_t i, int32_t j)
{
    const int32_t *b = P.colidx.data() + P.rowptr[i], *e = P.colidx.data() + P.rowptr[i + 1];
    const int32_t *p = std::lower_bound(b, e, j);
    return (p != e && *p == j) ? (p - b) : -1;
}

int build_plan(int nen, int64_t N, const double *coords, int64_t E, const int32_t *conn, bool renumber,
               Plan &P, std::string &err)
{
    if ((nen != 4 && nen != 8) || N <= 0 || E <= 0 || !coords || !conn) {
        err = "invalid mesh arguments";
        return FE_EINVAL;
    }
    if (N >= (int64_t)1 << 31 || E >= (int64_t)1 << 31) {
        err = "mesh too large for int32 ids";
        return FE_EINVAL;
    }
    for (int64_t k = 0; k < E * nen; ++k)
        if (conn[k] < 0 || conn[k] >= N) {
            err = "connectivity entry " + std::to_string(k) + " out of range";
            return FE_EBADMESH;
        }
    P = Plan();
    P.nen = nen;
    P.N = N;
    P.E = E;

    // 1. element order
    if (renumber) {
        morton_order(nen, N, coords, E, conn, P.elem_perm);
    } else {
        P.elem_perm.resize(E);
        std::iota(P.elem_perm.begin(), P.elem_perm.end(), 0);
    }
    // 2. node order: first touch along the element order (or identity)
    P.node_iperm.assign(N, -1);
    P.node_perm.assign(N, -1);
    if (renumber) {
        int32_t next = 0;
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nen; ++a) {
                int32_t v = conn[(int64_t)P.elem_perm[e] * nen + a];
                if (P.node_iperm[v] < 0) {
                    P.node_iperm[v] = next;
                    P.node_perm[next] = v;
                    ++next;
                }
            }
        if (next != N) {
            err = "mesh has nodes that belong to no element";
            return FE_EBADMESH;
        }
    } else {
        std::vector<char> used(N, 0);
        for (int64_t k = 0; k < E * nen; ++k) used[conn[k]] = 1;
        for (int64_t i = 0; i < N; ++i) {
            if (!used[i]) {
                err = "node " + std::to_string(i) + " belongs to no element";
                return FE_EBADMESH;
            }
            P.node_iperm[i] = (int32_t)i;
            P.node_perm[i] = (int32_t)i;
        }
    }
    P.conn.resize(E * nen);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nen; ++a) P.conn[e * nen + a] = P.node_iperm[conn[(int64_t)P.elem_perm[e] * nen + a]];
    P.X.resize(3 * N);
    for (int64_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) P.X[d * N + i] = coords[(int64_t)P.node_perm[i] * 3 + d];

    // 3. CSR pattern
    build_pattern(P);
    if (P.max_row > kMaxRow) {
        err = "a CSR row has " + std::to_string(P.max_row) + " entries (limit 255)";
        return FE_EBADMESH;
    }

    // 4. blocks: consecutive elements, <= 64, LDS image within budget
    const int nn2 = nen * nen;
    std::vector<int32_t> stamp(N, -1), local(N, 0);
    P.blk_elem_ptr.push_back(0);
    P.blk_node_ptr.push_back(0);
    {
        std::vector<int32_t> cur;  // touched nodes of the open block
        int64_t L = 0;
        int32_t bid = 0;
        auto lds_bytes = [&](int64_t T, int64_t Limg) {
            return (T * (kNodeFields + kMaxRhs)) * 8 + T * 4 + 8 + Limg * 8;
        };
        auto close_block = [&](int64_t e_end) {
            std::sort(cur.begin(), cur.end());
            P.blk_nodes.insert(P.blk_nodes.end(), cur.begin(), cur.end());
            P.blk_elem_ptr.push_back((int32_t)e_end);
            P.blk_node_ptr.push_back((int32_t)P.blk_nodes.size());
            P.max_T = std::max<int>(P.max_T, (int)cur.size());
            P.max_L = std::max<int>(P.max_L, (int)L);
            cur.clear();
            L = 0;
            ++bid;
        };
        int64_t start = 0;
        for (int64_t e = 0; e < E; ++e) {
            int newT = 0;
            int64_t newL = 0;
            for (int a = 0; a < nen; ++a) {
                int32_t v = P.conn[e * nen + a];
                if (stamp[v] != bid) {
                    bool dup = false;
                    for (int b = 0; b < a; ++b) dup |= (P.conn[e * nen + b] == v);
                    if (!dup) {
                        ++newT;
                        newL += P.rowptr[v + 1] - P.rowptr[v];
                    }
                }
            }
            if (e > start && (e - start >= kBlockElems ||
                              lds_bytes((int64_t)cur.size() + newT, L + newL) > kLdsBudget)) {
                close_block(e);
                start = e;
                newT = 0;
                newL = 0;
                for (int a = 0; a < nen; ++a) {
                    int32_t v = P.conn[e * nen + a];
                    bool dup = false;
                    for (int b = 0; b < a; ++b) dup |= (P.conn[e * nen + b] == v);
                    if (!dup) newL += P.rowptr[v + 1] - P.rowptr[v];
                }
            }
            for (int a = 0; a < nen; ++a) {
                int32_t v = P.conn[e * nen + a];
                if (stamp[v] != bid) {
                    stamp[v] = bid;
                    cur.push_back(v);
                    L += P.rowptr[v + 1] - P.rowptr[v];
                }
            }
            if (lds_bytes((int64_t)cur.size(), L) > kLdsBudget) {
                err = "one element's rows exceed the LDS budget";
                return FE_EBADMESH;
            }
        }
        close_block(E);
    }
    const int64_t nblk = P.n_blocks();

    // 5. per element: local rows, in-row offsets, phases
    P.elem_lnode.assign(nen * E, 0);
    P.elem_off.assign(E * nn2, 0);
    P.elem_phase.assign(E, 0);
    P.blk_nphase.assign(nblk, 1);
    std::atomic<int> bad{0};
    std::atomic<int> maxph{1};
    parallel_for(nblk, [&](int64_t b0, int64_t b1) {
        std::vector<uint64_t> used;   // [T][nen] phase masks
        for (int64_t b = b0; b < b1; ++b) {
            const int32_t *nb = P.blk_nodes.data() + P.blk_node_ptr[b];
            const int T = P.blk_node_ptr[b + 1] - P.blk_node_ptr[b];
            used.assign((size_t)T * nen, 0);
            int nph = 1;
            for (int64_t e = P.blk_elem_ptr[b]; e < P.blk_elem_ptr[b + 1]; ++e) {
                int ln[8];
                for (int a = 0; a < nen; ++a) {
                    int32_t v = P.conn[e * nen + a];
                    ln[a] = (int)(std::lower_bound(nb, nb + T, v) - nb);
                    P.elem_lnode[(int64_t)a * E + e] = (uint16_t)ln[a];
                }
                uint64_t m = 0;
                for (int a = 0; a < nen; ++a) m |= used[(size_t)ln[a] * nen + a];
                int ph = 0;
                while (ph < 64 && ((m >> ph) & 1)) ++ph;
                if (ph >= 64) { bad = 1; ph = 63; }
                for (int a = 0; a < nen; ++a) used[(size_t)ln[a] * nen + a] |= (1ull << ph);
                P.elem_phase[e] = (uint8_t)ph;
                nph = std::max(nph, ph + 1);
                for (int a = 0; a < nen; ++a)
                    for (int c = 0; c < nen; ++c) {
                        int64_t s = slot_in_row(P, P.conn[e * nen + a], P.conn[e * nen + c]);
                        if (s < 0) bad = 1;
                        P.elem_off[e * nn2 + a * nen + c] = (uint8_t)s;
                    }
            }
            P.blk_nphase[b] = (uint8_t)nph;
            int cur = maxph.load();
            while (nph > cur && !maxph.compare_exchange_weak(cur, nph)) {}
        }
    });
    if (bad) {
        err = "internal: scatter plan construction failed";
        return FE_EBADMESH;
    }
    P.max_phase = maxph;

    // 6. block colouring: blocks sharing a node get different colours
    {
        std::vector<int64_t> np(N + 1, 0);
        for (int32_t v : P.blk_nodes) np[v + 1]++;
        for (int64_t i = 0; i < N; ++i) np[i + 1] += np[i];
        std::vector<int32_t> nblks(np[N]);
        {
            std::vector<int64_t> fill(np.begin(), np.end() - 1);
            for (int64_t b = 0; b < nblk; ++b)
                for (int32_t k = P.blk_node_ptr[b]; k < P.blk_node_ptr[b + 1]; ++k)
                    nblks[fill[P.blk_nodes[k]]++] = (int32_t)b;
        }
        P.blk_color.assign(nblk, -1);
        std::vector<int64_t> seen;   // colour -> last block that saw it
        int ncol = 0;
        for (int64_t b = 0; b < nblk; ++b) {
            for (int32_t k = P.blk_node_ptr[b]; k < P.blk_node_ptr[b + 1]; ++k) {
                int32_t v = P.blk_nodes[k];
                for (int64_t q = np[v]; q < np[v + 1]; ++q) {
                    int c = P.blk_color[nblks[q]];
                    if (c >= 0) {
                        if ((int)seen.size() <= c) seen.resize(c + 1, -1);
                        seen[c] = b;
                    }
                }
            }
            int c = 0;
            while (c < (int)seen.size() && seen[c] == b) ++c;
            P.blk_color[b] = c;
            ncol = std::max(ncol, c + 1);
        }
        P.n_colors = ncol;
        P.color_ptr.assign(ncol + 1, 0);
        for (int64_t b = 0; b < nblk; ++b) P.color_ptr[P.blk_color[b] + 1]++;
        for (int c = 0; c < ncol; ++c) P.color_ptr[c + 1] += P.color_ptr[c];
        P.color_blk.resize(nblk);
        std::vector<int32_t> fill(P.color_ptr.begin(), P.color_ptr.end() - 1);
        for (int64_t b = 0; b < nblk; ++b) P.color_blk[fill[P.blk_color[b]]++] = (int32_t)b;
    }

    // 7. row descriptors: image offset, length and first-writer flag (launch
    //    order = colour order), and the CSR start of every touched row
    P.blk_rdesc.assign(P.blk_nodes.size(), 0);
    P.blk_rowstart.assign(P.blk_nodes.size(), 0);
    {
        std::vector<char> written(N, 0);
        for (int64_t q = 0; q < nblk; ++q) {
            int32_t b = P.color_blk[q];
            int32_t off = 0;
            for (int32_t k = P.blk_node_ptr[b]; k < P.blk_node_ptr[b + 1]; ++k) {
                int32_t v = P.blk_nodes[k];
                const int32_t len = P.rowptr[v + 1] - P.rowptr[v];
                uint32_t w = (uint32_t)off | ((uint32_t)len << 16);
                if (!written[v]) {
                    written[v] = 1;
                    w |= kFirstBit;
                }
                P.blk_rdesc[k] = (int32_t)w;
                P.blk_rowstart[k] = P.rowptr[v];
                off += len;
            }
            if (off >= (1 << 16)) {
                err = "internal: block image exceeds 65536 entries";
                return FE_EBADMESH;
            }
        }
    }
    return FE_OK;
}

}  // namespace feasm
