// plan.cpp -- host preprocessing: renumbering, CSR pattern, blocks, colours.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
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

int parallel_workers(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n));
}

void parallel_chunks_w(int64_t n, const std::function<void(int64_t, int)> &f)
{
    const int nt = parallel_workers(n);
    if (nt <= 1) {
        for (int64_t c = 0; c < n; ++c) f(c, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    auto run = [&](int w) {
        for (int64_t c = next.fetch_add(1); c < n; c = next.fetch_add(1)) f(c, w);
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(run, t);
    run(0);
    for (auto &x : th) x.join();
}

void parallel_chunks(int64_t n, const std::function<void(int64_t)> &f)
{
    parallel_chunks_w(n, [&](int64_t c, int) { f(c); });
}

// Sorts idx by less, a strict total order (so the result does not depend on
// how the work is split): runs sorted in parallel, then merged pairwise.
template <class Less>
static void parallel_sort(std::vector<int32_t> &idx, Less less)
{
    const int64_t n = (int64_t)idx.size();
    int parts = 1;
    while (parts < host_threads() && n / (2 * parts) >= 32768) parts *= 2;
    if (parts == 1) {
        std::sort(idx.begin(), idx.end(), less);
        return;
    }
    std::vector<int64_t> b(parts + 1);
    for (int k = 0; k <= parts; ++k) b[k] = n * k / parts;
    parallel_chunks(parts, [&](int64_t k) { std::sort(idx.begin() + b[k], idx.begin() + b[k + 1], less); });
    std::vector<int32_t> buf(n);
    for (int w = 1; w < parts; w *= 2) {
        parallel_chunks(parts / (2 * w), [&](int64_t q) {
            const int64_t lo = b[2 * w * q], mid = b[2 * w * q + w], hi = b[2 * w * q + 2 * w];
            std::merge(idx.begin() + lo, idx.begin() + mid, idx.begin() + mid, idx.begin() + hi, buf.begin() + lo,
                       less);
        });
        idx.swap(buf);
    }
}

void Plan::clear()
{
    nen = off_stride = 0;
    N = E = nnz = 0;
    max_row = n_colors = max_T = max_L = max_phase = 0;
    for (auto *v : {&node_perm, &node_iperm, &elem_perm, &conn, &rowptr, &colidx, &diagpos, &blk_elem_ptr,
                    &blk_node_ptr, &blk_nodes, &blk_img, &blk_rdesc, &blk_rowstart, &blk_color, &color_ptr,
                    &color_blk})
        v->clear();
    for (auto *v : {&etype, &blk_nphase, &elem_off, &blk_nen, &elem_phase}) v->clear();
    X.clear();
    elem_lnode.clear();
    segs.clear();
}

// Temporaries of one planning call, kept per calling thread (see
// kPlanScratchKeep).
struct PlanScratch {
    std::vector<uint64_t> key;             // Morton keys
    std::vector<int64_t> ip, np;           // node -> incident elements / blocks (offsets)
    std::vector<int32_t> inc, len, nblks;  // the lists, row lengths
    std::vector<std::vector<int32_t>> cols;   // pattern rows of each thread's range
    std::vector<std::vector<int32_t>> mark;   // per worker: node -> the last row / block that took it
    std::vector<std::vector<uint8_t>> pos;    // per worker: node -> its position in that row
    size_t bytes() const
    {
        size_t b = key.capacity() * 8 + ip.capacity() * 8 + np.capacity() * 8 +
                   (inc.capacity() + len.capacity() + nblks.capacity()) * 4;
        for (const auto &c : cols) b += c.capacity() * 4;
        for (const auto &c : mark) b += c.capacity() * 4;
        for (const auto &c : pos) b += c.capacity();
        return b;
    }
};
static thread_local PlanScratch t_scratch;

static void release_scratch_if_large()
{
    if (t_scratch.bytes() > kPlanScratchKeep) t_scratch = PlanScratch();
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

// Element order along a Morton curve of the centroids (ties: user order);
// with several element types, grouped by type first (type_rank).
static void morton_order(int S, const uint8_t *types, int64_t N, const double *coords, int64_t E,
                         const int32_t *conn, std::vector<int32_t> &order)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], coords[i * 3 + d]);
            hi[d] = std::max(hi[d], coords[i * 3 + d]);
        }
    std::vector<uint64_t> &key = t_scratch.key;
    key.resize(E);
    parallel_for(E, [&](int64_t a, int64_t b) {
        for (int64_t e = a; e < b; ++e) {
            const int nen = types ? types[e] : S;
            uint64_t k = 0;
            for (int d = 0; d < 3; ++d) {
                double c = 0.0;
                for (int j = 0; j < nen; ++j) c += coords[(int64_t)conn[e * S + j] * 3 + d];
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
    // ties keep the user order
    if (types) {
        parallel_sort(order, [&](int32_t a, int32_t b) {
            const int ra = type_rank(types[a]), rb = type_rank(types[b]);
            if (ra != rb) return ra < rb;
            return key[a] != key[b] ? key[a] < key[b] : a < b;
        });
    } else {
        parallel_sort(order, [&](int32_t a, int32_t b) { return key[a] != key[b] ? key[a] < key[b] : a < b; });
    }
}

// CSR pattern in mesh numbering: row i = sorted unique nodes of the elements
// containing i.  One pass over the rows, parallel over row ranges: a row's
// candidates (nen per incident element) are de-duplicated in a 512-slot
// open-addressing table and the survivors (<= max row length) are sorted by
// insertion; each range writes its rows to a buffer of its own, then the
// buffers are concatenated behind the row pointers.  The same pass fills the
// scatter offsets: with the row sorted, the table maps each column to its
// position, and every incident element e (node i at local position a) gets
// elem_off[e][a][c] = position of its node c in row i.  Element e has n_e
// nodes (its type) and its connectivity at stride S.
static void build_pattern(Plan &P)
{
    const int S = P.nen;
    const int64_t N = P.N, E = P.E;
    const uint8_t *ty = P.etype.empty() ? nullptr : P.etype.data();
    auto nen_of = [&](int64_t e) { return ty ? (int)ty[e] : S; };
    // node -> incident elements, ascending (an element repeating a node
    // appears once per repeat): counted and filled in parallel, then each
    // list sorted
    std::vector<int64_t> &ip = t_scratch.ip;
    std::vector<int32_t> &inc = t_scratch.inc;
    ip.assign(N + 1, 0);
    if (host_threads() <= 1 || E < 65536) {
        // one thread: counted and filled in element order (ascending as is)
        for (int64_t e = 0; e < E; ++e)
            for (int q = 0; q < nen_of(e); ++q) ip[P.conn[e * S + q] + 1]++;
        for (int64_t i = 0; i < N; ++i) ip[i + 1] += ip[i];
        inc.resize(ip[N]);
        std::vector<int64_t> fill(ip.begin(), ip.end() - 1);
        for (int64_t e = 0; e < E; ++e)
            for (int q = 0; q < nen_of(e); ++q) inc[fill[P.conn[e * S + q]]++] = (int32_t)e;
    } else {
        std::unique_ptr<std::atomic<int32_t>[]> cnt(new std::atomic<int32_t>[N]);
        parallel_for(N, [&](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i) cnt[i].store(0, std::memory_order_relaxed);
        });
        parallel_for(E, [&](int64_t a, int64_t b) {
            for (int64_t e = a; e < b; ++e)
                for (int q = 0; q < nen_of(e); ++q) cnt[P.conn[e * S + q]].fetch_add(1, std::memory_order_relaxed);
        });
        for (int64_t i = 0; i < N; ++i) {
            ip[i + 1] = ip[i] + cnt[i].load(std::memory_order_relaxed);
            cnt[i].store(0, std::memory_order_relaxed);
        }
        inc.resize(ip[N]);
        parallel_for(E, [&](int64_t a, int64_t b) {
            for (int64_t e = a; e < b; ++e)
                for (int q = 0; q < nen_of(e); ++q) {
                    const int32_t v = P.conn[e * S + q];
                    inc[ip[v] + cnt[v].fetch_add(1, std::memory_order_relaxed)] = (int32_t)e;
                }
        });
        cnt.reset();
        parallel_for(N, [&](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i) {
                int32_t *l = inc.data() + ip[i];
                const int64_t d = ip[i + 1] - ip[i];
                for (int64_t x = 1; x < d; ++x) {   // insertion sort: lists are short, mostly ascending
                    const int32_t v = l[x];
                    int64_t y = x;
                    while (y > 0 && l[y - 1] > v) {
                        l[y] = l[y - 1];
                        --y;
                    }
                    l[y] = v;
                }
            }
        });
    }
    std::vector<int32_t> &len = t_scratch.len;
    len.resize(N);
    const int OS = P.off_stride;
    P.elem_off.assign((size_t)E * OS, 0);
    const int nt = std::max(1, (int)std::min<int64_t>(host_threads(), (N + 4095) / 4096));
    const int64_t chunk = (N + nt - 1) / nt;
    std::vector<std::vector<int32_t>> &cols = t_scratch.cols;
    if ((int)cols.size() < nt) cols.resize(nt);
    for (auto &c : cols) c.clear();
    std::atomic<bool> overflow{false};
    // (the workers run on threads of their own: they reach the caller's
    // scratch only through these references)
    std::vector<std::vector<int32_t>> &marks = t_scratch.mark;
    std::vector<std::vector<uint8_t>> &poss = t_scratch.pos;
    if ((int)marks.size() < nt) marks.resize(nt);
    if ((int)poss.size() < nt) poss.resize(nt);
    auto work = [&](int t) {
        const int64_t lo = t * chunk, hi = std::min(N, lo + chunk);
        std::vector<int32_t> &out = cols[t];
        out.reserve((size_t)std::max<int64_t>(0, hi - lo) * 27);
        // a column is new to row i while mark[v] != i; pos[v] is its place
        // in the sorted row (so the scatter offsets are one lookup each)
        std::vector<int32_t> &mark = marks[t];
        std::vector<uint8_t> &pos = poss[t];
        mark.assign(N, -1);
        pos.resize(N);
        constexpr int kMaxCols = 256;   // one past the longest admissible row
        int32_t tmp[kMaxCols + 1];      // columns in first-touch order (+1: a non-fresh store at the end)
        int32_t rank[kMaxCols];
        std::vector<uint8_t> where;     // per incident element: bit a set where node a is the row's node
        for (int64_t i = lo; i < hi; ++i) {
            const size_t start = out.size();
            const int64_t deg = ip[i + 1] - ip[i];
            if ((int64_t)where.size() < deg) where.resize(deg);
            int nused = 0;
            for (int64_t k = 0; k < deg; ++k) {
                const int64_t ek = inc[ip[i] + k];
                const int32_t *c = &P.conn[ek * S];
                const int nen = nen_of(ek);
                uint32_t mk = 0;
                for (int a = 0; a < nen; ++a) {
                    const int32_t v = c[a];
                    mk |= (uint32_t)(v == (int32_t)i) << a;
                    // branch-free insert (whether a column is new is unpredictable)
                    const bool fresh = mark[v] != (int32_t)i;
                    if (fresh & (nused == kMaxCols)) {   // row longer than any admissible one
                        overflow = true;
                        continue;
                    }
                    mark[v] = (int32_t)i;
                    tmp[nused] = v;
                    nused += fresh;
                }
                where[k] = (uint8_t)mk;
            }
            const int n = nused;
            out.resize(start + n);
            int32_t *r = out.data() + start;
            len[i] = n;
            if (n <= 255) {   // longer rows are rejected by the caller
                // sort by rank: the columns are distinct, so the number of
                // smaller ones is each column's position (branch-free counting)
                for (int x = 0; x < n; ++x) {
                    const int32_t key = tmp[x];
                    int cnt = 0;
                    for (int y = 0; y < n; ++y) cnt += tmp[y] < key;
                    rank[x] = cnt;
                }
                for (int x = 0; x < n; ++x) {
                    r[rank[x]] = tmp[x];
                    pos[tmp[x]] = (uint8_t)rank[x];
                }
                int prev_a = -1;
                for (int64_t k = 0; k < deg; ++k) {
                    const int64_t e = inc[ip[i] + k];
                    const int nen = nen_of(e);
                    // the k-th occurrence of i in e (an element may repeat a
                    // node; its repeats are consecutive in inc)
                    uint32_t mk = where[k];
                    if (k > 0 && inc[ip[i] + k - 1] == e) mk &= ~((2u << prev_a) - 1);
                    const int a = mk ? __builtin_ctz(mk) : nen;
                    prev_a = a;
                    if (a == nen) continue;
                    uint8_t *off = &P.elem_off[(size_t)e * OS + (size_t)a * nen];
                    const int32_t *c = &P.conn[e * S];
                    for (int q = 0; q < nen; ++q) off[q] = pos[c[q]];
                }
            } else {
                std::copy(tmp, tmp + n, r);
                std::sort(r, r + n);
            }
        }
    };
    if (nt == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t) th.emplace_back(work, t);
        for (auto &x : th) x.join();
    }
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
    // a row reaching kSlots / 2 = 256 distinct nodes is over kMaxRow anyway
    P.max_row = overflow ? (1 << 30) : mx;
    P.colidx.reserve(s + 16);   // the device copy is padded later: no reallocation then
    P.colidx.resize(s);
    P.diagpos.assign(N, 0);
    parallel_for(nt, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t lo = t * chunk;
            if (lo >= N || cols[t].empty()) continue;
            std::copy(cols[t].begin(), cols[t].end(), P.colidx.begin() + P.rowptr[lo]);
        }
    });
    parallel_for(N, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            const int32_t *r0 = P.colidx.data() + P.rowptr[i], *r1 = P.colidx.data() + P.rowptr[i + 1];
            P.diagpos[i] = P.rowptr[i] + (int32_t)(std::lower_bound(r0, r1, (int32_t)i) - r0);
        }
    });
}

static int build_plan_impl(int S, const uint8_t *types, int64_t N, const double *coords, int64_t E,
                           const int32_t *conn, bool renumber, Plan &P, std::string &err)
{
    const bool typed_stride = types ? (S >= 4 && S <= 8) : (S == 4 || S == 5 || S == 6 || S == 8);
    if (!typed_stride || N <= 0 || E <= 0 || !coords || !conn) {
        err = "invalid mesh arguments";
        return FE_EINVAL;
    }
    if (N >= (int64_t)1 << 31 || E >= (int64_t)1 << 31) {
        err = "mesh too large for int32 ids";
        return FE_EINVAL;
    }
    auto nen_u = [&](int64_t e) { return types ? (int)types[e] : S; };
    bool one_type = true;
    int maxt = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int t = nen_u(e);
        if ((t != 4 && t != 5 && t != 6 && t != 8) || t > S) {
            err = "element " + std::to_string(e) + " has an unknown type (" + std::to_string(t) + " nodes)";
            return FE_EINVAL;
        }
        one_type &= t == nen_u(0);
        maxt = std::max(maxt, t);
        for (int a = 0; a < t; ++a)
            if (conn[e * S + a] < 0 || conn[e * S + a] >= N) {
                err = "connectivity entry " + std::to_string(e * S + a) + " out of range";
                return FE_EBADMESH;
            }
    }
    P.clear();
    P.nen = maxt;   // the plan's connectivity stride
    P.off_stride = (maxt * maxt + 3) & ~3;
    const int PS = maxt;
    P.N = N;
    P.E = E;

    // 1. element order (grouped by type when several are present)
    if (renumber) {
        morton_order(S, types, N, coords, E, conn, P.elem_perm);
    } else {
        P.elem_perm.resize(E);
        std::iota(P.elem_perm.begin(), P.elem_perm.end(), 0);
    }
    if (types && !one_type) {
        P.etype.resize(E);
        for (int64_t e = 0; e < E; ++e) P.etype[e] = types[P.elem_perm[e]];
    }
    auto nen_of = [&](int64_t e) { return P.etype.empty() ? PS : (int)P.etype[e]; };
    // 2. node order: first touch along the element order (or identity)
    P.node_iperm.assign(N, -1);
    P.node_perm.assign(N, -1);
    if (renumber) {
        int32_t next = 0;
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nen_of(e); ++a) {
                int32_t v = conn[(int64_t)P.elem_perm[e] * S + a];
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
        for (int64_t e = 0; e < E; ++e)
            for (int a = 0; a < nen_u(e); ++a) used[conn[e * S + a]] = 1;
        for (int64_t i = 0; i < N; ++i) {
            if (!used[i]) {
                err = "node " + std::to_string(i) + " belongs to no element";
                return FE_EBADMESH;
            }
            P.node_iperm[i] = (int32_t)i;
            P.node_perm[i] = (int32_t)i;
        }
    }
    // mesh connectivity; the unused slots of a short element repeat its first node
    P.conn.resize(E * PS);
    parallel_for(E, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t *c = conn + (int64_t)P.elem_perm[e] * S;
            const int t = nen_of(e);
            for (int a = 0; a < PS; ++a) P.conn[e * PS + a] = P.node_iperm[c[a < t ? a : 0]];
        }
    });
    P.X.resize(3 * N);
    parallel_for(N, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            for (int d = 0; d < 3; ++d) P.X[d * N + i] = coords[(int64_t)P.node_perm[i] * 3 + d];
    });

    // 3. CSR pattern
    build_pattern(P);
    if (P.max_row > kMaxRow) {
        err = "a CSR row has " + std::to_string(P.max_row) + " entries (limit 255)";
        return FE_EBADMESH;
    }

    // 4. blocks: consecutive elements of one type, <= 64, LDS image within
    //    budget, none across a kPlanElemChunk boundary (chunks in parallel)
    {
        auto lds_bytes = [&](int64_t T, int64_t Limg) {
            return (T * (kNodeFields + kMaxRhs)) * 8 + T * 4 + 8 + Limg * 8;
        };
        struct Chunk {
            std::vector<int32_t> eptr, nptr, nodes, img;   // per block: end element, end of its nodes, image
            int max_T = 0, max_L = 0;
            bool too_big = false;
        };
        const int64_t nchunk = (E + kPlanElemChunk - 1) / kPlanElemChunk;
        std::vector<Chunk> ch(nchunk);
        // a node is in the open block while mark[v] == its id (ids unique per
        // worker, so nothing is cleared between blocks)
        const int nw = parallel_workers(nchunk);
        std::vector<std::vector<int32_t>> &marks = t_scratch.mark;
        if ((int)marks.size() < nw) marks.resize(nw);
        std::vector<char> ready(nw, 0);
        std::vector<int32_t> next_id(nw, 0);
        parallel_chunks_w(nchunk, [&](int64_t c, int w) {
            Chunk &C = ch[c];
            const int64_t e0 = c * kPlanElemChunk, e1 = std::min(E, e0 + kPlanElemChunk);
            std::vector<int32_t> &mark = marks[w];
            if (!ready[w]) {
                mark.assign(N, -1);
                ready[w] = 1;
            }
            int32_t bid = next_id[w]++;
            std::vector<int32_t> cur;
            int64_t L = 0;
            auto close_block = [&](int64_t e_end) {
                std::sort(cur.begin(), cur.end());
                C.nodes.insert(C.nodes.end(), cur.begin(), cur.end());
                C.eptr.push_back((int32_t)e_end);
                C.nptr.push_back((int32_t)C.nodes.size());
                C.img.push_back((int32_t)L);
                C.max_T = std::max<int>(C.max_T, (int)cur.size());
                C.max_L = std::max<int>(C.max_L, (int)L);
                cur.clear();
                L = 0;
                bid = next_id[w]++;
            };
            int64_t start = e0;
            for (int64_t e = e0; e < e1; ++e) {
                const int nen = nen_of(e);
                const int32_t *ce = &P.conn[e * PS];
                int newT = 0;
                int64_t newL = 0;
                for (int a = 0; a < nen; ++a) {
                    const int32_t v = ce[a];
                    if (mark[v] != bid) {
                        bool dup = false;
                        for (int b = 0; b < a; ++b) dup |= (ce[b] == v);
                        if (!dup) {
                            ++newT;
                            newL += P.rowptr[v + 1] - P.rowptr[v];
                        }
                    }
                }
                if (e > start && (e - start >= kBlockElems || nen != nen_of(start) ||
                                  lds_bytes((int64_t)cur.size() + newT, L + newL) > kLdsBudget)) {
                    close_block(e);
                    start = e;
                }
                for (int a = 0; a < nen; ++a) {
                    const int32_t v = ce[a];
                    if (mark[v] != bid) {
                        mark[v] = bid;
                        cur.push_back(v);
                        L += P.rowptr[v + 1] - P.rowptr[v];
                    }
                }
                if (lds_bytes((int64_t)cur.size(), L) > kLdsBudget) {
                    C.too_big = true;
                    return;
                }
            }
            close_block(e1);
        });
        P.blk_elem_ptr.assign(1, 0);
        P.blk_node_ptr.assign(1, 0);
        for (const Chunk &C : ch) {
            if (C.too_big) {
                err = "one element's rows exceed the LDS budget";
                return FE_EBADMESH;
            }
            const int32_t base = (int32_t)P.blk_nodes.size();
            P.blk_nodes.insert(P.blk_nodes.end(), C.nodes.begin(), C.nodes.end());
            for (size_t k = 0; k < C.eptr.size(); ++k) {
                P.blk_elem_ptr.push_back(C.eptr[k]);
                P.blk_node_ptr.push_back(base + C.nptr[k]);
            }
            P.blk_img.insert(P.blk_img.end(), C.img.begin(), C.img.end());
            P.max_T = std::max(P.max_T, C.max_T);
            P.max_L = std::max(P.max_L, C.max_L);
        }
    }
    const int64_t nblk = P.n_blocks();

    // 5. per element: local rows, in-row offsets, phases
    P.elem_lnode.assign((size_t)PS * E, 0);
    P.elem_phase.assign(E, 0);
    P.blk_nphase.assign(nblk, 1);
    P.blk_nen.assign(nblk, (uint8_t)PS);
    for (int64_t b = 0; b < nblk; ++b) P.blk_nen[b] = (uint8_t)nen_of(P.blk_elem_ptr[b]);
    std::atomic<int> bad{0};
    std::atomic<int> maxph{1};
    parallel_for(nblk, [&](int64_t b0, int64_t b1) {
        std::vector<uint64_t> used;   // [T][nen] phase masks
        // node -> local row of the current block: open addressing over
        // 1024 slots (a block touches far fewer nodes, the LDS budget caps it)
        constexpr int kSlots = 1024;
        std::vector<int32_t> key(kSlots, -1);
        std::vector<uint16_t> val(kSlots, 0);
        auto hslot = [](int32_t v) { return ((uint32_t)v * 2654435761u) >> 22; };
        for (int64_t b = b0; b < b1; ++b) {
            const int32_t *nb = P.blk_nodes.data() + P.blk_node_ptr[b];
            const int T = P.blk_node_ptr[b + 1] - P.blk_node_ptr[b];
            if (T >= kSlots) {
                bad = 1;
                continue;
            }
            for (int k = 0; k < T; ++k) {
                uint32_t h = hslot(nb[k]);
                while (key[h] != -1) h = (h + 1) & (kSlots - 1);
                key[h] = nb[k];
                val[h] = (uint16_t)k;
            }
            const int nen = P.blk_nen[b];
            used.assign((size_t)T * nen, 0);
            int nph = 1;
            for (int64_t e = P.blk_elem_ptr[b]; e < P.blk_elem_ptr[b + 1]; ++e) {
                int ln[8];
                for (int a = 0; a < nen; ++a) {
                    int32_t v = P.conn[e * PS + a];
                    uint32_t h = hslot(v);
                    while (key[h] != v) h = (h + 1) & (kSlots - 1);
                    ln[a] = val[h];
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
            }
            P.blk_nphase[b] = (uint8_t)nph;
            for (int k = 0; k < T; ++k) {
                uint32_t h = hslot(nb[k]);
                while (key[h] != nb[k]) h = (h + 1) & (kSlots - 1);
                key[h] = -1;
            }
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
        std::vector<int64_t> &np = t_scratch.np;
        np.assign(N + 1, 0);
        for (int32_t v : P.blk_nodes) np[v + 1]++;
        for (int64_t i = 0; i < N; ++i) np[i + 1] += np[i];
        std::vector<int32_t> &nblks = t_scratch.nblks;
        nblks.resize(np[N]);
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
        // inside a colour, blocks by type; one launch per (colour, type)
        P.segs.clear();
        for (int c = 0; c < ncol; ++c) {
            int32_t *b0 = P.color_blk.data() + P.color_ptr[c], *b1 = P.color_blk.data() + P.color_ptr[c + 1];
            std::stable_sort(b0, b1, [&](int32_t x, int32_t y) {
                return type_rank(P.blk_nen[x]) < type_rank(P.blk_nen[y]);
            });
            for (int32_t *q = b0; q < b1;) {
                int32_t *r = q;
                while (r < b1 && P.blk_nen[*r] == P.blk_nen[*q]) ++r;
                P.segs.push_back(AsmSeg{P.blk_nen[*q], (int)(q - P.color_blk.data()), (int)(r - q)});
                q = r;
            }
        }
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

int build_plan(int S, const uint8_t *types, int64_t N, const double *coords, int64_t E, const int32_t *conn,
               bool renumber, Plan &P, std::string &err)
{
    const int st = build_plan_impl(S, types, N, coords, E, conn, renumber, P, err);
    release_scratch_if_large();
    return st;
}

}  // namespace feasm
