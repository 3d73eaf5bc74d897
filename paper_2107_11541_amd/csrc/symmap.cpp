// symmap.cpp -- row blocks of the symmetric PCG SpMV, built on the host.
//
// The PCG matrix is symmetric (Section 5.2 solves the SPD pressure system).
// Inside a row block both entries of a pair (i, j), (j, i) are in the same
// work-group's LDS once the block's values are staged, so the block stores
// the upper one and reads it again for the lower one (a mirror entry).  The
// layout is described with SymMap in plan.h.
#include <algorithm>

#include "../../include/feasm.h"
#include "plan.h"

namespace feasm {

namespace {

// Per row chunk: its blocks, with packed positions and mirror indices local
// to the chunk (the chunk's packed entries start at a multiple of 4, so
// positions modulo 4 are the same locally and globally).
struct SymChunk {
    std::vector<int32_t> r0, bp, mb, cb;   // per block: first row, packed start, first mirror, set start
    std::vector<uint32_t> roff;            // rows + 1 per block
    std::vector<uint8_t> lidx;             // per packed entry
    std::vector<uint16_t> mir;             // per mirror entry, each block's run of even length
    std::vector<int32_t> cols;
    std::vector<int32_t> added, sidx;      // scratch: the open block's columns, stored index per CSR entry
    std::string err;
};

// CSR position of column v in row c, or -1.
int64_t find_in_row(const int32_t *rowptr, const int32_t *colidx, int64_t c, int32_t v)
{
    const int32_t *b = colidx + rowptr[c], *e = colidx + rowptr[c + 1];
    const int32_t *it = std::lower_bound(b, e, v);
    if (it != e && *it == v) return it - colidx;
    for (const int32_t *q = b; q < e; ++q)   // rows are sorted; kept for any other pattern
        if (*q == v) return q - colidx;
    return -1;
}

}  // namespace

int build_sym_map(int64_t N, const int32_t *rowptr, const int32_t *colidx, SymMap &S, std::string &err)
{
    S.mstart.assign((size_t)N, 0);
    const int64_t nch = (N + kPlanRowChunk - 1) / kPlanRowChunk;
    std::vector<SymChunk> ch((size_t)nch);
    const int nw = parallel_workers(nch);
    std::vector<std::vector<int32_t>> stamps(nw), locs(nw);
    std::vector<int32_t> next_id(nw, 0);
    parallel_chunks_w(nch, [&](int64_t c, int w) {
        SymChunk &C = ch[c];
        std::vector<int32_t> &stamp = stamps[w], &loc = locs[w];
        if (stamp.empty()) {
            stamp.assign((size_t)N, -1);
            loc.assign((size_t)N, 0);
        }
        const int64_t R0 = c * kPlanRowChunk, R1 = std::min<int64_t>(N, R0 + kPlanRowChunk);
        int64_t packed = 0;
        for (int64_t r = R0; r < R1;) {
            // grow the block row by row while it fits
            const int32_t bid = next_id[w]++;
            C.added.clear();
            int64_t nst = 0, nmi = 0, r1 = r;
            for (; r1 < R1; ++r1) {
                const size_t mark = C.added.size();
                auto add = [&](int32_t v) {
                    if (stamp[v] != bid) {
                        stamp[v] = bid;
                        C.added.push_back(v);
                    }
                };
                add((int32_t)r1);   // own rows are always in the set
                int64_t st = 0, mi = 0;
                for (int32_t q = rowptr[r1]; q < rowptr[r1 + 1]; ++q) {
                    const int32_t v = colidx[q];
                    if (v >= r && v < r1) ++mi;
                    else ++st;
                    add(v);
                }
                const bool fits = r1 - r < kSymRows && nst + st <= kSymStored && nmi + mi <= kSymMirrors &&
                                  (int64_t)C.added.size() <= kSymCols;
                if (!fits) {
                    for (size_t k = mark; k < C.added.size(); ++k) stamp[C.added[k]] = -1;
                    C.added.resize(mark);
                    if (r1 == r) {
                        C.err = "row " + std::to_string(r) + " does not fit a symmetric SpMV block";
                        return;
                    }
                    break;
                }
                nst += st;
                nmi += mi;
            }
            // set slots: own rows first, then the other columns in first-touch order
            const int32_t R = (int32_t)(r1 - r), slot_id = next_id[w]++;
            C.r0.push_back((int32_t)r);
            C.bp.push_back((int32_t)packed);
            C.mb.push_back((int32_t)C.mir.size());
            C.cb.push_back((int32_t)C.cols.size());
            for (int32_t i = 0; i < R; ++i) C.cols.push_back((int32_t)(r + i));
            int32_t nslot = R;
            const int64_t p0 = rowptr[r];
            C.sidx.assign((size_t)(rowptr[r1] - p0), -1);
            const int shift = (int)(packed & 3);
            int32_t ns = 0, nm = 0;
            for (int64_t i = r; i < r1; ++i) {
                C.roff.push_back((uint32_t)ns | (uint32_t)nm << 16);
                S.mstart[(size_t)i] = (uint8_t)(rowptr[i + 1] - rowptr[i]);   // no mirror: the row's end
                bool run = false;
                for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
                    const int32_t v = colidx[q];
                    if (q > rowptr[i] && v <= colidx[q - 1]) {
                        C.err = "row " + std::to_string(i) + " is not sorted";
                        return;
                    }
                    if (v >= r && v < i) {
                        if (!run) S.mstart[(size_t)i] = (uint8_t)(q - rowptr[i]);
                        run = true;
                        // mirror of (v, i), stored earlier in row v (i > v)
                        const int64_t pq = find_in_row(rowptr, colidx, v, (int32_t)i);
                        if (pq < 0) {
                            C.err = "pattern not symmetric: (" + std::to_string(i) + ", " + std::to_string(v) +
                                    ") has no transpose";
                            return;
                        }
                        const int32_t k = C.sidx[(size_t)(pq - p0)];
                        C.mir.push_back((uint16_t)((shift + k) | (int32_t)(v - r) << 10));
                        ++nm;
                        continue;
                    }
                    int32_t sl;
                    if (v >= r && v < r1) {
                        sl = v - (int32_t)r;
                    } else {
                        if (stamp[v] != slot_id) {
                            stamp[v] = slot_id;
                            loc[v] = nslot++;
                            C.cols.push_back(v);
                        }
                        sl = loc[v];
                    }
                    C.sidx[(size_t)(q - p0)] = ns;
                    C.lidx.push_back((uint8_t)sl);
                    ++ns;
                }
            }
            C.roff.push_back((uint32_t)ns | (uint32_t)nm << 16);
            if (nm & 1) C.mir.push_back(0);
            packed += ns;
            r = r1;
        }
    });
    for (const SymChunk &C : ch)
        if (!C.err.empty()) {
            err = C.err;
            return FE_EBADMESH;
        }
    // chunk bases: packed entries (each chunk at a multiple of 4), mirror
    // words, set columns, blocks
    std::vector<int64_t> pb(nch + 1, 0), wb(nch + 1, 0), cb(nch + 1, 0), bb(nch + 1, 0);
    for (int64_t c = 0; c < nch; ++c) {
        const SymChunk &C = ch[c];
        const int64_t np = (int64_t)C.lidx.size();
        pb[c + 1] = c + 1 < nch ? (pb[c] + np + 3) & ~(int64_t)3 : pb[c] + np;
        wb[c + 1] = wb[c] + (int64_t)C.mir.size() / 2;
        cb[c + 1] = cb[c] + (int64_t)C.cols.size();
        bb[c + 1] = bb[c] + (int64_t)C.r0.size();
    }
    if (pb[nch] > INT32_MAX - 8 || cb[nch] > INT32_MAX) {
        err = "matrix too large for the symmetric SpMV map";
        return FE_EBADMESH;
    }
    S.nrb = bb[nch];
    S.n_packed = pb[nch];
    S.n_mirror_words = wb[nch];
    S.desc.assign((size_t)(S.nrb + 1) * 4, 0);
    S.roff.assign((size_t)(N + S.nrb), 0);
    S.lidx.assign((size_t)S.n_packed + 4, 0);
    S.mir.assign((size_t)S.n_mirror_words + 1, 0);
    S.cols.assign((size_t)cb[nch], 0);
    parallel_chunks(nch, [&](int64_t c) {
        const SymChunk &C = ch[c];
        for (size_t j = 0; j < C.r0.size(); ++j) {
            int32_t *d = &S.desc[(size_t)(bb[c] + (int64_t)j) * 4];
            d[0] = C.r0[j];
            d[1] = (int32_t)(pb[c] + C.bp[j]);
            d[2] = (int32_t)(wb[c] + C.mb[j] / 2);
            d[3] = (int32_t)(cb[c] + C.cb[j]);
        }
        const int64_t R0 = c * kPlanRowChunk;
        std::copy(C.roff.begin(), C.roff.end(), S.roff.begin() + (R0 + bb[c]));
        std::copy(C.lidx.begin(), C.lidx.end(), S.lidx.begin() + pb[c]);
        for (size_t k = 0; k < C.mir.size(); k += 2)
            S.mir[(size_t)wb[c] + k / 2] = (uint32_t)C.mir[k] | (uint32_t)C.mir[k + 1] << 16;
        std::copy(C.cols.begin(), C.cols.end(), S.cols.begin() + cb[c]);
    });
    int32_t *d = &S.desc[(size_t)S.nrb * 4];
    d[0] = (int32_t)N;
    d[1] = (int32_t)S.n_packed;
    d[2] = (int32_t)S.n_mirror_words;
    d[3] = (int32_t)cb[nch];
    return 0;
}

}  // namespace feasm
