// meshes.h -- small synthetic meshes for the sanitizer drivers (test
// infrastructure): a jittered n^3 cube of HEX08, its Kuhn split into TET04,
// and a mesh mixing the two, with node and element ids shuffled.
#pragma once
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t n_nodes, n_elems;
    int stride;        // connectivity stride (8)
    double *coords;    // [n_nodes][3]
    int32_t *conn;     // [n_elems][stride]
    uint8_t *types;    // [n_elems] node counts, or NULL (every element has stride nodes)
} SanMesh;

static uint64_t san_rng = 88172645463325252ull;
static double san_uniform(void)
{
    san_rng ^= san_rng << 13;
    san_rng ^= san_rng >> 7;
    san_rng ^= san_rng << 17;
    return (double)(san_rng >> 11) / 9007199254740992.0;
}

static void san_shuffle(int64_t n, int32_t *perm)
{
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)(san_uniform() * (double)(i + 1));
        if (j > i) j = i;
        int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
}

// kind 0: HEX08 (stride 8), 1: TET04 (stride 4), 2: mixed (stride 8, types)
static SanMesh san_cube(int n, int kind)
{
    static const int kuhn[6][4] = {{0, 1, 2, 6}, {0, 2, 3, 6}, {0, 3, 7, 6}, {0, 7, 4, 6}, {0, 4, 5, 6}, {0, 5, 1, 6}};
    SanMesh m;
    const int n1 = n + 1;
    m.n_nodes = (int64_t)n1 * n1 * n1;
    int64_t ne = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) ne += (kind == 1 || (kind == 2 && i >= n / 2)) ? 6 : 1;
    m.n_elems = ne;
    m.stride = kind == 1 ? 4 : 8;
    m.coords = (double *)malloc(sizeof(double) * 3 * (size_t)m.n_nodes);
    m.conn = (int32_t *)calloc((size_t)ne * m.stride, sizeof(int32_t));
    m.types = kind == 2 ? (uint8_t *)malloc((size_t)ne) : NULL;
    int32_t *np = (int32_t *)malloc(sizeof(int32_t) * (size_t)m.n_nodes);
    san_shuffle(m.n_nodes, np);
    for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n1; ++i) {
                const int64_t v = np[((int64_t)k * n1 + j) * n1 + i];
                const double h = 1.0 / n;
                m.coords[3 * v] = i * h + ((i > 0 && i < n) ? 0.2 * h * (san_uniform() - 0.5) : 0.0);
                m.coords[3 * v + 1] = j * h + ((j > 0 && j < n) ? 0.2 * h * (san_uniform() - 0.5) : 0.0);
                m.coords[3 * v + 2] = k * h + ((k > 0 && k < n) ? 0.2 * h * (san_uniform() - 0.5) : 0.0);
            }
    int32_t *ep = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne);
    san_shuffle(ne, ep);
    int64_t e = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int32_t c[8];
                const int di[8] = {0, 1, 1, 0, 0, 1, 1, 0}, dj[8] = {0, 0, 1, 1, 0, 0, 1, 1},
                          dk[8] = {0, 0, 0, 0, 1, 1, 1, 1};
                for (int a = 0; a < 8; ++a) c[a] = np[((int64_t)(k + dk[a]) * n1 + (j + dj[a])) * n1 + (i + di[a])];
                if (kind == 1 || (kind == 2 && i >= n / 2)) {
                    for (int t = 0; t < 6; ++t, ++e) {
                        int32_t *d = m.conn + (int64_t)ep[e] * m.stride;
                        for (int a = 0; a < 4; ++a) d[a] = c[kuhn[t][a]];
                        if (m.types) m.types[ep[e]] = 4;
                    }
                } else {
                    int32_t *d = m.conn + (int64_t)ep[e] * m.stride;
                    for (int a = 0; a < 8; ++a) d[a] = c[a];
                    if (m.types) m.types[ep[e]] = 8;
                    ++e;
                }
            }
    free(np);
    free(ep);
    return m;
}

static void san_free(SanMesh *m)
{
    free(m->coords);
    free(m->conn);
    free(m->types);
}
