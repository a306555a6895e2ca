/*
 * CPU oracle for the fixed-radius nearest-neighbour (FRNN) graph.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header, constant or helper with the HIP library.
 *
 * What it computes (paper, Section 2 and Section 3.4): the graph that joins every
 * spacepoint to all spacepoints lying within a constant radius of it in the
 * learned embedding space.  The paper leaves the arithmetic unstated; this oracle
 * fixes it as follows (each reading is listed in the design notes):
 *
 *   r2      = fl32(r * r)
 *   D(i,j)  = s_{d-1}, with s_{-1} = +0.0f and, for k = 0 .. d-1 in that order,
 *             t = fl32(X[i][k] - X[j][k]),  s_k = fl32(s_{k-1} + fl32(t * t))
 *             (every operation rounded on its own: no fused multiply-add)
 *   N(i)    = { j != i : D(i,j) < r2 }                       (strict)
 *   Out(i)  = N(i) if |N(i)| <= K, else the K members of N(i) that come first in
 *             the order of (D(i,j), j)                       (nearest K, index breaks ties;
 *             the nearest-k-then-radius reading of Section 3.1)
 *   edges   = { (i, j) : j in Out(i) }, listed by i ascending, then j ascending;
 *             row 0 holds i (the query), row 1 holds j (the neighbour).
 *
 * Two routes to that set are given:
 *   oracle_frnn_brute  the definition written out: every ordered pair is tested;
 *   oracle_frnn_grid   the grid-cell technique of Section 3.4: points are binned
 *                      into cubic cells over coordinates 0, 1, 2 and each query
 *                      visits only the 3 x 3 x 3 cells around its own.  The cell
 *                      edge is r * (1 + 2^-10) in double precision, so any pair
 *                      the float32 test accepts lies in adjacent cells (see the
 *                      margin argument in the design notes).
 *
 * Build with a plain C compiler and -ffp-contract=off (never -ffast-math).
 *
 * Status codes: 0 ok, 1 bad argument, 2 non-finite coordinate, 3 output capacity
 * too small (the required edge count is still written to *n_edges).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG 1
#define OR_ERR_NONFINITE 2
#define OR_ERR_CAPACITY 3

/* D(i,j) of the definition above: ascending coordinates, separately rounded. */
static float sq_dist(const float *xi, const float *xj, int d)
{
    float s = 0.0f;
    for (int k = 0; k < d; ++k) {
        float t = xi[k] - xj[k];
        float t2 = t * t;
        s = s + t2;
    }
    return s;
}

typedef struct {
    float dist;
    int64_t j;
} hit_t;

static int cmp_hit_dist_then_index(const void *a, const void *b)
{
    const hit_t *x = (const hit_t *)a, *y = (const hit_t *)b;
    if (x->dist < y->dist) return -1;
    if (x->dist > y->dist) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

static int cmp_hit_index(const void *a, const void *b)
{
    const hit_t *x = (const hit_t *)a, *y = (const hit_t *)b;
    return (x->j > y->j) - (x->j < y->j);
}

/* Growable list of accepted neighbours of one query. */
typedef struct {
    hit_t *v;
    int64_t len, cap;
} hits_t;

static int hits_push(hits_t *h, float dist, int64_t j)
{
    if (h->len == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 64;
        hit_t *nv = (hit_t *)realloc(h->v, (size_t)nc * sizeof(hit_t));
        if (!nv) return -1;
        h->v = nv;
        h->cap = nc;
    }
    h->v[h->len].dist = dist;
    h->v[h->len].j = j;
    h->len++;
    return 0;
}

/* Applies the cap of the definition to one query's neighbours and appends the
 * kept ones, j ascending, to the output.  Returns the number kept. */
static int64_t emit_query(int64_t i, hits_t *h, int K, int64_t *src, int64_t *dst,
                          int64_t cap, int64_t at)
{
    int64_t keep = h->len;
    if (keep > K) {
        qsort(h->v, (size_t)h->len, sizeof(hit_t), cmp_hit_dist_then_index);
        keep = K;
    }
    if (keep > 1) /* an empty list has no storage yet, and qsort needs a valid base */
        qsort(h->v, (size_t)keep, sizeof(hit_t), cmp_hit_index);
    for (int64_t t = 0; t < keep; ++t) {
        if (at + t < cap) {
            src[at + t] = i;
            dst[at + t] = h->v[t].j;
        }
    }
    return keep;
}

static int check_args(const float *X, int64_t n, int32_t d, float r, int32_t K,
                      int64_t *n_edges)
{
    if (!n_edges || n < 0 || d < 1 || !(r > 0.0f) || isinf(r) || K < 1) return OR_ERR_ARG;
    if (n > 0 && !X) return OR_ERR_ARG;
    for (int64_t q = 0; q < n * (int64_t)d; ++q)
        if (!isfinite(X[q])) return OR_ERR_NONFINITE;
    return OR_OK;
}

/* The definition, every ordered pair tested: O(n^2). */
int oracle_frnn_brute(const float *X, int64_t n, int32_t d, float r, int32_t K,
                      int64_t *src, int64_t *dst, int64_t cap, int64_t *n_edges)
{
    int st = check_args(X, n, d, r, K, n_edges);
    if (st != OR_OK) return st;
    const float r2 = r * r;
    hits_t h = {0, 0, 0};
    int64_t at = 0;
    for (int64_t i = 0; i < n; ++i) {
        h.len = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            float D = sq_dist(X + i * d, X + j * d, d);
            if (D < r2 && hits_push(&h, D, j) != 0) {
                free(h.v);
                return OR_ERR_ARG;
            }
        }
        at += emit_query(i, &h, K, src, dst, cap, at);
    }
    free(h.v);
    *n_edges = at;
    return at > cap ? OR_ERR_CAPACITY : OR_OK;
}

/* |N(i)| before the cap, by the definition (O(n^2)); used by the invariant checks. */
int oracle_frnn_degrees(const float *X, int64_t n, int32_t d, float r, int64_t *deg)
{
    int64_t dummy;
    int st = check_args(X, n, d, r, 1, &dummy);
    if (st != OR_OK) return st;
    const float r2 = r * r;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && sq_dist(X + i * d, X + j * d, d) < r2) ++c;
        deg[i] = c;
    }
    return OR_OK;
}

/* ---- grid route ------------------------------------------------------- */

typedef struct {
    double cell[3]; /* floor(x_p / c) for the binned coordinates p = 0, 1, 2 */
    int64_t idx;
} binned_t;

static int cmp_cell(const double *a, const double *b)
{
    for (int p = 0; p < 3; ++p) {
        if (a[p] < b[p]) return -1;
        if (a[p] > b[p]) return 1;
    }
    return 0;
}

static int cmp_binned(const void *a, const void *b)
{
    const binned_t *x = (const binned_t *)a, *y = (const binned_t *)b;
    int c = cmp_cell(x->cell, y->cell);
    if (c) return c;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* First position in the sorted bins whose cell is not less than `cell`. */
static int64_t first_not_before(const binned_t *b, int64_t n, const double *cell)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cmp_cell(b[mid].cell, cell) < 0) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* Grid-cell route (Section 3.4): bin into cells over coordinates 0..2 and scan
 * the 27 cells around each query.  Needs d >= 3.  A coordinate whose cell index
 * would exceed 2^50 in magnitude is left unbinned (every point gets cell 0 along
 * it), which keeps the search exact at the cost of visiting more points. */
int oracle_frnn_grid(const float *X, int64_t n, int32_t d, float r, int32_t K,
                     int64_t *src, int64_t *dst, int64_t cap, int64_t *n_edges)
{
    int st = check_args(X, n, d, r, K, n_edges);
    if (st != OR_OK) return st;
    if (d < 3) return OR_ERR_ARG;
    const float r2 = r * r;
    const double c = (double)r * (1.0 + 1.0 / 1024.0);

    int binned[3] = {1, 1, 1};
    for (int p = 0; p < 3; ++p)
        for (int64_t i = 0; i < n; ++i)
            if (fabs((double)X[i * d + p]) / c > 1125899906842624.0 /* 2^50 */) binned[p] = 0;

    binned_t *b = (binned_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(binned_t));
    if (!b) return OR_ERR_ARG;
    for (int64_t i = 0; i < n; ++i) {
        for (int p = 0; p < 3; ++p)
            b[i].cell[p] = binned[p] ? floor((double)X[i * d + p] / c) : 0.0;
        b[i].idx = i;
    }
    qsort(b, (size_t)n, sizeof(binned_t), cmp_binned);

    /* Where each original point sits in the sorted bins. */
    int64_t *where = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!where) {
        free(b);
        return OR_ERR_ARG;
    }
    for (int64_t s = 0; s < n; ++s) where[b[s].idx] = s;

    hits_t h = {0, 0, 0};
    int64_t at = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double *own = b[where[i]].cell;
        h.len = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int off[3] = {dx, dy, dz};
                    double nb[3];
                    int skip = 0;
                    for (int p = 0; p < 3; ++p) {
                        if (!binned[p] && off[p] != 0) skip = 1;
                        nb[p] = own[p] + off[p];
                    }
                    if (skip) continue;
                    int64_t s = first_not_before(b, n, nb);
                    for (; s < n && cmp_cell(b[s].cell, nb) == 0; ++s) {
                        int64_t j = b[s].idx;
                        if (j == i) continue;
                        float D = sq_dist(X + i * d, X + j * d, d);
                        if (D < r2 && hits_push(&h, D, j) != 0) {
                            free(h.v);
                            free(where);
                            free(b);
                            return OR_ERR_ARG;
                        }
                    }
                }
        at += emit_query(i, &h, K, src, dst, cap, at);
    }
    free(h.v);
    free(where);
    free(b);
    *n_edges = at;
    return at > cap ? OR_ERR_CAPACITY : OR_OK;
}

/* D(i,j) for a list of pairs, for checks of emitted edges. */
void oracle_pair_dist(const float *X, int32_t d, const int64_t *i, const int64_t *j,
                      int64_t m, float *out)
{
    for (int64_t q = 0; q < m; ++q) out[q] = sq_dist(X + i[q] * d, X + j[q] * d, d);
}
