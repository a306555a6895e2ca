/*
 * Runs the CPU oracles on one input file, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure: tests/test_oracle_sanitized.py
 * compiles it together with oracle/frnn_oracle.c and oracle/components_oracle.c).
 *
 * Input:  int64 n, int32 d, float r, int32 K, then n*d float32 coordinates.
 * Output: for the grid route: int64 E, then E sources and E destinations; for the
 *         O(n^2) route (n <= 4000, else E = -1): the same; for n <= 4000 the
 *         uncapped degrees (n int64); the distances of the grid route's edges (E
 *         float32); the component labels of the grid route's graph (n int64).
 * The oracles' argument checks and capacity reporting are exercised too; any
 * mismatch in those exits with status 3.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_frnn_brute(const float *X, int64_t n, int32_t d, float r, int32_t K,
                      int64_t *src, int64_t *dst, int64_t cap, int64_t *n_edges);
int oracle_frnn_grid(const float *X, int64_t n, int32_t d, float r, int32_t K,
                     int64_t *src, int64_t *dst, int64_t cap, int64_t *n_edges);
int oracle_frnn_degrees(const float *X, int64_t n, int32_t d, float r, int64_t *deg);
void oracle_pair_dist(const float *X, int32_t d, const int64_t *i, const int64_t *j, int64_t m, float *out);
int oracle_components(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n,
                      const float *scores, float threshold, int64_t *label);

typedef int (*route_fn)(const float *, int64_t, int32_t, float, int32_t, int64_t *, int64_t *, int64_t,
                        int64_t *);

/* Runs one route twice: first with a capacity one below the count it reports
 * (when there are edges), then with exactly that count. */
static int64_t run_route(route_fn f, const float *X, int64_t n, int32_t d, float r, int32_t K,
                         int64_t **src, int64_t **dst)
{
    int64_t E = 0;
    int st = f(X, n, d, r, K, NULL, NULL, 0, &E);
    if (st != 0 && st != 3) exit(3);
    if (E > 0) {
        int64_t *s = malloc(sizeof(int64_t) * (size_t)E), *t = malloc(sizeof(int64_t) * (size_t)E);
        int64_t E2 = 0;
        if (f(X, n, d, r, K, s, t, E - 1, &E2) != 3 || E2 != E) exit(3);
        if (f(X, n, d, r, K, s, t, E, &E2) != 0 || E2 != E) exit(3);
        *src = s;
        *dst = t;
    } else {
        if (st != 0) exit(3);
        *src = malloc(sizeof(int64_t));
        *dst = malloc(sizeof(int64_t));
    }
    return E;
}

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 2;
    int64_t n;
    int32_t d, K;
    float r;
    if (fread(&n, 8, 1, in) != 1 || fread(&d, 4, 1, in) != 1 || fread(&r, 4, 1, in) != 1 ||
        fread(&K, 4, 1, in) != 1)
        return 2;
    float *X = malloc(sizeof(float) * (size_t)(n * d + 1));
    if ((int64_t)fread(X, sizeof(float), (size_t)(n * d), in) != n * d) return 2;
    fclose(in);

    /* Argument checks. */
    int64_t E = 0;
    if (oracle_frnn_grid(X, n, d, -r, K, NULL, NULL, 0, &E) != 1) return 3;
    if (oracle_frnn_grid(X, n, d, r, 0, NULL, NULL, 0, &E) != 1) return 3;
    if (oracle_frnn_brute(X, -1, d, r, K, NULL, NULL, 0, &E) != 1) return 3;
    if (oracle_components(NULL, NULL, 1, n, NULL, 0.0f, NULL) != 1) return 3;

    FILE *out = fopen(argv[2], "wb");
    if (!out) return 2;
    int64_t *gs, *gd;
    const int64_t Eg = run_route(oracle_frnn_grid, X, n, d, r, K, &gs, &gd);
    fwrite(&Eg, 8, 1, out);
    fwrite(gs, 8, (size_t)Eg, out);
    fwrite(gd, 8, (size_t)Eg, out);
    const int small = n <= 4000;
    int64_t *bs = NULL, *bd = NULL;
    const int64_t Eb = small ? run_route(oracle_frnn_brute, X, n, d, r, K, &bs, &bd) : -1;
    fwrite(&Eb, 8, 1, out);
    if (small) {
        fwrite(bs, 8, (size_t)Eb, out);
        fwrite(bd, 8, (size_t)Eb, out);
        int64_t *deg = malloc(sizeof(int64_t) * (size_t)(n + 1));
        if (oracle_frnn_degrees(X, n, d, r, deg) != 0) return 3;
        fwrite(deg, 8, (size_t)n, out);
        free(deg);
    }
    float *dist = malloc(sizeof(float) * (size_t)(Eg + 1));
    oracle_pair_dist(X, d, gs, gd, Eg, dist);
    fwrite(dist, 4, (size_t)Eg, out);
    int64_t *label = malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (oracle_components(gs, gd, Eg, n, NULL, 0.0f, label) != 0) return 3;
    fwrite(label, 8, (size_t)n, out);
    fclose(out);
    free(label);
    free(dist);
    free(bs);
    free(bd);
    free(gs);
    free(gd);
    free(X);
    return 0;
}
