/*
 * CPU oracle for track labeling by weakly connected components.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header, constant or helper with the HIP library.
 *
 * What it computes (paper, Section 2: edges whose GNN score is above a threshold
 * are kept, and the weakly connected components of that graph are the track
 * candidates; Section 3.2: the labeling runs on the existing edge list instead of
 * building a new neighbour graph):
 *
 *   kept(e)   = scores == NULL or scores[e] > threshold      (strict)
 *   u ~ v     when some kept edge joins them, in either direction
 *   label[v]  = the smallest vertex id reachable from v through kept edges
 *               (v itself included), so every component is named by its
 *               smallest member and an isolated vertex is its own label.
 *
 * Route: the kept edges are stored both ways in adjacency lists; vertices are
 * visited in increasing order and every vertex not yet labeled starts a
 * breadth-first search that labels everything it reaches with its own id.  The
 * start vertex is the smallest of its component, because every smaller vertex
 * was visited earlier and either labeled this component already (then the start
 * would have been labeled too) or belongs to another one.
 *
 * Status codes: 0 ok, 1 bad argument (negative sizes, null pointers, an endpoint
 * outside [0, n)), 4 out of host memory.
 */
#include <stdint.h>
#include <stdlib.h>

int oracle_components(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n,
                      const float *scores, float threshold, int64_t *label)
{
    if (n < 0 || n_edges < 0 || (n > 0 && !label) || (n_edges > 0 && (!src || !dst)))
        return 1;
    for (int64_t e = 0; e < n_edges; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n)
            return 1;
    if (n == 0)
        return 0;

    /* Adjacency lists of the kept edges, both directions (compressed rows). */
    int64_t *first = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *fill = calloc((size_t)n, sizeof(int64_t));
    int64_t *adj = malloc(sizeof(int64_t) * (size_t)(2 * n_edges + 1));
    int64_t *queue = malloc(sizeof(int64_t) * (size_t)n);
    if (!first || !fill || !adj || !queue) {
        free(first); free(fill); free(adj); free(queue);
        return 4;
    }
    for (int64_t e = 0; e < n_edges; ++e) {
        if (scores && !(scores[e] > threshold))
            continue;
        first[src[e] + 1] += 1;
        first[dst[e] + 1] += 1;
    }
    for (int64_t v = 0; v < n; ++v)
        first[v + 1] += first[v];
    for (int64_t e = 0; e < n_edges; ++e) {
        if (scores && !(scores[e] > threshold))
            continue;
        const int64_t a = src[e], b = dst[e];
        adj[first[a] + fill[a]++] = b;
        adj[first[b] + fill[b]++] = a;
    }

    for (int64_t v = 0; v < n; ++v)
        label[v] = -1;
    for (int64_t v = 0; v < n; ++v) {
        if (label[v] >= 0)
            continue;
        int64_t head = 0, tail = 0;
        label[v] = v;
        queue[tail++] = v;
        while (head < tail) {
            const int64_t u = queue[head++];
            for (int64_t k = first[u]; k < first[u + 1]; ++k) {
                const int64_t w = adj[k];
                if (label[w] < 0) {
                    label[w] = v;
                    queue[tail++] = w;
                }
            }
        }
    }
    free(first); free(fill); free(adj); free(queue);
    return 0;
}
