/*
 * frnn.h - C interface of the MI355X fixed-radius nearest-neighbour graph builder.
 *
 * The operation (paper, Section 2 "Description of the Exa.TrkX Pipeline": the
 * graph built in the learned embedding space joins points that lie within a
 * constant radius of each other; Section 3.4 "Fixed-Radius Nearest Neighbors":
 * the points are projected to three coordinates and searched with a grid of
 * cells).  For points X (n rows of d float32 coordinates), radius r and cap K:
 *
 *   r2      = fl32(r * r)
 *   D(i,j)  = float32 sum over k = 0..d-1, in that order, of fl32(t_k * t_k),
 *             t_k = fl32(X[i][k] - X[j][k]); every operation separately rounded,
 *             no fused multiply-add, subnormals kept
 *   N(i)    = { j != i : D(i,j) < r2 }
 *   Out(i)  = N(i) if |N(i)| <= K, else its K members first in (D(i,j), j) order
 *   edges   = { (i, j) : j in Out(i) }, i ascending then j ascending
 *
 * The result is unique, so two correct implementations produce identical bytes.
 * The cell grid only limits which pairs are tested: it bins three coordinates as
 * the paper does, or four (the default for d >= 5, which leaves far fewer
 * candidates per query), and the edges depend on neither choice.
 *
 * Conventions shared by every entry point:
 *   - Device pointers are HIP device allocations (for example PyTorch CUDA
 *     tensors on ROCm); host pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     All device work is enqueued on it.  Inputs must stay alive and unchanged
 *     until that work has finished.
 *   - The caller owns every buffer.  The library allocates no device memory
 *     (frnn_build_noalloc works in a fixed device array of the library's own);
 *     it keeps one small pinned host buffer per calling thread for results.
 *   - Errors are returned as status codes; nothing is thrown across this
 *     interface.  On any status other than FRNN_OK the output buffers hold
 *     unspecified values.
 *   - Calls on different streams may overlap if they use different workspaces.
 */
#ifndef FRNN_H
#define FRNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum frnn_status {
    FRNN_OK = 0,
    FRNN_ERR_ARG = 1,         /* n < 0, d outside [3, 64], r not finite or <= 0, K outside
                                 [1, FRNN_MAX_K], bad config, or a null pointer that is needed */
    FRNN_ERR_NONFINITE = 2,   /* some coordinate is NaN or infinite; no edges are written */
    FRNN_ERR_CAPACITY = 3,    /* more edges than edge_capacity; *n_edges holds the number needed */
    FRNN_ERR_WORKSPACE = 4,   /* workspace smaller than frnn_workspace_bytes() */
    FRNN_ERR_UNSUPPORTED = 5, /* n >= 2^31 */
    FRNN_ERR_HIP = 6          /* a HIP runtime call failed */
};

#define FRNN_MAX_D 64
#define FRNN_MAX_K 4096

/* Tunables of the grid search.  They change speed only: every setting yields
 * the same edges.  Zero-initialise and set what you need. */
typedef struct frnn_config {
    int32_t dims[4];   /* coordinates binned by the grid, used when dims[0] != dims[1]: the
                          first `axes` entries, all different, in [0, d); dims[0] is the
                          fastest-varying cell axis.  Default: the last `axes` coordinates
                          d-axes .. d-1, so the leading coordinates of the distance sum
                          are unbinned. */
    int32_t axes;      /* number of binned coordinates, 3 or 4 (at most d).  0: 3 when dims
                          are given, else 4 when d >= 5 and cell_div <= 1, else 3.  Four
                          binned coordinates need cell_div 1. */
    int32_t cell_div;  /* cell edge = r * (1 + 2^-10) / cell_div, cell_div in {1, 2, 3}
                          (0 means 1).  Neighbours are searched cell_div cells away. */
    int32_t grid_mult; /* search workgroups as a multiple of those that fit on the GPU at
                          once: 1, 2, 4 or 8; 0 (default) chooses from the rows per wave
                          (1 up to 128 rows per resident wave, up to 4 beyond).  With 1,
                          waves order their issue priority by progress. */
    int32_t flags;     /* FRNN_FLAG_* bits */
} frnn_config;

/* frnn_config.flags: time every stage with HIP events on the call's stream and
 * report the durations in frnn_stats.stage_ms (adds a few microseconds). */
#define FRNN_FLAG_TIMING 1
/* frnn_config.flags, frnn_build_batch_async only: the workspace already holds the
 * event table of an earlier call with the same event_offsets and d, so nothing is
 * copied to the device and the call only enqueues kernels (it can then be
 * captured into a HIP graph and replayed). */
#define FRNN_FLAG_EVENTS_RESIDENT 2

/* Stages reported in frnn_stats.stage_ms. */
enum frnn_stage {
    FRNN_STAGE_BOUNDS = 0,   /* bounds of the binned coordinates, non-finite check */
    FRNN_STAGE_KEYS = 1,     /* grid plan, cell keys, histogram */
    FRNN_STAGE_CELLS = 2,    /* scan of the histogram */
    FRNN_STAGE_SCATTER = 3,  /* rows copied into cell order */
    FRNN_STAGE_SEARCH = 4,   /* neighbour-cell search */
    FRNN_STAGE_TOTALS = 5,   /* kept neighbours per tile of 256 queries */
    FRNN_STAGE_PLACE = 6,    /* output offsets, long neighbour lists and the K cap; edges
                                written in (i, j) order */
    FRNN_STAGES = 7
};

/* Counts describing one call, for diagnostics and benchmarks. */
typedef struct frnn_stats {
    int64_t n_edges;            /* edges written (= *n_edges on success) */
    int64_t candidates;         /* (query, candidate) pairs examined by the search */
    int64_t n_cells;            /* cells of the grid */
    int32_t axes;               /* binned coordinates (3 or 4) */
    int32_t grid[4];            /* cells per binned axis (1 past `axes`) */
    int32_t dims[4];            /* binned coordinates (-1 past `axes`) */
    float cell[4];              /* cell edge per binned axis (infinite past `axes`) */
    int32_t capped_queries;     /* queries with |N(i)| > K */
    int32_t overflow_queries;   /* queries with more than 16 neighbours, whose lists the
                                   placement pass collects again */
    float stage_ms[FRNN_STAGES]; /* per-stage device time with FRNN_FLAG_TIMING, else 0 */
    int64_t survivors;          /* examined pairs whose leading partial sum stayed below r2, so
                                   that the search added the remaining terms of the distance */
} frnn_stats;

/* Bytes of device workspace frnn_build needs for n points of dimension d.
 * Host-only arithmetic; returns 0 for invalid arguments (n outside [0, 2^31),
 * d outside [3, 64]). */
size_t frnn_workspace_bytes(int64_t n, int32_t d);

/* Builds the FRNN graph of the points.
 *   points          device, float32, row-major [n, d] (row i at points + i*d)
 *   n, d            point count (0 <= n < 2^31) and dimension (3 <= d <= 64)
 *   r, K            radius (finite, > 0) and cap (1 <= K <= FRNN_MAX_K)
 *   workspace       device scratch of at least frnn_workspace_bytes(n, d)
 *                   bytes, 256-byte aligned; its contents on entry do not matter
 *   src, dst        device, int64 [edge_capacity] each: edge e is (src[e], dst[e]),
 *                   src the query i, dst the neighbour j, sorted by (i, j)
 *   n_edges         host: receives E, or the E needed when it returns FRNN_ERR_CAPACITY
 *   config          host, may be NULL for defaults
 *   stats           host, may be NULL
 *   stream          hipStream_t as void*
 * Blocks the calling thread until the edge count is known (one device-to-host
 * copy at the end of the work enqueued on `stream`). */
int frnn_build(const float *points, int64_t n, int32_t d, float r, int32_t K,
               void *workspace, size_t workspace_bytes,
               int64_t *src, int64_t *dst, int64_t edge_capacity, int64_t *n_edges,
               const frnn_config *config, frnn_stats *stats, void *stream);

/* Size of the device array frnn_build_noalloc works in, in MiB (per device). */
#define FRNN_NOALLOC_SCRATCH_MIB 64

/* frnn_build for callers that cannot allocate device memory (code that must not
 * call hipMalloc: a tight serving loop, a harness that forbids it): the same
 * result, with no workspace argument.  The library works in a device array of
 * FRNN_NOALLOC_SCRATCH_MIB MiB that each device holds from the first such call
 * on it until the process ends; the call itself allocates no device or pinned
 * memory (its report is copied into the caller's frame).  The first call on a
 * device looks the array up; later calls only enqueue kernels and copy the
 * report back.
 *   Arguments as for frnn_build, without workspace / workspace_bytes.
 *   FRNN_ERR_WORKSPACE     frnn_workspace_bytes(n, d) exceeds the array
 *                          (checked on the host before any device work; for example
 *                          120,000 points of d = 8 with room for 16 edges per point fit)
 *   FRNN_ERR_ARG           also for FRNN_FLAG_TIMING (timing would create HIP events)
 * Every call on one device shares that device's array: calls that overlap in
 * time on one device (from several host threads, or on several streams) race
 * and must be serialised by the caller.  Nothing need be cleared between calls:
 * each call clears what it counts. */
int frnn_build_noalloc(const float *points, int64_t n, int32_t d, float r, int32_t K,
                       int64_t *src, int64_t *dst, int64_t edge_capacity, int64_t *n_edges,
                       const frnn_config *config, frnn_stats *stats, void *stream);

/* Bytes of device workspace frnn_build_batch needs for the given events (see
 * below).  Returns 0 for invalid arguments. */
size_t frnn_batch_workspace_bytes(const int64_t *event_offsets, int32_t n_events, int32_t d);

/* Builds the FRNN graphs of several independent events in one pass (one launch
 * sequence and one synchronisation for the whole batch).  Each event is searched
 * on its own: its own grid, no edges between events.
 *   points          device, float32, the events' rows back to back; event e is rows
 *                   [event_offsets[e], event_offsets[e+1]) of points (row-major, d columns)
 *   event_offsets   host, int64 [n_events + 1], non-decreasing; 1 <= n_events <= 65535;
 *                   total rows < 2^31
 *   src, dst        device, int64 [edge_capacity] each: the events' edge lists back to back;
 *                   indices are local to their event (0 .. n_e - 1); each list sorted by (i, j)
 *   edge_offsets    host, int64 [n_events + 1]: event e's edges are
 *                   [edge_offsets[e], edge_offsets[e+1]); on FRNN_ERR_CAPACITY only
 *                   edge_offsets[n_events] is set, to the total needed
 * Other arguments as for frnn_build; a non-finite coordinate in any event fails the
 * whole batch with FRNN_ERR_NONFINITE.  stats describe the batch (grid fields: event 0). */
int frnn_build_batch(const float *points, const int64_t *event_offsets, int32_t n_events, int32_t d,
                     float r, int32_t K, void *workspace, size_t workspace_bytes,
                     int64_t *src, int64_t *dst, int64_t edge_capacity, int64_t *edge_offsets,
                     const frnn_config *config, frnn_stats *stats, void *stream);

/* frnn_build_batch without waiting: checks the arguments, enqueues the work on
 * `stream` and returns.  Results stay on the device:
 *   edge_offsets_device  device, int64 [n_events + 2]: entries 0..n_events as for
 *                        frnn_build_batch's edge_offsets (entry n_events is the total E,
 *                        also when it exceeds edge_capacity), then a status word:
 *                        0 ok, FRNN_ERR_NONFINITE or FRNN_ERR_CAPACITY.
 * The total row count must be positive.  FRNN_FLAG_TIMING is not accepted.  With
 * more than one event the event table is copied to the workspace first, from
 * pinned staging memory the library keeps per calling thread (a call may wait for
 * that thread's copy of four calls earlier to have run); that copy cannot be
 * captured, so a call that needs it on a capturing stream returns FRNN_ERR_ARG.
 * With FRNN_FLAG_EVENTS_RESIDENT (see above) only kernels are enqueued, so the
 * call can be captured into a HIP graph; the points, workspace and outputs must
 * then stay at the same addresses for every replay.  Calls that share a workspace
 * must not overlap in time. */
int frnn_build_batch_async(const float *points, const int64_t *event_offsets, int32_t n_events, int32_t d,
                           float r, int32_t K, void *workspace, size_t workspace_bytes,
                           int64_t *src, int64_t *dst, int64_t edge_capacity, int64_t *edge_offsets_device,
                           const frnn_config *config, void *stream);

/* frnn_build_batch_async for events held in separate buffers: event e has
 * event_sizes[e] rows at event_points[e] (device, row-major, d columns; a null
 * pointer is allowed for an empty event).  event_points and event_sizes are host
 * arrays of n_events entries.  The workspace size is frnn_batch_workspace_bytes of
 * the offsets 0, s0, s0+s1, ...; outputs and status as for frnn_build_batch_async. */
int frnn_build_events_async(const float *const *event_points, const int64_t *event_sizes, int32_t n_events,
                            int32_t d, float r, int32_t K, void *workspace, size_t workspace_bytes,
                            int64_t *src, int64_t *dst, int64_t edge_capacity, int64_t *edge_offsets_device,
                            const frnn_config *config, void *stream);

/* ---- Track labeling ------------------------------------------------------
 * Weakly connected components of an edge list (paper, Section 2: the edges whose
 * score passes a threshold are kept, and each weakly connected component is a
 * track candidate; Section 3.2: the labeling uses the edge list that exists):
 *
 *   kept(e)   = scores == NULL or scores[e] > threshold (strict)
 *   label[v]  = the smallest vertex id joined to v by a path of kept edges taken
 *               in either direction (v itself when there is none)
 *
 * The labels are unique, so two correct implementations produce identical bytes.
 * Self-loops and repeated edges are allowed.
 */

/* Bytes of device workspace for a graph of n_vertices vertices (0 for
 * n_vertices < 0 or >= 2^31).  Host-only arithmetic. */
size_t frnn_components_workspace_bytes(int64_t n_vertices);

/* Labels the vertices of the graph.
 *   src, dst      device, int64 [n_edges] each: edge e joins src[e] and dst[e]
 *                 (for instance the output of frnn_build); every endpoint must lie in
 *                 [0, n_vertices), else FRNN_ERR_ARG
 *   n_edges       >= 0 (0: every vertex is its own component)
 *   n_vertices    0 <= n_vertices < 2^31 (FRNN_ERR_UNSUPPORTED above)
 *   scores        device, float32 [n_edges], or NULL to keep every edge
 *   threshold     edges with scores[e] > threshold are kept
 *   workspace     device scratch of at least frnn_components_workspace_bytes(n_vertices)
 *                 bytes, 256-byte aligned; contents on entry do not matter
 *   labels        device, int64 [n_vertices]: receives label[v]
 *   n_components  host, may be NULL: receives the number of components
 *   stream        hipStream_t as void*
 * Blocks until the work enqueued on `stream` has finished.  FRNN_ERR_HIP also
 * reports the (never expected) case of the hook loop reaching its internal bound. */
int frnn_components(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n_vertices,
                    const float *scores, float threshold, void *workspace, size_t workspace_bytes,
                    int64_t *labels, int64_t *n_components, void *stream);

/* frnn_components without waiting: enqueues the work on `stream` and returns.
 *   result_device  device, int64 [2]: receives the number of components, then a
 *                  status word (FRNN_OK, FRNN_ERR_ARG for an endpoint out of range,
 *                  FRNN_ERR_HIP for the internal bound)
 * Only kernels are enqueued, so the call can be captured into a HIP graph. */
int frnn_components_async(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n_vertices,
                          const float *scores, float threshold, void *workspace, size_t workspace_bytes,
                          int64_t *labels, int64_t *result_device, void *stream);

/* Static name of a status code. */
const char *frnn_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* FRNN_H */
