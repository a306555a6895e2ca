// Host side of the C interface declared in include/frnn.h: argument checks,
// workspace carving, the launch sequence and the single read-back of the edge
// count.  Arguments are checked before any HIP call, so invalid calls return
// without touching a device.

#include <math.h>
#include <string.h>

#include <map>
#include <mutex>
#include <utility>

#include "frnn.h"
#include "frnn_internal.h"

namespace frnn {

int64_t cells_max_for(int64_t n) {
    int64_t c = 4 * n;
    if (c < (int64_t{1} << 15)) c = int64_t{1} << 15;
    if (c > (int64_t{1} << 22)) c = int64_t{1} << 22;
    return c;
}

int dpad_for(int d) {
    static const int pads[] = {4, 8, 12, 16, 24, 32, 48, 64};
    for (int p : pads)
        if (d <= p) return p;
    return -1;
}

namespace {

size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct Carver {
    char *base;
    size_t at = 0;
    template <typename T>
    T *take(size_t count) {
        T *p = base ? reinterpret_cast<T *>(base + at) : nullptr;
        at += align_up(count * sizeof(T) + 1);
        return p;
    }
};

bool config_ok(const frnn_config *c, int d) {
    if (!c) return true;
    if (c->dims[0] != c->dims[1]) {
        for (int p = 0; p < 3; ++p)
            if (c->dims[p] < 0 || c->dims[p] >= d) return false;
        if (c->dims[0] == c->dims[2] || c->dims[1] == c->dims[2]) return false;
    }
    if (c->cell_div < 0 || c->cell_div > kMaxReach) return false;
    if (c->tile != 0 && c->tile != 32 && c->tile != 64) return false;
    if (c->flags & ~FRNN_FLAG_TIMING) return false;
    return true;
}

// Resident search workgroups per (device, padded width), computed once.
std::mutex g_blocks_mu;
std::map<std::pair<int, int>, int> g_blocks;

int search_blocks_cached(int dpad) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lock(g_blocks_mu);
    auto it = g_blocks.find({dev, dpad});
    if (it != g_blocks.end()) return it->second;
    int b = search_blocks_for(dpad);
    if (b > kMaxSearchBlocks) b = kMaxSearchBlocks;
    g_blocks[{dev, dpad}] = b;
    return b;
}

thread_local Report *t_report = nullptr;  // pinned host copy of the device report
thread_local hipEvent_t t_events[FRNN_STAGES + 1] = {};
thread_local bool t_events_ready = false;

}  // namespace

Workspace layout(void *base, int64_t n, int d, int64_t edge_capacity) {
    const int dpad = dpad_for(d);
    const int64_t cells = cells_max_for(n);
    const int64_t tiles_cells = (cells + 1 + kScanTile - 1) / kScanTile;
    const int64_t tiles_kept = (n + 1 + kScanTile - 1) / kScanTile;
    Carver cv{static_cast<char *>(base)};
    Workspace ws;
    ws.part = cv.take<BoundsPartial>(kBoundsBlocks);
    ws.plan = cv.take<Plan>(1);
    ws.ctr = cv.take<Counters>(1);
    ws.report = cv.take<Report>(1);
    ws.key = cv.take<unsigned int>(n);
    ws.rank = cv.take<unsigned int>(n);
    ws.cell_count = cv.take<unsigned int>(cells);
    ws.cell_start = cv.take<unsigned int>(cells + 1);
    ws.sums_cells = cv.take<unsigned long long>(tiles_cells);
    ws.sums_kept = cv.take<unsigned long long>(tiles_kept);
    ws.sorted = cv.take<float>(static_cast<size_t>(n) * dpad);
    ws.sorted_id = cv.take<unsigned int>(n);
    ws.kept = cv.take<unsigned int>(n);
    ws.tpos = cv.take<unsigned long long>(n);
    ws.off = cv.take<long long>(n + 1);
    ws.heavy = cv.take<HeavyEntry>(n);
    ws.temp = cv.take<unsigned int>(static_cast<size_t>(n) * kListCap + static_cast<size_t>(edge_capacity));
    ws.tested = cv.take<unsigned long long>(kMaxSearchBlocks);
    ws.tiles_cells_n = static_cast<int>(tiles_cells);
    ws.tiles_kept_n = static_cast<int>(tiles_kept);
    ws.total_bytes = cv.at;
    return ws;
}

}  // namespace frnn

using namespace frnn;

extern "C" size_t frnn_workspace_bytes(int64_t n, int32_t d, int64_t edge_capacity) {
    if (n < 0 || n >= (int64_t{1} << 31) || d < 3 || d > FRNN_MAX_D || edge_capacity < 0) return 0;
    return layout(nullptr, n, d, edge_capacity).total_bytes;
}

extern "C" const char *frnn_status_string(int status) {
    switch (status) {
        case FRNN_OK: return "ok";
        case FRNN_ERR_ARG: return "invalid argument";
        case FRNN_ERR_NONFINITE: return "non-finite coordinate";
        case FRNN_ERR_CAPACITY: return "edge capacity too small";
        case FRNN_ERR_WORKSPACE: return "workspace too small";
        case FRNN_ERR_UNSUPPORTED: return "unsupported size";
        case FRNN_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

extern "C" int frnn_build(const float *points, int64_t n, int32_t d, float r, int32_t K,
                          void *workspace, size_t workspace_bytes, int64_t *src, int64_t *dst,
                          int64_t edge_capacity, int64_t *n_edges, const frnn_config *config,
                          frnn_stats *stats, void *stream) {
    if (!n_edges || n < 0 || d < 3 || d > FRNN_MAX_D || !(r > 0.0f) || !isfinite(r) || K < 1 ||
        K > FRNN_MAX_K || edge_capacity < 0 || !config_ok(config, d))
        return FRNN_ERR_ARG;
    if (n >= (int64_t{1} << 31)) return FRNN_ERR_UNSUPPORTED;
    int dims[3] = {d - 3, d - 2, d - 1};
    if (config && config->dims[0] != config->dims[1])
        for (int p = 0; p < 3; ++p) dims[p] = config->dims[p];
    const int cell_div = (config && config->cell_div) ? config->cell_div : 1;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        for (int p = 0; p < 3; ++p) stats->dims[p] = dims[p];
    }
    *n_edges = 0;
    if (n == 0) return FRNN_OK;
    if (!points || !workspace || (edge_capacity > 0 && (!src || !dst))) return FRNN_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FRNN_ERR_ARG;
    const size_t need = frnn_workspace_bytes(n, d, edge_capacity);
    if (workspace_bytes < need) return FRNN_ERR_WORKSPACE;

    LaunchArgs a;
    a.points = points;
    a.n = static_cast<int>(n);
    a.d = d;
    a.dpad = dpad_for(d);
    for (int p = 0; p < 3; ++p) a.dims[p] = dims[p];
    a.r = r;
    a.r2 = r * r;
    a.K = K;
    a.cell_div = cell_div;
    a.tile = (config && config->tile) ? config->tile : 64;
    a.cells_max = cells_max_for(n);
    a.edge_capacity = static_cast<unsigned long long>(edge_capacity);
    a.src = reinterpret_cast<long long *>(src);
    a.dst = reinterpret_cast<long long *>(dst);
    a.stream = static_cast<hipStream_t>(stream);
    a.search_blocks = search_blocks_cached(a.dpad);
    const Workspace ws = layout(workspace, n, d, edge_capacity);
    const bool timing = config && (config->flags & FRNN_FLAG_TIMING);
    a.events = nullptr;
    if (timing) {
        if (!t_events_ready) {
            for (auto &e : t_events)
                if (hipEventCreate(&e) != hipSuccess) return FRNN_ERR_HIP;
            t_events_ready = true;
        }
        a.events = t_events;
    }

    if (!t_report) {
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(Report), hipHostMallocDefault) != hipSuccess) return FRNN_ERR_HIP;
        t_report = static_cast<Report *>(p);
    }
    if (enqueue_build(a, ws) != hipSuccess) return FRNN_ERR_HIP;
    if (hipMemcpyAsync(t_report, ws.report, sizeof(Report), hipMemcpyDeviceToHost, a.stream) != hipSuccess)
        return FRNN_ERR_HIP;
    if (hipStreamSynchronize(a.stream) != hipSuccess) return FRNN_ERR_HIP;
    const Report rep = *t_report;
    if (stats) {
        stats->n_edges = rep.n_edges;
        stats->candidates = static_cast<int64_t>(rep.tested);
        stats->n_cells = rep.n_cells;
        for (int p = 0; p < 3; ++p) {
            stats->grid[p] = rep.G[p];
            stats->cell[p] = rep.c[p];
        }
        stats->capped_queries = static_cast<int32_t>(rep.capped);
        stats->overflow_queries = static_cast<int32_t>(rep.heavy);
        if (timing)
            for (int k = 0; k < FRNN_STAGES; ++k)
                if (hipEventElapsedTime(&stats->stage_ms[k], t_events[k], t_events[k + 1]) != hipSuccess)
                    return FRNN_ERR_HIP;
    }
    if (rep.abort) return FRNN_ERR_NONFINITE;
    *n_edges = rep.n_edges;
    if (rep.n_edges > edge_capacity) return FRNN_ERR_CAPACITY;
    return FRNN_OK;
}
