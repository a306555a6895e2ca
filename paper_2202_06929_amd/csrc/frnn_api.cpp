// Host side of the C interface declared in include/frnn.h: argument checks,
// workspace carving, the launch sequence and the single read-back of the edge
// count.  Arguments are checked before any HIP call, so invalid calls return
// without touching a device.

#include <math.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "frnn.h"
#include "frnn_internal.h"

namespace frnn {

// Cell capacity of an event: 2 n cells, at least 2^15 and at most 2^24.  The grid
// plan coarsens its cells until the grid fits (a speed choice only: the search is
// exact for any grid).  A grid of r-sized cells over four binned coordinates of a
// workload event has about 2 n cells (mostly empty); every cell of the capacity is
// cleared and scanned per call.
int64_t cells_max_for(int64_t n) {
    if (n <= 0) return 1;
    int64_t c = 2 * n;
    if (c < (int64_t{1} << 15)) c = int64_t{1} << 15;
    if (c > (int64_t{1} << 24)) c = int64_t{1} << 24;
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

// Binned coordinates of a call: 4 by default when d >= 5 and the cell divisor is 1,
// else 3; explicit dims without an axis count are 3.
int axes_for(const frnn_config *c, int d) {
    if (c && c->axes) return c->axes;
    if (c && c->dims[0] != c->dims[1]) return 3;
    const int div = c && c->cell_div ? c->cell_div : 1;
    return d >= 5 && div == 1 ? 4 : 3;
}

bool config_ok(const frnn_config *c, int d) {
    if (!c) return true;
    if (c->axes != 0 && c->axes != 3 && c->axes != 4) return false;
    const int axes = axes_for(c, d);
    if (axes > d) return false;
    if (axes == 4 && c->cell_div > 1) return false;  // (2R+1)^3 runs must fit a wave
    if (c->dims[0] != c->dims[1]) {
        for (int p = 0; p < axes; ++p) {
            if (c->dims[p] < 0 || c->dims[p] >= d) return false;
            for (int q = 0; q < p; ++q)
                if (c->dims[q] == c->dims[p]) return false;
        }
    }
    if (c->cell_div < 0 || c->cell_div > kMaxReach) return false;
    if (c->grid_mult != 0 && c->grid_mult != 1 && c->grid_mult != 2 && c->grid_mult != 4 && c->grid_mult != 8)
        return false;
    if (c->flags & ~(FRNN_FLAG_TIMING | FRNN_FLAG_EVENTS_RESIDENT)) return false;
    return true;
}

// Resident search workgroups per (device, padded width), computed once.
std::mutex g_blocks_mu;
std::map<std::pair<int, int>, int> g_blocks;

int search_blocks_cached(int dpad, bool sel) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const int key = dpad * 2 + (sel ? 1 : 0);
    std::lock_guard<std::mutex> lock(g_blocks_mu);
    auto it = g_blocks.find({dev, key});
    if (it != g_blocks.end()) return it->second;
    int b = search_blocks_for(dpad, sel);
    if (b > kMaxSearchBlocks) b = kMaxSearchBlocks;
    g_blocks[{dev, key}] = b;
    return b;
}

// Event tables of batched calls are copied to the device from pinned host memory
// that stays valid until the copy has run: a small ring of staging buffers per
// calling thread, each reused only after the event recorded behind its last copy
// has completed.
struct Staging {
    EventDesc *host = nullptr;
    size_t count = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
constexpr int kStagingSlots = 4;
thread_local Staging t_staging[kStagingSlots];
thread_local int t_staging_next = 0;

// Copies n_events descriptors to dev on the stream through the next staging slot.
int upload_events(const EventDesc *descs, int n_events, EventDesc *dev, hipStream_t stream) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return FRNN_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone) return FRNN_ERR_ARG;  // captured calls pass FRNN_FLAG_EVENTS_RESIDENT
    Staging &st = t_staging[t_staging_next];
    t_staging_next = (t_staging_next + 1) % kStagingSlots;
    if (st.pending) {
        if (hipEventSynchronize(st.done) != hipSuccess) return FRNN_ERR_HIP;
        st.pending = false;
    }
    if (!st.done && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) return FRNN_ERR_HIP;
    if (st.count < static_cast<size_t>(n_events)) {
        if (st.host && hipHostFree(st.host) != hipSuccess) return FRNN_ERR_HIP;
        st.host = nullptr;
        st.count = 0;
        void *p = nullptr;
        const size_t want = static_cast<size_t>(n_events) < 64 ? 64 : static_cast<size_t>(n_events);
        if (hipHostMalloc(&p, sizeof(EventDesc) * want, hipHostMallocDefault) != hipSuccess) return FRNN_ERR_HIP;
        st.host = static_cast<EventDesc *>(p);
        st.count = want;
    }
    memcpy(st.host, descs, sizeof(EventDesc) * n_events);
    if (hipMemcpyAsync(dev, st.host, sizeof(EventDesc) * n_events, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipEventRecord(st.done, stream) != hipSuccess)
        return FRNN_ERR_HIP;
    st.pending = true;
    return FRNN_OK;
}

thread_local Report *t_report = nullptr;    // pinned host copy of the device report
thread_local Report *t_report_dev = nullptr;  // its device-visible address (null: copy instead)
thread_local hipEvent_t t_events[FRNN_STAGES + 1] = {};
thread_local bool t_events_ready = false;

}  // namespace

long long describe_events(const int64_t *event_offsets, int n_events, EventDesc *descs) {
    long long cells = 0;
    for (int e = 0; e < n_events; ++e) {
        const int64_t n = event_offsets[e + 1] - event_offsets[e];
        const int64_t cm = cells_max_for(n);
        if (descs) {
            descs[e].pts = nullptr;
            descs[e].row0 = event_offsets[e] - event_offsets[0];
            descs[e].cell0 = cells;
            descs[e].n = static_cast<int>(n);
            descs[e].cells_max = static_cast<int>(cm);
            descs[e].tile0 = static_cast<int>(cells / kScanTile);
            descs[e].pad = 0;
        }
        cells += cm;
    }
    return cells;
}

Workspace layout(void *base, long long rows, long long cells, int n_events, int d) {
    const int dpad = dpad_for(d);
    const int64_t tiles_cells = (cells + 1 + kScanTile - 1) / kScanTile;
    const int64_t tiles_kept = rows > 0 ? (rows + kPlaceTile - 1) / kPlaceTile : 1;
    Carver cv{static_cast<char *>(base)};
    Workspace ws;
    ws.ev = cv.take<EventDesc>(n_events);
    ws.plans = cv.take<Plan>(n_events);
    ws.part = cv.take<BoundsPartial>(static_cast<size_t>(n_events) * kBoundsBlocks);
    ws.ctr = cv.take<Counters>(1);
    ws.report = cv.take<Report>(1);
    ws.edge_off = cv.take<long long>(static_cast<size_t>(n_events) + 2);
    ws.pcell = cv.take<unsigned int>(rows);
    ws.rank = cv.take<unsigned int>(rows);
    ws.cell_count = cv.take<unsigned int>(cells);
    ws.cell_start = cv.take<unsigned int>(cells + 1);
    ws.sums_cells = cv.take<unsigned long long>(tiles_cells);
    const int64_t groups_kept = (tiles_kept + kKeptGroup - 1) / kKeptGroup;
    ws.sums_kept = cv.take<unsigned long long>(tiles_kept);
    ws.sums_kept2 = cv.take<unsigned long long>(groups_kept);
    // One padding row after the last: the search requests the row after each query.
    ws.sorted = cv.take<float>(static_cast<size_t>(rows + 1) * dpad);
    ws.sorted_id = cv.take<unsigned int>(2 * rows);
    ws.kept = cv.take<unsigned int>(rows);
    ws.long_slots = cv.take<unsigned int>(rows);
    ws.temp = cv.take<unsigned int>(static_cast<size_t>(rows) * kListCap);
    ws.tested = cv.take<unsigned long long>(2 * kMaxSearchBlocks);
    ws.capped_blk = cv.take<unsigned int>(kMaxSearchBlocks);
    ws.wave_start = cv.take<unsigned int>(static_cast<size_t>(kMaxSearchBlocks) * kWaves * kMaxPieces + 1);
    ws.claims = cv.take<unsigned int>(8 * kPools * kPoolStride);
    ws.rows = rows;
    ws.cells = cells;
    ws.tiles_cells_n = static_cast<int>(tiles_cells);
    ws.tiles_kept_n = static_cast<int>(tiles_kept);
    ws.groups_kept_n = static_cast<int>(groups_kept);
    ws.total_bytes = cv.at;
    return ws;
}

}  // namespace frnn

using namespace frnn;

namespace {

// Arguments shared by the single-event and batched calls.
int check_common(int32_t d, float r, int32_t K, int64_t edge_capacity, const frnn_config *config) {
    if (d < 3 || d > FRNN_MAX_D || !(r > 0.0f) || !isfinite(r) || K < 1 || K > FRNN_MAX_K || edge_capacity < 0 ||
        !config_ok(config, d))
        return FRNN_ERR_ARG;
    return FRNN_OK;
}

int check_events(const int64_t *event_offsets, int32_t n_events, long long *rows, int *max_n, long long *cells) {
    if (!event_offsets || n_events < 1 || n_events > kMaxEvents) return FRNN_ERR_ARG;
    long long mx = 0;
    for (int e = 0; e < n_events; ++e) {
        const int64_t n = event_offsets[e + 1] - event_offsets[e];
        if (n < 0) return FRNN_ERR_ARG;
        if (n > mx) mx = n;
    }
    *rows = event_offsets[n_events] - event_offsets[0];
    if (*rows >= (int64_t{1} << 31)) return FRNN_ERR_UNSUPPORTED;
    *cells = describe_events(event_offsets, n_events, nullptr);
    if (*cells >= (int64_t{1} << 31)) return FRNN_ERR_UNSUPPORTED;
    *max_n = static_cast<int>(mx);
    return FRNN_OK;
}

// Enqueues the pipeline for checked arguments (descriptors uploaded first unless
// they are already resident).  Returns a status and the workspace view.
int enqueue(const EventDesc *descs, int n_events, long long rows, long long cells, int max_n,
            int32_t d, float r, int32_t K, void *workspace, int64_t *src, int64_t *dst, int64_t edge_capacity,
            const frnn_config *config, hipStream_t stream, bool upload, long long *edge_off_out, Workspace *ws_out,
            bool *timing_out, Report *report_out = nullptr) {
    const int axes = axes_for(config, d);
    int dims[kMaxAxes] = {-1, -1, -1, -1};
    for (int p = 0; p < axes; ++p)
        dims[p] = (config && config->dims[0] != config->dims[1]) ? config->dims[p] : d - axes + p;
    LaunchArgs a;
    a.vec4 = d % 4 == 0 ? 1 : 0;
    for (int e = 0; e < n_events && a.vec4; ++e)
        if (reinterpret_cast<uintptr_t>(descs[e].pts) % 16 != 0) a.vec4 = 0;
    a.n_events = n_events;
    a.max_n = max_n;
    a.d = d;
    a.dpad = dpad_for(d);
    a.axes = axes;
    for (int p = 0; p < kMaxAxes; ++p) a.dims[p] = dims[p];
    a.r = r;
    a.r2 = r * r;
    a.K = K;
    a.cell_div = (config && config->cell_div) ? config->cell_div : 1;
    a.edge_capacity = static_cast<unsigned long long>(edge_capacity);
    a.src = reinterpret_cast<long long *>(src);
    a.dst = reinterpret_cast<long long *>(dst);
    a.stream = stream;
    // One round of resident workgroups (whose waves then order their issue by
    // progress) unless each resident wave would get more than 128 rows; then up to
    // four times as many workgroups as fit at once, so that the hardware hands the
    // remaining shares to whichever workgroups finish first.
    {
        const int resident = search_blocks_cached(a.dpad, K < kListCap);
        const long long per_wave = rows / (static_cast<long long>(resident) * kWaves);
        long long m = per_wave < 128 ? 1 : per_wave / 128 + 1;
        m = m > 4 ? 4 : m;
        if (config && config->grid_mult > 0) m = config->grid_mult;
        const long long b = resident * m;
        a.search_blocks = static_cast<int>(b > kMaxSearchBlocks ? kMaxSearchBlocks : b);
        a.search_prio = a.search_blocks <= resident ? 1 : 0;
    }
    // About 16 coordinates per thread of the bounds pass, at most kBoundsBlocks blocks per event.
    const long long bb = (static_cast<long long>(max_n) * d + 16 * kBlock - 1) / (16 * kBlock);
    a.bounds_blocks = static_cast<int>(bb < 1 ? 1 : (bb > kBoundsBlocks ? kBoundsBlocks : bb));
    a.ev0 = descs ? descs[0] : EventDesc{};
    a.ev_from_arg = n_events == 1 ? 1 : 0;
    a.edge_off_out = edge_off_out;
    a.report_out = report_out;
    const Workspace ws = layout(workspace, rows, cells, n_events, d);
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
    // Batches: descriptors go to the device first, from pinned staging memory.
    if (n_events > 1 && upload) {
        const int us = upload_events(descs, n_events, ws.ev, stream);
        if (us != FRNN_OK) return us;
    }
    if (enqueue_build(a, ws) != hipSuccess) return FRNN_ERR_HIP;
    *ws_out = ws;
    *timing_out = timing;
    return FRNN_OK;
}

int report_status(const Report &rep, frnn_stats *stats, bool timing, int64_t edge_capacity);

// Enqueues, copies the report (and the per-event edge ranges) back and waits.
int run(const EventDesc *descs, int n_events, long long rows, long long cells, int max_n,
        int32_t d, float r, int32_t K, void *workspace, int64_t *src, int64_t *dst, int64_t edge_capacity,
        const frnn_config *config, frnn_stats *stats, hipStream_t stream, Report *rep_out,
        int64_t *edge_offsets_host) {
    // The last kernel writes the report straight into pinned host memory when the
    // runtime maps it for the device; otherwise it is copied back.
    if (!t_report) {
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(Report), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            if (hipHostMalloc(&p, sizeof(Report), hipHostMallocDefault) != hipSuccess) return FRNN_ERR_HIP;
        } else {
            void *dp = nullptr;
            if (hipHostGetDevicePointer(&dp, p, 0) == hipSuccess) t_report_dev = static_cast<Report *>(dp);
        }
        t_report = static_cast<Report *>(p);
    }
    Workspace ws;
    bool timing = false;
    t_report->n_edges = -1;
    const int st = enqueue(descs, n_events, rows, cells, max_n, d, r, K, workspace, src, dst, edge_capacity,
                           config, stream, true, nullptr, &ws, &timing, t_report_dev);
    if (st != FRNN_OK) return st;
    if (!t_report_dev &&
        hipMemcpyAsync(t_report, ws.report, sizeof(Report), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return FRNN_ERR_HIP;
    if (edge_offsets_host &&
        hipMemcpyAsync(edge_offsets_host, ws.edge_off, sizeof(long long) * (n_events + 1), hipMemcpyDeviceToHost,
                       stream) != hipSuccess)
        return FRNN_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return FRNN_ERR_HIP;
    std::atomic_thread_fence(std::memory_order_acquire);
    memcpy(rep_out, t_report, sizeof(Report));
    return report_status(*rep_out, stats, timing, edge_capacity);
}

// Status of a finished call from its report; fills the stats.
int report_status(const Report &rep, frnn_stats *stats, bool timing, int64_t edge_capacity) {
    if (rep.n_edges < 0) return FRNN_ERR_HIP;  // the report never arrived
    if (stats) {
        stats->n_edges = rep.n_edges;
        stats->candidates = static_cast<int64_t>(rep.tested);
        stats->survivors = static_cast<int64_t>(rep.survived);
        stats->n_cells = rep.n_cells;
        for (int p = 0; p < kMaxAxes; ++p) {
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
    if (rep.n_edges > edge_capacity) return FRNN_ERR_CAPACITY;
    return FRNN_OK;
}

void init_stats(frnn_stats *stats, const frnn_config *config, int d) {
    if (!stats) return;
    memset(stats, 0, sizeof(*stats));
    const bool set = config && config->dims[0] != config->dims[1];
    const int axes = axes_for(config, d);
    stats->axes = axes;
    for (int p = 0; p < kMaxAxes; ++p)
        stats->dims[p] = p >= axes ? -1 : (set ? config->dims[p] : d - axes + p);
}

}  // namespace

extern "C" size_t frnn_workspace_bytes(int64_t n, int32_t d) {
    if (n < 0 || n >= (int64_t{1} << 31) || d < 3 || d > FRNN_MAX_D) return 0;
    const int64_t offs[2] = {0, n};
    return layout(nullptr, n, describe_events(offs, 1, nullptr), 1, d).total_bytes;
}

extern "C" size_t frnn_batch_workspace_bytes(const int64_t *event_offsets, int32_t n_events, int32_t d) {
    long long rows = 0, cells = 0;
    int max_n = 0;
    if (d < 3 || d > FRNN_MAX_D) return 0;
    if (check_events(event_offsets, n_events, &rows, &max_n, &cells) != FRNN_OK) return 0;
    return layout(nullptr, rows, cells, n_events, d).total_bytes;
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
    if (!n_edges || n < 0) return FRNN_ERR_ARG;
    const int st = check_common(d, r, K, edge_capacity, config);
    if (st != FRNN_OK) return st;
    if (n >= (int64_t{1} << 31)) return FRNN_ERR_UNSUPPORTED;
    init_stats(stats, config, d);
    *n_edges = 0;
    if (n == 0) return FRNN_OK;
    if (!points || !workspace || (edge_capacity > 0 && (!src || !dst))) return FRNN_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FRNN_ERR_ARG;
    if (workspace_bytes < frnn_workspace_bytes(n, d)) return FRNN_ERR_WORKSPACE;
    const int64_t offs[2] = {0, n};
    EventDesc desc;
    const long long cells = describe_events(offs, 1, &desc);
    desc.pts = points;
    Report rep;
    const int rs = run(&desc, 1, n, cells, static_cast<int>(n), d, r, K, workspace, src, dst, edge_capacity,
                       config, stats, static_cast<hipStream_t>(stream), &rep, nullptr);
    if (rs == FRNN_OK || rs == FRNN_ERR_CAPACITY) *n_edges = rep.n_edges;
    return rs;
}

extern "C" int frnn_build_batch(const float *points, const int64_t *event_offsets, int32_t n_events, int32_t d,
                                float r, int32_t K, void *workspace, size_t workspace_bytes, int64_t *src,
                                int64_t *dst, int64_t edge_capacity, int64_t *edge_offsets,
                                const frnn_config *config, frnn_stats *stats, void *stream) {
    if (!edge_offsets) return FRNN_ERR_ARG;
    const int st = check_common(d, r, K, edge_capacity, config);
    if (st != FRNN_OK) return st;
    long long rows = 0, cells = 0;
    int max_n = 0;
    const int se = check_events(event_offsets, n_events, &rows, &max_n, &cells);
    if (se != FRNN_OK) return se;
    init_stats(stats, config, d);
    for (int e = 0; e <= n_events; ++e) edge_offsets[e] = 0;
    if (rows == 0) return FRNN_OK;
    if (!points || !workspace || (edge_capacity > 0 && (!src || !dst))) return FRNN_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FRNN_ERR_ARG;
    if (workspace_bytes < layout(nullptr, rows, cells, n_events, d).total_bytes)
        return FRNN_ERR_WORKSPACE;
    std::vector<EventDesc> descs(n_events);
    describe_events(event_offsets, n_events, descs.data());
    for (int e = 0; e < n_events; ++e) descs[e].pts = points + static_cast<size_t>(event_offsets[e]) * d;
    Report rep;
    const int rs = run(descs.data(), n_events, rows, cells, max_n, d, r, K, workspace, src, dst,
                       edge_capacity, config, stats, static_cast<hipStream_t>(stream), &rep, edge_offsets);
    if (rs == FRNN_ERR_CAPACITY) {
        for (int e = 0; e < n_events; ++e) edge_offsets[e] = 0;
        edge_offsets[n_events] = rep.n_edges;
    }
    return rs;
}

extern "C" int frnn_build_batch_async(const float *points, const int64_t *event_offsets, int32_t n_events,
                                      int32_t d, float r, int32_t K, void *workspace, size_t workspace_bytes,
                                      int64_t *src, int64_t *dst, int64_t edge_capacity,
                                      int64_t *edge_offsets_device, const frnn_config *config, void *stream) {
    if (!edge_offsets_device) return FRNN_ERR_ARG;
    if (config && (config->flags & FRNN_FLAG_TIMING)) return FRNN_ERR_ARG;
    const int st = check_common(d, r, K, edge_capacity, config);
    if (st != FRNN_OK) return st;
    long long rows = 0, cells = 0;
    int max_n = 0;
    const int se = check_events(event_offsets, n_events, &rows, &max_n, &cells);
    if (se != FRNN_OK) return se;
    if (rows == 0) return FRNN_ERR_ARG;
    if (!points || !workspace || (edge_capacity > 0 && (!src || !dst))) return FRNN_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FRNN_ERR_ARG;
    if (workspace_bytes < layout(nullptr, rows, cells, n_events, d).total_bytes)
        return FRNN_ERR_WORKSPACE;
    std::vector<EventDesc> descs(n_events);
    describe_events(event_offsets, n_events, descs.data());
    for (int e = 0; e < n_events; ++e) descs[e].pts = points + static_cast<size_t>(event_offsets[e]) * d;
    const bool resident = config && (config->flags & FRNN_FLAG_EVENTS_RESIDENT);
    Workspace ws;
    bool timing = false;
    return enqueue(descs.data(), n_events, rows, cells, max_n, d, r, K, workspace, src, dst, edge_capacity,
                   config, static_cast<hipStream_t>(stream), !resident,
                   reinterpret_cast<long long *>(edge_offsets_device), &ws, &timing);
}

extern "C" int frnn_build_events_async(const float *const *event_points, const int64_t *event_sizes,
                                       int32_t n_events, int32_t d, float r, int32_t K, void *workspace,
                                       size_t workspace_bytes, int64_t *src, int64_t *dst, int64_t edge_capacity,
                                       int64_t *edge_offsets_device, const frnn_config *config, void *stream) {
    if (!edge_offsets_device || !event_points || !event_sizes || n_events < 1 || n_events > kMaxEvents)
        return FRNN_ERR_ARG;
    if (config && (config->flags & FRNN_FLAG_TIMING)) return FRNN_ERR_ARG;
    const int st = check_common(d, r, K, edge_capacity, config);
    if (st != FRNN_OK) return st;
    std::vector<int64_t> offs(n_events + 1, 0);
    for (int e = 0; e < n_events; ++e) {
        if (event_sizes[e] < 0 || (event_sizes[e] > 0 && !event_points[e])) return FRNN_ERR_ARG;
        offs[e + 1] = offs[e] + event_sizes[e];
    }
    long long rows = 0, cells = 0;
    int max_n = 0;
    const int se = check_events(offs.data(), n_events, &rows, &max_n, &cells);
    if (se != FRNN_OK) return se;
    if (rows == 0) return FRNN_ERR_ARG;
    if (!workspace || (edge_capacity > 0 && (!src || !dst))) return FRNN_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FRNN_ERR_ARG;
    if (workspace_bytes < layout(nullptr, rows, cells, n_events, d).total_bytes)
        return FRNN_ERR_WORKSPACE;
    std::vector<EventDesc> descs(n_events);
    describe_events(offs.data(), n_events, descs.data());
    for (int e = 0; e < n_events; ++e) descs[e].pts = event_points[e];
    const bool resident = config && (config->flags & FRNN_FLAG_EVENTS_RESIDENT);
    Workspace ws;
    bool timing = false;
    return enqueue(descs.data(), n_events, rows, cells, max_n, d, r, K, workspace, src, dst, edge_capacity, config,
                   static_cast<hipStream_t>(stream), !resident, reinterpret_cast<long long *>(edge_offsets_device),
                   &ws, &timing);
}

// ------------------------------------------------------- no-allocation build

namespace {

// Workspace of frnn_build_noalloc: one array per device, held until the process
// ends.  Host code never passes this name to a kernel or a copy (on the host it
// only stands for the symbol); it uses the device address looked up below.
constexpr size_t kNoAllocBytes = size_t{FRNN_NOALLOC_SCRATCH_MIB} << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocDevices] = {};

// The current device's address of `scratch`, looked up once per device (with
// that device current).  The same first call also fills the search-grid cache
// for every row width, so that later calls insert nothing into it.
int noalloc_workspace(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FRNN_ERR_HIP;
    if (dev < 0 || dev >= kNoAllocDevices) return FRNN_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FRNN_ERR_HIP;
        if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return FRNN_ERR_HIP;
        for (int dp : {4, 8, 12, 16, 24, 32, 48, 64}) {
            search_blocks_cached(dp, false);
            search_blocks_cached(dp, true);
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return FRNN_OK;
}

}  // namespace

extern "C" int frnn_build_noalloc(const float *points, int64_t n, int32_t d, float r, int32_t K, int64_t *src,
                                  int64_t *dst, int64_t edge_capacity, int64_t *n_edges,
                                  const frnn_config *config, frnn_stats *stats, void *stream) {
    if (!n_edges || n < 0) return FRNN_ERR_ARG;
    const int st = check_common(d, r, K, edge_capacity, config);
    if (st != FRNN_OK) return st;
    if (config && (config->flags & FRNN_FLAG_TIMING)) return FRNN_ERR_ARG;  // would create HIP events
    if (n >= (int64_t{1} << 31)) return FRNN_ERR_UNSUPPORTED;
    init_stats(stats, config, d);
    *n_edges = 0;
    if (n == 0) return FRNN_OK;
    if (!points || (edge_capacity > 0 && (!src || !dst))) return FRNN_ERR_ARG;
    if (frnn_workspace_bytes(n, d) > kNoAllocBytes) return FRNN_ERR_WORKSPACE;
    void *workspace = nullptr;
    const int sw = noalloc_workspace(&workspace);
    if (sw != FRNN_OK) return sw;
    const int64_t offs[2] = {0, n};
    EventDesc desc;
    const long long cells = describe_events(offs, 1, &desc);
    desc.pts = points;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace ws;
    bool timing = false;
    const int se = enqueue(&desc, 1, n, cells, static_cast<int>(n), d, r, K, workspace, src, dst, edge_capacity,
                           config, s, false, nullptr, &ws, &timing);
    if (se != FRNN_OK) return se;
    // The report stays in the scratch array and is copied into this frame.
    Report rep;
    rep.n_edges = -1;
    if (hipMemcpyAsync(&rep, ws.report, sizeof(Report), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FRNN_ERR_HIP;
    const int rs = report_status(rep, stats, false, edge_capacity);
    if (rs == FRNN_OK || rs == FRNN_ERR_CAPACITY) *n_edges = rep.n_edges;
    return rs;
}
