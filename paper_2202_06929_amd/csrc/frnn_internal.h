// Internal declarations shared by the host driver (frnn_api.cpp) and the HIP
// kernels (frnn_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace frnn {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kBoundsBlocks = 128;   // partial results of the bounds pass
constexpr int kScanTile = 4096;      // elements per workgroup in the scans
constexpr int kListCap = 32;         // neighbours a query may collect in the main search
constexpr int kQTile = 32;           // queries of one cell handled together by a wave
constexpr int kMaxReach = 3;         // largest cell_div
constexpr int kMaxRuns = (2 * kMaxReach + 1) * (2 * kMaxReach + 1);
constexpr int kGridAxisMax = 1024;   // cells per binned axis (bounds the key rounding error)
constexpr int kMaxK = 4096;
constexpr int kMaxSearchBlocks = 8192;
constexpr int kKeysBlock = 1024;     // threads per workgroup of the key/histogram pass

// Per-block min/max of the binned coordinates and a non-finite flag.
struct BoundsPartial {
    float mn[3];
    float mx[3];
    int nonfinite;
    int pad;
};

// The grid of one call, derived on the device from the bounds.
struct Plan {
    float lo[3];      // smallest binned coordinate per axis
    float inv_c[3];   // 1 / cell edge per axis (float32)
    float c[3];       // cell edge per axis
    int G[3];         // cells per axis
    int n_cells;      // G[0] * G[1] * G[2]
    int reach;        // neighbour cells searched on each side, per axis
    int abort;        // a coordinate was NaN or infinite
    int pad;
};

// Counters cleared at the start of every call.
// Single-address atomics serialise across the chip (about 11 ns each), so these
// are touched only by rare events (long lists, capped queries).
struct Counters {
    unsigned long long heavy_top;  // next free slot of the long-list store
    unsigned int heavy_count;      // queries sent to the long-list path
    unsigned int capped;           // queries with more than K neighbours
};

// Result summary copied to the host at the end of a call.
struct Report {
    long long n_edges;
    unsigned long long tested;
    int abort;
    unsigned int capped;
    unsigned int heavy;
    int n_cells;
    int G[3];
    float c[3];
};

// A query whose neighbour list did not fit the list of the main search.
struct HeavyEntry {
    unsigned int slot;    // position of the query in cell order
    unsigned int count;   // |N(i)| before the cap
    unsigned int cell;    // its cell key
    unsigned int pad;
};

// Device buffers of one call, carved from the caller's workspace.
struct Workspace {
    BoundsPartial *part;
    Plan *plan;
    Counters *ctr;
    Report *report;
    unsigned int *key;          // [n] cell key of each point
    unsigned int *rank;         // [n] arrival rank inside its cell
    unsigned int *cell_count;   // [cells_max] histogram
    unsigned int *cell_start;   // [cells_max + 1] exclusive scan of the histogram
    unsigned long long *sums_cells;  // [tiles of cells_max + 1] per-tile histogram totals
    unsigned long long *sums_kept;   // [tiles of n + 1] per-tile kept totals
    float *sorted;              // [n, dpad] points in cell order, zero-padded rows
    unsigned int *sorted_id;    // [n] original index of each sorted row
    unsigned int *kept;         // [n] neighbours kept per original index
    unsigned long long *tpos;   // [n] where each query's list sits in `temp`
    long long *off;             // [n + 1] exclusive scan of kept (output offsets)
    HeavyEntry *heavy;          // [n]
    unsigned int *temp;         // [n * kListCap + edge_capacity] neighbour lists
    unsigned long long *tested; // [kMaxSearchBlocks] pairs examined per search workgroup
    int tiles_cells_n;
    int tiles_kept_n;
    size_t total_bytes;
};

int64_t cells_max_for(int64_t n);
int dpad_for(int d);
Workspace layout(void *base, int64_t n, int d, int64_t edge_capacity);

struct LaunchArgs {
    const float *points;
    int n;
    int d;
    int dpad;
    int dims[3];
    float r;
    float r2;
    int K;
    int cell_div;
    int tile;
    int64_t cells_max;
    unsigned long long edge_capacity;
    long long *src;
    long long *dst;
    hipStream_t stream;
    hipEvent_t *events;  // 9 events bracketing the 8 stages, or null
    int search_blocks;   // resident workgroups of the search kernel
};

// Enqueues the whole pipeline on a.stream; the report lands in ws.report.
hipError_t enqueue_build(const LaunchArgs &a, const Workspace &ws);

// Resident workgroups of the search kernel for rows padded to dpad (per device).
int search_blocks_for(int dpad);

}  // namespace frnn
