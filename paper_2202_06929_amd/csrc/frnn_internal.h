// Internal declarations shared by the host driver (frnn_api.cpp) and the HIP
// kernels (frnn_kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace frnn {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kBoundsBlocks = 256;   // most bounds partials per event
constexpr int kScanTile = 4096;      // elements per workgroup in the scans
constexpr int kListCap = 16;         // neighbours a query may collect in the main search
constexpr int kQTile = 32;           // queries of one cell handled together by a wave
constexpr int kRing = 128;           // first-stage survivors queued per wave (a power of two)
constexpr int kMaxReach = 3;         // largest cell_div
constexpr int kMaxAxes = 4;          // binned coordinates: 3, or 4 with cell_div 1
// Cells per binned axis.  The bound keeps the float32 rounding of a cell
// coordinate under the cell margin; with four axes it also lets the four
// coordinates of a cell pack into one 32-bit word (8 bits each; 10 bits each
// with three axes).
constexpr int kGridAxisMax3 = 1024;
constexpr int kGridAxisMax4 = 256;
constexpr int kMaxK = 4096;
constexpr int kMaxSearchBlocks = 8192;
// A cell's fixed cost in the search (its runs' bounds, its candidates' first
// loads), in queries, when the queries are divided among the waves by work.
constexpr unsigned int kTileWeight = 4;
// The search's queries are cut into search_pieces(DP) pieces of equal work per
// wave: each wave takes one piece of its XCD's share, then claims the share's
// other pieces one at a time from kPools counters per XCD, so that waves that
// finish early take work from the others.  Rows of up to 24 floats keep one piece
// per wave: their queries cost about the same, and the claims and the cells cut
// twice cost more than they even out (the 120k-point 8-D search took 34.9 us with
// two pieces against 30.9 with one; whole 120k-point builds with 16- and 24-float
// rows 0.089 and 0.120 ms against 0.085 and 0.117).  Wider rows, whose queries
// cost more and which run fewer waves per SIMD, take two (32-, 48- and 64-float
// rows: 0.173, 0.292 and 0.558 ms against 0.181, 0.340 and 0.713 with one).
constexpr int kMaxPieces = 2;
constexpr int search_pieces(int dpad) { return dpad <= 24 ? 1 : 2; }
constexpr int kPools = 8;
constexpr int kPoolStride = 32;  // counters 128 bytes apart
constexpr int kKeysBlock = 1024;     // threads per workgroup of the key/histogram pass
constexpr long long kKeysTwoFrom = 196608;  // events above this many rows: two points per thread in k_keys
constexpr int kPlaceBlock = 256;     // threads per workgroup of the placement pass
constexpr int kPlaceTile = 256;      // queries per workgroup of the placement pass (and kept tile)
constexpr int kKeptGroup = 64;       // kept tiles per second-level total
constexpr int kFlatTiles = 4096;     // up to this many kept tiles, placement sums the tile totals directly
constexpr int kOwnerWindow = 4096;   // output positions formed in LDS at a time in placement
constexpr int kPlaceMinBlocks = 512; // placement workgroups at least (all of them collect long lists)
constexpr int kMaxEvents = 65535;  // events per call (the second grid dimension)
// A kept count with this bit set belongs to a long list (more than kListCap
// neighbours, or more than K without the search's own selection), which the
// placement pass collects again; other lists sit at kListCap slots per original row.
constexpr unsigned int kKeptLong = 1u << 31;

// One event of a call: its rows in the concatenated points and its share of the
// cell-key space.  The first event starts at row 0 and cell 0.
struct EventDesc {
    const float *pts;  // the event's points (device, row-major [n, d])
    long long row0;    // first row of the event in the call's row numbering
    long long cell0;   // first cell key of the event
    int n;             // rows of the event
    int cells_max;     // cells reserved for the event
    int tile0;         // first scan tile of the event's cells (cell0 / kScanTile)
    int pad;
};

// Per-block min/max of the binned coordinates and a non-finite flag.
struct BoundsPartial {
    float mn[kMaxAxes];
    float mx[kMaxAxes];
    int nonfinite;
    int pad;
};

// The grid of one event, derived on the device from its bounds.
// Axis 0 varies fastest in a cell key.  Axes past the binned count have one cell.
struct Plan {
    float lo[kMaxAxes];     // smallest binned coordinate per axis
    float inv_c[kMaxAxes];  // 1 / cell edge per axis (float32)
    float c[kMaxAxes];      // cell edge per axis
    int G[kMaxAxes];        // cells per axis
    int n_cells;            // product of G
    int reach;              // neighbour cells searched on each side, per axis
    int abort;              // a coordinate was NaN or infinite
    int axes;               // binned coordinates (3 or 4)
};

// Bits per axis in a packed cell coordinate word (axis p at bits [p b, p b + b)).
__host__ __device__ constexpr int cell_bits(int axes) { return axes == 4 ? 8 : 10; }

// Single-address atomics serialise across the chip (about 11 ns each), so these
// are touched only by rare events (long lists, bad input).
struct Counters {
    unsigned int heavy_count;      // queries whose list is long (entries of the long-list queue)
    unsigned int abort;            // some event had a non-finite coordinate
    unsigned int capped;           // queries with more than K neighbours (summed after the search)
    unsigned int pad;
    unsigned long long tested;     // pairs examined, summed over the search workgroups
    unsigned long long survived;   // pairs that reached the second stage, likewise
};

// Result summary copied to the host at the end of a call (event 0's grid).
struct Report {
    long long n_edges;
    unsigned long long tested;
    unsigned long long survived;  // pairs that passed the first-stage partial test
    int abort;
    unsigned int capped;
    unsigned int heavy;
    int n_cells;
    int G[kMaxAxes];
    float c[kMaxAxes];
};

// Device buffers of one call, carved from the caller's workspace.
struct Workspace {
    EventDesc *ev;              // [n_events]
    Plan *plans;                // [n_events]
    BoundsPartial *part;        // [n_events * kBoundsBlocks]
    Counters *ctr;
    Report *report;
    long long *edge_off;        // [n_events + 2] first edge of each event, then E, then a status
    unsigned int *pcell;        // [rows] packed cell coordinates of each point
    unsigned int *rank;         // [rows] arrival rank inside its cell
    unsigned int *cell_count;   // [cells] histogram
    unsigned int *cell_start;   // [cells + 1] exclusive scan of the histogram
    unsigned long long *sums_cells;  // [tiles of cells + 1] per-tile histogram totals
    unsigned long long *sums_kept;   // [tiles of kPlaceTile rows] per-tile kept totals
    unsigned long long *sums_kept2;  // [groups of kKeptGroup tiles] per-group kept totals (more than kFlatTiles tiles)
    float *sorted;              // [rows, dpad] points in cell order, zero-padded rows
    unsigned int *sorted_id;    // [2 rows] per sorted row: its original row, then its packed cell
    unsigned int *kept;         // [rows] neighbours kept per original row (| kKeptLong for a long list)
    unsigned int *long_slots;   // [rows] sorted rows of the queries with long lists, in queue order
    unsigned int *temp;         // [rows * kListCap] neighbour lists of up to kListCap entries
    unsigned long long *tested; // [2 kMaxSearchBlocks] pairs examined, then pairs fully tested, per search workgroup
    unsigned int *capped_blk;   // [kMaxSearchBlocks] capped queries per search workgroup
    unsigned int *wave_start;   // [kMaxSearchBlocks kWaves kMaxPieces + 1] first sorted row of each search piece
    unsigned int *claims;       // [8 kPools kPoolStride] the search's piece counters, cleared by the cell scan
    long long rows;
    long long cells;
    int tiles_cells_n;
    int tiles_kept_n;
    int groups_kept_n;
    size_t total_bytes;
};

int64_t cells_max_for(int64_t n);
int dpad_for(int d);
// Fills descs[e] (if not null) for events given by row offsets; returns the total
// cell count.
// (pts stays null; callers set it).
long long describe_events(const int64_t *event_offsets, int n_events, EventDesc *descs);
// Workspace layout for events of the given sizes (host arithmetic; base may be null).
Workspace layout(void *base, long long rows, long long cells, int n_events, int d, int64_t edge_capacity);

struct LaunchArgs {
    int vec4;           // every event's rows are 16-byte aligned float4 groups (d % 4 == 0)
    int n_events;
    int max_n;          // rows of the largest event
    int d;
    int dpad;
    int axes;           // binned coordinates (3 or 4)
    int dims[kMaxAxes]; // binned coordinates, axis 0 first (unused entries -1)
    float r;
    float r2;
    int K;
    int cell_div;
    unsigned long long edge_capacity;
    long long *src;
    long long *dst;
    hipStream_t stream;
    hipEvent_t *events;     // 8 events bracketing the 7 stages, or null
    int search_blocks;      // resident workgroups of the search kernel
    int search_prio;        // 1: the search grid is one round of resident workgroups
    int bounds_blocks;      // bounds partials per event (<= kBoundsBlocks)
    EventDesc ev0;          // event 0, written to ws.ev by the first kernel when ev_from_arg
    int ev_from_arg;
    long long *edge_off_out;  // device [n_events + 2] for the edge ranges and status, or null (workspace)
    Report *report_out;       // device-visible pinned host report, or null (workspace)
};

// Enqueues the whole pipeline on a.stream; the report lands in ws.report and the
// per-event edge ranges in ws.edge_off.
hipError_t enqueue_build(const LaunchArgs &a, const Workspace &ws);

// Resident workgroups of the search kernel for rows padded to dpad (current device);
// sel: the variant for K below the list size.
int search_blocks_for(int dpad, bool sel);

}  // namespace frnn
