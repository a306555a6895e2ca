// HIP kernels of the FRNN graph builder for CDNA4 (gfx950, wave64).
//
// Pipeline of one call (paper, Section 3.4: bin the points by three projected
// coordinates into grid cells, then visit only the cells around each query):
//   k_bounds      min/max of the binned coordinates and a non-finite check over
//                 all coordinates; clears the histogram, tile totals, counters
//   k_keys        grid plan (cell edge, cells per axis), cell key of every point,
//                 histogram with in-cell arrival rank, per-tile histogram totals
//   k_scan_cells  exclusive scan of the histogram -> first sorted row of each cell;
//                 the search's shares of equal work (cells' fixed costs plus queries)
//   k_scatter     counting-sort scatter: rows copied into cell order
//   k_search      each wave takes a share of equal work in cell order: a
//                 cell's queries against the (2R+1)^(axes-1) contiguous runs of
//                 neighbouring cells along axis 0; each lane holds one candidate (its
//                 first four coordinates), query rows are wave-uniform; an exact
//                 early exit after the first two or three terms of the distance
//                 sum; ballots queue the survivors, whose sums are finished 64 at a
//                 time; the lists of pending queries are stored as found, in batches
//   k_kept_sums   kept totals per placement tile and per group of tiles
//   k_place       output offsets from the totals and a block scan; each short list
//                 sorted by its query's thread and the block's output formed in LDS,
//                 then written to its (i asc, j asc) positions with coalesced
//                 stores; then the queued lists longer than the search keeps, or
//                 longer than K, collected again, one per workgroup at a time (the K
//                 smallest by (D, j) from an MSB-first radix select)
//
// Distances follow one fixed order with every product and sum rounded on its
// own: this file is compiled with -ffp-contract=off and the pragma below.

#include <float.h>

#include "frnn_internal.h"

#pragma clang fp contract(off)

namespace frnn {
namespace {

__device__ __forceinline__ unsigned int prefix_count(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<unsigned int>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<unsigned int>(mask), 0u));
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
// Wave index inside the workgroup, marked wave-uniform for the compiler (so that
// values derived from it live in scalar registers and feed scalar loads).
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

__device__ __forceinline__ unsigned int uniform(unsigned int v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders the LDS accesses of one wave (lanes of a wave exchange data through LDS
// without a workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Partial sum of the definition over coordinates [K0, K1): ascending order, every
// product and sum rounded on its own.  Rows are zero-padded; adding +0 leaves a
// sum unchanged, so padded rows give the same D as unpadded ones.  Partial sums of
// non-negative terms never decrease, so s >= r2 after a prefix rejects exactly.
template <int K0, int K1, int DP>
__device__ __forceinline__ float add_terms(float s, const float (&a)[DP], const float *__restrict__ b) {
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        const float t = a[k] - b[k];
        const float t2 = t * t;
        s = s + t2;
    }
    return s;
}

// The same partial sum with the second row held in registers.
template <int K0, int K1, int DP, int NB>
__device__ __forceinline__ float add_terms_r(float s, const float (&a)[DP], const float (&b)[NB]) {
#pragma unroll
    for (int k = K0; k < K1; ++k) {
        const float t = a[k] - b[k];
        const float t2 = t * t;
        s = s + t2;
    }
    return s;
}

template <int DP>
__device__ __forceinline__ float sq_dist(const float (&a)[DP], const float *__restrict__ b) {
    return add_terms<0, DP, DP>(0.0f, a, b);
}

// Row `s` of the zero-padded sorted points (DP is a multiple of 4, rows 16-byte aligned).
template <int DP>
__device__ __forceinline__ void load_row(const float *__restrict__ sorted, unsigned int s, float (&c)[DP]) {
    const float4 *row = reinterpret_cast<const float4 *>(sorted + static_cast<size_t>(s) * DP);
#pragma unroll
    for (int k = 0; k < DP / 4; ++k) {
        const float4 v = row[k];
        c[4 * k] = v.x;
        c[4 * k + 1] = v.y;
        c[4 * k + 2] = v.z;
        c[4 * k + 3] = v.w;
    }
}

// Cross-lane steps with DPP (GFX9 encodings): row_shr:n moves lane i - n of the
// same 16-lane row into lane i (0 when that lane is in another row); row_bcast:15
// gives the rows selected by the row mask lane 15 of the row before; row_bcast:31
// gives them lane 31.  Rows the mask leaves out keep `old` (here 0).
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ unsigned int dpp_move(unsigned int v) {
    return static_cast<unsigned int>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROW_MASK, 0xf, true));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ unsigned long long dpp_move(unsigned long long v) {
    const unsigned int lo = dpp_move<CTRL, ROW_MASK>(static_cast<unsigned int>(v));
    const unsigned int hi = dpp_move<CTRL, ROW_MASK>(static_cast<unsigned int>(v >> 32));
    return static_cast<unsigned long long>(hi) << 32 | lo;
}
// The same moves for a min/max fold: lanes without a source keep their own value.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_keep(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xf,
                                                      false));
}
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

// Inclusive prefix sum across the 64 lanes (a scan within each row of 16 lanes,
// then the row totals carried into the rows after them), for 32- or 64-bit
// unsigned values.
template <typename T>
__device__ __forceinline__ T wave_scan_add(T x) {
    x += dpp_move<kRowShr1>(x);
    x += dpp_move<kRowShr2>(x);
    x += dpp_move<kRowShr4>(x);
    x += dpp_move<kRowShr8>(x);
    x += dpp_move<kRowBcast15, 0xa>(x);
    x += dpp_move<kRowBcast31, 0xc>(x);
    return x;
}

// Inclusive prefix maximum across the 64 lanes (values >= 0).
__device__ __forceinline__ unsigned int wave_scan_max(unsigned int x) {
    x = max(x, dpp_move<kRowShr1>(x));
    x = max(x, dpp_move<kRowShr2>(x));
    x = max(x, dpp_move<kRowShr4>(x));
    x = max(x, dpp_move<kRowShr8>(x));
    x = max(x, dpp_move<kRowBcast15, 0xa>(x));
    x = max(x, dpp_move<kRowBcast31, 0xc>(x));
    return x;
}

// Value of lane 63 in every lane.
__device__ __forceinline__ unsigned int lane63(unsigned int x) { return __builtin_amdgcn_readlane(x, 63); }
__device__ __forceinline__ unsigned long long lane63(unsigned long long x) {
    return static_cast<unsigned long long>(__builtin_amdgcn_readlane(static_cast<unsigned int>(x >> 32), 63)) << 32 |
           __builtin_amdgcn_readlane(static_cast<unsigned int>(x), 63);
}
__device__ __forceinline__ float lane63(float x) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Sum over the 64 lanes, in every lane (32- or 64-bit unsigned).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    return lane63(wave_scan_add(v));
}

// Inclusive prefix sum across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    return wave_scan_add(v);
}

// Minimum and maximum over the 64 lanes, in every lane.
__device__ __forceinline__ float wave_min(float x) {
    x = fminf(x, dpp_keep<kRowShr1>(x));
    x = fminf(x, dpp_keep<kRowShr2>(x));
    x = fminf(x, dpp_keep<kRowShr4>(x));
    x = fminf(x, dpp_keep<kRowShr8>(x));
    x = fminf(x, dpp_keep<kRowBcast15, 0xa>(x));
    x = fminf(x, dpp_keep<kRowBcast31, 0xc>(x));
    return lane63(x);
}
__device__ __forceinline__ float wave_max(float x) {
    x = fmaxf(x, dpp_keep<kRowShr1>(x));
    x = fmaxf(x, dpp_keep<kRowShr2>(x));
    x = fmaxf(x, dpp_keep<kRowShr4>(x));
    x = fmaxf(x, dpp_keep<kRowShr8>(x));
    x = fmaxf(x, dpp_keep<kRowBcast15, 0xa>(x));
    x = fmaxf(x, dpp_keep<kRowBcast31, 0xc>(x));
    return lane63(x);
}
__device__ __forceinline__ int wave_any(int x) { return __builtin_amdgcn_ballot_w64(x != 0) != 0ull ? 1 : 0; }

// Sum over the block; every thread gets the total.
__device__ unsigned long long block_sum(unsigned long long v, unsigned long long *scratch) {
    v = wave_sum(v);
    if (lane_id() == 0) scratch[wave_id()] = v;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += scratch[w];
    __syncthreads();
    return t;
}

// Exclusive prefix over the block in thread order.
__device__ unsigned long long block_exclusive_scan(unsigned long long v, unsigned long long *scratch) {
    unsigned long long inc = wave_inclusive_scan(v);
    if (lane_id() == 63) scratch[wave_id()] = inc;
    __syncthreads();
    unsigned long long before = 0;
    for (int w = 0; w < wave_id(); ++w) before += scratch[w];
    __syncthreads();
    return before + inc - v;
}

// Block sums of a and b and the exclusive prefix of c in thread order, with one
// barrier: red (3 kWaves entries) belongs to this call alone, so it needs no
// barrier after it.
__device__ void block_sums_and_scan(unsigned long long a, unsigned long long b, unsigned long long c,
                                    unsigned long long *red, unsigned long long &sum_a, unsigned long long &sum_b,
                                    unsigned long long &before_c) {
    a = wave_sum(a);
    b = wave_sum(b);
    const unsigned long long inc = wave_inclusive_scan(c);
    if (lane_id() == 63) {
        red[wave_id()] = a;
        red[kWaves + wave_id()] = b;
        red[2 * kWaves + wave_id()] = inc;
    }
    __syncthreads();
    unsigned long long sa = 0, sb = 0, pre = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        sa += red[w];
        sb += red[kWaves + w];
        pre += w < wave_id() ? red[2 * kWaves + w] : 0ull;
    }
    sum_a = sa;
    sum_b = sb;
    before_c = pre + inc - c;
}

// ------------------------------------------------------------------ bounds

// Binned coordinates of an event, axis 0 first; -1 for an axis that is not binned.
struct Dims {
    int c[kMaxAxes];
};

struct BoundsAcc {
    float mn[kMaxAxes] = {INFINITY, INFINITY, INFINITY, INFINITY};
    float mx[kMaxAxes] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    __device__ __forceinline__ void add(float v, int col, const Dims &dd) {
        bad |= !__builtin_isfinite(v);
#pragma unroll
        for (int p = 0; p < kMaxAxes; ++p)
            if (col == dd.c[p]) {
                mn[p] = fminf(mn[p], v);
                mx[p] = fmaxf(mx[p], v);
            }
    }
};

// Grid (bounds blocks, n_events): block (b, e) folds a share of event e's rows.
// The first blocks also clear the histogram, tile totals and counters of the call.
__global__ __launch_bounds__(kBlock) void k_bounds(int d, Dims dd,
                                                   int vec4, EventDesc *__restrict__ ev, EventDesc ev0,
                                                   int ev_from_arg, BoundsPartial *__restrict__ part,
                                                   unsigned int *__restrict__ cell_count, long long cells,
                                                   unsigned long long *__restrict__ sums_cells, int tiles_cells,
                                                   unsigned long long *__restrict__ sums_kept2, int groups_kept,
                                                   Counters *__restrict__ ctr) {
    const long long nblk = static_cast<long long>(gridDim.x) * gridDim.y;
    const long long bid = static_cast<long long>(blockIdx.y) * gridDim.x + blockIdx.x;
    const long long gtid = bid * kBlock + threadIdx.x;
    const long long gstride = nblk * kBlock;
    for (long long c = gtid; c < cells; c += gstride) cell_count[c] = 0u;
    for (long long c = gtid; c < tiles_cells; c += gstride) sums_cells[c] = 0ull;
    for (long long c = gtid; c < groups_kept; c += gstride) sums_kept2[c] = 0ull;
    if (gtid == 0) {
        Counters z = {};
        *ctr = z;
        if (ev_from_arg) ev[0] = ev0;
    }
    const EventDesc E = ev_from_arg ? ev0 : ev[blockIdx.y];
    const int tid = blockIdx.x * kBlock + threadIdx.x;
    const int stride = gridDim.x * kBlock;
    BoundsAcc acc;
    const long long total = static_cast<long long>(E.n) * d;
    const float *Xe = E.pts;
    // The column of a thread's element advances by a fixed step per stride, so it
    // is tracked incrementally instead of a 64-bit remainder per element.
    auto next_col = [d](int col, int step) {
        col += step;
        return col >= d ? col - d : col;
    };
    if (vec4) {
        const float4 *X4 = reinterpret_cast<const float4 *>(Xe);
        const long long nv = total / 4;
        const int step = static_cast<int>((4ll * stride) % d);
        int col = static_cast<int>((4ll * tid) % d);
        // Four independent loads in flight per thread, issued together also for the
        // last, partial round (the grid gives most threads exactly four), so that a
        // thread waits for one round trip per four loads.
        for (long long v = tid; v < nv; v += 4ll * stride) {
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long w = v + u * static_cast<long long>(stride);
                x[u] = w < nv ? X4[w] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (v + u * static_cast<long long>(stride) < nv) {
                    acc.add(x[u].x, col, dd);
                    acc.add(x[u].y, col + 1, dd);
                    acc.add(x[u].z, col + 2, dd);
                    acc.add(x[u].w, col + 3, dd);
                }
                col = next_col(col, step);
            }
        }
    } else {
        const int step = stride % d;
        int col = tid % d;
        for (long long e = tid; e < total; e += stride) {
            acc.add(Xe[e], col, dd);
            col = next_col(col, step);
        }
    }
#pragma unroll
    for (int p = 0; p < kMaxAxes; ++p) {
        acc.mn[p] = wave_min(acc.mn[p]);
        acc.mx[p] = wave_max(acc.mx[p]);
    }
    acc.bad = wave_any(acc.bad);
    __shared__ BoundsPartial sp[kWaves];
    if (lane_id() == 0) {
        BoundsPartial &p = sp[wave_id()];
        for (int q = 0; q < kMaxAxes; ++q) {
            p.mn[q] = acc.mn[q];
            p.mx[q] = acc.mx[q];
        }
        p.nonfinite = acc.bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BoundsPartial out = sp[0];
        for (int w = 1; w < kWaves; ++w) {
            for (int p = 0; p < kMaxAxes; ++p) {
                out.mn[p] = fminf(out.mn[p], sp[w].mn[p]);
                out.mx[p] = fmaxf(out.mx[p], sp[w].mx[p]);
            }
            out.nonfinite |= sp[w].nonfinite;
        }
        out.pad = 0;
        part[static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x] = out;
    }
}

// ------------------------------------------------------------------- keys

// Wave 0 of a block folds the bounds partials and lane 0 derives the grid.
// Every block derives the same plan from the same partials (min/max are exact).
// Axes from `axes` on are not binned: one cell each.
__device__ void derive_plan(const BoundsPartial *__restrict__ part, int nparts, float r,
                            int cell_div, int axes, int cells_max, Plan *out) {
    float mn[kMaxAxes] = {INFINITY, INFINITY, INFINITY, INFINITY};
    float mx[kMaxAxes] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    // Every lane loads its (at most kBoundsBlocks / 64) partials before folding them.
    constexpr int kPartsPerLane = kBoundsBlocks / 64;
    BoundsPartial pb[kPartsPerLane];
#pragma unroll
    for (int u = 0; u < kPartsPerLane; ++u) {
        const int b = lane_id() + 64 * u;
        if (b < nparts) pb[u] = part[b];
    }
#pragma unroll
    for (int u = 0; u < kPartsPerLane; ++u) {
        if (lane_id() + 64 * u >= nparts) continue;
        for (int p = 0; p < kMaxAxes; ++p) {
            mn[p] = fminf(mn[p], pb[u].mn[p]);
            mx[p] = fmaxf(mx[p], pb[u].mx[p]);
        }
        bad |= pb[u].nonfinite;
    }
#pragma unroll
    for (int p = 0; p < kMaxAxes; ++p) {
        mn[p] = wave_min(mn[p]);
        mx[p] = wave_max(mx[p]);
    }
    bad = wave_any(bad);
    if (lane_id() != 0) return;
    // Cell edge r (1 + 2^-10) / cell_div.  A pair that passes the float32 test has
    // |x_p - y_p| < r exactly along every coordinate (partial sums never exceed D,
    // rounding is monotone); the 2^-10 margin absorbs the float32 rounding of the
    // key computation (at most 3 * 2^-24 * G cells per point, G <= 1024), so such
    // a pair lands at most cell_div cells apart along every binned axis.  Larger
    // cells only keep such pairs closer.
    const float cbase = (r * 1.0009765625f) / static_cast<float>(cell_div);
    const int axis_max = axes == 4 ? kGridAxisMax4 : kGridAxisMax3;
    const float axis_soft = axes == 4 ? 250.0f : 1000.0f;
    float c[kMaxAxes], ext[kMaxAxes];
    int G[kMaxAxes];
    // An axis whose extent is not a finite float (no points, or max - min
    // overflowing), or that is not binned, gets a single cell: inv_c = 0 puts
    // every point in cell 0.
    bool single[kMaxAxes];
    for (int p = 0; p < kMaxAxes; ++p) {
        ext[p] = mx[p] - mn[p];
        single[p] = p >= axes || !(ext[p] >= 0.0f && ext[p] <= FLT_MAX);
        if (!(mn[p] <= mx[p])) mn[p] = 0.0f;
        c[p] = cbase;
        if (!single[p] && ext[p] / c[p] > axis_soft) c[p] = ext[p] / axis_soft;
    }
    // Grow the cells until the grid fits cells_max (bounded: after 128 rounds of
    // x1.25 every finite extent spans one cell).
    for (int round = 0;; ++round) {
        long long total = 1;
        for (int p = 0; p < kMaxAxes; ++p) {
            float g = single[p] ? 1.0f : floorf(ext[p] / c[p]) + 1.0f;
            if (!(g <= static_cast<float>(axis_max))) g = static_cast<float>(axis_max);
            if (!(g >= 1.0f)) g = 1.0f;
            G[p] = static_cast<int>(g);
            total *= G[p];
        }
        if (total <= cells_max) break;
        if (round >= 128) {
            for (int p = 0; p < kMaxAxes; ++p) single[p] = true;
            continue;
        }
        for (int p = 0; p < kMaxAxes; ++p) c[p] *= 1.25f;
    }
    for (int p = 0; p < kMaxAxes; ++p) {
        out->lo[p] = p < axes ? mn[p] : 0.0f;
        out->c[p] = single[p] ? INFINITY : c[p];
        out->inv_c[p] = single[p] ? 0.0f : 1.0f / c[p];
        out->G[p] = G[p];
    }
    out->n_cells = G[0] * G[1] * G[2] * G[3];
    out->reach = cell_div;
    out->abort = bad;
    out->axes = axes;
}

// Clamping is monotone and moves no coordinate by more than the clamp, so two
// points that are at most R cells apart stay at most R cells apart.
__device__ __forceinline__ int cell_coord(float x, float lo, float inv_c, int G) {
    float q = floorf((x - lo) * inv_c);
    q = fmaxf(q, 0.0f);  // also maps NaN to 0
    q = fminf(q, static_cast<float>(G - 1));
    return static_cast<int>(q);
}

// Cell coordinates of a point pack into one word (cell_bits per axis); the cell
// key orders cells with axis 0 fastest, so the cells along axis 0 around a cell
// are contiguous in cell order.
__device__ __forceinline__ unsigned int pack_cell(const int (&u)[kMaxAxes], int axes) {
    const int b = cell_bits(axes);
    return static_cast<unsigned int>(u[0]) | static_cast<unsigned int>(u[1]) << b |
           static_cast<unsigned int>(u[2]) << (2 * b) | static_cast<unsigned int>(u[3]) << (3 * b);
}

__device__ __forceinline__ void unpack_cell(unsigned int pc, int axes, int (&u)[kMaxAxes]) {
    const int b = cell_bits(axes);
    const unsigned int m = (1u << b) - 1u;
#pragma unroll
    for (int p = 0; p < kMaxAxes; ++p) u[p] = static_cast<int>((pc >> (p * b)) & m);
}

__device__ __forceinline__ unsigned int cell_key(const int (&u)[kMaxAxes], const Plan &P) {
    return static_cast<unsigned int>(((u[3] * P.G[2] + u[2]) * P.G[1] + u[1]) * P.G[0] + u[0]);
}

constexpr int kMaxCellTiles = ((1 << 24) + kScanTile - 1) / kScanTile + 2;

// Grid (blocks, n_events) of kKeysBlock threads: block 0 of event e derives and
// stores its plan; every block computes the cells of kKeysBlock x kKeysPer of the
// event's rows.  Two points per thread halve the blocks, and with them the
// blocks' atomic adds to each tile total, which pays for large events.
template <int kKeysPer>
__global__ __launch_bounds__(kKeysBlock) void k_keys(int d, Dims dd, int axes,
                                                     float r, int cell_div, const EventDesc *__restrict__ ev,
                                                     EventDesc ev0, int ev_from_arg,
                                                     const BoundsPartial *__restrict__ part, int nparts,
                                                     Plan *__restrict__ plans, Counters *__restrict__ ctr,
                                                     unsigned int *__restrict__ pcell,
                                                     unsigned int *__restrict__ rank,
                                                     unsigned int *__restrict__ cell_count,
                                                     unsigned long long *__restrict__ sums_cells) {
    __shared__ Plan P;
    // Per scan tile: points (low word) and newly occupied cells (high word).
    __shared__ unsigned long long tile_count[kMaxCellTiles];
    const int e = blockIdx.y;
    const EventDesc E = ev_from_arg ? ev0 : ev[e];  // one event: no load before the points'
    constexpr int kSpan = kKeysBlock * kKeysPer;
    if (blockIdx.x != 0 && static_cast<long long>(blockIdx.x) * kSpan >= E.n) return;
    // kKeysPer points per thread, kKeysBlock apart; their binned coordinates are
    // loaded before the plan is derived so that the two latencies overlap.
    float x[kKeysPer][kMaxAxes];
#pragma unroll
    for (int m = 0; m < kKeysPer; ++m) {
        const int i = blockIdx.x * kSpan + m * kKeysBlock + threadIdx.x;
#pragma unroll
        for (int p = 0; p < kMaxAxes; ++p) x[m][p] = 0.0f;
        if (i < E.n) {
            const float *row = E.pts + static_cast<size_t>(i) * d;
#pragma unroll
            for (int p = 0; p < kMaxAxes; ++p)
                if (p < axes) x[m][p] = row[dd.c[p]];
        }
    }
    if (wave_id() == 0)
        derive_plan(part + static_cast<size_t>(e) * nparts, nparts, r, cell_div, axes, E.cells_max, &P);
    const int tile_end = static_cast<int>((E.cell0 + E.cells_max - 1) / kScanTile);
    const int ntiles = tile_end - E.tile0 + 1;
    for (int t = threadIdx.x; t < ntiles; t += kKeysBlock) tile_count[t] = 0ull;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        plans[e] = P;
        if (P.abort) atomicOr(&ctr->abort, 1u);
    }
    if (P.abort) return;
    unsigned int k[kKeysPer], rk[kKeysPer];
#pragma unroll
    for (int m = 0; m < kKeysPer; ++m) {
        const int i = blockIdx.x * kSpan + m * kKeysBlock + threadIdx.x;
        if (i >= E.n) continue;
        const long long gi = E.row0 + i;
        int u[kMaxAxes];
#pragma unroll
        for (int p = 0; p < kMaxAxes; ++p) u[p] = cell_coord(x[m][p], P.lo[p], P.inv_c[p], P.G[p]);
        k[m] = static_cast<unsigned int>(E.cell0) + cell_key(u, P);
        pcell[gi] = pack_cell(u, axes);
        rk[m] = atomicAdd(&cell_count[k[m]], 1u);
    }
#pragma unroll
    for (int m = 0; m < kKeysPer; ++m) {
        const int i = blockIdx.x * kSpan + m * kKeysBlock + threadIdx.x;
        if (i >= E.n) continue;
        rank[E.row0 + i] = rk[m];
        // The first point of a cell (rank 0) also counts the cell as occupied.
        atomicAdd(&tile_count[k[m] / kScanTile - E.tile0], rk[m] == 0u ? (1ull << 32) | 1ull : 1ull);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += kKeysBlock)
        if (tile_count[t]) atomicAdd(&sums_cells[E.tile0 + t], tile_count[t]);
}

// ------------------------------------------------------------------- scans

// floor(a / b) for a < 2^52, b > 0: the quotient rounded in double is within one
// of the exact, and integer products settle it.
__device__ __forceinline__ unsigned long long floor_div(unsigned long long a, unsigned long long b) {
    unsigned long long f = static_cast<unsigned long long>(static_cast<double>(a) / static_cast<double>(b));
    if (f * b > a) --f;
    if ((f + 1) * b <= a) ++f;
    return f;
}

// cell_start[c] = points in cells [0, c) for c in [0, cells]; sums[t] holds tile
// t's points (low word) and occupied cells (high word).  The tile's counts are
// requested before the totals of the tiles before it are summed, so that the two
// round trips overlap.
//
// The same pass divides the queries into the search's n_waves pieces by work
// rather than by count: a cell weighs its points plus kTileWeight if it has any
// (a tile's fixed cost, in queries), the cells in order span weights [0, W), and
// wave k starts at weight floor(k W / n_waves), which falls in one cell; the wave
// starts there at the query that many weight units past the cell's fixed cost
// (at its first query if it falls within the cost), so a dense cell can still be
// split among waves.  wave_start[k] is that sorted row; wave_start[n_waves] =
// rows.
__global__ __launch_bounds__(kBlock) void k_scan_cells(const unsigned int *__restrict__ in, long long len,
                                                       const unsigned long long *__restrict__ sums, int tiles,
                                                       unsigned int *__restrict__ out,
                                                       unsigned int *__restrict__ wave_start, int n_waves,
                                                       long long rows, unsigned int *__restrict__ claims) {
    __shared__ unsigned long long red[4 * kWaves];
    const long long base = static_cast<long long>(blockIdx.x) * kScanTile;
    if (base > len) return;
    constexpr int kPer = kScanTile / kBlock;
    static_assert(kPer % 4 == 0, "a thread's counts are read as 16-byte groups");
    // A thread's kPer counts are consecutive (16-byte aligned: the tile and the
    // workspace arrays are): whole groups are read as uint4, the last thread's
    // partial group one by one.
    unsigned int v[kPer];
    const long long first = base + static_cast<long long>(threadIdx.x) * kPer;
    if (first + kPer <= len) {
        const uint4 *src = reinterpret_cast<const uint4 *>(in + first);
#pragma unroll
        for (int j = 0; j < kPer / 4; ++j) {
            const uint4 g = src[j];
            v[4 * j] = g.x;
            v[4 * j + 1] = g.y;
            v[4 * j + 2] = g.z;
            v[4 * j + 3] = g.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kPer; ++j) v[j] = first + j < len ? in[first + j] : 0u;
    }
    // Points and weight of the tiles before this one, and the weight of them all.
    unsigned long long c_before = 0, w_before = 0, w_all = 0;
    for (int t = threadIdx.x; t < tiles; t += kBlock) {
        const unsigned long long x = sums[t];
        const unsigned long long w = (x & 0xffffffffull) + kTileWeight * (x >> 32);
        w_all += w;
        if (t < static_cast<int>(blockIdx.x)) {
            c_before += x & 0xffffffffull;
            w_before += w;
        }
    }
    // This thread's points (low word) and weight (high word); a block's totals of
    // either stay below 2^32, so the packed scan carries nothing between them.
    unsigned long long mine = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        mine += (static_cast<unsigned long long>(v[j] + (v[j] ? kTileWeight : 0u)) << 32) | v[j];
    c_before = wave_sum(c_before);
    w_before = wave_sum(w_before);
    w_all = wave_sum(w_all);
    const unsigned long long inc = wave_inclusive_scan(mine);
    if (lane_id() == 63) {
        red[wave_id()] = c_before;
        red[kWaves + wave_id()] = w_before;
        red[2 * kWaves + wave_id()] = w_all;
        red[3 * kWaves + wave_id()] = inc;
    }
    __syncthreads();
    unsigned long long cb = 0, wb = 0, W = 0, pre = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        cb += red[w];
        wb += red[kWaves + w];
        W += red[2 * kWaves + w];
        pre += w < wave_id() ? red[3 * kWaves + w] : 0ull;
    }
    pre += inc - mine;
    unsigned long long run_c = cb + (pre & 0xffffffffull), run_w = wb + (pre >> 32);
    const unsigned long long nw = static_cast<unsigned long long>(n_waves);
    // Wave k starts at weight B_k = floor(k W / nw).  The thread's first wave is the
    // smallest k with k W >= run_w nw (then B_k >= run_w); later ones follow by
    // B_{k+1} = B_k + q + carry, with W = q nw + m and the remainder of k W / nw
    // carried, so no division runs per wave.
    unsigned int starts[kPer];
    unsigned long long k = nw, B = 0, rem = 0, q = 0, m = 0;
    if (W) {
        q = floor_div(W, nw);
        m = W - q * nw;
        const unsigned long long target = run_w * nw;
        k = floor_div(target + W - 1, W);
        if (k == 0) k = 1;  // wave 0 starts at row 0
        B = floor_div(k * W, nw);
        rem = k * W - B * nw;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        starts[j] = static_cast<unsigned int>(run_c);
        const unsigned long long w = v[j] + (v[j] ? kTileWeight : 0u);
        for (; k < nw && B < run_w + w; ++k) {
            // B lies in this cell: past its fixed cost, one weight unit per query.
            const unsigned long long past = B - run_w;
            wave_start[k] = static_cast<unsigned int>(run_c + (past > kTileWeight ? past - kTileWeight : 0ull));
            B += q;
            rem += m;
            if (rem >= nw) {
                rem -= nw;
                ++B;
            }
        }
        run_c += v[j];
        run_w += w;
    }
    // cell_start has len + 1 entries: whole groups as uint4, the rest one by one.
    if (first + kPer <= len + 1) {
        uint4 *dst = reinterpret_cast<uint4 *>(out + first);
#pragma unroll
        for (int j = 0; j < kPer / 4; ++j)
            dst[j] = make_uint4(starts[4 * j], starts[4 * j + 1], starts[4 * j + 2], starts[4 * j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (first + j <= len) out[first + j] = starts[j];
    }
    if (blockIdx.x == 0) {
        if (threadIdx.x < 8 * kPools) claims[threadIdx.x * kPoolStride] = 0u;
        if (W == 0) {  // no rows: every share is empty
            for (int t = threadIdx.x; t <= n_waves; t += kBlock) wave_start[t] = 0u;
        } else if (threadIdx.x == 0) {
            wave_start[0] = 0u;
            wave_start[n_waves] = static_cast<unsigned int>(rows);
        }
    }
}

// ----------------------------------------------------------------- scatter

// Grid (blocks, n_events): block (b, e) copies a share of event e's rows.
template <int DP>
__global__ __launch_bounds__(kBlock) void k_scatter(int d, int vec4, const EventDesc *__restrict__ ev,
                                                    EventDesc ev0, int ev_from_arg,
                                                    const Plan *__restrict__ plans,
                                                    const unsigned int *__restrict__ pcell,
                                                    const unsigned int *__restrict__ rank,
                                                    const unsigned int *__restrict__ cell_start,
                                                    const Counters *__restrict__ ctr,
                                                    float *__restrict__ sorted,
                                                    unsigned int *__restrict__ sorted_id) {
    // The point's packed cell, rank and row are requested before the abort flag is
    // known (they are in bounds whatever it says); the cell start, whose index needs
    // a valid plan, only when it is clear.
    const bool abort = ctr->abort != 0;
    const EventDesc E = ev_from_arg ? ev0 : ev[blockIdx.y];
    const Plan P = plans[blockIdx.y];
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < E.n; i += gridDim.x * kBlock) {
        const long long gi = E.row0 + i;
        const unsigned int pc = pcell[gi];
        const unsigned int rk = rank[gi];
        float row[DP];
        if (vec4) {
            const float4 *src = reinterpret_cast<const float4 *>(E.pts + static_cast<size_t>(i) * d);
#pragma unroll
            for (int k = 0; k < DP / 4; ++k) {
                float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (4 * k < d) v = src[k];
                row[4 * k] = v.x;
                row[4 * k + 1] = v.y;
                row[4 * k + 2] = v.z;
                row[4 * k + 3] = v.w;
            }
        } else {
            const float *src = E.pts + static_cast<size_t>(i) * d;
#pragma unroll
            for (int k = 0; k < DP; ++k) row[k] = k < d ? src[k] : 0.0f;
        }
        if (abort) return;
        int u[kMaxAxes];
        unpack_cell(pc, P.axes, u);
        const unsigned int slot = cell_start[static_cast<unsigned int>(E.cell0) + cell_key(u, P)] + rk;
        float4 *out = reinterpret_cast<float4 *>(sorted + static_cast<size_t>(slot) * DP);
#pragma unroll
        for (int k = 0; k < DP / 4; ++k)
            out[k] = make_float4(row[4 * k], row[4 * k + 1], row[4 * k + 2], row[4 * k + 3]);
        // The original row and the packed cell of a sorted row sit side by side, so
        // the scattered write is one 8-byte store instead of two 4-byte ones.
        reinterpret_cast<uint2 *>(sorted_id)[slot] = make_uint2(static_cast<unsigned int>(gi), pc);
    }
}

// ------------------------------------------------------------ neighbour runs

// Event of a row: the last event whose first row is <= row (empty events share
// their first row with the next event, so they are never returned for a row).
__device__ __forceinline__ int find_event(const EventDesc *__restrict__ ev, int n_events, long long row) {
    int lo = 0, hi = n_events - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ev[mid].row0 <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The neighbour cells of a cell are the cells at most R = reach cells away along
// every binned axis.  Along axis 0 (the fastest in cell order) each group of them
// is contiguous, so they form (2R+1)^(axes-1) runs of candidate rows.
__device__ __forceinline__ int run_count(const Plan &P) {
    const int side = 2 * P.reach + 1;
    return P.axes == 4 ? side * side * side : side * side;
}

// Offsets along axes 1..3 of the run a lane builds (lanes below run_count).
struct RunLane {
    int a[3];
    bool live;
};

__device__ __forceinline__ RunLane run_lane(const Plan &P) {
    const int R = P.reach, side = 2 * R + 1, t = lane_id();
    RunLane rl;
    rl.live = t < run_count(P);
    rl.a[0] = t % side - R;
    rl.a[1] = (t / side) % side - R;
    rl.a[2] = P.axes == 4 ? t / (side * side) - R : 0;
    return rl;
}

// Lane t < run_count builds run t around the cell with coordinates u (global keys
// start at cell0): its first sorted row (start) and its candidates [pre, end) in
// the tile's candidate numbering (other lanes: an empty run at the end).  Returns
// the candidate count, the same in every lane.  Call with the whole wave active.
__device__ __forceinline__ unsigned int wave_runs(const int (&u)[kMaxAxes], unsigned int cell0, const Plan &P,
                                                  const RunLane &rl, const unsigned int *__restrict__ cell_start,
                                                  unsigned int &start, unsigned int &pre, unsigned int &end) {
    const int R = P.reach;
    // Branch-free: every lane loads (a lane without a run reads the event's first
    // row of cells, a valid address) and keeps its run only if it is inside the grid
    // (the unsigned comparisons also reject negative coordinates).
    const int y = u[1] + rl.a[0], z = u[2] + rl.a[1], w = u[3] + rl.a[2];
    const bool ok = rl.live & (static_cast<unsigned int>(y) < static_cast<unsigned int>(P.G[1])) &
                    (static_cast<unsigned int>(z) < static_cast<unsigned int>(P.G[2])) &
                    (static_cast<unsigned int>(w) < static_cast<unsigned int>(P.G[3]));
    const int xlo = max(u[0] - R, 0), xhi = min(u[0] + R, P.G[0] - 1);
    const unsigned int row =
        cell0 + (ok ? static_cast<unsigned int>(((w * P.G[2] + z) * P.G[1] + y) * P.G[0]) : 0u);
    const unsigned int s0 = cell_start[row + xlo];
    const unsigned int s1 = cell_start[row + xhi + 1];
    start = ok ? s0 : 0u;
    const unsigned int len = ok ? s1 - s0 : 0u;
    end = wave_scan_add(len);
    pre = end - len;
    return __builtin_amdgcn_readlane(end, 63);
}

// ------------------------------------------------------------------ search

// Waves per SIMD the search asks the register allocator for: a lane holds only a
// candidate's first four coordinates, so rows of up to 16 floats fit in 64
// registers (8 waves, some scalar registers spilled to vector lanes); wider rows,
// whose second stage holds the rest of a row, keep the compiler's choice.
template <int DP>
constexpr int kSearchWaves = DP <= 16 ? 8 : 1;

// SEL: the cap K is below kListCap, so a list that fits may still need the K
// nearest of its hits: the lists then also hold each hit's distance.
template <int DP, bool SEL>
__global__ __launch_bounds__(kBlock, kSearchWaves<DP>) void k_search(const float *__restrict__ sorted,
                                                   const unsigned int *__restrict__ sorted_id,
                                                   const unsigned int *__restrict__ wave_start,
                                                   unsigned int *__restrict__ claims,
                                                   const EventDesc *__restrict__ ev, int n_events,
                                                   const unsigned int *__restrict__ cell_start,
                                                   const Plan *__restrict__ plans, float r2, int K,
                                                   unsigned int *__restrict__ kept,
                                                   unsigned int *__restrict__ temp,
                                                   unsigned int *__restrict__ long_slots,
                                                   Counters *__restrict__ ctr,
                                                   unsigned long long *__restrict__ tested_out,
                                                   unsigned int *__restrict__ capped_out, int prio) {
    // Queries per tile: 16 when the lists also hold distances (their LDS would
    // otherwise cost occupancy), else kQTile.
    constexpr int kQT = SEL ? 16 : kQTile;
    static_assert((kQT & (kQT - 1)) == 0 && kQT <= 64, "list slots are numbered modulo kQT");
    __shared__ __align__(16) unsigned int lst_all[kWaves][kQT * kListCap];
    __shared__ unsigned int lstd_all[SEL ? kWaves : 1][SEL ? kQT * kListCap : 1];  // D bits of each hit
    // Per list slot (kQT per wave, taken by the queries in turn): the query's sorted
    // and original rows.
    __shared__ unsigned int qrow_all[kWaves][kQT];
    __shared__ unsigned int qid_all[kWaves][kQT];
    __shared__ unsigned int pre_all[kWaves][kQT + 1];
    __shared__ unsigned int cnt_all[kWaves][kQT];
    __shared__ unsigned int qcnt_all[kWaves][kQT];
    // Queued first-stage survivors: query slot << 32 | candidate's sorted row, with
    // the partial sum in racc.
    __shared__ unsigned long long ring_all[kWaves][kRing];
    __shared__ float racc_all[kWaves][kRing];
    __shared__ unsigned int mark_all[kWaves][64];  // run starting at each lane of a chunk, plus one
    __shared__ unsigned long long tested_w[kWaves];
    __shared__ unsigned long long survived_w[kWaves];
    __shared__ unsigned int capped_w[kWaves];
    if (ctr->abort) return;
    unsigned int *lst = lst_all[wave_id()];
    unsigned int *lstd = lstd_all[SEL ? wave_id() : 0];
    unsigned int *qrow_s = qrow_all[wave_id()];
    unsigned int *qid = qid_all[wave_id()];
    unsigned int capped = 0;
    unsigned int *tpre = pre_all[wave_id()];
    unsigned int *tcnt = cnt_all[wave_id()];
    unsigned int *qcnt = qcnt_all[wave_id()];
    unsigned long long *ring = ring_all[wave_id()];
    float *racc = racc_all[wave_id()];
    unsigned int *mark = mark_all[wave_id()];
    const int lane = lane_id();
    // Terms before the first exact rejection test: two for rows of up to 12 floats
    // (a three-term test rejects few more pairs than two terms do, and the first
    // stage runs for every query and candidate; on the 300k-point 12-D event two,
    // three and four terms took 87.5, 88.7 and 89.6 us), three for wider rows (two
    // terms took whole 120k-point builds with 32-, 48- and 64-float rows from
    // 0.173, 0.292 and 0.558 ms to 0.204, 0.423 and 1.126 ms).
    constexpr int kLead = DP <= 12 ? 2 : 3;
    // Pairs examined (lane q counts those of query q of each group) and pairs that
    // reached the second stage (each lane counts those it queued).  Per-lane counts
    // in vector registers, summed once at the end: scalar registers are the scarce
    // ones in this kernel.
    unsigned long long tested = 0;
    unsigned long long survived = 0;

    // The cell scan cuts the queries, in cell order, into kPieces pieces per wave
    // (one for rows of up to 24 floats, two for wider ones) of equal work (its
    // cells' fixed costs plus its queries; a piece may start or end inside a cell,
    // so a dense cell is split instead of holding up one wave).
    // Workgroups are dealt to the 8 XCDs round-robin; the workgroups of one XCD
    // take a contiguous share of the pieces, so that they share their rows in its
    // L2: each wave first takes one piece of the share, then claims the share's
    // remaining pieces one at a time from one of the XCD's counters (workgroup w
    // of the XCD uses counter w mod kPools, which hands out every kPools-th piece),
    // so that a wave that finishes early takes work the others have not started.
    // A wave's pieces only move forward in row order.  With one piece per wave
    // the claims compile out.
    constexpr int kPieces = search_pieces(DP);
    const unsigned int nb = gridDim.x;
    const unsigned int xcd = blockIdx.x % 8u, per = nb / 8u, rest = nb % 8u;
    const unsigned int xnb = per + (xcd < rest ? 1u : 0u);  // workgroups on this XCD
    const unsigned int xb0 = xcd < rest ? xcd * (per + 1u) : rest * (per + 1u) + (xcd - rest) * per;
    const unsigned int xblk = blockIdx.x / 8u;              // this workgroup's number on its XCD
    const unsigned int x_first = kPieces * kWaves * xb0;    // the XCD's first piece
    const unsigned int x_dyn = x_first + kWaves * xnb;      // its first claimed piece
    const unsigned int x_end = x_first + kPieces * kWaves * xnb;
    const unsigned int pools = min(static_cast<unsigned int>(kPools), xnb);
    const unsigned int pool = xblk % pools;
    unsigned int *claim = claims + (xcd * kPools + pool) * kPoolStride;
    Plan P;
    RunLane rl;
    unsigned int cell0 = 0;
    unsigned int ev_end = 0;  // first row after the current event
    const uint2 *__restrict__ sid = reinterpret_cast<const uint2 *>(sorted_id);
    // Queries take the wave's kQT list slots in turn (query number k of the wave
    // uses slot k mod kQT).  First-stage survivors stay queued across tiles, and
    // the lists of the pending queries are written out together: when the next
    // group of queries would not find free slots (the queue is emptied first) and
    // at the end of the share.  A tile of a sparse cell holds a few queries, so
    // the queue's partial drain and the list stores are shared by many tiles.
    unsigned int head = 0, tail = 0;     // queued survivors [head, tail)
    unsigned int pend0 = 0, pend_n = 0;  // pending queries: numbers [pend0, pend0 + pend_n)
    // A pair that passes the full test joins the list of the query in slot q.
    auto keep = [&](bool pass, unsigned int q, unsigned int j, float D) {
        if (pass) {
            const unsigned int pos = atomicAdd(&qcnt[q], 1u);
            if (pos < static_cast<unsigned int>(kListCap)) {
                lst[q * kListCap + pos] = j;
                if (SEL) lstd[q * kListCap + pos] = __float_as_uint(D);
            }
        }
    };
    // Second stage for ring entries [h, h + nb): lane l takes entry h + l and
    // adds terms kLead.. of the definition to the first stage's partial sum, in
    // the same order.  An entry names its query's slot and the candidate's sorted
    // row; the remaining coordinates are loaded here (the chunk holds only the
    // first four), so entries outlive their chunk and tile.
    auto finish_rows = [&](unsigned int h, unsigned int nb) {
        wave_lds_sync();
        const bool act = static_cast<unsigned int>(lane) < nb;
        const unsigned int e = (h + lane) & (kRing - 1);
        const unsigned long long ent = act ? ring[e] : 0ull;
        const float a3 = act ? racc[e] : 0.0f;
        const unsigned int q = static_cast<unsigned int>(ent >> 32);
        const unsigned int s2 = static_cast<unsigned int>(ent);
        const unsigned int qr = qrow_s[q];
        const float *crow = sorted + static_cast<size_t>(s2) * DP;
        float cc[DP];
#pragma unroll
        for (int k = kLead; k < DP; ++k) cc[k] = crow[k];
        const unsigned int j2 = sorted_id[2u * s2];
        const float D = add_terms<kLead, DP, DP>(a3, cc, sorted + static_cast<size_t>(qr) * DP);
        keep(act && D < r2 && s2 != qr, q, j2, D);
        wave_lds_sync();
    };
    // Empties the queue.
    auto drain_all = [&]() {
        if (tail != head) {
            finish_rows(head, tail - head);
            head = tail;
        }
    };
    // Writes out the lists of pending queries [f0, f0 + nf), nf <= kQT, whose
    // survivors are all finished; lane l takes query f0 + l.  Kept counts for every
    // query; lists that fit go to their fixed place (kListCap slots per original
    // row) as found, in 16-byte pieces, and the placement pass orders every such
    // list by neighbour id; the sorted rows of longer ones are queued (one atomic
    // each) for the placement pass to collect again.  With the cap binding (SEL and
    // more than K hits), the entries of those lists are numbered through a prefix
    // over their lengths; each lane takes one entry, finds its query by binary
    // search, ranks it by its (D, j) key within its list (D >= 0, so its bits order
    // like the value; keys are distinct) and, if the rank is below K, writes it at
    // that rank: the list's first K slots then hold its K nearest.  The stores are
    // scattered, but everything about query i lands at places indexed by i, which
    // the placement pass then reads in order.
    auto flush = [&](unsigned int f0, unsigned int nf) {
        wave_lds_sync();
        const bool mine = static_cast<unsigned int>(lane) < nf;
        const unsigned int sl = (f0 + static_cast<unsigned int>(lane)) & (kQT - 1);
        const unsigned int cnt = mine ? qcnt[sl] : 0u;
        const unsigned int iq = qid[sl];
        const unsigned int Ku = static_cast<unsigned int>(K);
        const bool fits = mine && cnt <= static_cast<unsigned int>(kListCap) && (SEL || cnt <= Ku);
        if (mine) {
            kept[iq] = min(cnt, Ku) | (fits ? 0u : kKeptLong);
            if (cnt > Ku) ++capped;
            if (!fits) long_slots[atomicAdd(&ctr->heavy_count, 1u)] = qrow_s[sl];
        }
        if (fits && !(SEL && cnt > Ku)) {
            const uint4 *from = reinterpret_cast<const uint4 *>(lst + sl * kListCap);
            uint4 *to = reinterpret_cast<uint4 *>(temp + static_cast<size_t>(iq) * kListCap);
            for (unsigned int k = 0; 4u * k < cnt; ++k) to[k] = from[k];
        }
        if (SEL) {
            const unsigned int take = fits && cnt > Ku ? cnt : 0u;
            const unsigned int inc = wave_inclusive_scan(take);
            const unsigned int T = __builtin_amdgcn_readlane(inc, 63);
            if (mine) {
                tpre[lane] = inc - take;
                tcnt[lane] = take;
            }
            wave_lds_sync();
            auto entry_query = [&](unsigned int t) {
                int lo = 0, hi = static_cast<int>(nf) - 1;  // last query whose list starts at or before t
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (tpre[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                return lo;
            };
            for (unsigned int t0 = 0; t0 < T; t0 += 64) {
                const unsigned int t = t0 + lane;
                if (t < T) {
                    const int lo = entry_query(t);
                    const unsigned int ls = (f0 + static_cast<unsigned int>(lo)) & (kQT - 1);
                    const unsigned int cq = tcnt[lo];
                    const unsigned int *l = lst + ls * kListCap;
                    const unsigned int *ld = lstd + ls * kListCap;
                    const unsigned int x = t - tpre[lo];
                    const unsigned long long key = (static_cast<unsigned long long>(ld[x]) << 32) | l[x];
                    unsigned int sr = 0;  // the entry's rank by (D, j) in its list
                    for (unsigned int u = 0; u < cq; ++u)
                        sr += ((static_cast<unsigned long long>(ld[u]) << 32) | l[u]) < key ? 1u : 0u;
                    if (sr < Ku) temp[static_cast<size_t>(qid[ls]) * kListCap + sr] = l[x];
                }
            }
        }
        wave_lds_sync();
    };
    // The share is read in windows of 64 queries: lane l holds query win + l (its
    // original row and packed cell), and a tile is a run of consecutive lanes with the
    // same cell, found by a ballot (no per-tile lookup of where the cell ends).
    for (unsigned int piece = x_first + xblk * kWaves + wave_id(); piece < x_end;) {
        // The next piece is claimed before this one is worked off, so that the claim's
        // round trip overlaps the first loads.
        unsigned int claimed = 0;
        if (kPieces > 1 && lane == 0) claimed = atomicAdd(claim, 1u);
        const unsigned int q_lo = wave_start[piece];
        const unsigned int q_hi = wave_start[piece + 1u];
        for (unsigned int win = q_lo; win < q_hi;) {
            const unsigned int nwin = min(64u, q_hi - win);
            uint2 me = make_uint2(0u, 0u);
            if (static_cast<unsigned int>(lane) < nwin) me = sid[win + lane];
            const unsigned int v_orig = me.x, v_pc = me.y;
            for (unsigned int t0 = 0; t0 < nwin;) {
                const unsigned int qs = win + t0;
                if (qs >= ev_end) {
                    const int e = n_events == 1 ? 0 : find_event(ev, n_events, qs);
                    P = plans[e];
                    const EventDesc E = ev[e];
                    cell0 = static_cast<unsigned int>(E.cell0);
                    ev_end = static_cast<unsigned int>(E.row0) + static_cast<unsigned int>(E.n);
                    rl = run_lane(P);
                }
                const unsigned int pc = __builtin_amdgcn_readlane(v_pc, t0);
                const unsigned long long other =
                    __builtin_amdgcn_ballot_w64(static_cast<unsigned int>(lane) >= nwin || v_pc != pc) &
                    (~0ull << t0);
                unsigned int t1 = other ? static_cast<unsigned int>(__builtin_ctzll(other)) : 64u;
                t1 = min(t1, ev_end - win);  // a tile never crosses into the next event
                const unsigned int qe = win + t1;
                int u[kMaxAxes];
                unpack_cell(pc, P.axes, u);
                unsigned int start, pre, end;
                const unsigned int M = wave_runs(u, cell0, P, rl, cell_start, start, pre, end);
                for (unsigned int q0 = qs; q0 < qe; q0 += kQT) {
                    const int Qn = static_cast<int>(uniform(min(static_cast<unsigned int>(kQT), qe - q0)));
                    if (prio) {
                        // A SIMD issues the oldest ready wave first, so with every workgroup
                        // resident from the start the waves dispatched last finish last and
                        // the SIMD runs its final stretch with few waves.  Issue priority
                        // falls as a wave works off its share (3 in the first quarter, 0 in
                        // the last), so that waves behind are issued first and the waves of
                        // a SIMD finish closer together.
                        const unsigned int left = q_hi - q0;
                        const unsigned int share = q_hi - q_lo;
                        if (4u * left > 3u * share) __builtin_amdgcn_s_setprio(3);
                        else if (4u * left > 2u * share) __builtin_amdgcn_s_setprio(2);
                        else if (4u * left > share) __builtin_amdgcn_s_setprio(1);
                        else __builtin_amdgcn_s_setprio(0);
                    }
                    // Slots for the group's queries; when they do not fit, the queue is
                    // emptied and the pending lists written out first.
                    if (pend_n + static_cast<unsigned int>(Qn) > static_cast<unsigned int>(kQT)) {
                        drain_all();
                        flush(pend0, pend_n);
                        pend0 += pend_n;
                        pend_n = 0;
                    }
                    const unsigned int gs = pend0 + pend_n;  // number of the group's first query
                    // Original row of query q0 + lane, held by lane q0 + lane - win.
                    const unsigned int iq = static_cast<unsigned int>(
                        __shfl(static_cast<int>(v_orig), static_cast<int>((q0 - win + lane) & 63u)));
                    if (lane < Qn) {
                        const unsigned int sl = (gs + static_cast<unsigned int>(lane)) & (kQT - 1);
                        qcnt[sl] = 0u;
                        qrow_s[sl] = q0 + lane;
                        qid[sl] = iq;
                    }
                    pend_n += static_cast<unsigned int>(Qn);
                    // Candidates are fetched one chunk ahead so that their latency overlaps
                    // the tests of the current chunk: each lane holds its candidate's first
                    // four coordinates (one 16-byte load).  Idle lanes read row 0 (any row
                    // is a valid address) and are masked out of every ballot.
                    constexpr int kHeld = 4;  // candidate coordinates held per lane
                    static_assert(kLead <= kHeld, "the first stage uses the held coordinates");
                    float cn[kHeld];
                    unsigned int sn;
                    // Candidate b + lane lies in the last run that starts at or before it:
                    // each run that starts inside the chunk marks its first lane (the run
                    // holding candidate b marks lane 0) and a prefix maximum spreads the
                    // marks over the lanes after them.
                    auto fetch = [&](unsigned int b) {
                        wave_lds_sync();
                        mark[lane] = 0u;
                        wave_lds_sync();
                        if (end > pre && pre < b + 64u && end > b) mark[pre > b ? pre - b : 0u] = lane + 1u;
                        wave_lds_sync();
                        const int r = static_cast<int>(wave_scan_max(mark[lane])) - 1;
                        const unsigned int mm = b + lane;
                        const unsigned int srow = static_cast<unsigned int>(__shfl(start, r)) +
                                                  (mm - static_cast<unsigned int>(__shfl(pre, r)));
                        sn = mm < M ? srow : 0u;
                        const float4 v = *reinterpret_cast<const float4 *>(sorted + static_cast<size_t>(sn) * DP);
                        cn[0] = v.x;
                        cn[1] = v.y;
                        cn[2] = v.z;
                        cn[3] = v.w;
                        // Lanes past the last candidate fail every first-stage test.
                        if (mm >= M) cn[0] = INFINITY;
                    };
                    fetch(0u);
                    for (unsigned int base = 0; base < M; base += 64) {
                        float c[kHeld];
#pragma unroll
                        for (int k = 0; k < kHeld; ++k) c[k] = cn[k];
                        const unsigned int s = sn;
                        if (base + 64 < M) fetch(base + 64);
                        // Query rows are wave-uniform (scalar loads); the next one is
                        // requested before the current one is tested (the sorted rows end with
                        // one padding row, so the request after the last query stays in bounds).
                        float qn[kLead];
#pragma unroll
                        for (int k = 0; k < kLead; ++k) qn[k] = sorted[static_cast<size_t>(q0) * DP + k];
                        const float *qrow = sorted + static_cast<size_t>(q0) * DP;
                        for (int q = 0; q < Qn; ++q, qrow += DP) {
                            float qc[kLead];
#pragma unroll
                            for (int k = 0; k < kLead; ++k) qc[k] = qn[k];
#pragma unroll
                            for (int k = 0; k < kLead; ++k) qn[k] = qrow[DP + k];
                            // First stage: kLead terms for all 64 candidates; pairs that are not
                            // yet at r2 are queued (exact: the remaining terms only add).
                            const float acc = add_terms_r<0, kLead, kHeld, kLead>(0.0f, c, qc);
                            const unsigned long long m1 = __builtin_amdgcn_ballot_w64(acc < r2);
                            if (m1 == 0ull) continue;
                            if (acc < r2) {
                                ++survived;
                                const unsigned int e = (tail + prefix_count(m1)) & (kRing - 1);
                                const unsigned int slot = uniform((gs + static_cast<unsigned int>(q)) & (kQT - 1));
                                ring[e] = (static_cast<unsigned long long>(slot) << 32) | s;
                                racc[e] = acc;
                            }
                            tail += static_cast<unsigned int>(__popcll(m1));
                            if (tail - head >= 64u) {
                                finish_rows(head, 64u);
                                head += 64u;
                            }
                        }
                    }
                    if (lane < Qn) tested += M;
                }
                t0 = t1;
            }
            win += nwin;
        }
        piece = kPieces > 1 ? x_dyn + pool + __builtin_amdgcn_readfirstlane(claimed) * pools : x_end;
    }
    drain_all();
    if (pend_n) flush(pend0, pend_n);
    capped = wave_sum(capped);
    tested = wave_sum(tested);
    survived = wave_sum(survived);
    if (lane == 0) {
        tested_w[wave_id()] = tested;
        survived_w[wave_id()] = survived;
        capped_w[wave_id()] = capped;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0, sv = 0;
        unsigned int c = 0;
        for (int w = 0; w < kWaves; ++w) {
            t += tested_w[w];
            sv += survived_w[w];
            c += capped_w[w];
        }
        tested_out[blockIdx.x] = t;
        tested_out[kMaxSearchBlocks + blockIdx.x] = sv;
        capped_out[blockIdx.x] = c;
    }
}

// --------------------------------------------------------------- kept totals

// Totals of the kept counts per placement tile, one wave per tile, and per group
// of kKeptGroup tiles (spread-address atomics into totals cleared by the bounds
// pass).  The last workgroup, which has no tiles, sums the search's per-workgroup
// counts for the report, beside the others and off the placement pass's path.
__global__ __launch_bounds__(kBlock) void k_kept_sums(int n, const unsigned int *__restrict__ kept,
                                                      unsigned long long *__restrict__ sums_kept,
                                                      unsigned long long *__restrict__ sums_kept2, int tiles_kept,
                                                      const unsigned long long *__restrict__ tested,
                                                      const unsigned int *__restrict__ capped_blk,
                                                      int search_blocks, Counters *__restrict__ ctr) {
    if (ctr->abort) return;
    if (blockIdx.x == gridDim.x - 1) {
        __shared__ unsigned long long red[3][kWaves];
        unsigned long long t = 0, sv = 0, cp = 0;
        for (int k = threadIdx.x; k < search_blocks; k += kBlock) {
            t += tested[k];
            sv += tested[kMaxSearchBlocks + k];
            cp += capped_blk[k];
        }
        t = wave_sum(t);
        sv = wave_sum(sv);
        cp = wave_sum(cp);
        if (lane_id() == 0) {
            red[0][wave_id()] = t;
            red[1][wave_id()] = sv;
            red[2][wave_id()] = cp;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            t = sv = cp = 0;
            for (int w = 0; w < kWaves; ++w) {
                t += red[0][w];
                sv += red[1][w];
                cp += red[2][w];
            }
            ctr->tested = t;
            ctr->survived = sv;
            ctr->capped = static_cast<unsigned int>(cp);
        }
        return;
    }
    const int nw = static_cast<int>(gridDim.x - 1) * kWaves;
    for (int t = static_cast<int>(blockIdx.x) * kWaves + wave_id(); t < tiles_kept; t += nw) {
        const long long b = static_cast<long long>(t) * kPlaceTile;
        unsigned long long s = 0;
#pragma unroll
        for (int k = 0; k < kPlaceTile / 64; ++k) {
            const long long idx = b + k * 64 + lane_id();
            if (idx < n) s += kept[idx] & ~kKeptLong;
        }
        s = wave_sum(s);
        if (lane_id() == 0) {
            sums_kept[t] = s;
            if (s && tiles_kept > kFlatTiles) atomicAdd(&sums_kept2[t / kKeptGroup], s);
        }
    }
}

// --------------------------------------------------------------- long lists

// LDS of the long-list collection (besides the hit keys and the kept ids, which
// use the placement pass's window arrays: they hold nothing at that point).
template <int DP>
struct LongLds {
    unsigned int hist[256];
    __align__(16) float qv[DP];
    unsigned int run_start[64];
    unsigned int run_pre[65];
    unsigned int fill;
    unsigned int left;
    unsigned long long prefix;
};

// Hit keys a long list keeps in LDS (the two window arrays of the placement pass);
// a list with more hits is selected by enumerating its candidates again per pass.
constexpr unsigned int kKeyCap = kOwnerWindow;

// One long list, collected again by the whole workgroup (every thread calls this
// with the same arguments): the query's candidates are enumerated over the same
// runs of cells as in the search and its hits keyed (bits(D) << 32 | j), which
// orders them by (D, j) since D is never negative.  With more hits than n_out
// (the cap binds) the n_out-th smallest key is found by an MSB-first radix select
// (8 passes of 8 bits; in each pass a scan over the 256 bin counts finds the bin
// that holds it), over the keys in LDS or, past kKeyCap hits, by enumerating the
// candidates again.  The kept ids are sorted by a bitonic network in LDS and
// written, local to the query's event, to out[0, n_out).
template <int DP>
__device__ void long_list(const float *__restrict__ sorted, const unsigned int *__restrict__ sorted_id,
                          const unsigned int *__restrict__ cell_start, const Plan &P, unsigned int cell0,
                          unsigned int slot, float r2, unsigned int n_out, long long row0,
                          long long *__restrict__ out, unsigned int *__restrict__ wbuf,
                          unsigned long long *__restrict__ scratch, LongLds<DP> &L) {
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(wbuf);  // [kKeyCap]
    unsigned int *ids = wbuf;                                                  // [kMaxK], after the keys are read
    const int nruns = run_count(P);
    for (int k = threadIdx.x; k < DP; k += kPlaceBlock) L.qv[k] = sorted[static_cast<size_t>(slot) * DP + k];
    if (wave_id() == 0) {
        int u[kMaxAxes];
        unpack_cell(sorted_id[2u * slot + 1u], P.axes, u);
        unsigned int start, pre, end;
        const unsigned int M = wave_runs(u, cell0, P, run_lane(P), cell_start, start, pre, end);
        L.run_start[lane_id()] = start;
        L.run_pre[lane_id()] = pre;
        if (lane_id() == 0) {
            L.run_pre[64] = M;
            L.fill = 0u;
        }
    }
    __syncthreads();
    const unsigned int M = L.run_pre[64];
    float q[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) q[k] = L.qv[k];

    // Candidate m lies in the last run that starts at or before it (runs are
    // numbered in order, so their starts ascend).
    auto hit_key = [&](unsigned int m, bool &ok) -> unsigned long long {
        int lo = 0, hi = nruns - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.run_pre[mid] <= m) lo = mid;
            else hi = mid - 1;
        }
        const unsigned int s = L.run_start[lo] + (m - L.run_pre[lo]);
        float c[DP];
        load_row<DP>(sorted, s, c);
        const float D = sq_dist<DP>(c, q);
        ok = (D < r2) && (s != slot);
        return (static_cast<unsigned long long>(__float_as_uint(D)) << 32) | sorted_id[2u * s];
    };
    // One radix pass: the bin of the left-th smallest key among those matching the
    // prefix above `shift + 8`, and how many of them lie in lower bins.
    auto pick_bin = [&](unsigned long long prefix, int shift) {
        const unsigned int c = L.hist[threadIdx.x];
        const unsigned int left = L.left;  // read before the scan's barriers; the winner writes after them
        const unsigned int below = static_cast<unsigned int>(block_exclusive_scan(c, scratch));
        if (below < left && left <= below + c) {
            L.left = left - below;
            L.prefix = prefix | (static_cast<unsigned long long>(threadIdx.x) << shift);
        }
        __syncthreads();
    };

    // Every hit, keyed, into LDS (as many as fit).
    for (unsigned int m = threadIdx.x; m < M; m += kPlaceBlock) {
        bool ok;
        const unsigned long long key = hit_key(m, ok);
        if (ok) {
            const unsigned int pos = atomicAdd(&L.fill, 1u);
            if (pos < kKeyCap) keys[pos] = key;
        }
    }
    __syncthreads();
    const unsigned int h = L.fill;
    const bool in_lds = h <= kKeyCap;
    unsigned long long limit = ~0ull;  // keep hits with key <= limit
    if (h > n_out) {
        if (threadIdx.x == 0) {
            L.prefix = 0ull;
            L.left = n_out;
        }
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            L.hist[threadIdx.x] = 0u;
            __syncthreads();
            const unsigned long long prefix = L.prefix;
            auto count = [&](unsigned long long key) {
                if (pass == 0 || (key >> (shift + 8)) == (prefix >> (shift + 8)))
                    atomicAdd(&L.hist[(key >> shift) & 255ull], 1u);
            };
            if (in_lds) {
                for (unsigned int k = threadIdx.x; k < h; k += kPlaceBlock) count(keys[k]);
            } else {
                for (unsigned int m = threadIdx.x; m < M; m += kPlaceBlock) {
                    bool ok;
                    const unsigned long long key = hit_key(m, ok);
                    if (ok) count(key);
                }
            }
            __syncthreads();
            pick_bin(prefix, shift);
        }
        limit = L.prefix;
    }
    // The kept ids, compacted into LDS (keys in LDS are read into registers first,
    // since the ids overwrite them).
    constexpr int kPer = kKeyCap / kPlaceBlock;
    if (in_lds) {
        unsigned long long mine[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const unsigned int k = threadIdx.x + static_cast<unsigned int>(j) * kPlaceBlock;
            mine[j] = k < h ? keys[k] : ~0ull;
        }
        __syncthreads();
        if (threadIdx.x == 0) L.fill = 0u;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (mine[j] != ~0ull && mine[j] <= limit) {
                const unsigned int pos = atomicAdd(&L.fill, 1u);
                if (pos < static_cast<unsigned int>(kMaxK)) ids[pos] = static_cast<unsigned int>(mine[j]);
            }
        }
    } else {
        __syncthreads();
        if (threadIdx.x == 0) L.fill = 0u;
        __syncthreads();
        for (unsigned int m = threadIdx.x; m < M; m += kPlaceBlock) {
            bool ok;
            const unsigned long long key = hit_key(m, ok);
            if (ok && key <= limit) {
                const unsigned int pos = atomicAdd(&L.fill, 1u);
                if (pos < static_cast<unsigned int>(kMaxK)) ids[pos] = static_cast<unsigned int>(key);
            }
        }
    }
    __syncthreads();
    // Bitonic sort of the ids by value; slots past the ids found hold the largest
    // value (only a corrupted kept count could leave any of them in [0, n_out)).
    const unsigned int found = min(L.fill, static_cast<unsigned int>(kMaxK));
    unsigned int size = 1;
    while (size < n_out) size <<= 1;
    for (unsigned int e = found + threadIdx.x; e < size; e += kPlaceBlock) ids[e] = 0xffffffffu;
    __syncthreads();
    for (unsigned int k = 2; k <= size; k <<= 1) {
        for (unsigned int j = k >> 1; j > 0; j >>= 1) {
            for (unsigned int e = threadIdx.x; e < size; e += kPlaceBlock) {
                const unsigned int o = e ^ j;
                if (o > e) {
                    const unsigned int a = ids[e], b = ids[o];
                    const bool up = (e & k) == 0;
                    if ((a > b) == up) {
                        ids[e] = b;
                        ids[o] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (unsigned int t = threadIdx.x; t < n_out; t += kPlaceBlock) out[t] = static_cast<long long>(ids[t]) - row0;
    __syncthreads();
}

// ------------------------------------------------------------------- place

// Block b < tiles_kept owns queries [kPlaceTile b, kPlaceTile (b + 1)), one per
// thread.  Its first output position is the sum of the kept totals before it
// (whole groups of kKeptGroup tiles, then the tiles of its own group); a block
// scan of its kept counts gives each query's offset.  Lists in the fixed
// kListCap-slot places come from the search in the order their hits were found:
// each query's thread sorts its list in registers.  The block's output is then
// formed in LDS a window at a time (each query's thread puts its row and its
// neighbours at its own positions), so that consecutive threads write consecutive
// int64 positions; the neighbour positions of a long list are left to its
// collector.  Indices are made local to each query's event.  Block 0 writes the
// report and the status; the block holding an event's first row writes its edge
// offset.  Then every block, including those past the tiles (the grid has at least
// kPlaceMinBlocks), collects the long lists of the search's queue in turn: the
// list's output position is the sum of the tile totals before its query's tile and
// of the kept counts before it in that tile.
template <int DP>
__global__ __launch_bounds__(kPlaceBlock) void k_place(long long rows, const EventDesc *__restrict__ ev,
                                                       int n_events, const unsigned int *__restrict__ kept,
                                                       const unsigned long long *__restrict__ sums_kept,
                                                       const unsigned long long *__restrict__ sums_kept2,
                                                       int groups_kept, int tiles_kept,
                                                       const unsigned int *__restrict__ long_slots,
                                                       const unsigned int *__restrict__ temp,
                                                       const float *__restrict__ sorted,
                                                       const unsigned int *__restrict__ sorted_id,
                                                       const unsigned int *__restrict__ cell_start, float r2, int K,
                                                       long long *__restrict__ src, long long *__restrict__ dst,
                                                       unsigned long long cap, const Plan *__restrict__ plans,
                                                       const Counters *__restrict__ ctr,
                                                       long long *__restrict__ edge_off,
                                                       Report *__restrict__ report) {
    static_assert(kPlaceBlock == kPlaceTile, "one query per thread");
    static_assert(kOwnerWindow >= kMaxK && kPlaceBlock == 256, "the window arrays hold a long list's keys");
    // A window of the block's output (event-local rows, then neighbours); a
    // neighbour entry of kSkip belongs to a long list, written by its collector.
    constexpr unsigned int kSkip = 0xffffffffu;
    __shared__ unsigned int o[kPlaceTile + 1];
    __shared__ __align__(16) unsigned int wbuf[2 * kOwnerWindow];
    unsigned int *wsrc = wbuf;
    unsigned int *wdst = wbuf + kOwnerWindow;
    __shared__ unsigned long long scratch[kWaves];
    __shared__ LongLds<DP> L;
    const bool abort = ctr->abort != 0;
    const int b = static_cast<int>(blockIdx.x);
    const bool tile_block = b < tiles_kept;
    const long long i0 = static_cast<long long>(b) * kPlaceTile;
    const int cnt = tile_block ? static_cast<int>(rows - i0 < kPlaceTile ? rows - i0 : kPlaceTile) : 0;
    const int q = threadIdx.x;
    // The query's kept count and its list of up to kListCap (at the query's own
    // fixed place) are requested first, so that their round trips overlap the sums
    // of the tile totals below.
    const bool mine = !abort && q < cnt;
    const unsigned int kraw = mine ? kept[i0 + q] : 0u;
    const unsigned int kq = kraw & ~kKeptLong;
    const bool is_long = mine && (kraw & kKeptLong) != 0u;
    const bool fixed = mine && kq > 0u && !is_long;
    unsigned int v[kListCap];
    if (fixed) {
        const uint4 *l4 = reinterpret_cast<const uint4 *>(temp + static_cast<size_t>(i0 + q) * kListCap);
#pragma unroll
        for (int c = 0; c < kListCap / 4; ++c) {
            const uint4 w = l4[c];
            v[4 * c] = w.x;
            v[4 * c + 1] = w.y;
            v[4 * c + 2] = w.z;
            v[4 * c + 3] = w.w;
        }
    }
    // Sum of the tile totals before tile t (and of all of them), one part per thread.
    auto tile_prefix = [&](int t, unsigned long long &before, unsigned long long &all) {
        before = 0;
        all = 0;
        if (tiles_kept <= kFlatTiles) {
            // Few tiles: the tile totals are summed directly.
            for (int x = threadIdx.x; x < tiles_kept; x += kPlaceBlock) {
                const unsigned long long y = sums_kept[x];
                all += y;
                if (x < t) before += y;
            }
        } else {
            const int gt = t / kKeptGroup;
            for (int x = threadIdx.x; x < groups_kept; x += kPlaceBlock) {
                const unsigned long long y = sums_kept2[x];
                all += y;
                if (x < gt) before += y;
            }
            const int x = gt * kKeptGroup + static_cast<int>(threadIdx.x);
            if (threadIdx.x < kKeptGroup && x < t) before += sums_kept[x];
        }
    };
    __shared__ unsigned long long red[3 * kWaves];
    unsigned long long pre = 0, tot = 0;
    if (!abort) tile_prefix(tile_block ? b : 0, pre, tot);
    // The block's first output position, E, and each query's offset in the block.
    unsigned long long oq64;
    block_sums_and_scan(pre, tot, static_cast<unsigned long long>(kq), red, pre, tot, oq64);
    const long long E = static_cast<long long>(tot);
    const bool overflow = static_cast<unsigned long long>(E) > cap;
    if (b == 0 && threadIdx.x == 0) {
        const Plan P = plans[0];
        Report rep;
        rep.n_edges = E;
        rep.tested = abort ? 0ull : ctr->tested;
        rep.survived = abort ? 0ull : ctr->survived;
        rep.abort = abort ? 1 : 0;
        rep.capped = abort ? 0u : ctr->capped;
        rep.heavy = ctr->heavy_count;
        rep.n_cells = P.n_cells;
        for (int p = 0; p < kMaxAxes; ++p) {
            rep.G[p] = P.G[p];
            rep.c[p] = P.c[p];
        }
        *report = rep;
        edge_off[n_events] = E;
        edge_off[n_events + 1] = abort ? 2 : (overflow ? 3 : 0);
    }
    if (tile_block) {
        const unsigned int oq = static_cast<unsigned int>(oq64);
        if (q < cnt) o[q] = oq;
        if (q == cnt - 1) o[cnt] = oq + kq;
        __syncthreads();
        // Edge ranges of the events whose first row lies in this block (events with no
        // rows at the very end start at E).
        {
            int lo = 0, hi = n_events;  // first event whose first row is >= i0
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (ev[mid].row0 < i0) lo = mid + 1;
                else hi = mid;
            }
            const bool last_tile = b == tiles_kept - 1;
            for (int e = lo + threadIdx.x; e < n_events; e += kPlaceBlock) {
                const long long r0 = ev[e].row0;
                if (r0 >= i0 + cnt && !(last_tile && r0 >= rows)) break;
                edge_off[e] = abort ? 0 : (r0 >= rows ? E : static_cast<long long>(pre + o[r0 - i0]));
            }
        }
        if (abort || overflow) return;
        const unsigned int brow =
            n_events == 1 || q >= cnt ? 0u : static_cast<unsigned int>(ev[find_event(ev, n_events, i0 + q)].row0);
        const unsigned int total = o[cnt];
        if (pre + total > cap) return;  // cannot happen when E <= cap; never write past the outputs
        // A list from a fixed place holds the query's hits in the order they were
        // found: its thread sorts it (a bitonic network over 16 slots, the unused
        // ones holding the largest value).
        if (fixed) {
#pragma unroll
            for (int u = 0; u < kListCap; ++u) v[u] = static_cast<unsigned int>(u) < kq ? v[u] : 0xffffffffu;
#pragma unroll
            for (int k = 2; k <= kListCap; k <<= 1) {
#pragma unroll
                for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
                    for (int u = 0; u < kListCap; ++u) {
                        const int l = u ^ j;
                        if (l > u) {
                            const unsigned int lo = v[u] < v[l] ? v[u] : v[l];
                            const unsigned int hi = v[u] < v[l] ? v[l] : v[u];
                            const bool up = (u & k) == 0;
                            v[u] = up ? lo : hi;
                            v[l] = up ? hi : lo;
                        }
                    }
                }
            }
        }
        const unsigned int il = static_cast<unsigned int>(i0 + q) - brow;  // the query's event-local row
        for (unsigned int w0 = 0; w0 < total; w0 += kOwnerWindow) {
            const unsigned int wend = total - w0 < kOwnerWindow ? total - w0 : kOwnerWindow;
            if (fixed) {
#pragma unroll
                for (int u = 0; u < kListCap; ++u) {
                    const unsigned int pw = oq + static_cast<unsigned int>(u) - w0;  // wraps when before the window
                    if (static_cast<unsigned int>(u) < kq && oq + u >= w0 && pw < wend) {
                        wsrc[pw] = il;
                        wdst[pw] = v[u] - brow;
                    }
                }
            } else if (is_long) {
                const unsigned int a0 = oq > w0 ? oq - w0 : 0u;
                const unsigned int a1 = oq + kq > w0 ? min(oq + kq - w0, wend) : 0u;
                for (unsigned int pw = a0; pw < a1; ++pw) {
                    wsrc[pw] = il;
                    wdst[pw] = kSkip;
                }
            }
            __syncthreads();
            for (unsigned int pw = threadIdx.x; pw < wend; pw += kPlaceBlock) {
                const long long at = static_cast<long long>(pre) + w0 + pw;
                src[at] = wsrc[pw];
                const unsigned int dv = wdst[pw];
                if (dv != kSkip) dst[at] = dv;
            }
            __syncthreads();
        }
    }
    if (abort || overflow) return;
    // Long lists of the search's queue, every gridDim-th one.
    const unsigned int n_long = ctr->heavy_count;
    for (unsigned int h = blockIdx.x; h < n_long; h += gridDim.x) {
        const unsigned int slot = long_slots[h];
        if (static_cast<long long>(slot) >= rows) continue;  // only a corrupted queue
        const long long gi = sorted_id[2u * slot];  // the query's original row
        const int t = static_cast<int>(gi / kPlaceTile);
        if (gi >= rows || t >= tiles_kept) continue;  // likewise
        unsigned long long at = 0, all = 0;
        tile_prefix(t, at, all);
        const long long x = static_cast<long long>(t) * kPlaceTile + threadIdx.x;
        if (x < gi) at += kept[x] & ~kKeptLong;
        at = block_sum(at, scratch);
        const unsigned int nq = kept[gi] & ~kKeptLong;
        if (at + nq > cap) continue;  // cannot happen when E <= cap
        const int e = n_events == 1 ? 0 : find_event(ev, n_events, gi);
        const Plan P = plans[e];
        long_list<DP>(sorted, sorted_id, cell_start, P, static_cast<unsigned int>(ev[e].cell0), slot, r2, nq,
                      ev[e].row0, dst + at, wbuf, scratch, L);
    }
}

// Launches the stages whose kernels depend on the padded row width.
template <int DP>
void launch_rows(const LaunchArgs &a, const Workspace &ws, int vec4) {
    auto mark = [&](int stage) {
        if (a.events) (void)hipEventRecord(a.events[stage], a.stream);
    };
    const long long rows = ws.rows;
    const long long nb = (static_cast<long long>(a.max_n) + kBlock - 1) / kBlock;
    const int gs = static_cast<int>(nb < 1 ? 1 : (nb > 4096 ? 4096 : nb));
    hipLaunchKernelGGL(k_scatter<DP>, dim3(gs, a.n_events), dim3(kBlock), 0, a.stream, a.d, vec4, ws.ev, a.ev0,
                       a.ev_from_arg, ws.plans,
                       ws.pcell, ws.rank, ws.cell_start, ws.ctr, ws.sorted, ws.sorted_id);
    mark(4);
    if (a.K < kListCap)
        hipLaunchKernelGGL((k_search<DP, true>), dim3(a.search_blocks), dim3(kBlock), 0, a.stream, ws.sorted,
                           ws.sorted_id, ws.wave_start, ws.claims, ws.ev, a.n_events, ws.cell_start, ws.plans,
                           a.r2, a.K, ws.kept, ws.temp, ws.long_slots, ws.ctr, ws.tested, ws.capped_blk,
                           a.search_prio);
    else
        hipLaunchKernelGGL((k_search<DP, false>), dim3(a.search_blocks), dim3(kBlock), 0, a.stream, ws.sorted,
                           ws.sorted_id, ws.wave_start, ws.claims, ws.ev, a.n_events, ws.cell_start, ws.plans,
                           a.r2, a.K, ws.kept, ws.temp, ws.long_slots, ws.ctr, ws.tested, ws.capped_blk,
                           a.search_prio);
    mark(5);
    const long long kb = (static_cast<long long>(ws.tiles_kept_n) + kWaves - 1) / kWaves;
    const int kblocks = static_cast<int>(kb > 2048 ? 2048 : kb) + 1;  // and one for the search's counts
    hipLaunchKernelGGL(k_kept_sums, dim3(kblocks), dim3(kBlock), 0, a.stream, static_cast<int>(rows), ws.kept,
                       ws.sums_kept, ws.sums_kept2, ws.tiles_kept_n, ws.tested, ws.capped_blk, a.search_blocks,
                       ws.ctr);
    mark(6);
    const int place_blocks = ws.tiles_kept_n > kPlaceMinBlocks ? ws.tiles_kept_n : kPlaceMinBlocks;
    hipLaunchKernelGGL(k_place<DP>, dim3(static_cast<unsigned int>(place_blocks)), dim3(kPlaceBlock), 0, a.stream,
                       rows, ws.ev, a.n_events, ws.kept, ws.sums_kept, ws.sums_kept2, ws.groups_kept_n,
                       ws.tiles_kept_n, ws.long_slots, ws.temp, ws.sorted, ws.sorted_id, ws.cell_start, a.r2, a.K,
                       a.src, a.dst, a.edge_capacity, ws.plans, ws.ctr, a.edge_off_out ? a.edge_off_out : ws.edge_off,
                       a.report_out ? a.report_out : ws.report);
}

template <int DP>
int occupancy_blocks(bool sel) {
    int per_cu = 0;
    const hipError_t e = sel ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_search<DP, true>, kBlock, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_search<DP, false>, kBlock, 0);
    if (e != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return per_cu * cus;
}

}  // namespace

int search_blocks_for(int dpad, bool sel) {
    switch (dpad) {
        case 4: return occupancy_blocks<4>(sel);
        case 8: return occupancy_blocks<8>(sel);
        case 12: return occupancy_blocks<12>(sel);
        case 16: return occupancy_blocks<16>(sel);
        case 24: return occupancy_blocks<24>(sel);
        case 32: return occupancy_blocks<32>(sel);
        case 48: return occupancy_blocks<48>(sel);
        default: return occupancy_blocks<64>(sel);
    }
}

hipError_t enqueue_build(const LaunchArgs &a, const Workspace &ws) {
    auto mark = [&](int stage) {
        if (a.events) (void)hipEventRecord(a.events[stage], a.stream);
    };
    const int vec4 = a.vec4;
    const int keys_per = a.max_n > kKeysTwoFrom ? 2 : 1;  // points per thread
    const long long kb = (static_cast<long long>(a.max_n) + kKeysBlock * keys_per - 1) / (kKeysBlock * keys_per);
    const int gkeys = static_cast<int>(kb < 1 ? 1 : kb);
    Dims dd;
    for (int p = 0; p < kMaxAxes; ++p) dd.c[p] = p < a.axes ? a.dims[p] : -1;
    mark(0);
    hipLaunchKernelGGL(k_bounds, dim3(a.bounds_blocks, a.n_events), dim3(kBlock), 0, a.stream, a.d, dd, vec4,
                       ws.ev, a.ev0, a.ev_from_arg, ws.part, ws.cell_count, ws.cells, ws.sums_cells,
                       ws.tiles_cells_n, ws.sums_kept2, ws.groups_kept_n, ws.ctr);
    mark(1);
    if (keys_per == 2)
        hipLaunchKernelGGL(k_keys<2>, dim3(gkeys, a.n_events), dim3(kKeysBlock), 0, a.stream, a.d, dd, a.axes,
                           a.r, a.cell_div, ws.ev, a.ev0, a.ev_from_arg, ws.part, a.bounds_blocks, ws.plans, ws.ctr,
                           ws.pcell, ws.rank, ws.cell_count, ws.sums_cells);
    else
        hipLaunchKernelGGL(k_keys<1>, dim3(gkeys, a.n_events), dim3(kKeysBlock), 0, a.stream, a.d, dd, a.axes,
                           a.r, a.cell_div, ws.ev, a.ev0, a.ev_from_arg, ws.part, a.bounds_blocks, ws.plans, ws.ctr,
                           ws.pcell, ws.rank, ws.cell_count, ws.sums_cells);
    mark(2);
    hipLaunchKernelGGL(k_scan_cells, dim3(ws.tiles_cells_n), dim3(kBlock), 0, a.stream, ws.cell_count, ws.cells,
                       ws.sums_cells, ws.tiles_cells_n, ws.cell_start, ws.wave_start,
                       a.search_blocks * kWaves * search_pieces(a.dpad), ws.rows, ws.claims);
    mark(3);
    switch (a.dpad) {
        case 4: launch_rows<4>(a, ws, vec4); break;
        case 8: launch_rows<8>(a, ws, vec4); break;
        case 12: launch_rows<12>(a, ws, vec4); break;
        case 16: launch_rows<16>(a, ws, vec4); break;
        case 24: launch_rows<24>(a, ws, vec4); break;
        case 32: launch_rows<32>(a, ws, vec4); break;
        case 48: launch_rows<48>(a, ws, vec4); break;
        default: launch_rows<64>(a, ws, vec4); break;
    }
    mark(7);
    return hipGetLastError();
}

}  // namespace frnn
