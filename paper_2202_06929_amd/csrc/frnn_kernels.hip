// HIP kernels of the FRNN graph builder for CDNA4 (gfx950, wave64).
//
// Pipeline of one call (paper, Section 3.4: bin the projected points into grid
// cells, then visit only the cells around each query):
//   k_bounds      min/max of the three binned coordinates, non-finite check,
//                 clears the cell histogram and counters
//   k_keys        plan of the grid (cell edge, cells per axis), cell key of every
//                 point, histogram with in-cell arrival rank
//   k_tile_sums / k_scan_tiles
//                 exclusive scan of the histogram -> first row of every cell
//   k_scatter     counting-sort scatter: rows copied into cell order
//   k_search      one workgroup per cell: the queries of the cell against the
//                 (2*reach+1)^2 contiguous x-runs of neighbouring cells, each lane
//                 one candidate with its coordinates in registers, wave ballots
//                 to collect hits into per-query lists in LDS, lists sorted and
//                 stored in an unsorted edge store
//   k_heavy       queries whose list overflowed LDS or exceeded K: exact K
//                 smallest by (D, j) through an MSB-first radix select
//   k_scan_tiles  exclusive scan of kept counts -> int64 output offsets
//   k_place       edges copied to their final (i asc, j asc) position
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
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Squared distance of the definition: ascending coordinates, separately rounded.
// Rows are zero-padded to DP coordinates; adding +0 leaves the sum unchanged.
template <int DP>
__device__ __forceinline__ float sq_dist(const float (&a)[DP], const float *b) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < DP; ++k) {
        float t = a[k] - b[k];
        float t2 = t * t;
        s = s + t2;
    }
    return s;
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

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Inclusive prefix sum across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    return v;
}

// Sum over the block; every thread gets the total.
__device__ unsigned long long block_sum(unsigned long long v, unsigned long long *scratch) {
    v = wave_sum(v);
    if (lane_id() == 0) scratch[wave_id()] = v;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += scratch[w];
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

// ------------------------------------------------------------------ bounds

__global__ __launch_bounds__(kBlock) void k_bounds(const float *__restrict__ X, int n, int d,
                                                   int d0, int d1, int d2,
                                                   BoundsPartial *__restrict__ part,
                                                   unsigned int *__restrict__ cell_count,
                                                   int cells_max, Counters *__restrict__ ctr) {
    const int tid = blockIdx.x * kBlock + threadIdx.x;
    const int stride = gridDim.x * kBlock;
    for (int c = tid; c < cells_max; c += stride) cell_count[c] = 0u;
    if (tid == 0) {
        ctr->temp_top = 0ull;
        ctr->tested = 0ull;
        ctr->heavy_count = 0u;
        ctr->capped = 0u;
        ctr->heavy_next = 0u;
    }
    float mn0 = INFINITY, mn1 = INFINITY, mn2 = INFINITY;
    float mx0 = -INFINITY, mx1 = -INFINITY, mx2 = -INFINITY;
    int bad = 0;
    for (int i = tid; i < n; i += stride) {
        const float *row = X + static_cast<size_t>(i) * d;
        for (int k = 0; k < d; ++k) bad |= !__builtin_isfinite(row[k]);
        const float a = row[d0], b = row[d1], c = row[d2];
        mn0 = fminf(mn0, a); mx0 = fmaxf(mx0, a);
        mn1 = fminf(mn1, b); mx1 = fmaxf(mx1, b);
        mn2 = fminf(mn2, c); mx2 = fmaxf(mx2, c);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn0 = fminf(mn0, __shfl_xor(mn0, o)); mx0 = fmaxf(mx0, __shfl_xor(mx0, o));
        mn1 = fminf(mn1, __shfl_xor(mn1, o)); mx1 = fmaxf(mx1, __shfl_xor(mx1, o));
        mn2 = fminf(mn2, __shfl_xor(mn2, o)); mx2 = fmaxf(mx2, __shfl_xor(mx2, o));
        bad |= __shfl_xor(bad, o);
    }
    __shared__ BoundsPartial sp[kBlock / 64];
    if (lane_id() == 0) {
        BoundsPartial &p = sp[wave_id()];
        p.mn[0] = mn0; p.mn[1] = mn1; p.mn[2] = mn2;
        p.mx[0] = mx0; p.mx[1] = mx1; p.mx[2] = mx2;
        p.nonfinite = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BoundsPartial out = sp[0];
        for (int w = 1; w < kBlock / 64; ++w)
            for (int p = 0; p < 3; ++p) {
                out.mn[p] = fminf(out.mn[p], sp[w].mn[p]);
                out.mx[p] = fmaxf(out.mx[p], sp[w].mx[p]);
                out.nonfinite |= sp[w].nonfinite;
            }
        out.pad = 0;
        part[blockIdx.x] = out;
    }
}

// ------------------------------------------------------------------- keys

// Wave 0 of a block folds the bounds partials and lane 0 derives the grid.
// Every block derives the same plan from the same partials (min/max are exact).
__device__ void derive_plan(const BoundsPartial *__restrict__ part, int nparts, float r,
                            int cell_div, int cells_max, Plan *out) {
    float mn[3] = {INFINITY, INFINITY, INFINITY};
    float mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int b = lane_id(); b < nparts; b += 64) {
        for (int p = 0; p < 3; ++p) {
            mn[p] = fminf(mn[p], part[b].mn[p]);
            mx[p] = fmaxf(mx[p], part[b].mx[p]);
        }
        bad |= part[b].nonfinite;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        for (int p = 0; p < 3; ++p) {
            mn[p] = fminf(mn[p], __shfl_xor(mn[p], o));
            mx[p] = fmaxf(mx[p], __shfl_xor(mx[p], o));
        }
        bad |= __shfl_xor(bad, o);
    }
    if (lane_id() != 0) return;
    // Cell edge r (1 + 2^-10) / cell_div: the margin absorbs the float32 rounding
    // of the key computation (at most 3 * 2^-24 * G cells per point, G <= 1024),
    // so two points whose float32 distance test can pass land at most cell_div
    // cells apart along every binned axis.
    const float cbase = (r * 1.0009765625f) / static_cast<float>(cell_div);
    float c[3], ext[3];
    int G[3];
    // An axis whose extent is not a finite float (no points, or max - min
    // overflowing) gets a single cell: inv_c = 0 puts every point in cell 0.
    bool single[3];
    for (int p = 0; p < 3; ++p) {
        ext[p] = mx[p] - mn[p];
        single[p] = !(ext[p] >= 0.0f && ext[p] <= FLT_MAX);
        if (!(mn[p] <= mx[p])) mn[p] = 0.0f;
        c[p] = cbase;
        if (!single[p] && ext[p] / c[p] > 1000.0f) c[p] = ext[p] / 1000.0f;
    }
    // Grow the cells until the grid fits cells_max (bounded: after 128 rounds of
    // x1.25 every finite extent spans one cell).
    for (int round = 0;; ++round) {
        long long total = 1;
        for (int p = 0; p < 3; ++p) {
            float g = single[p] ? 1.0f : floorf(ext[p] / c[p]) + 1.0f;
            if (!(g <= static_cast<float>(kGridAxisMax))) g = static_cast<float>(kGridAxisMax);
            if (!(g >= 1.0f)) g = 1.0f;
            G[p] = static_cast<int>(g);
            total *= G[p];
        }
        if (total <= cells_max) break;
        if (round >= 128) {
            for (int p = 0; p < 3; ++p) single[p] = true;
            continue;
        }
        for (int p = 0; p < 3; ++p) c[p] *= 1.25f;
    }
    for (int p = 0; p < 3; ++p) {
        out->lo[p] = mn[p];
        out->c[p] = single[p] ? INFINITY : c[p];
        out->inv_c[p] = single[p] ? 0.0f : 1.0f / c[p];
        out->G[p] = G[p];
    }
    out->n_cells = G[0] * G[1] * G[2];
    out->reach = cell_div;
    out->abort = bad;
    out->pad = 0;
}

__device__ __forceinline__ int cell_coord(float x, float lo, float inv_c, int G) {
    float q = floorf((x - lo) * inv_c);
    q = fmaxf(q, 0.0f);  // also maps NaN to 0
    q = fminf(q, static_cast<float>(G - 1));
    return static_cast<int>(q);
}

__global__ __launch_bounds__(kBlock) void k_keys(const float *__restrict__ X, int n, int d,
                                                 int d0, int d1, int d2, float r, int cell_div,
                                                 int cells_max,
                                                 const BoundsPartial *__restrict__ part, int nparts,
                                                 Plan *__restrict__ plan_out,
                                                 unsigned int *__restrict__ key,
                                                 unsigned int *__restrict__ rank,
                                                 unsigned int *__restrict__ cell_count) {
    __shared__ Plan P;
    if (wave_id() == 0) derive_plan(part, nparts, r, cell_div, cells_max, &P);
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *plan_out = P;
    if (P.abort) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const float *row = X + static_cast<size_t>(i) * d;
        const int u0 = cell_coord(row[d0], P.lo[0], P.inv_c[0], P.G[0]);
        const int u1 = cell_coord(row[d1], P.lo[1], P.inv_c[1], P.G[1]);
        const int u2 = cell_coord(row[d2], P.lo[2], P.inv_c[2], P.G[2]);
        const unsigned int k = static_cast<unsigned int>((u2 * P.G[1] + u1) * P.G[0] + u0);
        key[i] = k;
        rank[i] = atomicAdd(&cell_count[k], 1u);
    }
}

// ------------------------------------------------------------------- scans

__global__ __launch_bounds__(kBlock) void k_tile_sums(const unsigned int *__restrict__ in,
                                                      int host_len, const int *__restrict__ dev_len,
                                                      unsigned long long *__restrict__ sums) {
    __shared__ unsigned long long scratch[kBlock / 64];
    const long long len = dev_len ? *dev_len : host_len;
    const long long base = static_cast<long long>(blockIdx.x) * kScanTile;
    unsigned long long s = 0;
    for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
        const long long idx = base + k;
        if (idx < len) s += in[idx];
    }
    s = block_sum(s, scratch);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// out[i] = sum of in[0..i) for i in [0, len]; out[len] is the total.
template <typename OutT>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const unsigned int *__restrict__ in,
                                                       int host_len, const int *__restrict__ dev_len,
                                                       const unsigned long long *__restrict__ sums,
                                                       OutT *__restrict__ out) {
    __shared__ unsigned long long scratch[kBlock / 64];
    const long long len = dev_len ? *dev_len : host_len;
    const long long base = static_cast<long long>(blockIdx.x) * kScanTile;
    if (base > len) return;
    unsigned long long off = 0;
    for (unsigned int t = threadIdx.x; t < blockIdx.x; t += kBlock) off += sums[t];
    off = block_sum(off, scratch);
    constexpr int kPer = kScanTile / kBlock;
    unsigned int v[kPer];
    unsigned long long tsum = 0;
    const long long first = base + static_cast<long long>(threadIdx.x) * kPer;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const long long idx = first + j;
        v[j] = idx < len ? in[idx] : 0u;
        tsum += v[j];
    }
    unsigned long long run = block_exclusive_scan(tsum, scratch) + off;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const long long idx = first + j;
        if (idx <= len) out[idx] = static_cast<OutT>(run);
        run += v[j];
    }
}

// ----------------------------------------------------------------- scatter

__global__ __launch_bounds__(kBlock) void k_scatter(const float *__restrict__ X, int n, int d, int dpad,
                                                    const unsigned int *__restrict__ key,
                                                    const unsigned int *__restrict__ rank,
                                                    const unsigned int *__restrict__ cell_start,
                                                    const Plan *__restrict__ plan,
                                                    float *__restrict__ sorted,
                                                    unsigned int *__restrict__ sorted_id) {
    if (plan->abort) return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const unsigned int slot = cell_start[key[i]] + rank[i];
        const float *row = X + static_cast<size_t>(i) * d;
        float *out = sorted + static_cast<size_t>(slot) * dpad;
        for (int k = 0; k < d; ++k) out[k] = row[k];
        for (int k = d; k < dpad; ++k) out[k] = 0.0f;
        sorted_id[slot] = static_cast<unsigned int>(i);
    }
}

// ------------------------------------------------------------ neighbour runs

// The neighbour cells of `cell` form (2*reach+1)^2 runs that are contiguous in
// cell order (x is the fastest axis).  Threads of wave 0 build one run each and
// publish run starts and the prefix of run lengths in LDS.  Returns nothing;
// run_pre[nruns] is the candidate count.  Must be called by the whole block.
__device__ void build_runs(unsigned int cell, const Plan &P, const unsigned int *__restrict__ cell_start,
                           unsigned int *run_start, unsigned int *run_pre, int *nruns_out) {
    const int G0 = P.G[0], G1 = P.G[1], G2 = P.G[2];
    const int ux = static_cast<int>(cell % static_cast<unsigned int>(G0));
    const int uy = static_cast<int>((cell / static_cast<unsigned int>(G0)) % static_cast<unsigned int>(G1));
    const int uz = static_cast<int>(cell / static_cast<unsigned int>(G0 * G1));
    const int R = P.reach;
    const int side = 2 * R + 1;
    const int nr = side * side;
    if (wave_id() == 0) {
        const int t = lane_id();
        unsigned int start = 0, len = 0;
        if (t < nr) {
            const int yy = uy + (t % side) - R;
            const int zz = uz + (t / side) - R;
            if (yy >= 0 && yy < G1 && zz >= 0 && zz < G2) {
                const int xlo = max(ux - R, 0), xhi = min(ux + R, G0 - 1);
                const unsigned int row = static_cast<unsigned int>((zz * G1 + yy) * G0);
                start = cell_start[row + xlo];
                len = cell_start[row + xhi + 1] - start;
            }
        }
        const unsigned int inc = wave_inclusive_scan(len);
        if (t < nr) {
            run_start[t] = start;
            run_pre[t + 1] = inc;
        }
        if (t == 0) {
            run_pre[0] = 0;
            *nruns_out = nr;
        }
    }
    __syncthreads();
}

// Maps candidate number m in [0, run_pre[nruns]) to its sorted row.
__device__ __forceinline__ unsigned int candidate_row(unsigned int m, const unsigned int *run_start,
                                                      const unsigned int *run_pre, int nruns) {
    int r = 0;
    while (r + 1 < nruns && run_pre[r + 1] <= m) ++r;
    return run_start[r] + (m - run_pre[r]);
}

// ------------------------------------------------------------------ search

constexpr int kQTile = 64;

template <int DP>
__global__ __launch_bounds__(kBlock) void k_search(const float *__restrict__ sorted,
                                                   const unsigned int *__restrict__ sorted_id,
                                                   const unsigned int *__restrict__ cell_start,
                                                   const Plan *__restrict__ plan, float r2, int K,
                                                   unsigned int *__restrict__ kept,
                                                   unsigned long long *__restrict__ tpos,
                                                   unsigned int *__restrict__ temp,
                                                   unsigned long long temp_cap,
                                                   HeavyEntry *__restrict__ heavy,
                                                   Counters *__restrict__ ctr) {
    __shared__ __align__(16) float qx[kQTile * DP];
    __shared__ unsigned int cnt[kQTile];
    __shared__ unsigned int lst[kQTile * kListCap];
    __shared__ unsigned long long qbase[kQTile];
    __shared__ unsigned int run_start[kMaxRuns];
    __shared__ unsigned int run_pre[kMaxRuns + 1];
    __shared__ int nruns_s;

    const Plan P = *plan;
    if (P.abort) return;
    const int lane = lane_id();
    unsigned long long tested = 0;

    for (unsigned int cell = blockIdx.x; cell < static_cast<unsigned int>(P.n_cells); cell += gridDim.x) {
        const unsigned int qs = cell_start[cell], qe = cell_start[cell + 1];
        if (qs == qe) continue;
        build_runs(cell, P, cell_start, run_start, run_pre, &nruns_s);
        const int nruns = nruns_s;
        const unsigned int M = run_pre[nruns];

        for (unsigned int q0 = qs; q0 < qe; q0 += kQTile) {
            const int Qn = static_cast<int>(min(static_cast<unsigned int>(kQTile), qe - q0));
            for (int e = threadIdx.x; e < Qn * DP; e += kBlock) qx[e] = sorted[static_cast<size_t>(q0) * DP + e];
            for (int q = threadIdx.x; q < kQTile; q += kBlock) cnt[q] = 0u;
            __syncthreads();
            tested += static_cast<unsigned long long>(Qn) * M;

            for (unsigned int mb = static_cast<unsigned int>(wave_id()) * 64u; mb < M; mb += kBlock) {
                const unsigned int m = mb + lane;
                const bool valid = m < M;
                unsigned int s = 0;
                float c[DP];
                if (valid) {
                    s = candidate_row(m, run_start, run_pre, nruns);
                    load_row<DP>(sorted, s, c);
                } else {
#pragma unroll
                    for (int k = 0; k < DP; ++k) c[k] = 0.0f;
                }
                const unsigned int jid = valid ? sorted_id[s] : 0u;
                for (int q = 0; q < Qn; ++q) {
                    const float D = sq_dist<DP>(c, &qx[q * DP]);
                    const bool pass = valid && (D < r2) && (s != q0 + q);
                    const unsigned long long mask = __ballot(pass);
                    if (mask) {
                        const int leader = __ffsll(static_cast<long long>(mask)) - 1;
                        unsigned int base = 0;
                        if (lane == leader) base = atomicAdd(&cnt[q], static_cast<unsigned int>(__popcll(mask)));
                        base = __shfl(base, leader);
                        if (pass) {
                            const unsigned int pos = base + prefix_count(mask);
                            if (pos < kListCap) lst[q * kListCap + pos] = jid;
                        }
                    }
                }
            }
            __syncthreads();

            // Lists that fit (at most kListCap and at most K entries) go to the edge
            // store; the others are handed to the long-list kernel.
            if (wave_id() == 0) {
                const int q = lane;
                unsigned int c = 0, take = 0;
                if (q < Qn) {
                    c = cnt[q];
                    take = (c <= static_cast<unsigned int>(kListCap) && c <= static_cast<unsigned int>(K)) ? c : 0u;
                }
                const unsigned int inc = wave_inclusive_scan(take);
                const unsigned int total = __shfl(inc, 63);
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(&ctr->temp_top, static_cast<unsigned long long>(total));
                base = __shfl(base, 0);
                if (q < Qn) {
                    const unsigned int i = sorted_id[q0 + q];
                    const bool fits = c <= static_cast<unsigned int>(kListCap) && c <= static_cast<unsigned int>(K);
                    if (fits) {
                        kept[i] = c;
                        tpos[i] = base + (inc - take);
                        qbase[q] = base + (inc - take);
                    } else {
                        qbase[q] = ~0ull;
                        const unsigned int h = atomicAdd(&ctr->heavy_count, 1u);
                        HeavyEntry he;
                        he.slot = q0 + q;
                        he.count = c;
                        he.cell = cell;
                        he.pad = 0;
                        heavy[h] = he;
                        if (c > static_cast<unsigned int>(K)) atomicAdd(&ctr->capped, 1u);
                    }
                }
            }
            __syncthreads();
            for (int e = threadIdx.x; e < Qn * kListCap; e += kBlock) {
                const int q = e / kListCap, t = e % kListCap;
                const unsigned long long b = qbase[q];
                const unsigned int c = cnt[q];
                if (b == ~0ull || static_cast<unsigned int>(t) >= c) continue;
                const unsigned int j = lst[q * kListCap + t];
                unsigned int rk = 0;
                for (unsigned int u = 0; u < c; ++u) rk += lst[q * kListCap + u] < j;
                const unsigned long long pos = b + rk;
                if (pos < temp_cap) temp[pos] = j;
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0 && tested) atomicAdd(&ctr->tested, tested);
}

// --------------------------------------------------------------- long lists

constexpr int kHeavyBlocks = 256;

template <int DP>
__global__ __launch_bounds__(kBlock) void k_heavy(const float *__restrict__ sorted,
                                                  const unsigned int *__restrict__ sorted_id,
                                                  const unsigned int *__restrict__ cell_start,
                                                  const Plan *__restrict__ plan, float r2, int K,
                                                  unsigned int *__restrict__ kept,
                                                  unsigned long long *__restrict__ tpos,
                                                  unsigned int *__restrict__ temp,
                                                  unsigned long long temp_cap,
                                                  const HeavyEntry *__restrict__ heavy,
                                                  Counters *__restrict__ ctr) {
    __shared__ unsigned int buf[kMaxK];
    __shared__ unsigned int hist[256];
    __shared__ __align__(16) float qv[DP];
    __shared__ unsigned int run_start[kMaxRuns];
    __shared__ unsigned int run_pre[kMaxRuns + 1];
    __shared__ int nruns_s;
    __shared__ unsigned int h_s, fill_s;
    __shared__ unsigned long long prefix_s, base_s;
    __shared__ unsigned int remaining_s;

    const Plan P = *plan;
    if (P.abort) return;
    const unsigned int n_heavy = ctr->heavy_count;

    for (;;) {
        if (threadIdx.x == 0) h_s = atomicAdd(&ctr->heavy_next, 1u);
        __syncthreads();
        const unsigned int h = h_s;
        if (h >= n_heavy) break;
        const HeavyEntry he = heavy[h];
        for (int k = threadIdx.x; k < DP; k += kBlock) qv[k] = sorted[static_cast<size_t>(he.slot) * DP + k];
        build_runs(he.cell, P, cell_start, run_start, run_pre, &nruns_s);
        const int nruns = nruns_s;
        const unsigned int M = run_pre[nruns];
        float q[DP];
#pragma unroll
        for (int k = 0; k < DP; ++k) q[k] = qv[k];

        // (D bits << 32 | j) orders hits by (D, j): D is never negative.
        auto hit_key = [&](unsigned int m, bool &ok) -> unsigned long long {
            const unsigned int s = candidate_row(m, run_start, run_pre, nruns);
            float c[DP];
            load_row<DP>(sorted, s, c);
            const float D = sq_dist<DP>(c, q);
            ok = (D < r2) && (s != he.slot);
            return (static_cast<unsigned long long>(__float_as_uint(D)) << 32) | sorted_id[s];
        };

        unsigned int n_out;
        unsigned long long limit = ~0ull;  // keep hits with key <= limit
        if (he.count > static_cast<unsigned int>(K)) {
            if (threadIdx.x == 0) {
                prefix_s = 0ull;
                remaining_s = static_cast<unsigned int>(K);
            }
            for (int pass = 0; pass < 8; ++pass) {
                const int shift = 56 - 8 * pass;
                for (int b = threadIdx.x; b < 256; b += kBlock) hist[b] = 0u;
                __syncthreads();
                const unsigned long long prefix = prefix_s;
                for (unsigned int m = threadIdx.x; m < M; m += kBlock) {
                    bool ok;
                    const unsigned long long key = hit_key(m, ok);
                    const bool match = pass == 0 || (key >> (shift + 8)) == (prefix >> (shift + 8));
                    if (ok && match) atomicAdd(&hist[(key >> shift) & 255ull], 1u);
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    unsigned int rem = remaining_s, b = 0;
                    while (b < 255 && hist[b] < rem) {
                        rem -= hist[b];
                        ++b;
                    }
                    remaining_s = rem;
                    prefix_s = prefix | (static_cast<unsigned long long>(b) << shift);
                }
                __syncthreads();
            }
            limit = prefix_s;
            n_out = static_cast<unsigned int>(K);
        } else {
            n_out = he.count;
        }
        if (threadIdx.x == 0) fill_s = 0u;
        __syncthreads();
        for (unsigned int m = threadIdx.x; m < M; m += kBlock) {
            bool ok;
            const unsigned long long key = hit_key(m, ok);
            if (ok && key <= limit) {
                const unsigned int pos = atomicAdd(&fill_s, 1u);
                if (pos < static_cast<unsigned int>(kMaxK)) buf[pos] = static_cast<unsigned int>(key & 0xffffffffull);
            }
        }
        __syncthreads();
        // Bitonic sort of buf[0, n_out) by neighbour id.
        unsigned int size = 1;
        while (size < n_out) size <<= 1;
        for (unsigned int e = n_out + threadIdx.x; e < size; e += kBlock) buf[e] = 0xffffffffu;
        __syncthreads();
        for (unsigned int k = 2; k <= size; k <<= 1) {
            for (unsigned int j = k >> 1; j > 0; j >>= 1) {
                for (unsigned int e = threadIdx.x; e < size; e += kBlock) {
                    const unsigned int o = e ^ j;
                    if (o > e) {
                        const unsigned int a = buf[e], b = buf[o];
                        const bool up = (e & k) == 0;
                        if ((a > b) == up) {
                            buf[e] = b;
                            buf[o] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) {
            base_s = atomicAdd(&ctr->temp_top, static_cast<unsigned long long>(n_out));
            const unsigned int i = sorted_id[he.slot];
            kept[i] = n_out;
            tpos[i] = base_s;
        }
        __syncthreads();
        const unsigned long long base = base_s;
        for (unsigned int t = threadIdx.x; t < n_out; t += kBlock)
            if (base + t < temp_cap) temp[base + t] = buf[t];
        __syncthreads();
    }
}

// ------------------------------------------------------------------- place

__global__ __launch_bounds__(kBlock) void k_place(int n, const unsigned int *__restrict__ kept,
                                                  const unsigned long long *__restrict__ tpos,
                                                  const long long *__restrict__ off,
                                                  const unsigned int *__restrict__ temp,
                                                  unsigned long long temp_cap,
                                                  long long *__restrict__ src, long long *__restrict__ dst,
                                                  unsigned long long cap, const Plan *__restrict__ plan,
                                                  const Counters *__restrict__ ctr,
                                                  Report *__restrict__ report) {
    const Plan P = *plan;
    const long long E = P.abort ? 0 : off[n];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Report rep;
        rep.n_edges = E;
        rep.tested = ctr->tested;
        rep.abort = P.abort;
        rep.capped = ctr->capped;
        rep.heavy = ctr->heavy_count;
        rep.n_cells = P.n_cells;
        for (int p = 0; p < 3; ++p) {
            rep.G[p] = P.G[p];
            rep.c[p] = P.c[p];
        }
        *report = rep;
    }
    if (P.abort || static_cast<unsigned long long>(E) > cap || static_cast<unsigned long long>(E) > temp_cap)
        return;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const unsigned int c = kept[i];
        const long long o = off[i];
        const unsigned long long p = tpos[i];
        for (unsigned int t = 0; t < c; ++t) {
            src[o + t] = i;
            dst[o + t] = static_cast<long long>(temp[p + t]);
        }
    }
}

template <int DP>
void launch_search(const LaunchArgs &a, const Workspace &ws, int grid) {
    hipLaunchKernelGGL(k_search<DP>, dim3(grid), dim3(kBlock), 0, a.stream, ws.sorted, ws.sorted_id,
                       ws.cell_start, ws.plan, a.r2, a.K, ws.kept, ws.tpos, ws.temp, a.edge_capacity,
                       ws.heavy, ws.ctr);
    if (a.events) hipEventRecord(a.events[5], a.stream);
    hipLaunchKernelGGL(k_heavy<DP>, dim3(kHeavyBlocks), dim3(kBlock), 0, a.stream, ws.sorted,
                       ws.sorted_id, ws.cell_start, ws.plan, a.r2, a.K, ws.kept, ws.tpos, ws.temp,
                       a.edge_capacity, ws.heavy, ws.ctr);
}

int blocks_for(long long work, int cap) {
    long long b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<int>(b);
}

}  // namespace

hipError_t enqueue_build(const LaunchArgs &a, const Workspace &ws) {
    const int cells_max = static_cast<int>(a.cells_max);
    auto mark = [&](int stage) {
        if (a.events) hipEventRecord(a.events[stage], a.stream);
    };
    mark(0);
    hipLaunchKernelGGL(k_bounds, dim3(kBoundsBlocks), dim3(kBlock), 0, a.stream, a.points, a.n, a.d,
                       a.dims[0], a.dims[1], a.dims[2], ws.part, ws.cell_count, cells_max, ws.ctr);
    mark(1);
    const int gk = blocks_for(a.n, 4096);
    hipLaunchKernelGGL(k_keys, dim3(gk), dim3(kBlock), 0, a.stream, a.points, a.n, a.d, a.dims[0],
                       a.dims[1], a.dims[2], a.r, a.cell_div, cells_max, ws.part, kBoundsBlocks, ws.plan,
                       ws.key, ws.rank, ws.cell_count);
    mark(2);
    const int cell_tiles = static_cast<int>((a.cells_max + 1 + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_tile_sums, dim3(cell_tiles), dim3(kBlock), 0, a.stream, ws.cell_count, 0,
                       &ws.plan->n_cells, ws.scan_sums);
    hipLaunchKernelGGL(k_scan_tiles<unsigned int>, dim3(cell_tiles), dim3(kBlock), 0, a.stream,
                       ws.cell_count, 0, &ws.plan->n_cells, ws.scan_sums, ws.cell_start);
    mark(3);
    hipLaunchKernelGGL(k_scatter, dim3(gk), dim3(kBlock), 0, a.stream, a.points, a.n, a.d, a.dpad, ws.key,
                       ws.rank, ws.cell_start, ws.plan, ws.sorted, ws.sorted_id);
    mark(4);
    const int gs = static_cast<int>(a.cells_max < 2048 ? a.cells_max : 2048);
    switch (a.dpad) {
        case 4: launch_search<4>(a, ws, gs); break;
        case 8: launch_search<8>(a, ws, gs); break;
        case 12: launch_search<12>(a, ws, gs); break;
        case 16: launch_search<16>(a, ws, gs); break;
        case 24: launch_search<24>(a, ws, gs); break;
        case 32: launch_search<32>(a, ws, gs); break;
        case 48: launch_search<48>(a, ws, gs); break;
        default: launch_search<64>(a, ws, gs); break;
    }
    mark(6);
    const int kept_tiles = static_cast<int>((static_cast<long long>(a.n) + 1 + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_tile_sums, dim3(kept_tiles), dim3(kBlock), 0, a.stream, ws.kept, a.n, nullptr,
                       ws.scan_sums);
    hipLaunchKernelGGL(k_scan_tiles<long long>, dim3(kept_tiles), dim3(kBlock), 0, a.stream, ws.kept, a.n,
                       nullptr, ws.scan_sums, ws.off);
    mark(7);
    hipLaunchKernelGGL(k_place, dim3(blocks_for(a.n, 8192)), dim3(kBlock), 0, a.stream, a.n, ws.kept,
                       ws.tpos, ws.off, ws.temp, a.edge_capacity, a.src, a.dst, a.edge_capacity, ws.plan,
                       ws.ctr, ws.report);
    mark(8);
    return hipGetLastError();
}

}  // namespace frnn
