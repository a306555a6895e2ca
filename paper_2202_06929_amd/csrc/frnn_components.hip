// Track labeling on the FRNN edge list: weakly connected components of the kept
// edges, every vertex labeled with the smallest vertex id of its component
// (paper, Section 2: the edges whose score passes a threshold are kept and each
// weakly connected component is a track candidate; Section 3.2: the labeling
// runs on the edge list that already exists).
//
// Lock-free union-find on a parent array (one 32-bit entry per vertex):
//   k_cc_init     parent[v] = v
//   k_cc_minhook  each source hooked under its smallest neighbour (see there), so
//                 that clusters whose vertices all neighbour their smallest vertex
//                 are stars before the next pass
//   k_cc_hook     one lane per kept edge: find both roots (plain reads: the only
//                 writes of this kernel are the hooks, device-scope atomics that are
//                 performed beyond the per-XCD caches and cost memory traffic), hook
//                 the larger root under the smaller one with a compare-and-swap,
//                 retry from the new roots if another thread hooked it first
//   k_cc_label    label[v] = root of v (path halving); counts the roots; the last
//                 workgroup writes the component count and the status
// Parent pointers only ever point to smaller ids (hooks go from the larger root
// to the smaller, halving jumps to an ancestor), so there are no cycles and every
// find ends.  When all edges are done each component is one tree, and its root is
// its smallest vertex: that vertex's parent cannot be smaller, so it is a root.
// Finds read the parent array with ordinary (cached) loads: a stale entry is still
// an ancestor, because entries only ever move up the tree, so a find returns a
// vertex of the right tree, perhaps not its current root.  Equal results therefore
// prove two vertices share a tree.  Hooks are device-scope compare-and-swaps on
// the presumed root; a failed one returns that vertex's current parent, a
// strictly smaller id, and the hook resumes from there, so every retry makes
// progress on fresh data.  Path-halving stores (labeling pass) are device-scope
// atomic stores.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "frnn.h"

namespace {

constexpr int kCcBlock = 256;
// Rounds of the hook loop per edge before the call reports an internal error.  A
// round repeats only after another thread merged one of the two trees, so a
// correct run needs at most one round per merge; the bound is a safety net.
constexpr unsigned int kMaxHookRounds = 1u << 20;

struct CcState {
    unsigned int status;             // bit 0: endpoint out of range; bit 1: hook bound reached
    unsigned int pad;
    // Labeling workgroups done (bits 44..63) and roots counted so far (bits 0..43),
    // one word so that a single atomic add both counts and tells the last workgroup.
    unsigned long long done_roots;
};

constexpr int kRootBits = 44;
constexpr unsigned long long kRootMask = (1ull << kRootBits) - 1;

__device__ __forceinline__ long long status_code(unsigned int s) {
    return (s & 1u) ? FRNN_ERR_ARG : ((s & 2u) ? FRNN_ERR_HIP : FRNN_OK);
}

__device__ __forceinline__ unsigned int ld(const unsigned int *p) { return *p; }

__device__ __forceinline__ void st(unsigned int *p, unsigned int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, halving the path on the way (x is pointed at its grandparent).
__device__ unsigned int cc_find(unsigned int *parent, unsigned int x) {
    for (;;) {
        const unsigned int p = ld(parent + x);
        if (p == x) return x;
        const unsigned int gp = ld(parent + p);
        if (gp == p) return p;
        st(parent + x, gp);
        x = gp;
    }
}

// Root of x by plain reads (no path halving).
__device__ __forceinline__ unsigned int cc_root(unsigned int *parent, unsigned int x) {
    for (;;) {
        const unsigned int p = ld(parent + x);
        if (p == x) return x;
        x = p;
    }
}

// Roots of x and y by plain reads, the two walks interleaved so that their loads
// overlap.
__device__ void cc_find2(unsigned int *parent, unsigned int &x, unsigned int &y) {
    bool dx = false, dy = false;
    while (!(dx && dy)) {
        const unsigned int px = dx ? x : ld(parent + x);
        const unsigned int py = dy ? y : ld(parent + y);
        dx = dx || px == x;
        dy = dy || py == y;
        const unsigned int gx = dx ? x : ld(parent + px);
        const unsigned int gy = dy ? y : ld(parent + py);
        if (!dx) {
            if (gx == px) {
                x = px;
                dx = true;
            } else {
                x = gx;
            }
        }
        if (!dy) {
            if (gy == py) {
                y = py;
                dy = true;
            } else {
                y = gy;
            }
        }
    }
}

// Joins the trees of u and v: hooks the larger root under the smaller with a
// compare-and-swap.  u and v need not be roots: a failed swap returns the larger
// vertex's current parent, a strictly smaller id, and the join resumes from its
// root, so the larger of the pair decreases every round.
__device__ void cc_union(unsigned int *parent, unsigned int u, unsigned int v, CcState *state) {
    for (unsigned int round = 0; u != v; ++round) {
        if (round >= kMaxHookRounds) {
            atomicOr(&state->status, 2u);
            return;
        }
        const unsigned int hi = u > v ? u : v, lo = u > v ? v : u;
        unsigned int expected = hi;
        if (__hip_atomic_compare_exchange_strong(parent + hi, &expected, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        u = cc_root(parent, expected);
        v = lo;
    }
}

__global__ __launch_bounds__(kCcBlock) void k_cc_init(unsigned int *parent, long long n, CcState *state) {
    const long long stride = static_cast<long long>(gridDim.x) * kCcBlock;
    for (long long v = static_cast<long long>(blockIdx.x) * kCcBlock + threadIdx.x; v < n; v += stride)
        parent[v] = static_cast<unsigned int>(v);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        CcState z = {};
        *state = z;
    }
}

// Hooks each edge's larger endpoint under its smallest neighbour first, so that a
// cluster whose vertices all neighbour its smallest vertex (the FRNN graph of a
// track: its points lie within r of one another) is a star before the union-find
// pass, which then finds equal roots for its edges and swaps nothing.  Lanes of a
// wave that share a source take the minimum of their targets below it by a
// segmented reduction (edges come grouped by source), and one lane per source does
// a device-scope atomicMin on the source's parent.  The parent array then still
// points only to smaller ids and every entry to a neighbour or itself: each
// vertex is hooked at most under one neighbour, a valid union of two trees, as
// every vertex is still a root before this pass.  Whatever this pass leaves
// unjoined, the union-find pass joins.
// Edges (or vertices) per lane in the hook and label passes: their loads are all
// issued before any is used, so a wave keeps several round trips in flight.
constexpr int kPerLane = 4;

__global__ __launch_bounds__(kCcBlock) void k_cc_minhook(const long long *__restrict__ src,
                                                         const long long *__restrict__ dst, long long n_edges,
                                                         long long n, const float *__restrict__ scores,
                                                         float threshold, unsigned int *parent) {
    const long long stride = static_cast<long long>(gridDim.x) * kCcBlock;
    const int lane = static_cast<int>(threadIdx.x & 63u);
    // Wave-aligned bases, so that every lane of a wave takes the same trip count.
    for (long long e0 = static_cast<long long>(blockIdx.x) * kCcBlock + (threadIdx.x & ~63u); e0 < n_edges;
         e0 += stride) {
        const long long e = e0 + lane;
        unsigned int a = 0xffffffffu, m = 0xffffffffu;
        if (e < n_edges && !(scores && !(scores[e] > threshold))) {
            const long long x = src[e], y = dst[e];
            if (x >= 0 && x < n && y >= 0 && y < n) {  // out-of-range edges are reported by the hook pass
                a = static_cast<unsigned int>(x);
                m = static_cast<unsigned int>(y);
            }
        }
        // Minimum over the lanes at or after this one with the same source.
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned int a2 = static_cast<unsigned int>(__shfl_down(static_cast<int>(a), o));
            const unsigned int m2 = static_cast<unsigned int>(__shfl_down(static_cast<int>(m), o));
            if (lane + o < 64 && a2 == a && m2 < m) m = m2;
        }
        const unsigned int a_prev = static_cast<unsigned int>(__shfl_up(static_cast<int>(a), 1));
        const bool head = lane == 0 || a_prev != a;
        if (head && a != 0xffffffffu && m < a) atomicMin(parent + a, m);
    }
}

__global__ __launch_bounds__(kCcBlock) void k_cc_hook(const long long *__restrict__ src,
                                                      const long long *__restrict__ dst, long long n_edges,
                                                      long long n, const float *__restrict__ scores,
                                                      float threshold, unsigned int *parent, CcState *state) {
    const long long span = static_cast<long long>(kCcBlock) * kPerLane;
    const long long stride = static_cast<long long>(gridDim.x) * span;
    for (long long e0 = static_cast<long long>(blockIdx.x) * span + threadIdx.x; e0 < n_edges; e0 += stride) {
        unsigned int ra[kPerLane], rb[kPerLane];
        bool act[kPerLane];
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            const long long e = e0 + static_cast<long long>(kCcBlock) * j;
            act[j] = e < n_edges && !(scores && !(scores[e] > threshold));
            const long long a = act[j] ? src[e] : 0, b = act[j] ? dst[e] : 0;
            if (act[j] && (a < 0 || a >= n || b < 0 || b >= n)) {
                atomicOr(&state->status, 1u);
                act[j] = false;
            }
            ra[j] = static_cast<unsigned int>(a);
            rb[j] = static_cast<unsigned int>(b);
        }
        // Endpoints with the same parent are in one tree already (the common case
        // after the min-neighbour pass): no walk to the roots.
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            ra[j] = act[j] ? ld(parent + ra[j]) : 0u;
            rb[j] = act[j] ? ld(parent + rb[j]) : 0u;
        }
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            if (!act[j] || ra[j] == rb[j]) continue;
            cc_find2(parent, ra[j], rb[j]);
            if (ra[j] != rb[j]) cc_union(parent, ra[j], rb[j], state);
        }
    }
}

// Labels every vertex with its root and counts the roots; the last workgroup to
// finish writes the caller's result [n_components, status].
__global__ __launch_bounds__(kCcBlock) void k_cc_label(unsigned int *parent, long long n, long long *labels,
                                                       CcState *state, long long *result) {
    __shared__ unsigned long long part[kCcBlock / 64];
    const long long span = static_cast<long long>(kCcBlock) * kPerLane;
    const long long stride = static_cast<long long>(gridDim.x) * span;
    unsigned long long roots = 0;
    for (long long v0 = static_cast<long long>(blockIdx.x) * span + threadIdx.x; v0 < n; v0 += stride) {
        // Parents and grandparents of kPerLane vertices requested together; most
        // trees are one or two levels deep by now.
        unsigned int p[kPerLane], g[kPerLane];
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            const long long v = v0 + static_cast<long long>(kCcBlock) * j;
            p[j] = v < n ? ld(parent + v) : 0u;
        }
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) g[j] = ld(parent + p[j]);
#pragma unroll
        for (int j = 0; j < kPerLane; ++j) {
            const long long v = v0 + static_cast<long long>(kCcBlock) * j;
            if (v >= n) continue;
            const unsigned int r = g[j] == p[j] ? p[j] : cc_find(parent, g[j]);
            labels[v] = static_cast<long long>(r);
            roots += r == static_cast<unsigned int>(v) ? 1ull : 0ull;
        }
    }
    for (int o = 32; o > 0; o >>= 1) roots += __shfl_xor(roots, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = roots;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kCcBlock / 64; ++w) t += part[w];
        const unsigned long long old = atomicAdd(&state->done_roots, (1ull << kRootBits) | t);
        if ((old >> kRootBits) == gridDim.x - 1u) {
            result[0] = static_cast<long long>((old & kRootMask) + t);
            result[1] = status_code(state->status);
        }
    }
}

// The caller's device result [n_components, status] of a graph without vertices.
__global__ void k_cc_result(const CcState *state, long long *result) {
    result[0] = 0;
    result[1] = status_code(state->status);
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int grid_for(long long items) {
    const long long b = (items + kCcBlock - 1) / kCcBlock;
    return static_cast<int>(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

int check(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n_vertices, void *workspace,
          size_t workspace_bytes, int64_t *labels) {
    if (n_edges < 0 || n_vertices < 0) return FRNN_ERR_ARG;
    if (n_vertices >= (int64_t{1} << 31)) return FRNN_ERR_UNSUPPORTED;
    if (n_edges > 0 && (!src || !dst)) return FRNN_ERR_ARG;
    if (n_vertices > 0 && !labels) return FRNN_ERR_ARG;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return FRNN_ERR_ARG;
    if (workspace_bytes < frnn_components_workspace_bytes(n_vertices)) return FRNN_ERR_WORKSPACE;
    return FRNN_OK;
}

int enqueue(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n_vertices, const float *scores,
            float threshold, void *workspace, int64_t *labels, int64_t *result_device, hipStream_t s) {
    CcState *state = static_cast<CcState *>(workspace);
    unsigned int *parent = reinterpret_cast<unsigned int *>(static_cast<char *>(workspace) + 256);
    const long long n = n_vertices;
    hipLaunchKernelGGL(k_cc_init, dim3(grid_for(n)), dim3(kCcBlock), 0, s, parent, n, state);
    if (n_edges > 0)
        hipLaunchKernelGGL(k_cc_minhook, dim3(grid_for(n_edges)), dim3(kCcBlock), 0, s,
                           reinterpret_cast<const long long *>(src), reinterpret_cast<const long long *>(dst),
                           static_cast<long long>(n_edges), n, scores, threshold, parent);
    if (n_edges > 0)
        hipLaunchKernelGGL(k_cc_hook, dim3(grid_for((n_edges + kPerLane - 1) / kPerLane)), dim3(kCcBlock), 0, s,
                           reinterpret_cast<const long long *>(src), reinterpret_cast<const long long *>(dst),
                           static_cast<long long>(n_edges), n, scores, threshold, parent, state);
    if (n > 0)
        hipLaunchKernelGGL(k_cc_label, dim3(grid_for((n + kPerLane - 1) / kPerLane)), dim3(kCcBlock), 0, s, parent, n,
                           reinterpret_cast<long long *>(labels), state, reinterpret_cast<long long *>(result_device));
    else
        hipLaunchKernelGGL(k_cc_result, dim3(1), dim3(1), 0, s, state, reinterpret_cast<long long *>(result_device));
    return hipGetLastError() == hipSuccess ? FRNN_OK : FRNN_ERR_HIP;
}

thread_local long long *t_result = nullptr;  // pinned host copy of [n_components, status]

}  // namespace

extern "C" size_t frnn_components_workspace_bytes(int64_t n_vertices) {
    if (n_vertices < 0 || n_vertices >= (int64_t{1} << 31)) return 0;
    // state, a 16-byte device result, then the parent array
    return 256 + align256(sizeof(unsigned int) * static_cast<size_t>(n_vertices)) + 256;
}

extern "C" int frnn_components_async(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n_vertices,
                                     const float *scores, float threshold, void *workspace, size_t workspace_bytes,
                                     int64_t *labels, int64_t *result_device, void *stream) {
    const int st = check(src, dst, n_edges, n_vertices, workspace, workspace_bytes, labels);
    if (st != FRNN_OK) return st;
    if (!result_device) return FRNN_ERR_ARG;
    return enqueue(src, dst, n_edges, n_vertices, scores, threshold, workspace, labels, result_device,
                   static_cast<hipStream_t>(stream));
}

extern "C" int frnn_components(const int64_t *src, const int64_t *dst, int64_t n_edges, int64_t n_vertices,
                               const float *scores, float threshold, void *workspace, size_t workspace_bytes,
                               int64_t *labels, int64_t *n_components, void *stream) {
    const int st = check(src, dst, n_edges, n_vertices, workspace, workspace_bytes, labels);
    if (st != FRNN_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!t_result) {
        void *p = nullptr;
        if (hipHostMalloc(&p, 2 * sizeof(long long), hipHostMallocDefault) != hipSuccess) return FRNN_ERR_HIP;
        t_result = static_cast<long long *>(p);
    }
    int64_t *result_device = reinterpret_cast<int64_t *>(
        static_cast<char *>(workspace) + 256 + align256(sizeof(unsigned int) * static_cast<size_t>(n_vertices)));
    const int e = enqueue(src, dst, n_edges, n_vertices, scores, threshold, workspace, labels, result_device, s);
    if (e != FRNN_OK) return e;
    if (hipMemcpyAsync(t_result, result_device, 2 * sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FRNN_ERR_HIP;
    if (n_components) *n_components = t_result[0];
    return static_cast<int>(t_result[1]);
}
