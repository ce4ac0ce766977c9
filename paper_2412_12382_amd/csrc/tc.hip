// Per-edge triangle counts t(u,v) = |N(u) n N(v)| on the degree-ordered
// orientation.
//
// Vertices are numbered by rank, every edge points from the lower to the
// higher id, and row u of the CSR lists N+(u) (out-neighbours) in increasing
// id.  A triangle {u < v < w} is found exactly once, at edge u->v, as the
// common element w of N+(u) and N+(v).  Only the part of N+(u) after v can
// meet N+(v) (whose ids all exceed v).  Each find credits the three edges
// u->v, u->w and v->w; integer atomics are commutative, so the counts do not
// depend on scheduling.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;

// First index in [lo, hi) whose value is >= x.
__device__ __forceinline__ int64_t lower_bound(const int32_t* __restrict__ a, int64_t lo, int64_t hi,
                                               int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void k_tc_edge(const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ adj, int64_t m,
                                                      int32_t* __restrict__ t) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[e], v = adj[e];
        int64_t a0 = e + 1, a1 = off[u + 1];
        int64_t b0 = off[v], b1 = off[v + 1];
        if (a0 >= a1 || b0 >= b1) continue;
        int32_t c = 0;
        if (a1 - a0 <= b1 - b0) {
            // walk N+(u) after v, search each w in N+(v); searches move right
            for (int64_t i = a0; i < a1 && b0 < b1; ++i) {
                const int32_t w = adj[i];
                b0 = lower_bound(adj, b0, b1, w);
                if (b0 < b1 && adj[b0] == w) {
                    atomicAdd(&t[i], 1);
                    atomicAdd(&t[b0], 1);
                    ++c;
                    ++b0;
                }
            }
        } else {
            for (int64_t j = b0; j < b1 && a0 < a1; ++j) {
                const int32_t w = adj[j];
                a0 = lower_bound(adj, a0, a1, w);
                if (a0 < a1 && adj[a0] == w) {
                    atomicAdd(&t[a0], 1);
                    atomicAdd(&t[j], 1);
                    ++c;
                    ++a0;
                }
            }
        }
        if (c) atomicAdd(&t[e], c);
    }
}

}  // namespace

void launch_triangles(const mcd_graph* g, int32_t* t, hipStream_t s) {
    fill_i32(t, g->m, 0, s);
    if (g->m <= 0) return;
    int64_t blocks = (g->m + kThreads - 1) / kThreads;
    if (blocks > 1 << 20) blocks = 1 << 20;
    hipLaunchKernelGGL(k_tc_edge, dim3((unsigned)blocks), dim3(kThreads), 0, s, g->off, g->src, g->adj,
                       g->m, t);
}

}  // namespace mcd
