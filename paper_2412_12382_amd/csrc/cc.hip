// Connected components of (V, kept edges), the second step of Algorithm 1.
//
// Lock-free union-find over the rank-numbered vertices: every kept edge
// unites its endpoints by hooking the root with the larger ORIGINAL id under
// the root with the smaller one (compare-and-swap on the root's parent),
// and finds use path halving, i.e. pointer jumping to the grandparent.  The
// original id strictly decreases along every parent chain, so the root of a
// component is its smallest original id: the canonical label.  Parent reads
// and halving writes use device-scope atomics so no wave spins on a stale
// per-CU cache line.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t N, int64_t cap) {
    int64_t b = (N + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__device__ __forceinline__ int32_t ld_parent(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_parent(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t find_root(int32_t* parent, int32_t x) {
    for (;;) {
        const int32_t p = ld_parent(&parent[x]);
        if (p == x) return x;
        const int32_t gp = ld_parent(&parent[p]);
        if (gp != p) st_parent(&parent[x], gp);
        x = gp;
    }
}

__device__ __forceinline__ void unite(int32_t* parent, const int32_t* __restrict__ perm, int32_t a,
                                      int32_t b) {
    for (;;) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (perm[a] < perm[b]) {
            const int32_t x = a;
            a = b;
            b = x;
        }
        int32_t expected = a;
        if (__hip_atomic_compare_exchange_strong(&parent[a], &expected, b, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
    }
}

__global__ __launch_bounds__(kThreads) void k_cc_init(int32_t* __restrict__ parent, int64_t n) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        parent[v] = (int32_t)v;
}

__global__ __launch_bounds__(kThreads) void k_cc_union(const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ adj,
                                                       const uint32_t* __restrict__ keep, int64_t m,
                                                       const int32_t* __restrict__ perm,
                                                       int32_t* parent) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (keep && !((keep[e >> 5] >> (e & 31)) & 1u)) continue;
        unite(parent, perm, src[e], adj[e]);
    }
}

__global__ __launch_bounds__(kThreads) void k_cc_label(int32_t* parent, const int32_t* __restrict__ perm,
                                                       int64_t n, int32_t* __restrict__ labels,
                                                       unsigned long long* __restrict__ ncc) {
    __shared__ unsigned long long wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long roots = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nround = (n + stride - 1) / stride;
    for (int64_t rd = 0; rd < nround; ++rd) {
        const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + rd * stride;
        bool is_root = false;
        if (v < n) {
            const int32_t r = find_root(parent, (int32_t)v);
            labels[perm[v]] = perm[r];
            is_root = (r == (int32_t)v);
        }
        const uint64_t bal = __ballot(is_root);
        if (lane == 0) roots += (unsigned long long)__popcll(bal);
    }
    if (!ncc) return;
    if (lane == 0) wsum[w] = roots;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kThreads / 64; ++i) s += wsum[i];
        if (s) atomicAdd(ncc, s);
    }
}

}  // namespace

void launch_components(const mcd_graph* g, const uint32_t* keep_bits, int32_t* labels,
                       int64_t* n_components, int32_t* parent, hipStream_t s) {
    if (n_components) fill_i64(n_components, 1, 0, s);
    if (g->n <= 0) return;
    hipLaunchKernelGGL(k_cc_init, dim3(grid_for(g->n, 1 << 16)), dim3(kThreads), 0, s, parent, g->n);
    if (g->m > 0)
        hipLaunchKernelGGL(k_cc_union, dim3(grid_for(g->m, 1 << 16)), dim3(kThreads), 0, s, g->src, g->adj,
                           keep_bits, g->m, g->perm, parent);
    hipLaunchKernelGGL(k_cc_label, dim3(grid_for(g->n, 8192)), dim3(kThreads), 0, s, parent, g->perm, g->n,
                       labels, (unsigned long long*)n_components);
}

}  // namespace mcd
