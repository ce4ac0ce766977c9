// Connected components of (V, kept edges), the second step of Algorithm 1.
//
// Lock-free union-find over the rank-numbered vertices: every kept edge
// unites its endpoints by hooking the root of lower rank under the root of
// higher rank (compare-and-swap on the root's parent), and finds use path
// halving, i.e. pointer jumping to the grandparent.  Parents only ever point
// to higher ranks, so chains are acyclic; roots end at high-degree vertices,
// which keeps trees shallow on skewed graphs.  The canonical label of a
// component is its smallest original id.  The label array itself holds the
// running minimum: every label starts as its own original id, a root's label
// cell takes the atomic minimum of its members' ids, and each member then
// copies its root's cell.  Singletons, most vertices of a pruned graph, are
// touched only by the first write.  Parent reads and halving writes use
// device-scope atomics so no wave spins on a stale per-CU cache line.
#include "common.hpp"
#include "unionfind.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t N, int64_t cap) {
    int64_t b = (N + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// Singletons: parent[v] = v, and every label (indexed by original id) its
// own original id.
__global__ __launch_bounds__(kThreads) void k_cc_init(int32_t* __restrict__ parent, int32_t* __restrict__ labels,
                                                      int64_t n) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        parent[v] = (int32_t)v;
        labels[v] = (int32_t)v;
    }
}

__global__ __launch_bounds__(kThreads) void k_cc_union(const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ adj,
                                                       const uint32_t* __restrict__ keep, int64_t m,
                                                       int32_t* parent) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (keep && !((keep[e >> 5] >> (e & 31)) & 1u)) continue;
        uf_unite(parent, src[e], adj[e]);
    }
}

// One wave per segment of a kept-edge list, walked from its end: a segment
// lists its edge groups in ascending rank of the lower endpoint, so all waves
// together unite the edges among high-degree vertices first and the rest of
// the graph then hooks straight under the roots that core has formed.
__global__ __launch_bounds__(kThreads) void k_cc_union_kept(const int2* __restrict__ kept,
                                                            const int32_t* __restrict__ counts, int64_t seg_len,
                                                            int32_t* parent) {
    const int lane = threadIdx.x & 63;
    const int64_t seg = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int32_t cnt = counts[seg];
    const int2* p = kept + seg * seg_len;
    for (int32_t i = cnt - 1 - lane; i >= 0; i -= 64) {
        const int2 e = p[i];
        uf_unite(parent, e.x, e.y);
    }
}

// The label cell of every root, labels[perm[root]], takes the minimum of its
// members' original ids.
__global__ __launch_bounds__(kThreads) void k_cc_min(int32_t* parent, const int32_t* __restrict__ perm, int64_t n,
                                                     int32_t* __restrict__ labels) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nround = (n + stride - 1) / stride;
    for (int64_t rd = 0; rd < nround; ++rd) {
        const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + rd * stride;
        int32_t r = -1, id = 0x7fffffff;
        if (v < n) {
            const int32_t p = uf_load(&parent[v]);
            if (p != (int32_t)v) {
                r = uf_find(parent, p);
                id = perm[v];
            }
        }
        const uint64_t act = __ballot(r >= 0);
        if (act == 0) continue;  // wave-uniform: only roots here
        // lanes sharing the first active lane's root reduce first
        const int lead = __ffsll((unsigned long long)act) - 1;
        const int32_t r0 = __shfl(r, lead);
        int32_t x = r == r0 ? id : 0x7fffffff;
        for (int o = 32; o > 0; o >>= 1) {
            const int32_t y = __shfl_xor(x, o);
            x = y < x ? y : x;
        }
        if ((threadIdx.x & 63) == lead) atomicMin(&labels[perm[r0]], x);
        if (r != r0 && r >= 0) atomicMin(&labels[perm[r]], id);
    }
}

// Every non-root copies its root's label cell (final after k_cc_min: root
// cells are only read here, non-root cells only written); roots are counted.
__global__ __launch_bounds__(kThreads) void k_cc_label(int32_t* parent, const int32_t* __restrict__ perm, int64_t n,
                                                       int32_t* __restrict__ labels,
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
            const int32_t p = uf_load(&parent[v]);
            is_root = p == (int32_t)v;
            if (!is_root) {
                const int32_t r = uf_find(parent, p);
                labels[perm[v]] = labels[perm[r]];
            }
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

void init_components(const mcd_graph* g, int32_t* parent, int32_t* labels, int64_t* n_components,
                     hipStream_t s) {
    if (n_components) fill_i64(n_components, 1, 0, s);
    if (g->n <= 0) return;
    hipLaunchKernelGGL(k_cc_init, dim3(grid_for(g->n, 1 << 16)), dim3(kThreads), 0, s, parent, labels, g->n);
}

void finish_components(const mcd_graph* g, int32_t* labels, int64_t* n_components, int32_t* parent,
                       hipStream_t s) {
    if (g->n <= 0) return;
    // (the label pass ends with one atomic per block on the component count,
    // so its grid stays small)
    hipLaunchKernelGGL(k_cc_min, dim3(grid_for(g->n, 8192)), dim3(kThreads), 0, s, parent, g->perm, g->n, labels);
    hipLaunchKernelGGL(k_cc_label, dim3(grid_for(g->n, 8192)), dim3(kThreads), 0, s, parent, g->perm, g->n, labels,
                       (unsigned long long*)n_components);
}

// Every edge of the graph kept (a threshold no similarity falls below),
// after the sampling idea of Sutton et al. (Afforest): each vertex first
// unites its first two out-edges, which links most of the large component
// of a skewed graph; the root most of 1024 evenly spaced vertices reach is
// taken as that component's; then every vertex outside it unites all its
// edges, out-edges from the CSR and in-edges from the in-edge lists.  An edge
// with both endpoints inside that component when they are looked at joins
// nothing new (components only grow), and every other edge is in the lists
// of an endpoint outside it, so the partition is the edge-by-edge union's.
constexpr int kSampleVerts = 1024;

__global__ __launch_bounds__(kThreads) void k_cc_sample(const int64_t* __restrict__ off,
                                                        const int32_t* __restrict__ adj, int64_t n,
                                                        int32_t* parent) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e0 = off[x], e1 = min(off[x + 1], e0 + 2);
        for (int64_t e = e0; e < e1; ++e) uf_unite(parent, (int32_t)x, adj[e]);
    }
}

// One workgroup of kSampleVerts threads: the most frequent root of the
// samples (ties: the smaller root) into *giant.
__global__ __launch_bounds__(kSampleVerts) void k_cc_giant(int32_t* parent, int64_t n, int32_t* __restrict__ giant) {
    __shared__ int32_t key[2 * kSampleVerts];
    __shared__ uint32_t cnt[2 * kSampleVerts];
    __shared__ unsigned long long wbest[kSampleVerts / 64];
    const int tid = threadIdx.x;
    for (int i = tid; i < 2 * kSampleVerts; i += kSampleVerts) {
        key[i] = -1;
        cnt[i] = 0u;
    }
    __syncthreads();
    const int32_t r = uf_find(parent, (int32_t)((int64_t)tid * n / kSampleVerts));
    uint32_t h = ((uint32_t)r * 2654435761u) >> 21;  // 11 bits: 2 kSampleVerts slots
    for (;;) {
        const int32_t k = atomicCAS(&key[h], -1, r);
        if (k == -1 || k == r) break;
        h = (h + 1) & (2 * kSampleVerts - 1);
    }
    atomicAdd(&cnt[h], 1u);
    __syncthreads();
    unsigned long long best = 0;
    for (int i = tid; i < 2 * kSampleVerts; i += kSampleVerts)
        if (key[i] >= 0) {
            const unsigned long long c = ((unsigned long long)cnt[i] << 32) | (uint32_t)~(uint32_t)key[i];
            best = c > best ? c : best;
        }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(best, o);
        best = y > best ? y : best;
    }
    if ((tid & 63) == 0) wbest[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kSampleVerts / 64; ++w) best = wbest[w] > best ? wbest[w] : best;
        *giant = (int32_t)~(uint32_t)best;
    }
}

__global__ __launch_bounds__(kThreads) void k_cc_rest(const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ adj,
                                                      const int64_t* __restrict__ in_off,
                                                      const int2* __restrict__ in_ea,
                                                      const int32_t* __restrict__ src, int64_t n, int32_t* parent,
                                                      const int32_t* __restrict__ giant) {
    const int32_t c = *giant;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        if (uf_find(parent, (int32_t)x) == c) continue;
        for (int64_t e = off[x]; e < off[x + 1]; ++e) uf_unite(parent, (int32_t)x, adj[e]);
        for (int64_t k = in_off[x]; k < in_off[x + 1]; ++k) uf_unite(parent, (int32_t)x, src[in_ea[k].x]);
    }
}

}  // namespace

// parent (n int32) and one more int32 behind it (the vertex-by-vertex union
// of every edge keeps its sampled root there)
size_t cc_scratch_bytes(const mcd_graph* g) { return mcd_align(sizeof(int32_t) * ((size_t)g->n + 1)); }

void launch_components_all_edges(const mcd_graph* g, int32_t* parent, int32_t* giant, hipStream_t s) {
    if (g->n <= 0 || g->m <= 0) return;
    hipLaunchKernelGGL(k_cc_sample, dim3(grid_for(g->n, 1 << 16)), dim3(kThreads), 0, s, g->off, g->adj, g->n, parent);
    hipLaunchKernelGGL(k_cc_giant, dim3(1), dim3(kSampleVerts), 0, s, parent, g->n, giant);
    hipLaunchKernelGGL(k_cc_rest, dim3(grid_for(g->n, 1 << 16)), dim3(kThreads), 0, s, g->off, g->adj, g->in_off,
                       g->in_ea, g->src, g->n, parent, giant);
}

void launch_components(const mcd_graph* g, const uint32_t* keep_bits, int32_t* labels, int64_t* n_components,
                       void* ws, hipStream_t s) {
    int32_t* parent = (int32_t*)ws;
    init_components(g, parent, labels, n_components, s);
    if (g->n > 0 && g->m > 0)
        hipLaunchKernelGGL(k_cc_union, dim3(grid_for(g->m, 1 << 16)), dim3(kThreads), 0, s, g->src, g->adj,
                           keep_bits, g->m, parent);
    finish_components(g, labels, n_components, parent, s);
}

void launch_components_kept(const mcd_graph* g, const int32_t* kept_pairs, const int32_t* kept_counts,
                            int32_t* labels, int64_t* n_components, void* ws, hipStream_t s) {
    int32_t* parent = (int32_t*)ws;
    init_components(g, parent, labels, n_components, s);
    if (g->n > 0 && g->m > 0)
        hipLaunchKernelGGL(k_cc_union_kept, dim3(MCD_KEPT_SEGMENTS / (kThreads / 64)), dim3(kThreads), 0, s,
                           (const int2*)kept_pairs, kept_counts, kept_segment_len(g->m), parent);
    finish_components(g, labels, n_components, parent, s);
}

int32_t* launch_components_init(const mcd_graph* g, int32_t* labels, int64_t* n_components, void* ws,
                                hipStream_t s) {
    int32_t* parent = (int32_t*)ws;
    init_components(g, parent, labels, n_components, s);
    return parent;
}

void launch_components_finish(const mcd_graph* g, int32_t* labels, int64_t* n_components, void* ws,
                              hipStream_t s) {
    finish_components(g, labels, n_components, (int32_t*)ws, s);
}

}  // namespace mcd
