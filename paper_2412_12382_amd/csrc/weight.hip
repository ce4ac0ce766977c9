// Edge similarities (Table tab:simfunctions) and the prune step of Algorithm 1.
//
// Tectonic(e) = t / D and TW(e) = 3t - D + 2 with D = deg u + deg v; the TW
// form is t - wedge with |N(u) u N(v)| = deg u + deg v - t (Eq. eq:tw and the
// notation paragraph of Sec. 1).  The keep decision never uses floating point:
// with delta = num/den (den > 0), Tectonic keeps iff t*den >= num*D and TW
// keeps iff TW*den >= num, evaluated in int64.
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

__global__ __launch_bounds__(kThreads) void k_weights(const int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ adj,
                                                      const int32_t* __restrict__ deg,
                                                      const int32_t* __restrict__ t, int64_t m,
                                                      int measure, float* __restrict__ wf,
                                                      int32_t* __restrict__ wi) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t D = deg[src[e]] + deg[adj[e]];
        const int32_t tt = t[e];
        if (measure == MCD_SIM_TECTONIC) {
            if (wf) wf[e] = (float)tt / (float)D;  // IEEE-correct fp32 division
        } else {
            const int32_t tw = 3 * tt - D + 2;
            if (wi) wi[e] = tw;
            if (wf) wf[e] = (float)tw;
        }
    }
}

// One wave handles 64 consecutive edges at a time; its keep decisions form a
// 64-bit ballot = two keep words.  Kept counts are reduced per block.
__global__ __launch_bounds__(kThreads) void k_prune(const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ adj,
                                                    const int32_t* __restrict__ deg,
                                                    const int32_t* __restrict__ t, int64_t m,
                                                    int measure, int64_t num, int64_t den,
                                                    uint32_t* __restrict__ keep,
                                                    unsigned long long* __restrict__ n_kept) {
    __shared__ unsigned long long wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nchunks = (m + 63) >> 6;
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    unsigned long long kept = 0;
    for (int64_t c = (int64_t)blockIdx.x * (kThreads / 64) + w; c < nchunks; c += waves) {
        const int64_t e = (c << 6) + lane;
        bool k = false;
        if (e < m) {
            const int64_t D = (int64_t)deg[src[e]] + deg[adj[e]];
            const int64_t tt = t[e];
            if (measure == MCD_SIM_TECTONIC) k = tt * den >= num * D;
            else k = (3 * tt - D + 2) * den >= num;
        }
        const uint64_t bal = __ballot(k);
        if (lane == 0) {
            keep[c * 2] = (uint32_t)bal;
            kept += (unsigned long long)__popcll(bal);
        } else if (lane == 1 && (c << 6) + 32 < m) {
            keep[c * 2 + 1] = (uint32_t)(bal >> 32);
        }
    }
    if (!n_kept) return;
    if (lane == 0) wsum[w] = kept;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kThreads / 64; ++i) s += wsum[i];
        if (s) atomicAdd(n_kept, s);
    }
}

__device__ __forceinline__ int graph_of(const int64_t* __restrict__ vbase, int G, int64_t x) {
    int lo = 0, hi = G;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (vbase[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Algorithm 1's removal rule with a per-graph threshold read from device
// memory (deltas[2g] / deltas[2g+1]); compared exactly in 128-bit integers.
__global__ __launch_bounds__(kThreads) void k_prune_graphs(const int32_t* __restrict__ src,
                                                           const int32_t* __restrict__ adj,
                                                           const int32_t* __restrict__ deg,
                                                           const int32_t* __restrict__ perm,
                                                           const int32_t* __restrict__ t, int64_t m,
                                                           int measure, int G, const int64_t* __restrict__ vbase,
                                                           const int64_t* __restrict__ deltas,
                                                           uint32_t* __restrict__ keep,
                                                           unsigned long long* __restrict__ n_kept) {
    __shared__ unsigned long long wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nchunks = (m + 63) >> 6;
    const int64_t waves = (int64_t)gridDim.x * (kThreads / 64);
    unsigned long long kept = 0;
    for (int64_t c = (int64_t)blockIdx.x * (kThreads / 64) + w; c < nchunks; c += waves) {
        const int64_t e = (c << 6) + lane;
        bool k = false;
        if (e < m) {
            const int32_t u = src[e];
            const int64_t D = (int64_t)deg[u] + deg[adj[e]];
            const int64_t tt = t[e];
            const int g = G == 1 ? 0 : graph_of(vbase, G, perm[u]);
            const int64_t num = deltas[2 * g], den = deltas[2 * g + 1];
            const int64_t sn = measure == MCD_SIM_TECTONIC ? tt : 3 * tt - D + 2;
            const int64_t sd = measure == MCD_SIM_TECTONIC ? D : 1;
            k = (__int128)sn * den >= (__int128)num * sd;
        }
        const uint64_t bal = __ballot(k);
        if (lane == 0) {
            keep[c * 2] = (uint32_t)bal;
            kept += (unsigned long long)__popcll(bal);
        } else if (lane == 1 && (c << 6) + 32 < m) {
            keep[c * 2 + 1] = (uint32_t)(bal >> 32);
        }
    }
    if (!n_kept) return;
    if (lane == 0) wsum[w] = kept;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kThreads / 64; ++i) s += wsum[i];
        if (s) atomicAdd(n_kept, s);
    }
}

}  // namespace

void launch_prune_graphs(const mcd_graph* g, int measure, const int32_t* t, int G, const int64_t* vbase,
                         const int64_t* deltas, uint32_t* keep_bits, int64_t* n_kept, hipStream_t s) {
    if (n_kept) fill_i64(n_kept, 1, 0, s);
    if (g->m <= 0) return;
    hipLaunchKernelGGL(k_prune_graphs, dim3(grid_for(g->m, 4096)), dim3(kThreads), 0, s, g->src, g->adj, g->deg,
                       g->perm, t, g->m, measure, G, vbase, deltas, keep_bits, (unsigned long long*)n_kept);
}

void launch_weights(const mcd_graph* g, int measure, const int32_t* t, float* wf, int32_t* wi,
                    hipStream_t s) {
    if (g->m <= 0) return;
    hipLaunchKernelGGL(k_weights, dim3(grid_for(g->m, 1 << 16)), dim3(kThreads), 0, s, g->src, g->adj,
                       g->deg, t, g->m, measure, wf, wi);
}

void launch_prune(const mcd_graph* g, int measure, const int32_t* t, int64_t num, int64_t den,
                  uint32_t* keep_bits, int64_t* n_kept, hipStream_t s) {
    if (n_kept) fill_i64(n_kept, 1, 0, s);
    if (g->m <= 0) return;
    hipLaunchKernelGGL(k_prune, dim3(grid_for(g->m, 4096)), dim3(kThreads), 0, s, g->src, g->adj, g->deg,
                       t, g->m, measure, num, den, keep_bits, (unsigned long long*)n_kept);
}

}  // namespace mcd
