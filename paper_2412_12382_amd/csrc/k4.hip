// kappa-clique participation for kappa = 4 (Table tab:simfunctions): for
// every edge, the number of 4-cliques that contain it.
//
// On the degree-ordered orientation a 4-clique {a < b < c < d} is found once,
// from its lowest edge a->b: c and d lie in L = N+(a) n N+(b) (both rows
// sorted, so L is the part of N+(a) after b that also lies in N+(b)), and the
// clique closes when d lies in N+(c).  One wave takes one edge at a time: it
// gathers L into LDS (value, position in row a, position in row b), then for
// every c in L tests the later elements d of L against row c by binary search.
// A clique credits its six edges: a->b once per wave (a single add), a->c and
// b->c once per c (summed over its hits), a->d, b->d and c->d per hit.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 64;  // one wave per workgroup

__device__ __forceinline__ void add_relaxed(int32_t* p, int32_t x) {
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// position of x in the sorted slice adj[lo, hi), or -1
__device__ __forceinline__ int64_t find_sorted(const int32_t* __restrict__ adj, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t y = adj[mid];
        if (y < x) lo = mid + 1;
        else if (y > x) hi = mid;
        else return mid;
    }
    return -1;
}

__global__ __launch_bounds__(kThreads) void k_k4(const int32_t* __restrict__ src, const int32_t* __restrict__ adj,
                                                 const int64_t* __restrict__ off, int64_t m,
                                                 int32_t* __restrict__ k4) {
    __shared__ int32_t lv[MCD_K4_MAX_COMMON];   // elements c of L
    __shared__ int32_t lpa[MCD_K4_MAX_COMMON];  // edge a->c
    __shared__ int32_t lpb[MCD_K4_MAX_COMMON];  // edge b->c
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t e = blockIdx.x; e < m; e += gridDim.x) {
        const int32_t a = src[e], b = adj[e];
        const int64_t a1 = off[a + 1];
        const int64_t b0 = off[b], b1 = off[b + 1];
        // L: the suffix of row a after b that also lies in row b
        int nL = 0;
        for (int64_t i0 = e + 1; i0 < a1; i0 += 64) {
            const int64_t i = i0 + lane;
            int64_t pb = -1;
            int32_t c = 0;
            if (i < a1) {
                c = adj[i];
                pb = find_sorted(adj, b0, b1, c);
            }
            const bool hit = pb >= 0;
            const uint64_t bal = __ballot(hit);
            if (hit) {
                const int slot = nL + __popcll(bal & below);
                lv[slot] = c;
                lpa[slot] = (int32_t)i;
                lpb[slot] = (int32_t)pb;
            }
            nL += __popcll(bal);
        }
        __syncthreads();
        int32_t cliques = 0;
        for (int x = 0; x + 1 < nL; ++x) {
            const int32_t c = lv[x];
            const int64_t c0 = off[c], c1 = off[c + 1];
            uint32_t hits = 0;
            for (int y0 = x + 1; y0 < nL; y0 += 64) {
                const int y = y0 + lane;
                bool hit = false;
                if (y < nL) {
                    const int64_t pcd = find_sorted(adj, c0, c1, lv[y]);
                    if (pcd >= 0) {
                        hit = true;
                        add_relaxed(&k4[lpa[y]], 1);  // a->d
                        add_relaxed(&k4[lpb[y]], 1);  // b->d
                        add_relaxed(&k4[pcd], 1);     // c->d
                    }
                }
                hits += (uint32_t)__popcll(__ballot(hit));
            }
            if (lane == 0 && hits) {
                add_relaxed(&k4[lpa[x]], (int32_t)hits);  // a->c
                add_relaxed(&k4[lpb[x]], (int32_t)hits);  // b->c
            }
            cliques += (int32_t)hits;
        }
        if (lane == 0 && cliques) add_relaxed(&k4[e], cliques);
        __syncthreads();
    }
}

}  // namespace

void launch_k4(const mcd_graph* g, int32_t* k4, hipStream_t s) {
    fill_i32(k4, g->m, 0, s);
    if (g->m <= 0) return;
    const int64_t blocks = g->m < 65536 ? g->m : 65536;
    hipLaunchKernelGGL(k_k4, dim3((unsigned)blocks), dim3(kThreads), 0, s, g->src, g->adj, g->off, g->m, k4);
}

}  // namespace mcd
