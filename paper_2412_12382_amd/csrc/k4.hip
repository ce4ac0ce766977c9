// kappa-clique participation for kappa = 4 (Table tab:simfunctions): for
// every edge, the number of 4-cliques that contain it.
//
// On the degree-ordered orientation a 4-clique {a < b < c < d} is found once,
// from its lowest edge a->b: c and d lie in L = N+(a) n N+(b) (both rows
// sorted, so L is the part of N+(a) after b that also lies in N+(b)), and the
// clique closes when d lies in N+(c).  One wave takes one edge at a time and
// tests every element of the suffix of row a against row b by binary search;
// then for every c in L it tests the later elements d of L against row c.  A
// clique credits its six edges: a->b once per wave (a single add), a->c and
// b->c once per c (summed over its hits), a->d, b->d and c->d per hit.
//
// |L| is at most min(suffix length, outd(b)), known from the offsets alone:
// an edge whose bound is below 2 closes no clique and is skipped.  The suffix
// length sorts the rest into two kernels.  Up to 64 * kRegChunks elements the
// suffix stays in registers, lane i holding element i of each 64-element
// chunk with a ballot mask of the hits, so that kernel needs no LDS and runs
// at full occupancy.  Longer suffixes (hub rows) gather L into LDS sized by
// the graph's longest row.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kRegChunks = 4;     // register path: suffixes of at most 256 elements
constexpr int kRegThreads = 256;  // 4 waves per workgroup
constexpr int kRegSuffix = 64 * kRegChunks;

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

// upper bound of |L| for edge e = a->b
__device__ __forceinline__ int64_t common_bound(int64_t e, int64_t a1, int64_t b0, int64_t b1) {
    const int64_t suf = a1 - e - 1;
    const int64_t ob = b1 - b0;
    return suf < ob ? suf : ob;
}

__global__ __launch_bounds__(kRegThreads) void k_k4_reg(const int32_t* __restrict__ src,
                                                        const int32_t* __restrict__ adj,
                                                        const int64_t* __restrict__ off, int64_t m,
                                                        int32_t* __restrict__ k4) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (kRegThreads / 64);
    const int64_t w0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kRegThreads / 64) + (threadIdx.x >> 6)));
    for (int64_t e = w0; e < m; e += nw) {
        const int32_t a = src[e], b = adj[e];
        const int64_t a1 = off[a + 1];
        const int64_t b0 = off[b], b1 = off[b + 1];
        if (a1 - e - 1 > kRegSuffix || common_bound(e, a1, b0, b1) < 2) continue;
        // L: hits of the suffix of row a (after b) in row b, kept in place
        int32_t cv[kRegChunks], pb[kRegChunks];
        uint64_t hm[kRegChunks];
        int nL = 0;
#pragma unroll
        for (int r = 0; r < kRegChunks; ++r) {
            cv[r] = 0;
            pb[r] = -1;
            hm[r] = 0;
            const int64_t i0 = e + 1 + 64 * r;
            if (i0 < a1) {
                const int64_t i = i0 + lane;
                if (i < a1) {
                    cv[r] = adj[i];
                    pb[r] = (int32_t)find_sorted(adj, b0, b1, cv[r]);
                }
                hm[r] = __ballot(pb[r] >= 0);
                nL += __popcll(hm[r]);
            }
        }
        if (nL < 2) continue;
        int32_t cliques = 0;
#pragma unroll
        for (int xr = 0; xr < kRegChunks; ++xr) {
            uint64_t bits = hm[xr];
            while (bits) {
                const int xl = __builtin_ctzll(bits);
                bits &= bits - 1;
                const int32_t c = __builtin_amdgcn_readlane(cv[xr], xl);
                const int32_t pbc = __builtin_amdgcn_readlane(pb[xr], xl);
                const int64_t c0 = off[c], c1 = off[c + 1];
                uint32_t hits = 0;
#pragma unroll
                for (int yr = xr; yr < kRegChunks; ++yr) {
                    // the hits after c: later lanes of c's chunk, all of later chunks
                    const uint64_t cand = yr == xr ? (hm[yr] & ~((2ull << xl) - 1ull)) : hm[yr];
                    if (cand == 0) continue;
                    bool hit = false;
                    if ((cand >> lane) & 1ull) {
                        const int64_t pcd = find_sorted(adj, c0, c1, cv[yr]);
                        if (pcd >= 0) {
                            hit = true;
                            add_relaxed(&k4[e + 1 + 64 * yr + lane], 1);  // a->d
                            add_relaxed(&k4[pb[yr]], 1);                 // b->d
                            add_relaxed(&k4[pcd], 1);                    // c->d
                        }
                    }
                    hits += (uint32_t)__popcll(__ballot(hit));
                }
                if (lane == 0 && hits) {
                    add_relaxed(&k4[e + 1 + 64 * xr + xl], (int32_t)hits);  // a->c
                    add_relaxed(&k4[pbc], (int32_t)hits);                  // b->c
                }
                cliques += (int32_t)hits;
            }
        }
        if (lane == 0 && cliques) add_relaxed(&k4[e], cliques);  // a->b
    }
}

// edges whose suffix is longer than the register path holds: L gathered into LDS (value,
// position in row a, position in row b), cap entries each
__global__ __launch_bounds__(64) void k_k4_lds(const int32_t* __restrict__ src, const int32_t* __restrict__ adj,
                                               const int64_t* __restrict__ off, int64_t m, int cap,
                                               int32_t* __restrict__ k4) {
    extern __shared__ int32_t lds[];
    int32_t* lv = lds;             // elements c of L
    int32_t* lpa = lds + cap;      // edge a->c
    int32_t* lpb = lds + 2 * cap;  // edge b->c
    const int lane = threadIdx.x;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int64_t e = blockIdx.x; e < m; e += gridDim.x) {
        const int32_t a = src[e], b = adj[e];
        const int64_t a1 = off[a + 1];
        const int64_t b0 = off[b], b1 = off[b + 1];
        if (a1 - e - 1 <= kRegSuffix || common_bound(e, a1, b0, b1) < 2) continue;
        int nL = 0;
        for (int64_t i0 = e + 1; i0 < a1; i0 += 64) {
            const int64_t i = i0 + lane;
            int64_t pbi = -1;
            int32_t c = 0;
            if (i < a1) {
                c = adj[i];
                pbi = find_sorted(adj, b0, b1, c);
            }
            const bool hit = pbi >= 0;
            const uint64_t bal = __ballot(hit);
            if (hit) {
                const int slot = nL + __popcll(bal & below);
                lv[slot] = c;
                lpa[slot] = (int32_t)i;
                lpb[slot] = (int32_t)pbi;
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
    // the LDS path only has work when some row is longer than the register path's suffix
    if (g->max_outdeg > kRegSuffix) {
        const int cap = (g->max_outdeg + 63) & ~63;
        const int64_t blocks = g->m < 16384 ? g->m : 16384;
        hipLaunchKernelGGL(k_k4_lds, dim3((unsigned)blocks), dim3(64), (size_t)cap * 3 * sizeof(int32_t), s,
                           g->src, g->adj, g->off, g->m, cap, k4);
    }
    const int64_t waves = g->m < (int64_t)1 << 16 ? g->m : (int64_t)1 << 16;
    const int64_t blocks = (waves + kRegThreads / 64 - 1) / (kRegThreads / 64);
    hipLaunchKernelGGL(k_k4_reg, dim3((unsigned)blocks), dim3(kRegThreads), 0, s, g->src, g->adj, g->off, g->m, k4);
}

}  // namespace mcd
