// kappa-clique participation for kappa = 4 (Table tab:simfunctions): for
// every edge, the number of 4-cliques that contain it.
//
// On the degree-ordered orientation a 4-clique {a < b < c < d} is found once,
// from its lowest edge a->b: c and d lie in L = N+(a) n N+(b) (both rows
// sorted, so L is the part of N+(a) after b that also lies in N+(b)), and the
// clique closes when d lies in N+(c).  Per edge a->b: every element of the
// suffix of row a after b is tested against row b by binary search and the
// hits are gathered into LDS (value; its offsets in the suffix and in row b,
// packed in one word; the row offsets of c); then the nL(nL-1)/2 pairs
// c < d of L are spread over the lanes, one pair per lane, and d is searched
// in row c.
//
// Credits: a clique credits its six edges.  c->d is a global atomic at the
// position the search found.  The others are summed on chip first: a->x and
// b->x, for x in L, both gain the degree of x in the subgraph that L induces
// (counted in LDS, written once per element), and a->b gains that subgraph's
// number of edges (one add per wave).
//
// |L| is at most min(suffix length, outd(b)), known from the offsets alone:
// an edge whose bound is below 2 closes no clique and is skipped.  Edges are
// dealt round-robin to the waves (or workgroups), which test 64 (or 256) of
// theirs at a time and work only on the candidates.  A suffix of at most
// kWaveSuffix elements is one wave's work; longer ones (hub rows) take a
// workgroup of four waves that share L in LDS sized by the graph's longest
// row.  The two kernels run at once, on the context's stream and one of its
// side streams.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kWaveSuffix = 256;   // longest suffix one wave takes
constexpr int kWaveBlock = 4;      // waves per workgroup of the wave kernel
constexpr int kBlockThreads = 256; // workgroup of the long-suffix kernel

__device__ __forceinline__ void add_relaxed(int32_t* p, int32_t x) {
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_lds(int32_t* p) {
    __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS written by other lanes of this wave: order the writes before the reads
// (one wave: no barrier needed)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// an element of L by its offset in the suffix of row a and in row b, both
// below 4096 (rows hold at most 4096 edges), in one word
__device__ __forceinline__ int32_t pack_pos(int64_t in_suffix, int64_t in_b) {
    return (int32_t)((uint32_t)in_suffix | ((uint32_t)in_b << 16));
}

// pairs (x, y), x < y < nL, numbered row by row: row x starts at
// x (2 nL - x - 1) / 2
__device__ __forceinline__ int pair_row_start(int x, int nL) { return (x * (2 * nL - x - 1)) >> 1; }

__device__ __forceinline__ void pair_of(int p, int nL, int& x, int& y) {
    // the row from the quadratic's smaller root, then exact integer correction
    const float bb = (float)(2 * nL - 1);
    int r = (int)((bb - sqrtf(fmaxf(bb * bb - 8.0f * (float)p, 0.0f))) * 0.5f);
    r = r < 0 ? 0 : (r > nL - 2 ? nL - 2 : r);
    while (r > 0 && pair_row_start(r, nL) > p) --r;
    while (r < nL - 2 && pair_row_start(r + 1, nL) <= p) ++r;
    x = r;
    y = p - pair_row_start(r, nL) + r + 1;
}

// whether edge e (row a ending at a1, head b with row [b0, b1)) goes to the
// wave kernel (LONG = false) or the workgroup kernel (LONG = true)
template <bool LONG>
__device__ __forceinline__ bool k4_candidate(int64_t e, int64_t a1, int64_t b0, int64_t b1) {
    const int64_t suf = a1 - e - 1;
    const int64_t bound = suf < b1 - b0 ? suf : b1 - b0;
    return bound >= 2 && (LONG ? suf > kWaveSuffix : suf <= kWaveSuffix);
}

__global__ __launch_bounds__(64 * kWaveBlock) void k_k4_wave(const int32_t* __restrict__ src,
                                                            const int32_t* __restrict__ adj,
                                                            const int64_t* __restrict__ off, int64_t m,
                                                            int32_t* __restrict__ k4) {
    __shared__ int32_t sv[kWaveBlock][kWaveSuffix], spk[kWaveBlock][kWaveSuffix];
    __shared__ int32_t scnt[kWaveBlock][kWaveSuffix], sc0[kWaveBlock][kWaveSuffix], sc1[kWaveBlock][kWaveSuffix];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    int32_t *lv = sv[w], *lpk = spk[w], *lcnt = scnt[w], *lc0 = sc0[w], *lc1 = sc1[w];
    const uint64_t below = (1ull << lane) - 1ull;
    // edges interleaved over the waves (edge e to wave e mod W): the heavy
    // edges of a hub row spread over many waves
    const int64_t W = (int64_t)gridDim.x * kWaveBlock;
    const int64_t wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kWaveBlock + w));
    for (int64_t r0 = 0; wid + r0 * W < m; r0 += 64) {
        // 64 of this wave's edges, one per lane
        const int64_t el = wid + (r0 + lane) * W;
        bool cand = false;
        if (el < m) {
            const int64_t a1 = off[src[el] + 1];
            const int32_t b = adj[el];
            cand = k4_candidate<false>(el, a1, off[b], off[b + 1]);
        }
        uint64_t todo = __ballot(cand);
        while (todo) {
            const int64_t e = wid + (r0 + __builtin_ctzll(todo)) * W;
            todo &= todo - 1;
            const int32_t a = src[e], b = adj[e];
            const int64_t a1 = off[a + 1];
            const int64_t b0 = off[b], b1 = off[b + 1];
            // L: the suffix's hits in row b, at most kWaveSuffix of them
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
                    lpk[slot] = pack_pos(i - e - 1, pb - b0);
                    lcnt[slot] = 0;
                    lc0[slot] = (int32_t)off[c];  // offsets < m < 2^31
                    lc1[slot] = (int32_t)off[c + 1];
                }
                nL += __popcll(bal);
            }
            if (nL < 2) continue;
            wave_lds_sync();
            const int P = nL * (nL - 1) / 2;
            int32_t total = 0;
            for (int p0 = 0; p0 < P; p0 += 64) {
                const int p = p0 + lane;
                bool hit = false;
                if (p < P) {
                    int x, y;
                    pair_of(p, nL, x, y);
                    const int64_t pcd = find_sorted(adj, lc0[x], lc1[x], lv[y]);
                    if (pcd >= 0) {
                        hit = true;
                        add_relaxed(&k4[pcd], 1);  // c->d
                        add_lds(&lcnt[x]);
                        add_lds(&lcnt[y]);
                    }
                }
                total += __popcll(__ballot(hit));
            }
            wave_lds_sync();
            for (int i = lane; i < nL; i += 64) {
                const int32_t k = lcnt[i];
                if (k) {
                    const uint32_t pk = (uint32_t)lpk[i];
                    add_relaxed(&k4[e + 1 + (pk & 0xFFFFu)], k);  // a->x
                    add_relaxed(&k4[b0 + (pk >> 16)], k);        // b->x
                }
            }
            if (lane == 0 && total) add_relaxed(&k4[e], total);  // a->b
            wave_lds_sync();  // reads done before the next edge's writes
        }
    }
}

// suffixes longer than one wave takes: four waves share L (cap entries per
// array; with ROWS the row offsets of every c are kept beside it, else they
// are read per pair)
template <bool ROWS>
__global__ __launch_bounds__(kBlockThreads) void k_k4_block(const int32_t* __restrict__ src,
                                                           const int32_t* __restrict__ adj,
                                                           const int64_t* __restrict__ off, int64_t m, int cap,
                                                           int32_t* __restrict__ k4) {
    extern __shared__ int32_t lds[];
    __shared__ uint64_t wmask[kBlockThreads / 64];
    __shared__ int32_t wcount[kBlockThreads / 64];
    int32_t *lv = lds, *lpk = lds + cap, *lcnt = lds + 2 * cap;
    int32_t *lc0 = lds + 3 * cap, *lc1 = lds + 4 * cap;  // ROWS only
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    constexpr int NW = kBlockThreads / 64;
    const uint64_t below = (1ull << lane) - 1ull;
    // edges interleaved over the workgroups (edge e to workgroup e mod G)
    const int64_t G = gridDim.x;
    for (int64_t r0 = 0; blockIdx.x + r0 * G < m; r0 += kBlockThreads) {
        const int64_t el = blockIdx.x + (r0 + tid) * G;
        bool cand = false;
        if (el < m) {
            const int64_t a1 = off[src[el] + 1];
            const int32_t b = adj[el];
            cand = k4_candidate<true>(el, a1, off[b], off[b + 1]);
        }
        const uint64_t bal0 = __ballot(cand);
        if (lane == 0) wmask[w] = bal0;
        __syncthreads();
        for (int ww = 0; ww < NW; ++ww) {
            uint64_t todo = wmask[ww];
            while (todo) {
                const int64_t e = blockIdx.x + (r0 + 64 * ww + __builtin_ctzll(todo)) * G;
                todo &= todo - 1;
                const int32_t a = src[e], b = adj[e];
                const int64_t a1 = off[a + 1];
                const int64_t b0 = off[b], b1 = off[b + 1];
                int nL = 0;
                for (int64_t i0 = e + 1; i0 < a1; i0 += kBlockThreads) {
                    const int64_t i = i0 + tid;
                    int64_t pb = -1;
                    int32_t c = 0;
                    if (i < a1) {
                        c = adj[i];
                        pb = find_sorted(adj, b0, b1, c);
                    }
                    const bool hit = pb >= 0;
                    const uint64_t bal = __ballot(hit);
                    if (lane == 0) wcount[w] = __popcll(bal);
                    __syncthreads();
                    int base = nL, add = 0;
                    for (int k = 0; k < NW; ++k) {
                        const int ck = wcount[k];
                        base += k < w ? ck : 0;
                        add += ck;
                    }
                    if (hit) {
                        const int slot = base + __popcll(bal & below);
                        lv[slot] = c;
                        lpk[slot] = pack_pos(i - e - 1, pb - b0);
                        lcnt[slot] = 0;
                        if (ROWS) {
                            lc0[slot] = (int32_t)off[c];
                            lc1[slot] = (int32_t)off[c + 1];
                        }
                    }
                    nL += add;
                    __syncthreads();  // entries written, wcount free again
                }
                if (nL < 2) continue;  // workgroup-uniform
                const int P = nL * (nL - 1) / 2;
                int32_t total = 0;
                for (int p0 = 0; p0 < P; p0 += kBlockThreads) {
                    const int p = p0 + tid;
                    bool hit = false;
                    if (p < P) {
                        int x, y;
                        pair_of(p, nL, x, y);
                        int64_t c0, c1;
                        if (ROWS) {
                            c0 = lc0[x];
                            c1 = lc1[x];
                        } else {
                            const int32_t c = lv[x];
                            c0 = off[c];
                            c1 = off[c + 1];
                        }
                        const int64_t pcd = find_sorted(adj, c0, c1, lv[y]);
                        if (pcd >= 0) {
                            hit = true;
                            add_relaxed(&k4[pcd], 1);  // c->d
                            add_lds(&lcnt[x]);
                            add_lds(&lcnt[y]);
                        }
                    }
                    total += __popcll(__ballot(hit));
                }
                if (lane == 0 && total) add_relaxed(&k4[e], total);  // a->b, one add per wave
                __syncthreads();
                for (int i = tid; i < nL; i += kBlockThreads) {
                    const int32_t k = lcnt[i];
                    if (k) {
                        const uint32_t pk = (uint32_t)lpk[i];
                        add_relaxed(&k4[e + 1 + (pk & 0xFFFFu)], k);  // a->x
                        add_relaxed(&k4[b0 + (pk >> 16)], k);        // b->x
                    }
                }
                __syncthreads();  // reads done before the next edge's writes
            }
        }
        __syncthreads();  // wmask read by every wave before the next chunk writes it
    }
}

}  // namespace

void launch_k4(const mcd_graph* g, int32_t* k4, hipStream_t s) {
    fill_i32(k4, g->m, 0, s);
    if (g->m <= 0) return;
    // |L| <= outd(b) <= the longest row; the workgroup kernel only has work
    // when some row is longer than one wave's suffix.  It runs beside the
    // wave kernel on a side stream of the context (forked from and joined
    // back into s), so that each fills the other's tail
    mcd_ctx* c = g->ctx;
    const bool two = g->max_outdeg > kWaveSuffix;
    if (two) {
        hipStream_t s1 = c->side[0];
        (void)hipEventRecord(c->fork, s);
        (void)hipStreamWaitEvent(s1, c->fork, 0);
        const int cap = (g->max_outdeg + 63) & ~63;  // <= 4096
        const unsigned blocks = (unsigned)(g->m < 8192 ? g->m : 8192);
        // the whole workgroup's LDS within 64 KB: 20 bytes per entry with
        // the row offsets (cap <= 3264), 12 without (cap <= 4096)
        const size_t with_rows = (size_t)cap * 5 * sizeof(int32_t), without = (size_t)cap * 3 * sizeof(int32_t);
        if (c->k4_row_cache && with_rows + 64 <= 65536)
            hipLaunchKernelGGL(k_k4_block<true>, dim3(blocks), dim3(kBlockThreads), with_rows, s1, g->src, g->adj,
                               g->off, g->m, cap, k4);
        else
            hipLaunchKernelGGL(k_k4_block<false>, dim3(blocks), dim3(kBlockThreads), without, s1, g->src, g->adj,
                               g->off, g->m, cap, k4);
    }
    const int64_t waves = g->m < ((int64_t)1 << 16) ? g->m : ((int64_t)1 << 16);
    const unsigned blocks = (unsigned)((waves + kWaveBlock - 1) / kWaveBlock);
    hipLaunchKernelGGL(k_k4_wave, dim3(blocks), dim3(64 * kWaveBlock), 0, s, g->src, g->adj, g->off, g->m, k4);
    if (two) {
        (void)hipEventRecord(c->join[0], c->side[0]);
        (void)hipStreamWaitEvent(s, c->join[0], 0);
    }
}

}  // namespace mcd
