// Threshold sweep over one graph or a batch of disjoint graphs, with
// per-threshold statistics and the adjusted Rand index against planted labels.
//
// Algorithm 1 keeps an edge at threshold delta iff NOT (sim < delta), so with
// thresholds sorted ascending an edge's "level" (the number of thresholds it
// survives) decides all K prune masks at once: kept at threshold i iff
// level > i.  Walking i from K-1 down to 0 only ever adds edges, so one
// union-find absorbs each level's edges in turn; after each level the
// partition is exactly the components of the edges kept at threshold i.  Roots
// hook under the higher-ranked root (as in the components step); a threshold
// whose labels are asked for gets the smallest original id per root.
//
// Per-graph sums and the sizes of large components are accumulated per block
// in LDS before one global atomic per block: with one graph (or one giant
// component) a global atomic per wave would serialise on a single address.
//
// ARI (Hubert & Arabie) per graph and threshold from exact pair counts:
//   S = sum over (cluster, class) cells of C(n_cc, 2)
//   A = sum over clusters of C(a, 2), B = sum over classes of C(b, 2), N = C(n, 2)
// each gathered as sum over vertices of (cell size - 1) / 2.
#include <algorithm>

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

#define GRID_STRIDE(i, N)                                                              \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (N);          \
         i += (int64_t)gridDim.x * blockDim.x)

__device__ __forceinline__ int rat_cmp(int64_t a, int64_t b, int64_t c, int64_t d) {
    const __int128 l = (__int128)a * d, r = (__int128)c * b;
    return (l > r) - (l < r);
}

// acc[key] += val, summing first over the lanes of the wave whose key equals
// lane 0's (the common case: one graph, one giant component).  All lanes of
// the wave that reach the call must be active together (grid-stride loops
// keep the active lanes a prefix of the wave).
__device__ __forceinline__ void agg_add(unsigned long long* acc, int64_t key, unsigned long long val) {
    const int64_t k0 = __shfl(key, 0);
    const bool same = key == k0;
    unsigned long long x = same ? val : 0ull;
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0) {
        if (x) atomicAdd(&acc[k0], x);
    }
    if (!same && val) atomicAdd(&acc[key], val);
}

// acc[key] = max(acc[key], val), reduced first over the lanes sharing lane 0's key
__device__ __forceinline__ void agg_max(unsigned long long* acc, int64_t key, unsigned long long val) {
    const int64_t k0 = __shfl(key, 0);
    const bool same = key == k0;
    unsigned long long x = same ? val : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    if ((threadIdx.x & 63) == 0) {
        if (x) atomicMax(&acc[k0], x);
    }
    if (!same && val) atomicMax(&acc[key], val);
}

constexpr int kLdsGraphs = 1024;  // per-graph accumulators held in LDS up to this many graphs
constexpr int kRootSlots = 1024;  // LDS table of component roots per block (power of two)

// Per-graph accumulator of a block: LDS when the graphs fit, else global.
struct GraphAcc {
    unsigned long long* lds;   // [G] in LDS, or nullptr
    unsigned long long* glob;  // [G] in global memory
    int G;
    __device__ void init() {
        if (lds)
            for (int i = threadIdx.x; i < G; i += blockDim.x) lds[i] = 0ull;
    }
    __device__ void add(int64_t key, unsigned long long val) {
        if (lds) agg_add(lds, key, val);
        else agg_add(glob, key, val);
    }
    __device__ void max(int64_t key, unsigned long long val) {
        if (lds) agg_max(lds, key, val);
        else agg_max(glob, key, val);
    }
    // after a barrier
    __device__ void flush_add() {
        if (lds)
            for (int i = threadIdx.x; i < G; i += blockDim.x)
                if (lds[i]) atomicAdd(&glob[i], lds[i]);
    }
    __device__ void flush_max() {
        if (lds)
            for (int i = threadIdx.x; i < G; i += blockDim.x)
                if (lds[i]) atomicMax(&glob[i], lds[i]);
    }
};

// LDS table root -> count; false when the probe sequence is full.
__device__ __forceinline__ bool root_table_add(int32_t* key, uint32_t* val, int32_t r, uint32_t c) {
    uint32_t h = ((uint32_t)r * 2654435761u) >> 22;  // 10 bits: kRootSlots
    for (int probe = 0; probe < 8; ++probe) {
        const int32_t k = atomicCAS(&key[h], -1, r);
        if (k == -1 || k == r) {
            atomicAdd(&val[h], c);
            return true;
        }
        h = (h + 1) & (kRootSlots - 1);
    }
    return false;
}

constexpr int kLevelBins = 8192;  // largest (graph, level) histogram kept in LDS

// level[e] = number of sorted thresholds delta_i with NOT (sim(e) < delta_i)
// and hist[g][level] (edge counts): with one graph the lanes of a wave that
// share a level are counted with one ballot, else an LDS histogram of
// (graph, level) when it fits.
// sign(a/b - c/d) for b, d > 0 in 64-bit products, exact when |a|, |c| < 2^31
// and b, d < 2^32 (NARROW inputs: every degree below 2^29, thresholds below
// 2^31 in magnitude)
__device__ __forceinline__ int rat_cmp64(int64_t a, int64_t b, int64_t c, int64_t d) {
    const int64_t l = a * d, r = c * b;
    return (l > r) - (l < r);
}

// gate (nullable): a device flag; when it reads 0 the sweep's kernels return
// at once (a caller that needs the sweep only for some inputs decides on the
// device, without a host round trip).
__device__ __forceinline__ bool gated_off(const int32_t* gate) { return gate && *gate == 0; }

template <bool NARROW>
__global__ __launch_bounds__(kThreads) void k_level(const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ dsum,
                                                    const int32_t* __restrict__ t, int64_t m, int measure,
                                                    SweepDeltas ds, uint8_t* __restrict__ level,
                                                    const int32_t* __restrict__ gid, int G,
                                                    unsigned long long* __restrict__ hist,
                                                    const int32_t* __restrict__ gate) {
    if (gated_off(gate)) return;
    extern __shared__ uint32_t h[];  // nbins counters when local (sized at launch)
    // the thresholds in LDS: the search's steps read them at lane-dependent
    // indices, which from the kernel arguments would be a global load (and
    // its latency) per step
    __shared__ int64_t tnum[MCD_SWEEP_MAX], tden[MCD_SWEEP_MAX];
    const int nbins = G * (ds.K + 1);
    const bool local = nbins <= kLevelBins;
    const int lane = threadIdx.x & 63;
    if (local)
        for (int i = threadIdx.x; i < nbins; i += blockDim.x) h[i] = 0;
    for (int i = threadIdx.x; i < ds.K; i += blockDim.x) {
        tnum[i] = ds.num[i];
        tden[i] = ds.den[i];
    }
    __syncthreads();
    GRID_STRIDE(e, m) {
        const int64_t D = (uint32_t)dsum[e];
        const int64_t tt = t[e];
        int64_t num = tt, den = 1;  // K3, K4
        if (measure == MCD_SIM_TECTONIC) den = D;
        else if (measure == MCD_SIM_JACCARD) den = D - tt;
        else if (measure == MCD_SIM_TW) num = 3 * tt - D + 2;
        int lo = 0, hi = ds.K;  // first threshold that prunes e
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int c = NARROW ? rat_cmp64(num, den, tnum[mid], tden[mid]) : rat_cmp(num, den, tnum[mid], tden[mid]);
            if (c >= 0) lo = mid + 1;
            else hi = mid;
        }
        level[e] = (uint8_t)lo;
        if (G == 1) {
            uint64_t pending = __ballot(true);
            while (pending) {  // once per distinct level in the wave
                const int first = __ffsll((long long)pending) - 1;
                const int l0 = __shfl(lo, first);
                const uint64_t same = __ballot(lo == l0) & pending;
                if (lane == first) atomicAdd(&h[l0], (uint32_t)__popcll(same));
                pending &= ~same;
            }
        } else {
            const int64_t key = (int64_t)gid[src[e]] * (ds.K + 1) + lo;
            if (local) atomicAdd(&h[key], 1u);
            else atomicAdd(&hist[key], 1ull);
        }
    }
    __syncthreads();
    if (local)
        for (int i = threadIdx.x; i < nbins; i += blockDim.x)
            if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

// graph id and class of every rank-numbered vertex
__global__ __launch_bounds__(kThreads) void k_vertex_info(const int32_t* __restrict__ perm, int64_t n,
                                                          const int64_t* __restrict__ vbase, int G,
                                                          const int32_t* __restrict__ truth,
                                                          int32_t* __restrict__ gid, int32_t* __restrict__ cls,
                                                          const int32_t* __restrict__ gate) {
    if (gated_off(gate)) return;
    GRID_STRIDE(v, n) {
        const int64_t x = perm[v];
        int lo = 0, hi = G;  // last g with vbase[g] <= x
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (vbase[mid] <= x) lo = mid;
            else hi = mid;
        }
        gid[v] = lo;
        if (truth) cls[v] = truth[x];
    }
}

__global__ __launch_bounds__(kThreads) void k_init_parent(int32_t* __restrict__ parent, int64_t n,
                                                          const int32_t* __restrict__ gate) {
    if (gated_off(gate)) return;
    GRID_STRIDE(v, n) parent[v] = (int32_t)v;
}

// ---- the level loop -------------------------------------------------------
//
// The passes below are device functions over grid-stride loops, run by one
// persistent kernel (k_sweep_levels) whose blocks are all resident and meet
// at grid barriers between phases.  `sh` is the block's LDS scratch
// (kShWords 64-bit words); a pass that uses it initialises it, and ends with
// a block barrier so the next pass may reuse it.

constexpr int kShWords = 2 * kLdsGraphs;  // 16 KB

// unite the endpoints of every edge at level lv.  Every level scans all m
// level bytes, most of them for a handful of edges, so the bytes are read 16
// at a time and a group without a match is passed over with one test.
__device__ __forceinline__ bool has_byte(uint32_t x, uint32_t pat) {
    const uint32_t v = x ^ pat;  // a zero byte where x matches
    return ((v - 0x01010101u) & ~v & 0x80808080u) != 0u;
}

__device__ void d_union_level(const int32_t* __restrict__ src, const int32_t* __restrict__ adj,
                              const uint8_t* __restrict__ level, int64_t m, int lv, int32_t* parent) {
    const int64_t head = min(m, (int64_t)((16u - ((uint32_t)(uintptr_t)level & 15u)) & 15u));
    const int64_t nq = (m - head) >> 4;
    const int64_t tail0 = head + 16 * nq;
    const uint32_t pat = 0x01010101u * (uint32_t)lv;
    GRID_STRIDE(q, nq) {
        const int64_t e0 = head + 16 * q;
        const uint4 x = *(const uint4*)(level + e0);
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (!has_byte(w[i], pat)) continue;
            for (int b = 0; b < 4; ++b)
                if (((w[i] >> (8 * b)) & 0xffu) == (uint32_t)lv) {
                    const int64_t e = e0 + 4 * i + b;
                    uf_unite(parent, src[e], adj[e]);
                }
        }
    }
    GRID_STRIDE(i, head + (m - tail0)) {  // unaligned head and tail bytes
        const int64_t e = i < head ? i : tail0 + (i - head);
        if (level[e] == lv) uf_unite(parent, src[e], adj[e]);
    }
}

// Compress every vertex to its root, count roots per graph, size of every
// component.
__device__ void d_pass_size(int32_t* parent, int64_t n, const int32_t* __restrict__ gid, int G,
                            int32_t* size, unsigned long long* ncc, unsigned long long* sh) {
    int32_t* rk = (int32_t*)(sh + kLdsGraphs);
    uint32_t* rv = (uint32_t*)(rk + kRootSlots);
    GraphAcc acc{G <= kLdsGraphs ? sh : nullptr, ncc, G};
    acc.init();
    for (int i = threadIdx.x; i < kRootSlots; i += blockDim.x) {
        rk[i] = -1;
        rv[i] = 0u;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    GRID_STRIDE(v, n) {
        const int32_t r = uf_find(parent, (int32_t)v);
        uf_store(&parent[v], r);
        const bool root = r == (int32_t)v;
        acc.add(gid[v], root ? 1ull : 0ull);
        // size[r] += 1, first summed over the lanes sharing lane 0's root;
        // roots shared by several lanes go through the LDS table
        const int32_t r0 = __shfl(r, 0);
        const uint64_t same = __ballot(r == r0);
        if (r == r0) {
            if (lane == 0) {
                const uint32_t c = (uint32_t)__popcll(same);
                if ((c == 1 && root) || !root_table_add(rk, rv, r0, c)) atomicAdd(&size[r0], (int32_t)c);
            }
        } else if (root || !root_table_add(rk, rv, r, 1u)) {
            atomicAdd(&size[r], 1);
        }
    }
    __syncthreads();
    acc.flush_add();
    for (int i = threadIdx.x; i < kRootSlots; i += blockDim.x)
        if (rk[i] >= 0) atomicAdd(&size[rk[i]], (int32_t)rv[i]);
    __syncthreads();
}

// Labels of one threshold: the smallest original id of every component
// (minid starts as perm, set with the other per-level resets).
__device__ void d_label_min(int32_t* parent, const int32_t* __restrict__ perm, int64_t n, int32_t* minid) {
    GRID_STRIDE(v, n) {
        const int32_t r = uf_find(parent, (int32_t)v);
        if (r != (int32_t)v) atomicMin(&minid[r], perm[v]);
    }
}

__device__ void d_label_write(int32_t* parent, const int32_t* __restrict__ perm, int64_t n, const int32_t* minid,
                              int32_t* __restrict__ labels) {
    GRID_STRIDE(v, n) labels[perm[v]] = __hip_atomic_load(&minid[uf_find(parent, (int32_t)v)], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t cell_key(int32_t r, int32_t c) {
    return ((uint64_t)(uint32_t)r << 32) | (uint32_t)c;
}

__device__ __forceinline__ uint32_t cell_slot(uint64_t k, int log2cap) {
    return (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> (64 - log2cap));
}

// A (same cluster pairs) and the largest component per graph, read off the
// component sizes: after the size pass only roots hold a nonzero size, and a
// root's graph is its own.
__device__ void d_pass_roots(int64_t n, const int32_t* __restrict__ gid, int G, const int32_t* size,
                             unsigned long long* acc_a, unsigned long long* largest, unsigned long long* sh) {
    const bool lds = G <= kLdsGraphs;
    GraphAcc A{lds ? sh : nullptr, acc_a, G}, Lg{lds ? sh + kLdsGraphs : nullptr, largest, G};
    A.init();
    Lg.init();
    __syncthreads();
    GRID_STRIDE(v, n) {
        const int32_t sz = __hip_atomic_load(&size[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t g = gid[v];
        A.add(g, (unsigned long long)sz * (unsigned long long)(sz > 0 ? sz - 1 : 0));
        Lg.max(g, (unsigned long long)sz);
    }
    __syncthreads();
    A.flush_add();
    Lg.flush_max();
    __syncthreads();
}

// With planted labels: count every (cluster, class) cell in a hash table.
__device__ void d_pass_cells(int32_t* parent, int64_t n, const int32_t* __restrict__ cls, unsigned long long* keys,
                             int32_t* counts, int log2cap) {
    const int lane = threadIdx.x & 63;
    GRID_STRIDE(v, n) {
        // the size pass compressed the paths, but a concurrent halving may
        // have left parent[v] at an ancestor below the root: follow to the root
        const int32_t r = uf_find(parent, (int32_t)v);
        const uint64_t k = cell_key(r, cls[v]);
        const uint32_t mask = (1u << log2cap) - 1u;
        uint32_t h = cell_slot(k, log2cap);
        for (;;) {
            const unsigned long long prev = atomicCAS(&keys[h], ~0ull, (unsigned long long)k);
            if (prev == ~0ull || prev == k) break;
            h = (h + 1) & mask;
        }
        const uint64_t k0 = __shfl(k, 0);
        const uint64_t same = __ballot(k == k0);
        if (k == k0) {
            if ((same & ((1ull << lane) - 1ull)) == 0) atomicAdd(&counts[h], (int32_t)__popcll(same));
        } else {
            atomicAdd(&counts[h], 1);
        }
    }
}

// S (pairs sharing cluster and class) per graph.
__device__ void d_pass_s(int32_t* parent, int64_t n, const int32_t* __restrict__ gid, int G,
                         const int32_t* __restrict__ cls, const unsigned long long* keys, const int32_t* counts,
                         int log2cap, unsigned long long* acc_s, unsigned long long* sh) {
    GraphAcc S{G <= kLdsGraphs ? sh : nullptr, acc_s, G};
    S.init();
    __syncthreads();
    GRID_STRIDE(v, n) {
        const uint64_t k = cell_key(uf_find(parent, (int32_t)v), cls[v]);
        const uint32_t mask = (1u << log2cap) - 1u;
        uint32_t h = cell_slot(k, log2cap);
        while (__hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != k) h = (h + 1) & mask;
        const int32_t c = __hip_atomic_load(&counts[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        S.add(gid[v], (unsigned long long)(c - 1));
    }
    __syncthreads();
    S.flush_add();
    __syncthreads();
}

// Precision, recall and F1 of Sec. 4 (Evaluation): every output community S
// (a component, root r, size s) is matched to the planted class C maximising
// the Jaccard overlap |C n S| / |C u S| = x / (s + b - x) (x = the cell count,
// b = |C|; ties go to the smaller class id); then p = x / s, r = x / b and,
// weighted by s, precision = sum x / n, recall = sum x s / b / n and
// F1 = sum 2 x s / (s + b) / n (2 p r / (p + r) = 2 x / (s + b)).
//
// best[r] holds (x << 32) | c of the best cell seen; cells compete by an exact
// compare-and-swap maximum.
__device__ void d_cells_best(const unsigned long long* keys, const int32_t* counts, int64_t cap, const int32_t* size,
                             const int32_t* __restrict__ csize, unsigned long long* best) {
    GRID_STRIDE(h, cap) {
        const unsigned long long k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == ~0ull) continue;
        const int32_t r = (int32_t)(k >> 32), c = (int32_t)(uint32_t)k;
        const int64_t x = __hip_atomic_load(&counts[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t sz = __hip_atomic_load(&size[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t b = csize[c];
        const unsigned long long mine = ((unsigned long long)x << 32) | (uint32_t)c;
        unsigned long long cur = __hip_atomic_load(&best[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
            if (cur != 0ull) {
                const int64_t x2 = (int64_t)(cur >> 32);
                const int32_t c2 = (int32_t)(uint32_t)cur;
                const int64_t b2 = csize[c2];
                // x / (sz + b - x) vs x2 / (sz + b2 - x2), both denominators >= 1
                const int64_t l = x * (sz + b2 - x2), rr = x2 * (sz + b - x);
                if (l < rr || (l == rr && c > c2)) break;  // the stored cell wins
            }
            const unsigned long long seen = atomicCAS(&best[r], cur, mine);
            if (seen == cur) break;
            cur = seen;
        }
    }
}

__device__ void d_prf_sums(int64_t n, const int32_t* __restrict__ gid, int G, const int32_t* size,
                           const int32_t* __restrict__ csize, const unsigned long long* best, double* acc,
                           unsigned long long* sh) {
    double* lp = (double*)sh;  // 3 doubles per graph
    const bool lds = 3 * G <= kShWords;
    if (lds)
        for (int i = threadIdx.x; i < 3 * G; i += blockDim.x) lp[i] = 0.0;
    __syncthreads();
    GRID_STRIDE(v, n) {
        const int32_t sz = __hip_atomic_load(&size[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (sz == 0) continue;  // not a root
        const unsigned long long rec = __hip_atomic_load(&best[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double x = (double)(rec >> 32), b = (double)csize[(int32_t)(uint32_t)rec], s = (double)sz;
        double* dst = lds ? lp + 3 * gid[v] : acc + 3 * (int64_t)gid[v];
        atomicAdd(dst + 0, x);
        atomicAdd(dst + 1, x * s / b);
        atomicAdd(dst + 2, 2.0 * x * s / (s + b));
    }
    __syncthreads();
    if (lds)
        for (int i = threadIdx.x; i < 3 * G; i += blockDim.x)
            if (lp[i] != 0.0) atomicAdd(&acc[i], lp[i]);
    __syncthreads();
}

// Modularity (the quality measure of the paper's threshold rule of thumb) of
// the partition at this threshold, on the input graph:
//   Q = sum over components c of e_c / m - (vol_c / 2m)^2,
// with e_c the input edges inside c and vol_c the sum of input degrees over c.
// vol[root] accumulates the degrees of each component (wave-aggregated, big
// components through the block's LDS table like the sizes).
__device__ void d_pass_volume(int32_t* parent, int64_t n, const int32_t* __restrict__ deg, unsigned long long* vol,
                              unsigned long long* sh) {
    unsigned long long* rv = sh;
    int32_t* rk = (int32_t*)(sh + kRootSlots);
    for (int i = threadIdx.x; i < kRootSlots; i += blockDim.x) {
        rk[i] = -1;
        rv[i] = 0ull;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    GRID_STRIDE(v, n) {
        const int32_t r = uf_find(parent, (int32_t)v);
        const unsigned long long d = (unsigned long long)deg[v];
        const int32_t r0 = __shfl(r, 0);
        unsigned long long x = r == r0 ? d : 0ull;
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        const bool done = r == r0;
        if (lane == 0 && x) {
            uint32_t h = ((uint32_t)r0 * 2654435761u) >> 22;
            bool put = false;
            for (int probe = 0; probe < 8 && !put; ++probe) {
                const int32_t k = atomicCAS(&rk[h], -1, r0);
                if (k == -1 || k == r0) {
                    atomicAdd(&rv[h], x);
                    put = true;
                }
                h = (h + 1) & (kRootSlots - 1);
            }
            if (!put) atomicAdd(&vol[r0], x);
        }
        if (!done && d) atomicAdd(&vol[r], d);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kRootSlots; i += blockDim.x)
        if (rk[i] >= 0 && rv[i]) atomicAdd(&vol[rk[i]], rv[i]);
    __syncthreads();
}

// Per graph: the input edges whose endpoints share a component at threshold
// slot lv_thresh (kept edges always do; a pruned edge iff its endpoints have
// one root).
__device__ void d_pass_intra(const int32_t* __restrict__ src, const int32_t* __restrict__ adj,
                             const uint8_t* __restrict__ level, int64_t m, int lv_thresh, int32_t* parent,
                             const int32_t* __restrict__ gid, int G, unsigned long long* acc_intra,
                             unsigned long long* sh) {
    GraphAcc I{G <= kLdsGraphs ? sh : nullptr, acc_intra, G};
    I.init();
    __syncthreads();
    GRID_STRIDE(e, m) {
        const int32_t u = src[e];
        bool in = level[e] > lv_thresh;
        if (!in) in = uf_find(parent, u) == uf_find(parent, adj[e]);
        I.add(G == 1 ? 0 : gid[u], in ? 1ull : 0ull);
    }
    __syncthreads();
    I.flush_add();
    __syncthreads();
}

// and the sum over components of vol_c^2
__device__ void d_pass_vsq(int64_t n, const int32_t* __restrict__ gid, int G, const unsigned long long* vol,
                           unsigned long long* acc_vsq, unsigned long long* sh) {
    GraphAcc Q{G <= kLdsGraphs ? sh : nullptr, acc_vsq, G};
    Q.init();
    __syncthreads();
    GRID_STRIDE(v, n) {
        const unsigned long long x = __hip_atomic_load(&vol[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Q.add(gid[v], x * x);  // nonzero only at roots
    }
    __syncthreads();
    Q.flush_add();
    __syncthreads();
}

// class sizes (truth ids lie in [0, n)), then B per graph
__global__ __launch_bounds__(kThreads) void k_class_size(const int32_t* __restrict__ cls, int64_t n,
                                                         int32_t* __restrict__ csize,
                                                         const int32_t* __restrict__ gate) {
    if (gated_off(gate)) return;
    const int lane = threadIdx.x & 63;
    GRID_STRIDE(v, n) {
        const int32_t c = cls[v];
        const int32_t c0 = __shfl(c, 0);
        const uint64_t same = __ballot(c == c0);
        if (c == c0) {
            if ((same & ((1ull << lane) - 1ull)) == 0) atomicAdd(&csize[c], (int32_t)__popcll(same));
        } else {
            atomicAdd(&csize[c], 1);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_class_b(const int32_t* __restrict__ cls, int64_t n,
                                                      const int32_t* __restrict__ gid, int G,
                                                      const int32_t* __restrict__ csize,
                                                      unsigned long long* __restrict__ acc_b,
                                                      const int32_t* __restrict__ gate) {
    if (gated_off(gate)) return;
    __shared__ unsigned long long lb[kLdsGraphs];
    GraphAcc B{G <= kLdsGraphs ? lb : nullptr, acc_b, G};
    B.init();
    __syncthreads();
    GRID_STRIDE(v, n) B.add(gid[v], (unsigned long long)(csize[cls[v]] - 1));
    __syncthreads();
    B.flush_add();
}

// Slots of the caller's thresholds: slot[i] = caller slot of the i-th smallest.
struct SlotOrder {
    int slot[MCD_SWEEP_MAX];
};

// Per-graph accumulators of one level; the level loop keeps two sets and
// alternates between them, so a level's statistics are written while the
// next level's set is being cleared.
enum { kAccNcc, kAccLargest, kAccA, kAccS, kAccIntra, kAccVsq, kAccFields };

// State of the grid barrier (in the sweep workspace, zeroed before launch):
// blocks arrive in groups (block index mod kSyncGroups), the last of a group
// arrives at the top counter, and the last group moves every group's
// generation on; each counter and generation sits on its own cache line, so
// arrivals and the blocks' polling spread over several addresses.
constexpr int kSyncGroups = 8;
struct GridSync {
    unsigned int top;  // groups arrived at the current barrier
    unsigned int pad0[31];
    struct Group {
        unsigned int count;  // blocks of the group arrived
        unsigned int gen;    // barriers completed
        unsigned int pad[30];
    } grp[kSyncGroups];
    int timed_out;  // a block waited longer than the limit
    int giant;      // root of the sampled large component of a dense level
    int pad1[30];
};

struct SweepArgs {
    const int32_t* src;
    const int32_t* adj;
    const int64_t* off;     // CSR row offsets (out-edges of every vertex)
    const int64_t* in_off;  // in-edge list offsets
    const int2* in_ea;      // in-edge lists: (edge id, suffix length)
    const uint8_t* level;
    const int32_t* perm;
    const int32_t* deg;
    const int32_t* gid;
    const int32_t* cls;    // planted class of every rank-numbered vertex, or null
    const int32_t* csize;  // class sizes (with planted labels)
    const int64_t* vbase;
    const unsigned long long* hist;   // [G][K+1] edges per (graph, level)
    const unsigned long long* acc_b;  // [G] B of every graph
    int32_t* parent;
    int32_t* size;
    int32_t* minid;
    unsigned long long* keys;
    int32_t* counts;
    unsigned long long* vol;
    unsigned long long* best;
    unsigned long long* acc[2];  // [kAccFields][G] per parity
    double* acc_prf[2];          // [G][3] per parity
    mcd_sweep_stats* stats;
    double* ari;
    double* modularity;
    double* prf;
    int32_t* labels;  // [K][n] or null
    GridSync* sync;
    int64_t n, m, cap;
    int G, K, log2cap;
    unsigned nblocks;
    unsigned long long limit;  // barrier wait limit in wall-clock ticks
    const int32_t* gate;       // nullable: run only when it reads nonzero
    SlotOrder out;
};

// Grid barrier over the resident blocks of k_sweep_levels (a sense-reversing
// central counter): each block's first thread releases the block's writes,
// arrives, and waits for the generation to move on.  Every wait is bounded by
// a wall-clock limit; a block that reaches it records the time-out and from
// then on no block waits any more, so the kernel always ends (its statistics
// are then marked invalid, n_components = -1).
__device__ void grid_sync(const SweepArgs& a) {
    // Every wave waits until its own stores and atomics have completed at the
    // L2: the block barrier alone orders them only within the CU, and the
    // first thread's agent-scope release below writes back the L2 as it
    // stands, so other waves' writes must have reached it by then.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        GridSync* s = a.sync;
        if (!__hip_atomic_load(&s->timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            // Arrival releases the block's writes (complete at the L2, see
            // above); the last block of a group acquires
            // its group's writes and releases them on at the top counter; the
            // last group acquires everything and releases it with the new
            // generation, which every waiting block then acquires.
            const unsigned ng = a.nblocks < kSyncGroups ? a.nblocks : kSyncGroups;
            const unsigned gi = blockIdx.x % ng;
            const unsigned members = a.nblocks / ng + (gi < a.nblocks % ng ? 1u : 0u);
            GridSync::Group* gr = &s->grp[gi];
            const unsigned g = __hip_atomic_load(&gr->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(&gr->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&gr->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (__hip_atomic_fetch_add(&s->top, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == ng - 1) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    __hip_atomic_store(&s->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    for (unsigned h = 0; h < ng; ++h)
                        __hip_atomic_fetch_add(&s->grp[h].gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(&gr->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(4);
                if (wall_clock64() - t0 > a.limit) {
                    __hip_atomic_store(&s->timed_out, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            // acquire every block's released writes (the block barrier below
            // passes them on to the other threads of the block)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
}

// A level that holds most of a single graph's edges (the lowest thresholds)
// is united vertex by vertex, skipping the vertices of one large component,
// after the sampling idea of Sutton et al. (Afforest): (A) every vertex is
// united with up to two of its first eight out-edges at the level, which
// links most vertices of the graph's large component; (B) the root that most
// of 1024 evenly spaced vertices reach is taken as that component's; (C) every
// vertex outside it unites all its edges at the level, out-edges and
// in-edges.  An edge with both endpoints inside the component at the time
// they are looked at joins nothing new (components only grow), and every
// other edge has an endpoint outside, whose lists hold it; so the partition
// equals the edge-by-edge union's.  Each phase ends at a grid barrier.
constexpr int kSampleVerts = 1024;

__device__ void d_union_level_dense(const SweepArgs& a, int lv, unsigned long long* sh) {
    const int64_t n = a.n;
    int32_t* parent = a.parent;
    GRID_STRIDE(x, n) {  // (A)
        const int64_t e0 = a.off[x], e1 = min(a.off[x + 1], e0 + 8);
        int linked = 0;
        for (int64_t e = e0; e < e1 && linked < 2; ++e)
            if (a.level[e] == lv) {
                uf_unite(parent, (int32_t)x, a.adj[e]);
                ++linked;
            }
    }
    grid_sync(a);
    if (blockIdx.x == 0) {  // (B): count the roots of the samples in an LDS table
        int32_t* key = (int32_t*)sh;
        uint32_t* cnt = (uint32_t*)(key + 2 * kSampleVerts);
        for (int i = threadIdx.x; i < 2 * kSampleVerts; i += blockDim.x) {
            key[i] = -1;
            cnt[i] = 0u;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kSampleVerts; i += blockDim.x) {
            const int32_t r = uf_find(parent, (int32_t)((int64_t)i * n / kSampleVerts));
            uint32_t h = ((uint32_t)r * 2654435761u) >> 21;  // 11 bits: 2 kSampleVerts slots
            for (;;) {
                const int32_t k = atomicCAS(&key[h], -1, r);
                if (k == -1 || k == r) break;
                h = (h + 1) & (2 * kSampleVerts - 1);
            }
            atomicAdd(&cnt[h], 1u);
        }
        __syncthreads();
        if (threadIdx.x < 64) {  // the most sampled root (ties: the smaller root)
            uint64_t best = 0;
            for (int i = threadIdx.x; i < 2 * kSampleVerts; i += 64)
                if (key[i] >= 0) {
                    const uint64_t c = ((uint64_t)cnt[i] << 32) | (uint32_t)~(uint32_t)key[i];
                    best = c > best ? c : best;
                }
            for (int o = 32; o > 0; o >>= 1) {
                const uint64_t y = __shfl_xor(best, o);
                best = y > best ? y : best;
            }
            if (threadIdx.x == 0) a.sync->giant = best ? (int32_t)~(uint32_t)best : -1;
        }
        __syncthreads();
    }
    grid_sync(a);
    const int32_t giant = __hip_atomic_load(&a.sync->giant, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    GRID_STRIDE(x, n) {  // (C)
        if (uf_find(parent, (int32_t)x) == giant) continue;
        for (int64_t e = a.off[x]; e < a.off[x + 1]; ++e)
            if (a.level[e] == lv) uf_unite(parent, (int32_t)x, a.adj[e]);
        for (int64_t k = a.in_off[x]; k < a.in_off[x + 1]; ++k) {
            const int32_t e = a.in_ea[k].x;
            if (a.level[e] == lv) uf_unite(parent, (int32_t)x, a.src[e]);
        }
    }
}

// Writes the statistics of threshold i (caller slot a.out.slot[i]) for every
// graph from the accumulator set `p`.
__device__ void d_write_stats(const SweepArgs& a, int i, int p) {
    const int G = a.G, K = a.K;
    const unsigned long long* acc = a.acc[p];
    const bool bad = __hip_atomic_load(&a.sync->timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const int out_i = a.out.slot[i];
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += (int64_t)gridDim.x * blockDim.x) {
        int64_t kept = 0, mg = 0;
        for (int l = 0; l <= K; ++l) {
            const int64_t c = (int64_t)a.hist[g * (K + 1) + l];
            mg += c;
            if (l > i) kept += c;
        }
        auto ld = [&](int field) {
            return (int64_t)__hip_atomic_load(&acc[field * G + g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        mcd_sweep_stats st;
        const int64_t nv = a.vbase[g + 1] - a.vbase[g];
        st.m_kept = kept;
        st.n_components = bad ? -1 : ld(kAccNcc);
        st.largest_component = ld(kAccLargest);
        st.pairs_cluster = ld(kAccA) / 2;
        st.pairs_class = a.cls ? (int64_t)(a.acc_b[g] / 2) : 0;
        st.pairs_both = a.cls ? ld(kAccS) / 2 : 0;
        st.pairs_total = nv * (nv - 1) / 2;
        st.intra_edges = a.modularity ? ld(kAccIntra) : 0;
        st.volume_sq = a.modularity ? ld(kAccVsq) : 0;
        a.stats[g * K + out_i] = st;
        if (a.prf) {
            const double* ap = a.acc_prf[p] + 3 * g;
            double* o = a.prf + (g * K + out_i) * 3;
            const double nn = (double)nv;
            for (int j = 0; j < 3; ++j)
                o[j] = nv ? __hip_atomic_load(&ap[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) / nn : 0.0;
        }
        if (a.modularity) {
            const double mm = (double)mg;
            a.modularity[g * K + out_i] =
                mg == 0 ? 0.0 : (double)st.intra_edges / mm - (double)st.volume_sq / (4.0 * mm * mm);
        }
        if (a.ari) {
            double r = 0.0;
            if (a.cls) {
                const double A = (double)st.pairs_cluster, B = (double)st.pairs_class;
                const double S = (double)st.pairs_both, N = (double)st.pairs_total;
                const double prod = (A * B) / N;
                const double den = 0.5 * (A + B) - prod;
                r = (st.pairs_total == 0 || den == 0.0) ? 1.0 : (S - prod) / den;
            }
            a.ari[g * K + out_i] = r;
        }
    }
}

// The whole level loop in one launch: from the highest threshold down, each
// level's edges are united, then the per-graph statistics of the partition
// are gathered, with grid barriers between the phases that depend on each
// other:
//   U : stats of the previous level | reset this level's accumulators and
//       per-vertex arrays | unite this level's edges
//   P1: roots and sizes (paths compressed) | label minima | (cluster, class)
//       cells | component volumes | intra-component edges
//   P2: A and largest | labels | S | best cells | sum of squared volumes
//   P3: precision / recall / F1 sums (when asked for)
// NT threads per block, at least WPE waves per SIMD (which bounds the
// registers per thread)
// The level loop's arguments live in device memory (written by one tiny
// kernel, so a captured graph holds them by value): read through a pointer,
// they do not occupy registers for the whole kernel.
__global__ void k_store_args(SweepArgs a, SweepArgs* __restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = a;
}

template <int NT, int WPE>
__global__ __launch_bounds__(NT, WPE) void k_sweep_levels(const SweepArgs* __restrict__ ap) {
    const SweepArgs& a = *ap;
    if (gated_off(a.gate)) return;  // uniform over the grid: no block waits for another
    __shared__ unsigned long long sh[kShWords];
    const int64_t n = a.n, m = a.m;
    const int G = a.G;
    for (int i = a.K - 1; i >= 0; --i) {
        const int p = i & 1;
        unsigned long long* acc = a.acc[p];
        if (i < a.K - 1) d_write_stats(a, i + 1, p ^ 1);
        // A level that adds no edge to any graph leaves every partition as it
        // was: its statistics are the previous threshold's (m_kept, the only
        // other input, is read from the level counts when written).  Without
        // label output, the accumulators are copied instead of recomputed.
        // The test reads the same counts in every block, so all skip together.
        if (i < a.K - 1 && !a.labels && G <= kLdsGraphs) {
            bool added = false;
            for (int g = 0; g < G && !added; ++g) added = a.hist[(int64_t)g * (a.K + 1) + i + 1] != 0ull;
            if (!added) {
                GRID_STRIDE(j, (int64_t)kAccFields * G) acc[j] = a.acc[p ^ 1][j];
                if (a.prf) GRID_STRIDE(j, 3 * (int64_t)G) a.acc_prf[p][j] = a.acc_prf[p ^ 1][j];
                grid_sync(a);
                continue;
            }
        }
        GRID_STRIDE(j, (int64_t)kAccFields * G) acc[j] = 0ull;
        if (a.prf) GRID_STRIDE(j, 3 * (int64_t)G) a.acc_prf[p][j] = 0.0;
        GRID_STRIDE(v, n) {
            a.size[v] = 0;
            if (a.modularity) a.vol[v] = 0ull;
            if (a.prf) a.best[v] = 0ull;
            if (a.labels) a.minid[v] = a.perm[v];
        }
        if (a.cls) GRID_STRIDE(h, a.cap) {
            a.keys[h] = ~0ull;
            a.counts[h] = 0;
        }
        // a single graph's level holding more than half its edges goes
        // vertex by vertex (uniform over the grid: every block reads the
        // same count)
        if (m > 0 && G == 1 && 2 * a.hist[i + 1] > (unsigned long long)m)
            d_union_level_dense(a, i + 1, sh);
        else if (m > 0)
            d_union_level(a.src, a.adj, a.level, m, i + 1, a.parent);
        grid_sync(a);
        d_pass_size(a.parent, n, a.gid, G, a.size, acc + kAccNcc * G, sh);
        if (a.labels) d_label_min(a.parent, a.perm, n, a.minid);
        if (a.cls) d_pass_cells(a.parent, n, a.cls, a.keys, a.counts, a.log2cap);
        if (a.modularity) {
            d_pass_volume(a.parent, n, a.deg, a.vol, sh);
            if (m > 0) d_pass_intra(a.src, a.adj, a.level, m, i, a.parent, a.gid, G, acc + kAccIntra * G, sh);
        }
        grid_sync(a);
        d_pass_roots(n, a.gid, G, a.size, acc + kAccA * G, acc + kAccLargest * G, sh);
        if (a.labels) d_label_write(a.parent, a.perm, n, a.minid, a.labels + (int64_t)a.out.slot[i] * n);
        if (a.cls) {
            d_pass_s(a.parent, n, a.gid, G, a.cls, a.keys, a.counts, a.log2cap, acc + kAccS * G, sh);
            if (a.prf) d_cells_best(a.keys, a.counts, a.cap, a.size, a.csize, a.best);
        }
        if (a.modularity) d_pass_vsq(n, a.gid, G, a.vol, acc + kAccVsq * G, sh);
        grid_sync(a);
        if (a.prf) {
            d_prf_sums(n, a.gid, G, a.size, a.csize, a.best, a.acc_prf[p], sh);
            grid_sync(a);
        }
    }
    d_write_stats(a, 0, 0);
}

// One thread per graph: the rule of thumb over the thresholds in ascending
// order (slot[i] = caller slot of the i-th smallest).

__global__ __launch_bounds__(kThreads) void k_sweep_rule(int G, SweepDeltas ds, SlotOrder so,
                                                         const int64_t* __restrict__ vbase,
                                                         const mcd_sweep_stats* __restrict__ stats,
                                                         const double* __restrict__ modularity, int64_t jump_num,
                                                         int64_t jump_den, int32_t* __restrict__ index,
                                                         int64_t* __restrict__ deltas) {
    const int K = ds.K;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
        const int64_t nv = vbase[g + 1] - vbase[g];
        const mcd_sweep_stats* row = stats + (int64_t)g * K;
        // largest increase of the largest component while the threshold falls;
        // the first maximum met walking downwards
        int64_t best_jump = 0;
        int jump_at = -1;
        for (int i = K - 2; i >= 0; --i) {
            const int64_t d = row[so.slot[i]].largest_component - row[so.slot[i + 1]].largest_component;
            if (d > best_jump) {
                best_jump = d;
                jump_at = i;
            }
        }
        int pick = K - 1;
        if (jump_at >= 0 && (__int128)best_jump * jump_den >= (__int128)jump_num * nv) {
            pick = jump_at + 1;
        } else if (modularity) {
            const double* q = modularity + (int64_t)g * K;
            double bq = q[so.slot[K - 1]];
            for (int i = K - 2; i >= 0; --i)
                if (q[so.slot[i]] > bq) {
                    bq = q[so.slot[i]];
                    pick = i;
                }
        }
        index[g] = so.slot[pick];
        if (deltas) {
            deltas[2 * g] = ds.num[pick];
            deltas[2 * g + 1] = ds.den[pick];
        }
    }
}

template <class T>
__global__ void k_fill_t(T* __restrict__ p, int64_t N, T v) {
    GRID_STRIDE(i, N) p[i] = v;
}

template <class T>
void fill_t(T* p, int64_t N, T v, hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_fill_t<T>, dim3(grid_for(N, 8192)), dim3(kThreads), 0, s, p, N, v);
}

int cells_log2(int64_t n) {
    int l = 4;
    while (((int64_t)1 << l) < 2 * n + 16) ++l;
    return l;
}

struct SweepLayout {
    uint8_t* level;
    int32_t* parent;
    int32_t* gid;
    int32_t* cls;
    int32_t* size;
    int32_t* minid;
    int32_t* csize;
    unsigned long long* keys;
    int32_t* counts;
    unsigned long long* hist;    // [G][K+1]
    unsigned long long* acc_b;   // [G]
    unsigned long long* acc[2];  // [kAccFields][G] per parity
    double* acc_prf[2];          // [G][3] per parity
    unsigned long long* vol;     // [n]
    unsigned long long* best;    // [n] (planted labels)
    GridSync* sync;
    SweepArgs* args;
    size_t bytes;
};

SweepLayout sweep_layout(void* p, const mcd_graph* g, int G, int K, bool truth) {
    Carve c{(char*)p, 0, 0};
    SweepLayout L;
    const int64_t n = g->n, m = g->m;
    L.level = c.take<uint8_t>((size_t)m);
    L.parent = c.take<int32_t>((size_t)n);
    L.gid = c.take<int32_t>((size_t)n);
    L.size = c.take<int32_t>((size_t)n);
    L.minid = c.take<int32_t>((size_t)n);
    L.cls = truth ? c.take<int32_t>((size_t)n) : nullptr;
    L.csize = truth ? c.take<int32_t>((size_t)n) : nullptr;
    const int64_t cap = truth ? ((int64_t)1 << cells_log2(n)) : 0;
    L.keys = truth ? c.take<unsigned long long>((size_t)cap) : nullptr;
    L.counts = truth ? c.take<int32_t>((size_t)cap) : nullptr;
    L.hist = c.take<unsigned long long>((size_t)G * (K + 1));
    L.acc_b = c.take<unsigned long long>((size_t)G);
    for (int q = 0; q < 2; ++q) {
        L.acc[q] = c.take<unsigned long long>((size_t)kAccFields * G);
        L.acc_prf[q] = c.take<double>((size_t)3 * G);
    }
    L.vol = c.take<unsigned long long>((size_t)n);
    L.best = truth ? c.take<unsigned long long>((size_t)n) : nullptr;
    L.sync = c.take<GridSync>(1);
    L.args = c.take<SweepArgs>(1);
    L.bytes = c.used;
    return L;
}

// Launch shapes of the level loop (threads per block, waves per SIMD): the
// context parameter sweep_shape picks (1024, 4), (512, 6) or (256, 8); all
// give the same results.
// Blocks of the level loop that are resident at once (by the occupancy
// query, and no more than the work needs), so that every block reaches every
// barrier.
template <int NT, int WPE>
unsigned sweep_blocks(int64_t work) {
    int dev = 0, cus = 1, per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_levels<NT, WPE>, NT, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t b = (int64_t)per_cu * cus;
    const int64_t need = (work + NT - 1) / NT;
    if (need < b) b = need;
    return (unsigned)std::max<int64_t>(b, 1);
}

template <int NT, int WPE>
void launch_levels(SweepArgs& a, SweepArgs* dev_args, int64_t work, hipStream_t s) {
    a.nblocks = sweep_blocks<NT, WPE>(work);
    hipLaunchKernelGGL(k_store_args, dim3(1), dim3(64), 0, s, a, dev_args);
    hipLaunchKernelGGL((k_sweep_levels<NT, WPE>), dim3(a.nblocks), dim3(NT), 0, s, dev_args);
}

// Barrier wait limit: 30 s of the device's constant-rate wall clock.
unsigned long long sweep_wait_limit() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
    return (unsigned long long)khz * 1000ull * 30ull;
}

}  // namespace

size_t sweep_scratch_bytes(const mcd_graph* g, int G, int K, bool truth) {
    return sweep_layout(nullptr, g, G, K, truth).bytes;
}

void launch_sweep(const mcd_graph* g, int measure, const int32_t* t, const SweepDeltas& ds,
                  const int* out_index, int G, const int64_t* vbase, const int32_t* truth,
                  mcd_sweep_stats* stats, double* ari, double* modularity, double* prf, int32_t* labels,
                  void* ws, hipStream_t s, const int32_t* gate) {
    const int K = ds.K;
    if (!truth) prf = nullptr;
    const int64_t n = g->n, m = g->m;
    SweepLayout L = sweep_layout(ws, g, G, K, truth != nullptr);
    const int l2 = truth ? cells_log2(n) : 0;
    const int64_t cap = truth ? ((int64_t)1 << l2) : 0;
    fill_t<unsigned long long>(L.hist, (int64_t)G * (K + 1), 0ull, s);
    fill_t<unsigned long long>(L.acc_b, G, 0ull, s);
    fill_t<int32_t>((int32_t*)L.sync, (int64_t)(sizeof(GridSync) / sizeof(int32_t)), 0, s);
    if (n > 0)
        hipLaunchKernelGGL(k_vertex_info, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, g->perm, n, vbase, G,
                           truth, L.gid, L.cls, gate);
    if (m > 0) {
        // thresholds reach the kernel validated to |num|, den < 2^31
        // LDS for the histogram only as large as it is (a few bins for one
        // graph), so that it does not limit the waves per CU
        const int nbins = G * (K + 1);
        const unsigned lds = nbins <= kLevelBins ? (unsigned)nbins * 4u : 0u;
        if (g->max_deg < (1 << 29))
            hipLaunchKernelGGL(k_level<true>, dim3(grid_for(m, 8192)), dim3(kThreads), lds, s, g->src, g->dsum, t, m,
                               measure, ds, L.level, L.gid, G, L.hist, gate);
        else
            hipLaunchKernelGGL(k_level<false>, dim3(grid_for(m, 8192)), dim3(kThreads), lds, s, g->src, g->dsum, t,
                               m, measure, ds, L.level, L.gid, G, L.hist, gate);
    }
    if (truth && n > 0) {
        fill_t<int32_t>(L.csize, n, 0, s);
        hipLaunchKernelGGL(k_class_size, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.cls, n, L.csize, gate);
        hipLaunchKernelGGL(k_class_b, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.cls, n, L.gid, G,
                           L.csize, L.acc_b, gate);
    }
    if (n > 0)
        hipLaunchKernelGGL(k_init_parent, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent, n, gate);
    SweepArgs a;
    a.src = g->src;
    a.adj = g->adj;
    a.off = g->off;
    a.in_off = g->in_off;
    a.in_ea = g->in_ea;
    a.level = L.level;
    a.perm = g->perm;
    a.deg = g->deg;
    a.gid = L.gid;
    a.cls = truth ? L.cls : nullptr;
    a.csize = L.csize;
    a.vbase = vbase;
    a.hist = L.hist;
    a.acc_b = L.acc_b;
    a.parent = L.parent;
    a.size = L.size;
    a.minid = L.minid;
    a.keys = L.keys;
    a.counts = L.counts;
    a.vol = L.vol;
    a.best = L.best;
    for (int q = 0; q < 2; ++q) {
        a.acc[q] = L.acc[q];
        a.acc_prf[q] = L.acc_prf[q];
    }
    a.stats = stats;
    a.ari = ari;
    a.modularity = modularity;
    a.prf = prf;
    a.labels = labels;
    a.sync = L.sync;
    a.n = n;
    a.m = m;
    a.cap = cap;
    a.G = G;
    a.K = K;
    a.log2cap = l2;
    for (int i = 0; i < K; ++i) a.out.slot[i] = out_index[i];
    const int64_t work = std::max<int64_t>(std::max<int64_t>(n, (m + 15) / 16), std::max<int64_t>(cap, G));
    a.limit = sweep_wait_limit();
    a.gate = gate;
    switch (g->ctx->sweep_shape) {
        case 1: launch_levels<512, 6>(a, L.args, work, s); break;
        case 2: launch_levels<256, 8>(a, L.args, work, s); break;
        default: launch_levels<1024, 4>(a, L.args, work, s); break;
    }
}

void launch_sweep_rule(const SweepDeltas& ds, const int* order, int G, const int64_t* vbase,
                       const mcd_sweep_stats* stats, const double* modularity, int64_t jump_num, int64_t jump_den,
                       int32_t* index, int64_t* deltas, hipStream_t s) {
    SlotOrder so;
    for (int i = 0; i < ds.K; ++i) so.slot[i] = order[i];
    hipLaunchKernelGGL(k_sweep_rule, dim3((G + kThreads - 1) / kThreads), dim3(kThreads), 0, s, G, ds, so, vbase,
                       stats, modularity, jump_num, jump_den, index, deltas);
}

}  // namespace mcd
