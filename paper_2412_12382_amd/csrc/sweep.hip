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

template <bool NARROW>
__global__ __launch_bounds__(kThreads) void k_level(const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ dsum,
                                                    const int32_t* __restrict__ t, int64_t m, int measure,
                                                    SweepDeltas ds, uint8_t* __restrict__ level,
                                                    const int32_t* __restrict__ gid, int G,
                                                    unsigned long long* __restrict__ hist) {
    extern __shared__ uint32_t h[];  // nbins counters when local (sized at launch)
    const int nbins = G * (ds.K + 1);
    const bool local = nbins <= kLevelBins;
    const int lane = threadIdx.x & 63;
    if (local)
        for (int i = threadIdx.x; i < nbins; i += blockDim.x) h[i] = 0;
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
            const int c = NARROW ? rat_cmp64(num, den, ds.num[mid], ds.den[mid])
                                 : rat_cmp(num, den, ds.num[mid], ds.den[mid]);
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
                                                          int32_t* __restrict__ gid, int32_t* __restrict__ cls) {
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

__global__ __launch_bounds__(kThreads) void k_init_parent(int32_t* __restrict__ parent, int64_t n) {
    GRID_STRIDE(v, n) parent[v] = (int32_t)v;
}

// unite the endpoints of every edge at level lv.  Every level scans all m
// level bytes, most of them for a handful of edges, so the bytes are read 16
// at a time and a group without a match is passed over with one test.
__device__ __forceinline__ bool has_byte(uint32_t x, uint32_t pat) {
    const uint32_t v = x ^ pat;  // a zero byte where x matches
    return ((v - 0x01010101u) & ~v & 0x80808080u) != 0u;
}

__global__ __launch_bounds__(kThreads) void k_union_level(const int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ adj,
                                                          const uint8_t* __restrict__ level, int64_t m,
                                                          int lv, int32_t* parent) {
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

// Pass 1 over vertices: compress to the root, count roots per graph, size of
// every component.
__global__ __launch_bounds__(kThreads) void k_pass_size(int32_t* parent, int64_t n,
                                                        const int32_t* __restrict__ gid, int G,
                                                        int32_t* __restrict__ size,
                                                        unsigned long long* __restrict__ ncc) {
    __shared__ unsigned long long gl[kLdsGraphs];
    __shared__ int32_t rk[kRootSlots];
    __shared__ uint32_t rv[kRootSlots];
    GraphAcc acc{G <= kLdsGraphs ? gl : nullptr, ncc, G};
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
}

// Labels of one threshold: the smallest original id of every component.
__global__ __launch_bounds__(kThreads) void k_label_init(const int32_t* __restrict__ perm, int64_t n,
                                                         int32_t* __restrict__ minid) {
    GRID_STRIDE(v, n) minid[v] = perm[v];
}

__global__ __launch_bounds__(kThreads) void k_label_min(int32_t* parent, const int32_t* __restrict__ perm, int64_t n,
                                                        int32_t* __restrict__ minid) {
    GRID_STRIDE(v, n) {
        const int32_t r = uf_find(parent, (int32_t)v);
        if (r != (int32_t)v) atomicMin(&minid[r], perm[v]);
    }
}

__global__ __launch_bounds__(kThreads) void k_label_write(int32_t* parent, const int32_t* __restrict__ perm,
                                                          int64_t n, const int32_t* __restrict__ minid,
                                                          int32_t* __restrict__ labels) {
    GRID_STRIDE(v, n) labels[perm[v]] = minid[uf_find(parent, (int32_t)v)];
}

__device__ __forceinline__ uint64_t cell_key(int32_t r, int32_t c) {
    return ((uint64_t)(uint32_t)r << 32) | (uint32_t)c;
}

__device__ __forceinline__ uint32_t cell_slot(uint64_t k, int log2cap) {
    return (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> (64 - log2cap));
}

// Pass 2: A (same cluster pairs) and the largest component per graph, read
// off the component sizes: after pass 1 only roots hold a nonzero size, and
// a root's graph is its own.  Streams size[] and gid[] once.
__global__ __launch_bounds__(kThreads) void k_pass_roots(int64_t n, const int32_t* __restrict__ gid, int G,
                                                         const int32_t* __restrict__ size,
                                                         unsigned long long* __restrict__ acc_a,
                                                         unsigned long long* __restrict__ largest) {
    __shared__ unsigned long long la[kLdsGraphs], ll[kLdsGraphs];
    const bool lds = G <= kLdsGraphs;
    GraphAcc A{lds ? la : nullptr, acc_a, G}, Lg{lds ? ll : nullptr, largest, G};
    A.init();
    Lg.init();
    __syncthreads();
    GRID_STRIDE(v, n) {
        const int32_t sz = size[v];
        const int32_t g = gid[v];
        A.add(g, (unsigned long long)sz * (unsigned long long)(sz > 0 ? sz - 1 : 0));
        Lg.max(g, (unsigned long long)sz);
    }
    __syncthreads();
    A.flush_add();
    Lg.flush_max();
}

// Pass 2b (with labels): count every (cluster, class) cell in a hash table.
__global__ __launch_bounds__(kThreads) void k_pass_cells(int32_t* parent, int64_t n,
                                                         const int32_t* __restrict__ cls,
                                                         unsigned long long* __restrict__ keys,
                                                         int32_t* __restrict__ counts, int log2cap) {
    const int lane = threadIdx.x & 63;
    GRID_STRIDE(v, n) {
        // pass 1 compressed the paths, but a concurrent halving may have left
        // parent[v] at an ancestor below the root: always follow to the root
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

// Pass 3: S (pairs sharing cluster and class) per graph.
__global__ __launch_bounds__(kThreads) void k_pass_s(int32_t* parent, int64_t n,
                                                     const int32_t* __restrict__ gid, int G,
                                                     const int32_t* __restrict__ cls,
                                                     const unsigned long long* __restrict__ keys,
                                                     const int32_t* __restrict__ counts, int log2cap,
                                                     unsigned long long* __restrict__ acc_s) {
    __shared__ unsigned long long ls[kLdsGraphs];
    GraphAcc S{G <= kLdsGraphs ? ls : nullptr, acc_s, G};
    S.init();
    __syncthreads();
    GRID_STRIDE(v, n) {
        const uint64_t k = cell_key(uf_find(parent, (int32_t)v), cls[v]);
        const uint32_t mask = (1u << log2cap) - 1u;
        uint32_t h = cell_slot(k, log2cap);
        while (keys[h] != k) h = (h + 1) & mask;
        S.add(gid[v], (unsigned long long)(counts[h] - 1));
    }
    __syncthreads();
    S.flush_add();
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
__global__ __launch_bounds__(kThreads) void k_cells_best(const unsigned long long* __restrict__ keys,
                                                         const int32_t* __restrict__ counts, int64_t cap,
                                                         const int32_t* __restrict__ size,
                                                         const int32_t* __restrict__ csize,
                                                         unsigned long long* best) {
    GRID_STRIDE(h, cap) {
        const unsigned long long k = keys[h];
        if (k == ~0ull) continue;
        const int32_t r = (int32_t)(k >> 32), c = (int32_t)(uint32_t)k;
        const int64_t x = counts[h], sz = size[r], b = csize[c];
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

__global__ __launch_bounds__(kThreads) void k_prf_sums(int64_t n, const int32_t* __restrict__ gid, int G,
                                                       const int32_t* __restrict__ size,
                                                       const int32_t* __restrict__ csize,
                                                       const unsigned long long* __restrict__ best,
                                                       double* __restrict__ acc) {
    __shared__ double lp[3 * 256];
    const bool lds = G <= 256;
    if (lds)
        for (int i = threadIdx.x; i < 3 * G; i += blockDim.x) lp[i] = 0.0;
    __syncthreads();
    GRID_STRIDE(v, n) {
        const int32_t sz = size[v];
        if (sz == 0) continue;  // not a root
        const unsigned long long rec = best[v];
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
}

// class sizes (truth ids lie in [0, n)), then B per graph
__global__ __launch_bounds__(kThreads) void k_class_size(const int32_t* __restrict__ cls, int64_t n,
                                                         int32_t* __restrict__ csize) {
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
                                                      unsigned long long* __restrict__ acc_b) {
    __shared__ unsigned long long lb[kLdsGraphs];
    GraphAcc B{G <= kLdsGraphs ? lb : nullptr, acc_b, G};
    B.init();
    __syncthreads();
    GRID_STRIDE(v, n) B.add(gid[v], (unsigned long long)(csize[cls[v]] - 1));
    __syncthreads();
    B.flush_add();
}

// Modularity (the quality measure of the paper's threshold rule of thumb) of
// the partition at this threshold, on the input graph:
//   Q = sum over components c of e_c / m - (vol_c / 2m)^2,
// with e_c the input edges inside c and vol_c the sum of input degrees over c.
// vol[root] accumulates the degrees of each component (wave-aggregated, big
// components through the block's LDS table like the sizes).
__global__ __launch_bounds__(kThreads) void k_pass_volume(int32_t* parent, int64_t n,
                                                          const int32_t* __restrict__ deg,
                                                          unsigned long long* __restrict__ vol) {
    __shared__ int32_t rk[kRootSlots];
    __shared__ unsigned long long rv[kRootSlots];
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
        bool done = r == r0;
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
}

// Per graph: the input edges whose endpoints share a component at threshold
// slot lv_thresh (kept edges always do; a pruned edge iff its endpoints have
// one root), and the sum over components of vol_c^2.
__global__ __launch_bounds__(kThreads) void k_pass_intra(const int32_t* __restrict__ src,
                                                         const int32_t* __restrict__ adj,
                                                         const uint8_t* __restrict__ level, int64_t m,
                                                         int lv_thresh, int32_t* parent,
                                                         const int32_t* __restrict__ gid, int G,
                                                         unsigned long long* __restrict__ acc_intra) {
    __shared__ unsigned long long li[kLdsGraphs];
    GraphAcc I{G <= kLdsGraphs ? li : nullptr, acc_intra, G};
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
}

__global__ __launch_bounds__(kThreads) void k_pass_vsq(int64_t n, const int32_t* __restrict__ gid, int G,
                                                       const unsigned long long* __restrict__ vol,
                                                       unsigned long long* __restrict__ acc_vsq) {
    __shared__ unsigned long long lq[kLdsGraphs];
    GraphAcc Q{G <= kLdsGraphs ? lq : nullptr, acc_vsq, G};
    Q.init();
    __syncthreads();
    GRID_STRIDE(v, n) {
        const unsigned long long x = vol[v];  // nonzero only at roots
        Q.add(gid[v], x * x);
    }
    __syncthreads();
    Q.flush_add();
}

// Writes the statistics of threshold slot `out_i` for every graph.
__global__ __launch_bounds__(kThreads) void k_write_stats(int G, int K, int lv_thresh, int out_i,
                                                          const unsigned long long* __restrict__ hist,
                                                          const unsigned long long* __restrict__ ncc,
                                                          const unsigned long long* __restrict__ largest,
                                                          const unsigned long long* __restrict__ acc_a,
                                                          const unsigned long long* __restrict__ acc_s,
                                                          const unsigned long long* __restrict__ acc_b,
                                                          const unsigned long long* __restrict__ acc_intra,
                                                          const unsigned long long* __restrict__ acc_vsq,
                                                          const int64_t* __restrict__ vbase, int has_truth,
                                                          mcd_sweep_stats* __restrict__ stats,
                                                          double* __restrict__ ari, double* __restrict__ modularity,
                                                          const double* __restrict__ acc_prf,
                                                          double* __restrict__ prf) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
        int64_t kept = 0, mg = 0;
        for (int l = 0; l <= K; ++l) {
            const int64_t c = (int64_t)hist[(int64_t)g * (K + 1) + l];
            mg += c;
            if (l > lv_thresh) kept += c;
        }
        mcd_sweep_stats st;
        const int64_t nv = vbase[g + 1] - vbase[g];
        st.m_kept = kept;
        st.n_components = (int64_t)ncc[g];
        st.largest_component = (int64_t)largest[g];
        st.pairs_cluster = (int64_t)(acc_a[g] / 2);
        st.pairs_class = has_truth ? (int64_t)(acc_b[g] / 2) : 0;
        st.pairs_both = has_truth ? (int64_t)(acc_s[g] / 2) : 0;
        st.pairs_total = nv * (nv - 1) / 2;
        st.intra_edges = modularity ? (int64_t)acc_intra[g] : 0;
        st.volume_sq = modularity ? (int64_t)acc_vsq[g] : 0;
        stats[(int64_t)g * K + out_i] = st;
        if (prf) {
            double* o = prf + ((int64_t)g * K + out_i) * 3;
            const double nn = (double)nv;
            o[0] = nv ? acc_prf[3 * g] / nn : 0.0;
            o[1] = nv ? acc_prf[3 * g + 1] / nn : 0.0;
            o[2] = nv ? acc_prf[3 * g + 2] / nn : 0.0;
        }
        if (modularity) {
            const double mm = (double)mg;
            modularity[(int64_t)g * K + out_i] =
                mg == 0 ? 0.0 : (double)st.intra_edges / mm - (double)st.volume_sq / (4.0 * mm * mm);
        }
        if (ari) {
            double r = 0.0;
            if (has_truth) {
                const double A = (double)st.pairs_cluster, B = (double)st.pairs_class;
                const double S = (double)st.pairs_both, N = (double)st.pairs_total;
                const double prod = (A * B) / N;
                const double den = 0.5 * (A + B) - prod;
                r = (st.pairs_total == 0 || den == 0.0) ? 1.0 : (S - prod) / den;
            }
            ari[(int64_t)g * K + out_i] = r;
        }
    }
}

// One thread per graph: the rule of thumb over the thresholds in ascending
// order (slot[i] = caller slot of the i-th smallest).
struct SlotOrder {
    int slot[MCD_SWEEP_MAX];
};

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
    unsigned long long* ncc;     // [G]
    unsigned long long* largest; // [G]
    unsigned long long* acc_a;   // [G]
    unsigned long long* acc_s;   // [G]
    unsigned long long* acc_b;   // [G]
    unsigned long long* acc_intra;  // [G]
    unsigned long long* acc_vsq;    // [G]
    unsigned long long* vol;        // [n]
    unsigned long long* best;       // [n] (planted labels)
    double* acc_prf;                // [G][3]
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
    L.ncc = c.take<unsigned long long>((size_t)G);
    L.largest = c.take<unsigned long long>((size_t)G);
    L.acc_a = c.take<unsigned long long>((size_t)G);
    L.acc_s = c.take<unsigned long long>((size_t)G);
    L.acc_b = c.take<unsigned long long>((size_t)G);
    L.acc_intra = c.take<unsigned long long>((size_t)G);
    L.acc_vsq = c.take<unsigned long long>((size_t)G);
    L.vol = c.take<unsigned long long>((size_t)n);
    L.best = truth ? c.take<unsigned long long>((size_t)n) : nullptr;
    L.acc_prf = c.take<double>((size_t)3 * G);
    L.bytes = c.used;
    return L;
}

}  // namespace

size_t sweep_scratch_bytes(const mcd_graph* g, int G, int K, bool truth) {
    return sweep_layout(nullptr, g, G, K, truth).bytes;
}

void launch_sweep(const mcd_graph* g, int measure, const int32_t* t, const SweepDeltas& ds,
                  const int* out_index, int G, const int64_t* vbase, const int32_t* truth,
                  mcd_sweep_stats* stats, double* ari, double* modularity, double* prf, int32_t* labels,
                  void* ws, hipStream_t s) {
    const int K = ds.K;
    if (!truth) prf = nullptr;
    const int64_t n = g->n, m = g->m;
    SweepLayout L = sweep_layout(ws, g, G, K, truth != nullptr);
    const int l2 = truth ? cells_log2(n) : 0;
    const int64_t cap = truth ? ((int64_t)1 << l2) : 0;
    fill_t<unsigned long long>(L.hist, (int64_t)G * (K + 1), 0ull, s);
    fill_t<unsigned long long>(L.acc_b, G, 0ull, s);
    if (n > 0)
        hipLaunchKernelGGL(k_vertex_info, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, g->perm, n, vbase, G,
                           truth, L.gid, L.cls);
    if (m > 0) {
        // thresholds reach the kernel validated to |num|, den < 2^31
        // LDS for the histogram only as large as it is (a few bins for one
        // graph), so that it does not limit the waves per CU
        const int nbins = G * (K + 1);
        const unsigned lds = nbins <= kLevelBins ? (unsigned)nbins * 4u : 0u;
        if (g->max_deg < (1 << 29))
            hipLaunchKernelGGL(k_level<true>, dim3(grid_for(m, 8192)), dim3(kThreads), lds, s, g->src, g->dsum, t, m,
                               measure, ds, L.level, L.gid, G, L.hist);
        else
            hipLaunchKernelGGL(k_level<false>, dim3(grid_for(m, 8192)), dim3(kThreads), lds, s, g->src, g->dsum, t,
                               m, measure, ds, L.level, L.gid, G, L.hist);
    }
    if (truth && n > 0) {
        fill_t<int32_t>(L.csize, n, 0, s);
        hipLaunchKernelGGL(k_class_size, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.cls, n, L.csize);
        hipLaunchKernelGGL(k_class_b, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.cls, n, L.gid, G,
                           L.csize, L.acc_b);
    }
    if (n > 0) hipLaunchKernelGGL(k_init_parent, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent, n);
    for (int i = K - 1; i >= 0; --i) {
        if (m > 0)
            hipLaunchKernelGGL(k_union_level, dim3(grid_for(m, 16384)), dim3(kThreads), 0, s, g->src, g->adj,
                               L.level, m, i + 1, L.parent);
        fill_t<unsigned long long>(L.ncc, G, 0ull, s);
        fill_t<unsigned long long>(L.largest, G, 0ull, s);
        fill_t<unsigned long long>(L.acc_a, G, 0ull, s);
        fill_t<unsigned long long>(L.acc_s, G, 0ull, s);
        fill_t<int32_t>(L.size, n, 0, s);
        if (modularity) {
            fill_t<unsigned long long>(L.acc_intra, G, 0ull, s);
            fill_t<unsigned long long>(L.acc_vsq, G, 0ull, s);
            fill_t<unsigned long long>(L.vol, n, 0ull, s);
        }
        int32_t* lab = labels ? labels + (int64_t)out_index[i] * n : nullptr;
        if (n > 0) {
            hipLaunchKernelGGL(k_pass_size, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent, n, L.gid, G,
                               L.size, L.ncc);
            if (lab) {
                hipLaunchKernelGGL(k_label_init, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, g->perm, n,
                                   L.minid);
                hipLaunchKernelGGL(k_label_min, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent, g->perm,
                                   n, L.minid);
                hipLaunchKernelGGL(k_label_write, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent,
                                   g->perm, n, L.minid, lab);
            }
            if (truth) {
                fill_t<unsigned long long>(L.keys, cap, ~0ull, s);
                fill_t<int32_t>(L.counts, cap, 0, s);
            }
            hipLaunchKernelGGL(k_pass_roots, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, n, L.gid, G, L.size,
                               L.acc_a, L.largest);
            if (modularity) {
                hipLaunchKernelGGL(k_pass_volume, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent, n, g->deg,
                                   L.vol);
                hipLaunchKernelGGL(k_pass_vsq, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, n, L.gid, G, L.vol,
                                   L.acc_vsq);
                if (m > 0)
                    hipLaunchKernelGGL(k_pass_intra, dim3(grid_for(m, 8192)), dim3(kThreads), 0, s, g->src, g->adj,
                                       L.level, m, i, L.parent, L.gid, G, L.acc_intra);
            }
            if (truth) {
                hipLaunchKernelGGL(k_pass_cells, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent, n,
                                   L.cls, L.keys, L.counts, l2);
                hipLaunchKernelGGL(k_pass_s, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.parent, n, L.gid, G,
                                   L.cls, L.keys, L.counts, l2, L.acc_s);
                if (prf) {
                    fill_t<unsigned long long>(L.best, n, 0ull, s);
                    fill_t<double>(L.acc_prf, 3 * (int64_t)G, 0.0, s);
                    hipLaunchKernelGGL(k_cells_best, dim3(grid_for(cap, 8192)), dim3(kThreads), 0, s, L.keys, L.counts,
                                       cap, L.size, L.csize, L.best);
                    hipLaunchKernelGGL(k_prf_sums, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, n, L.gid, G, L.size,
                                       L.csize, L.best, L.acc_prf);
                }
            }
        }
        hipLaunchKernelGGL(k_write_stats, dim3((G + kThreads - 1) / kThreads), dim3(kThreads), 0, s, G, K, i,
                           out_index[i], L.hist, L.ncc, L.largest, L.acc_a, L.acc_s, L.acc_b, L.acc_intra,
                           L.acc_vsq, vbase, truth ? 1 : 0, stats, ari, modularity, L.acc_prf, prf);
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
