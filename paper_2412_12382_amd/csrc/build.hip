// Graph construction kernels: raw pairs -> simple undirected graph -> vertices
// ranked by (degree, id) -> CSR of the orientation from lower to higher rank.
//
// Keys pack two vertex ids in 2*bits bits: (first << bits) | second.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t N, int64_t cap = 65536) {
    int64_t b = (N + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

#define GRID_STRIDE(i, N)                                                              \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (N);          \
         i += (int64_t)gridDim.x * blockDim.x)

// Undirected edge {u,v} of a raw pair as the packed key (min, max); dropped
// pairs (self-loops, ids outside [0,n)) become the sentinel.  Any invalid id
// raises *err.
__global__ __launch_bounds__(kThreads) void k_canon(const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ dst, int64_t P,
                                                    int64_t n, int bits, uint64_t* __restrict__ keys,
                                                    int64_t* __restrict__ err) {
    GRID_STRIDE(i, P) {
        const int64_t u = src[i], v = dst[i];
        const bool bad = u < 0 || u >= n || v < 0 || v >= n;
        if (bad) *err = 1;
        uint64_t k = MCD_SENTINEL;
        if (!bad && u != v) {
            const uint64_t a = (uint64_t)(u < v ? u : v), b = (uint64_t)(u < v ? v : u);
            k = (a << bits) | b;
        }
        keys[i] = k;
    }
}

// deg[x] += the number of occurrences of x in a sequence whose equal values
// are adjacent: the lanes of a wave hold runs of equal values and each run
// adds its length with one atomic (a hub's run would otherwise serialise 64
// same-address atomics per wave; a run crossing waves adds in parts).
template <class T>
__device__ __forceinline__ void add_runs(T x, int32_t* __restrict__ deg) {
    const int lane = threadIdx.x & 63;
    const T prev = __shfl_up(x, 1);
    const bool head = lane == 0 || prev != x;
    const uint64_t heads = __ballot(head);
    const uint64_t active = __ballot(true);
    if (head) {
        // run = lanes from this head up to the next head (or the last active lane)
        const uint64_t above = heads & ~((2ull << lane) - 1ull);
        const int end = above ? __ffsll((long long)above) - 1 : 64 - __clzll((long long)active);
        atomicAdd(&deg[x], end - lane);
    }
}

// Lower endpoints of the unique keys (sorted by lower endpoint).
__global__ __launch_bounds__(kThreads) void k_degree(const uint64_t* __restrict__ uniq, int64_t m,
                                                     int bits, int32_t* __restrict__ deg) {
    GRID_STRIDE(e, m) add_runs<int32_t>((int32_t)(uniq[e] >> bits), deg);
}

__global__ __launch_bounds__(kThreads) void k_upper_ends(const uint64_t* __restrict__ uniq, int64_t m, int bits,
                                                         uint32_t* __restrict__ hi) {
    const uint64_t mask = (1ull << bits) - 1;
    GRID_STRIDE(e, m) hi[e] = (uint32_t)(uniq[e] & mask);
}

// Upper endpoints after sorting: equal values are adjacent.
__global__ __launch_bounds__(kThreads) void k_count_runs(const uint32_t* __restrict__ sorted, int64_t m,
                                                         int32_t* __restrict__ deg) {
    GRID_STRIDE(e, m) add_runs<int32_t>((int32_t)sorted[e], deg);
}

__global__ __launch_bounds__(kThreads) void k_rank_keys(const int32_t* __restrict__ deg, int64_t n,
                                                        int bits, uint64_t* __restrict__ keys) {
    GRID_STRIDE(v, n) keys[v] = ((uint64_t)(uint32_t)deg[v] << bits) | (uint64_t)v;
}

__global__ __launch_bounds__(kThreads) void k_rank_apply(const uint64_t* __restrict__ sorted, int64_t n,
                                                         int bits, const int32_t* __restrict__ deg_orig,
                                                         int32_t* __restrict__ perm,
                                                         int32_t* __restrict__ inv,
                                                         int32_t* __restrict__ deg_new) {
    const uint64_t mask = (1ull << bits) - 1;
    GRID_STRIDE(p, n) {
        const int32_t v = (int32_t)(sorted[p] & mask);
        perm[p] = v;
        inv[v] = (int32_t)p;
        deg_new[p] = deg_orig[v];
    }
}

// dsum[e] = deg u + deg v of every oriented edge (as uint32): the degree term
// of both similarity measures, stored with the CSR so that every weight pass
// streams it instead of gathering two degrees per edge.
__global__ __launch_bounds__(kThreads) void k_edge_dsum(const int32_t* __restrict__ src,
                                                        const int32_t* __restrict__ adj,
                                                        const int32_t* __restrict__ deg, int64_t m,
                                                        int32_t* __restrict__ dsum) {
    GRID_STRIDE(e, m) dsum[e] = (int32_t)((uint32_t)deg[src[e]] + (uint32_t)deg[adj[e]]);
}

__global__ __launch_bounds__(kThreads) void k_orient_keys(const uint64_t* __restrict__ uniq, int64_t m,
                                                          int bits, const int32_t* __restrict__ inv,
                                                          uint64_t* __restrict__ keys) {
    const uint64_t mask = (1ull << bits) - 1;
    GRID_STRIDE(e, m) {
        const uint64_t k = uniq[e];
        const uint32_t a = (uint32_t)inv[k >> bits], c = (uint32_t)inv[k & mask];
        const uint64_t lo = a < c ? a : c, hi = a < c ? c : a;
        keys[e] = (lo << bits) | hi;
    }
}

// Splits sorted oriented keys into src/adj and counts the out-degree of each
// row; lanes of one wave that share a row add their count with one atomic.
__global__ __launch_bounds__(kThreads) void k_csr_fill(const uint64_t* __restrict__ sorted, int64_t m,
                                                       int bits, int32_t* __restrict__ src,
                                                       int32_t* __restrict__ adj,
                                                       int32_t* __restrict__ outdeg) {
    const uint64_t mask = (1ull << bits) - 1;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nround = (m + stride - 1) / stride;
    for (int64_t rd = 0; rd < nround; ++rd) {  // uniform trip count: ballots see the whole wave
        const int64_t e = start + rd * stride;
        const bool valid = e < m;
        int32_t r = -1;
        if (valid) {
            const uint64_t k = sorted[e];
            r = (int32_t)(k >> bits);
            src[e] = r;
            adj[e] = (int32_t)(k & mask);
        }
        const int32_t prev = __shfl_up(r, 1);
        const bool head = valid && (lane == 0 || prev != r);
        const uint64_t heads = __ballot(head);
        const uint64_t vmask = __ballot(valid);
        if (head) {
            const uint64_t after = heads & ~((2ull << lane) - 1ull);
            const int nxt = after ? __builtin_ctzll(after) : (64 - __builtin_clzll(vmask));
            atomicAdd(&outdeg[r], nxt - lane);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_max_i32(const int32_t* __restrict__ a, int64_t N,
                                                      unsigned long long* __restrict__ out) {
    int32_t mx = 0;
    GRID_STRIDE(i, N) mx = max(mx, a[i]);
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)mx);
}

// Words of the triangle count's hit bitmasks for a row of d out-neighbours:
// one bit per suffix element, the suffix after the row's j-th edge having
// d - 1 - j elements, each suffix in whole 64-bit words:
//   sum over L = 0 .. d-1 of ceil(L / 64) = 64 q (q + 1) / 2 + r (q + 1)
// with d - 1 = 64 q + r.
__global__ __launch_bounds__(kThreads) void k_bitmask_words(const int32_t* __restrict__ outdeg, int64_t n,
                                                            unsigned long long* __restrict__ out) {
    unsigned long long sum = 0;
    GRID_STRIDE(v, n) {
        const int64_t d = outdeg[v];
        if (d < 2) continue;
        const int64_t q = (d - 1) >> 6, r = (d - 1) & 63;
        sum += (unsigned long long)(32 * q * (q + 1) + r * (q + 1));
    }
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if ((threadIdx.x & 63) == 0 && sum) atomicAdd(out, sum);
}

__global__ __launch_bounds__(kThreads) void k_edges_orig(const int32_t* __restrict__ src,
                                                         const int32_t* __restrict__ adj,
                                                         const int32_t* __restrict__ perm, int64_t m,
                                                         int32_t* __restrict__ u, int32_t* __restrict__ v) {
    GRID_STRIDE(e, m) {
        u[e] = perm[src[e]];
        v[e] = perm[adj[e]];
    }
}

__global__ __launch_bounds__(kThreads) void k_scatter_by_perm(const int32_t* __restrict__ val,
                                                              const int32_t* __restrict__ perm, int64_t n,
                                                              int32_t* __restrict__ out) {
    GRID_STRIDE(v, n) out[perm[v]] = val[v];
}

__global__ __launch_bounds__(kThreads) void k_in_count(const int32_t* __restrict__ deg,
                                                       const int32_t* __restrict__ outdeg, int64_t n,
                                                       int32_t* __restrict__ in_cnt) {
    GRID_STRIDE(v, n) in_cnt[v] = deg[v] - outdeg[v];
}

// keys[e] = (head << 32) | e, and suf[e] = length of the tail's row after e
// (both in edge order, so the row offsets are read sequentially).
__global__ __launch_bounds__(kThreads) void k_in_keys(const int32_t* __restrict__ src,
                                                      const int32_t* __restrict__ adj,
                                                      const int64_t* __restrict__ off, int64_t m,
                                                      uint64_t* __restrict__ keys, int32_t* __restrict__ suf) {
    GRID_STRIDE(e, m) {
        keys[e] = ((uint64_t)(uint32_t)adj[e] << 32) | (uint64_t)e;
        suf[e] = (int32_t)(off[src[e] + 1] - e - 1);
    }
}

// In-edge lists grouped by head, each in increasing edge id (= increasing
// tail rank): the stable sort of (head, edge id) keys, which carried each
// edge's suffix length along (suf is in sorted order: no gather).
__global__ __launch_bounds__(kThreads) void k_in_fill(const uint64_t* __restrict__ sorted,
                                                      const int32_t* __restrict__ suf, int64_t m,
                                                      int2* __restrict__ in_ea) {
    GRID_STRIDE(i, m) in_ea[i] = make_int2((int32_t)(uint32_t)sorted[i], suf[i]);
}

}  // namespace

void launch_in_count(const int32_t* deg, const int32_t* outdeg, int64_t n, int32_t* in_cnt,
                     hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_in_count, dim3(grid_for(n)), dim3(kThreads), 0, s, deg, outdeg, n, in_cnt);
}

void launch_in_keys(const int32_t* src, const int32_t* adj, const int64_t* off, int64_t m, uint64_t* keys,
                    int32_t* suf, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_in_keys, dim3(grid_for(m)), dim3(kThreads), 0, s, src, adj, off, m, keys, suf);
}

void launch_in_fill(const uint64_t* sorted, const int32_t* suf, int64_t m, int2* in_ea, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_in_fill, dim3(grid_for(m)), dim3(kThreads), 0, s, sorted, suf, m, in_ea);
}

void launch_canon(const int32_t* src, const int32_t* dst, int64_t P, int64_t n, int bits,
                  uint64_t* keys, int64_t* d_err, hipStream_t s) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_canon, dim3(grid_for(P)), dim3(kThreads), 0, s, src, dst, P, n, bits, keys, d_err);
}

void launch_degree(const uint64_t* uniq, int64_t m, int bits, int32_t* deg, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_degree, dim3(grid_for(m)), dim3(kThreads), 0, s, uniq, m, bits, deg);
}

void launch_upper_ends(const uint64_t* uniq, int64_t m, int bits, uint32_t* hi, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_upper_ends, dim3(grid_for(m)), dim3(kThreads), 0, s, uniq, m, bits, hi);
}

void launch_count_runs(const uint32_t* sorted, int64_t m, int32_t* deg, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_count_runs, dim3(grid_for(m)), dim3(kThreads), 0, s, sorted, m, deg);
}

void launch_rank_keys(const int32_t* deg, int64_t n, int bits, uint64_t* keys, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rank_keys, dim3(grid_for(n)), dim3(kThreads), 0, s, deg, n, bits, keys);
}

void launch_rank_apply(const uint64_t* sorted, int64_t n, int bits, const int32_t* deg_orig,
                       int32_t* perm, int32_t* inv, int32_t* deg_new, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rank_apply, dim3(grid_for(n)), dim3(kThreads), 0, s, sorted, n, bits, deg_orig,
                       perm, inv, deg_new);
}

void launch_edge_dsum(const int32_t* src, const int32_t* adj, const int32_t* deg, int64_t m, int32_t* dsum,
                      hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_edge_dsum, dim3(grid_for(m)), dim3(kThreads), 0, s, src, adj, deg, m, dsum);
}

void launch_orient_keys(const uint64_t* uniq, int64_t m, int bits, const int32_t* inv,
                        uint64_t* keys, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_orient_keys, dim3(grid_for(m)), dim3(kThreads), 0, s, uniq, m, bits, inv, keys);
}

void launch_csr_fill(const uint64_t* sorted, int64_t m, int bits, int32_t* src, int32_t* adj,
                     int32_t* outdeg, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_csr_fill, dim3(grid_for(m)), dim3(kThreads), 0, s, sorted, m, bits, src, adj,
                       outdeg);
}

void launch_max_i32(const int32_t* a, int64_t N, int64_t* d_out, hipStream_t s) {
    fill_i64(d_out, 1, 0, s);
    if (N <= 0) return;
    hipLaunchKernelGGL(k_max_i32, dim3(grid_for(N, 4096)), dim3(kThreads), 0, s, a, N,
                       (unsigned long long*)d_out);
}

void launch_bitmask_words(const int32_t* outdeg, int64_t n, int64_t* d_out, hipStream_t s) {
    fill_i64(d_out, 1, 0, s);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bitmask_words, dim3(grid_for(n, 4096)), dim3(kThreads), 0, s, outdeg, n,
                       (unsigned long long*)d_out);
}

void launch_edges_orig(const int32_t* src, const int32_t* adj, const int32_t* perm, int64_t m,
                       int32_t* u, int32_t* v, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_edges_orig, dim3(grid_for(m)), dim3(kThreads), 0, s, src, adj, perm, m, u, v);
}

void launch_scatter_by_perm(const int32_t* val, const int32_t* perm, int64_t n, int32_t* out,
                            hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_by_perm, dim3(grid_for(n)), dim3(kThreads), 0, s, val, perm, n, out);
}

}  // namespace mcd
