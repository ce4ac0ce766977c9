// Edge similarities (Table tab:simfunctions) and the prune step of Algorithm 1.
//
// With D = deg u + deg v: Tectonic(e) = t / D, TW(e) = 3t - D + 2 (t - wedge
// with |N(u) u N(v)| = D - t, Eq. eq:tw and the notation paragraph of Sec. 1),
// K3(e) = t (triangles on the edge), K4(e) = the 4-clique count (passed in
// place of t) and Jaccard(e) = t / (D - t).  Every
// similarity is an exact rational sn / sd and the keep decision never uses
// floating point: with delta = num/den (den > 0) an edge is kept iff
// sn * den >= num * sd, in 64- or 128-bit integers.
#include "common.hpp"
#include "unionfind.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int graph_of(const int64_t* __restrict__ vbase, int G, int64_t x) {
    int lo = 0, hi = G;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (vbase[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// t / d in fp32 (Tectonic, Jaccard), defined as the fp64 quotient rounded to
// fp32.  While both integers fit 24 bits they are exact fp32 values and the
// single fp32 division gives the same result (double rounding of one
// division of 24-bit operands through 53 bits is innocuous, 53 >= 2 * 24 + 2),
// so it is the correctly rounded quotient.  Wider operands (degree sums of
// 2^24 or more) take the fp64 route itself; there the value can differ from
// the correctly rounded quotient by one ulp, but it is still the defined one.
__device__ __forceinline__ float ratio_f32(int32_t t, int64_t d) {
    if (t < (1 << 24) && d < (1 << 24)) return (float)t / (float)d;
    return (float)((double)t / (double)d);
}

constexpr int kUnroll = 8;  // 64-edge groups in flight per wave

// A device threshold whose terms fit the 64-bit products of keep_test<true>.
__device__ __forceinline__ bool small_delta(int64_t num, int64_t den) {
    return num > -(1ll << 31) && num < (1ll << 31) && den < (1ll << 31);
}

// The exact keep test sn / sd >= num / den (sd, den > 0).  64-bit products
// suffice when |sn| < 2^31, sd < 2^32 and |num|, den < 2^31 (NARROW, which
// the host establishes from the maximum degree and a validated threshold);
// otherwise 128-bit products are used.

template <bool NARROW>
__device__ __forceinline__ bool keep_test(int64_t sn, int64_t sd, int64_t num, int64_t den) {
    if (NARROW) return sn * den >= num * sd;
    return (__int128)sn * den >= (__int128)num * sd;
}

// One pass of weights + prune.  Wave `seg` owns edges [seg L, seg L + L),
// L a multiple of 64, in groups of 64 (one edge per lane); a group's keep
// decisions form one 64-bit ballot = two keep words, and its kept edges are
// appended, in edge order, at the wave's running count inside the wave's own
// run of the kept-pair array, so the compaction needs no atomics.  The
// degree sum deg u + deg v of every edge comes from the graph (dsum), so the
// pass streams its inputs.
//
// UNION (the fused weights + prune + components pass): instead of being
// listed, kept edges are united in the union-find `parent`: the kept edge ids
// of the wave's 8 groups in flight are compacted in LDS, then all lanes fetch
// their endpoints and unite them, 64 edges per round, so a round never runs
// with a few lanes.  The wave walks its run from the end, so that the edges
// among high-degree vertices (the high ranks) are united first and the rest
// hooks straight under the roots that core forms.
//
// Endpoints are streamed with t and dsum only where every edge needs them (a
// graph lookup); the kept list and the queue read them for kept edges alone.
// THR: 0 one host threshold (num0 / den0, validated); 1 one device threshold
// (deltas[0..1], read once per wave); 2 a device threshold per graph of a
// batch (deltas[2 g .. 2 g + 1], the graph found from vbase).  Only THR 2
// carries the endpoints and the graph lookup through the loop.
template <int MEASURE, int THR, bool NARROW, bool UNION>
__global__ __launch_bounds__(kThreads) void k_weigh_prune(
    const int32_t* __restrict__ src, const int32_t* __restrict__ adj, const int32_t* __restrict__ dsum,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ t, int64_t m, int64_t seg_len, int G,
    const int64_t* __restrict__ vbase, const int64_t* __restrict__ deltas, int64_t num0, int64_t den0,
    float* __restrict__ wf, int32_t* __restrict__ wi, uint32_t* __restrict__ keep, int2* __restrict__ kept,
    int32_t* __restrict__ kept_counts, unsigned long long* __restrict__ n_kept, int32_t* parent) {
    __shared__ unsigned long long wsum[kThreads / 64];
    __shared__ int32_t queue[UNION ? kThreads / 64 : 1][UNION ? 64 * kUnroll : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t seg = (int64_t)blockIdx.x * (kThreads / 64) + w;
    const int64_t e0 = seg * seg_len;
    const int64_t e1 = e0 + seg_len < m ? e0 + seg_len : m;
    const uint64_t below = (1ull << lane) - 1ull;
    constexpr bool need_uv = THR == 2;
    // one threshold for every edge: read once (a device threshold of one
    // graph too), not per edge
    int64_t num1 = num0, den1 = den0;
    if (THR == 1) {
        num1 = deltas[0];
        den1 = deltas[1];
    }
    const bool narrow1 = THR == 0 || small_delta(num1, den1);
    const int64_t ng = e1 > e0 ? (e1 - e0 + 63) >> 6 : 0;  // 64-edge groups of the run
    int64_t cnt = 0;
    for (int64_t gi = 0; gi < ng; gi += kUnroll) {
        int32_t u[kUnroll], v[kUnroll], tt[kUnroll], dd[kUnroll];
        int nq = 0;  // kept edges of this iteration queued for union (wave-uniform)
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int64_t gj = UNION ? ng - 1 - (gi + j) : gi + j;
            const int64_t e = gi + j < ng ? e0 + 64 * gj + lane : e1;
            u[j] = v[j] = tt[j] = 0;
            dd[j] = 1;
            if (e < e1) {
                tt[j] = __builtin_nontemporal_load(&t[e]);  // streamed once: no reuse to cache
                dd[j] = __builtin_nontemporal_load(&dsum[e]);
                if (need_uv) {
                    u[j] = src[e];
                    v[j] = adj[e];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            if (gi + j >= ng) break;  // wave-uniform
            const int64_t cj = e0 + 64 * (UNION ? ng - 1 - (gi + j) : gi + j);
            const int64_t e = cj + lane;
            bool k = false;
            if (e < e1) {
                const int64_t D = (uint32_t)dd[j];  // deg u + deg v < 2^32
                int64_t sn, sd;
                if (MEASURE == MCD_SIM_TECTONIC || MEASURE == MCD_SIM_JACCARD) {
                    sn = tt[j];
                    sd = MEASURE == MCD_SIM_TECTONIC ? D : D - tt[j];  // D - t >= t + 2 > 0
                    if (wf) __builtin_nontemporal_store(ratio_f32(tt[j], sd), &wf[e]);
                } else {
                    sn = MEASURE == MCD_SIM_TW ? 3 * (int64_t)tt[j] - D + 2 : (int64_t)tt[j];
                    sd = 1;
                    if (wi) __builtin_nontemporal_store((int32_t)sn, &wi[e]);
                    if (wf) __builtin_nontemporal_store((float)sn, &wf[e]);
                }
                if (THR == 2) {
                    const int g = graph_of(vbase, G, perm[u[j]]);
                    const int64_t num = deltas[2 * g], den = deltas[2 * g + 1];
                    k = small_delta(num, den) ? keep_test<NARROW>(sn, sd, num, den)
                                              : keep_test<false>(sn, sd, num, den);
                } else {
                    k = narrow1 ? keep_test<NARROW>(sn, sd, num1, den1) : keep_test<false>(sn, sd, num1, den1);
                }
            }
            const uint64_t bal = __ballot(k);
            if (keep) {
                if (lane == 0) keep[cj >> 5] = (uint32_t)bal;
                else if (lane == 1 && cj + 32 < m) keep[(cj >> 5) + 1] = (uint32_t)(bal >> 32);
            }
            if (kept && k) {
                if (!need_uv) {
                    u[j] = src[e];
                    v[j] = adj[e];
                }
                kept[e0 + cnt + __popcll(bal & below)] = make_int2(u[j], v[j]);
            }
            if (UNION && k) queue[w][nq + __popcll(bal & below)] = (int32_t)e;  // e < m < 2^31
            nq += __popcll(bal);
            cnt += __popcll(bal);
        }
        if (UNION && nq > 0) {  // wave-uniform
            // the queue was written by other lanes of this wave: order the
            // LDS writes before the reads (one wave: no barrier needed)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int r = lane; r < nq; r += 64) {
                const int32_t e = queue[w][r];
                uf_unite(parent, src[e], adj[e]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();  // reads done before the next writes
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            nq = 0;
        }
    }
    if (kept_counts && lane == 0) kept_counts[seg] = (int32_t)cnt;
    if (!n_kept) return;
    if (lane == 0) wsum[w] = (unsigned long long)cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < kThreads / 64; ++i) s += wsum[i];
        if (s) atomicAdd(n_kept, s);
    }
}

}  // namespace

int64_t kept_segment_len(int64_t m) {
    const int64_t groups = (m + 63) / 64;
    return 64 * ((groups + MCD_KEPT_SEGMENTS - 1) / MCD_KEPT_SEGMENTS);
}

void launch_weigh_prune(const mcd_graph* g, int measure, const int32_t* t, int64_t num, int64_t den, int G,
                        const int64_t* vbase, const int64_t* deltas, float* wf, int32_t* wi, uint32_t* keep_bits,
                        int32_t* kept_pairs, int32_t* kept_counts, int64_t* n_kept, hipStream_t s, int32_t* parent) {
    if (n_kept) fill_i64(n_kept, 1, 0, s);
    if (g->m <= 0 && !kept_counts) return;
    // |TW| < 2^31 and deg u + deg v < 2^30 whenever every degree is below 2^29;
    // host thresholds are validated to |num|, den < 2^31
    const bool narrow = g->max_deg < (1 << 29);
    const int64_t L = kept_segment_len(g->m);
    const dim3 grid(MCD_KEPT_SEGMENTS / (kThreads / 64)), block(kThreads);
    // 0: host threshold, 1: one device threshold, 2: per-graph device thresholds
    const int thr = deltas == nullptr ? 0 : (G == 1 ? 1 : 2);
    int2* kp = (int2*)kept_pairs;
    unsigned long long* nk = (unsigned long long*)n_kept;
#define MCD_WP_ARGS                                                                                          \
    g->src, g->adj, g->dsum, g->perm, t, g->m, L, G, vbase, deltas, num, den, wf, wi, keep_bits, kp, kept_counts, \
        nk, parent
#define MCD_WP_LAUNCH_U(MEAS, THR, UNION)                                                                      \
    do {                                                                                                     \
        if (narrow) hipLaunchKernelGGL((k_weigh_prune<MEAS, THR, true, UNION>), grid, block, 0, s, MCD_WP_ARGS); \
        else hipLaunchKernelGGL((k_weigh_prune<MEAS, THR, false, UNION>), grid, block, 0, s, MCD_WP_ARGS);      \
    } while (0)
#define MCD_WP_LAUNCH_T(MEAS, THR)                          \
    do {                                                \
        if (parent) MCD_WP_LAUNCH_U(MEAS, THR, true);   \
        else MCD_WP_LAUNCH_U(MEAS, THR, false);         \
    } while (0)
#define MCD_WP_LAUNCH(MEAS)                                   \
    do {                                                      \
        if (thr == 0) MCD_WP_LAUNCH_T(MEAS, 0);               \
        else if (thr == 1) MCD_WP_LAUNCH_T(MEAS, 1);          \
        else MCD_WP_LAUNCH_T(MEAS, 2);                        \
    } while (0)
    switch (measure) {
        case MCD_SIM_TECTONIC:
            MCD_WP_LAUNCH(MCD_SIM_TECTONIC);
            break;
        case MCD_SIM_TW:
            MCD_WP_LAUNCH(MCD_SIM_TW);
            break;
        case MCD_SIM_K3:
        case MCD_SIM_K4:  // the count array passed as t
            MCD_WP_LAUNCH(MCD_SIM_K3);
            break;
        default:
            MCD_WP_LAUNCH(MCD_SIM_JACCARD);
            break;
    }
#undef MCD_WP_LAUNCH
#undef MCD_WP_LAUNCH_T
#undef MCD_WP_LAUNCH_U
#undef MCD_WP_ARGS
}

void launch_prune_graphs(const mcd_graph* g, int measure, const int32_t* t, int G, const int64_t* vbase,
                         const int64_t* deltas, uint32_t* keep_bits, int64_t* n_kept, hipStream_t s) {
    launch_weigh_prune(g, measure, t, 0, 1, G, vbase, deltas, nullptr, nullptr, keep_bits, nullptr, nullptr,
                       n_kept, s);
}

void launch_weights(const mcd_graph* g, int measure, const int32_t* t, float* wf, int32_t* wi,
                    hipStream_t s) {
    launch_weigh_prune(g, measure, t, 0, 1, 1, nullptr, nullptr, wf, wi, nullptr, nullptr, nullptr, nullptr, s);
}

void launch_prune(const mcd_graph* g, int measure, const int32_t* t, int64_t num, int64_t den,
                  uint32_t* keep_bits, int64_t* n_kept, hipStream_t s) {
    launch_weigh_prune(g, measure, t, num, den, 1, nullptr, nullptr, nullptr, nullptr, keep_bits, nullptr, nullptr,
                       n_kept, s);
}

}  // namespace mcd
