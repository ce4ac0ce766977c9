// Per-edge triangle counts t(u,v) = |N(u) n N(v)| on the degree-ordered
// orientation.
//
// Vertices are numbered by rank, every edge points from the lower to the
// higher id, and row x of the CSR lists N+(x) in increasing id.  A triangle
// {u < v < w} is found exactly once: at the edge u->v, as an element w of the
// part of N+(u) after v that also lies in N+(v).  The work is organised around
// the middle vertex v: a work item is v together with a slice of its in-edges
// u->v.  The workgroup hashes N+(v) into LDS (key w -> position in N+(v)) and
// every wave streams, for one in-edge at a time, the suffix of row u after v
// in 64-element coalesced chunks, probing each element.  A hit w credits
//     t(u,v) : one atomic per in-edge (wave ballot count),
//     t(u,w) : a global atomic at the suffix position (same cache lines just read),
//     t(v,w) : an LDS counter of v's row, flushed once per work item.
// The probe count is the sum over edges of |suffix of N+(u) after v|, the
// smallest list the intersection needs to scan.  All increments are integer
// atomics, so the counts do not depend on scheduling.
//
// Items are grouped by |N+(v)| into LDS size classes (a wave, two waves or
// four waves per item); rows longer than the largest class (or than the
// configured cap) take a binary-search path.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;

struct Item {
    int32_t v;
    int32_t len;  // in-edges of this item
    int64_t s;    // first in-edge slot (index into in_ea)
};

__device__ __forceinline__ void add_relaxed(int32_t* p, int32_t x) {
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Hash table of N+(v) in LDS.  PACKED (every key of the row lies within 2^20
// ranks above v): one 32-bit word per slot, ((w - v - 1) << 12) | position, so
// a single LDS read yields key and position; the slot is the key's low bits
// folded once, which is collision-free when the row's rank range fits the
// table (the dense rows of the highest-ranked vertices).  WIDE: separate key
// and 16-bit position arrays for rows that span more ranks.
template <int LOG2S, bool PACKED>
struct RowHash;

// Fibonacci hashing: spreads runs of consecutive ranks over the table, so
// linear-probe clusters stay short.
template <int LOG2S>
__device__ __forceinline__ uint32_t fib_slot(uint32_t x) {
    return (x * 0x9E3779B1u) >> (32 - LOG2S);
}

template <int LOG2S>
struct RowHash<LOG2S, true> {
    static constexpr int S = 1 << LOG2S;
    uint32_t tab[S];
    static __device__ __forceinline__ uint32_t slot_of(uint32_t r) { return fib_slot<LOG2S>(r); }
    __device__ __forceinline__ void prepare(int, int, int32_t) {}
    __device__ __forceinline__ void clear(int tid, int nt) {
        for (int i = tid; i < S; i += nt) tab[i] = 0xffffffffu;
    }
    __device__ __forceinline__ void insert(int32_t w, int32_t v, int j) {
        const uint32_t r = (uint32_t)(w - v - 1);
        uint32_t h = slot_of(r);
        const uint32_t ent = (r << 12) | (uint32_t)j;
        while (atomicCAS(&tab[h], 0xffffffffu, ent) != 0xffffffffu) h = (h + 1) & (S - 1);
    }
    // position of w in the row, or -1
    __device__ __forceinline__ int find(int32_t w, int32_t v) const {
        const uint32_t r = (uint32_t)(w - v - 1);
        uint32_t h = slot_of(r);
        for (;;) {
            const uint32_t e = tab[h];
            if (e == 0xffffffffu) return -1;
            if ((e >> 12) == r) return (int)(e & 4095u);
            h = (h + 1) & (S - 1);
        }
    }
};

template <int LOG2S>
struct RowHash<LOG2S, false> {
    static constexpr int S = 1 << LOG2S;
    int32_t keys[S];
    uint16_t pos[S];
    static __device__ __forceinline__ uint32_t slot_of(uint32_t r) { return fib_slot<LOG2S>(r); }
    __device__ __forceinline__ void prepare(int, int, int32_t) {}
    __device__ __forceinline__ void clear(int tid, int nt) {
        for (int i = tid; i < S; i += nt) keys[i] = -1;
    }
    __device__ __forceinline__ void insert(int32_t w, int32_t, int j) {
        uint32_t h = slot_of((uint32_t)w);
        while (atomicCAS(&keys[h], -1, w) != -1) h = (h + 1) & (S - 1);
        pos[h] = (uint16_t)j;
    }
    __device__ __forceinline__ int find(int32_t w, int32_t) const {
        uint32_t h = slot_of((uint32_t)w);
        for (;;) {
            const int32_t k = keys[h];
            if (k == w) return pos[h];
            if (k == -1) return -1;
            h = (h + 1) & (S - 1);
        }
    }
};

// Rank window of N+(v) in LDS, for rows whose ranks all lie in (v, v + 2^LOG2R]:
// bit r of the bitmap marks rank v + 1 + r, and pre[k] counts the set bits
// before word k, so a lookup is two independent LDS reads (word and prefix)
// and a popcount, with no probe loop.  The prefix pass needs the whole
// workgroup (one item per workgroup).
template <int LOG2R>
struct RowWindow {
    static constexpr int NW = (1 << LOG2R) / 32;
    uint32_t bm[NW];
    uint16_t pre[NW];
    uint32_t part[4];
    __device__ __forceinline__ void clear(int tid, int nt) {
        for (int i = tid; i < NW; i += nt) bm[i] = 0;
    }
    __device__ __forceinline__ void insert(int32_t w, int32_t v, int) {
        const uint32_t r = (uint32_t)(w - v - 1);
        atomicOr(&bm[r >> 5], 1u << (r & 31));
    }
    // exclusive prefix of popcounts over the words that can hold ranks <= v + R
    __device__ __forceinline__ void prepare(int tid, int nt, int32_t R) {
        const int nw = (R + 31) >> 5;
        const int per = (nw + nt - 1) / nt;
        const int w0 = tid * per, w1 = min(nw, w0 + per);
        uint32_t s = 0;
        for (int i = w0; i < w1; ++i) s += __popc(bm[i]);
        uint32_t x = s;  // inclusive wave scan
        const int lane = tid & 63;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) part[tid >> 6] = x;
        __syncthreads();
        uint32_t run = x - s;
        for (int k = 0; k < (tid >> 6); ++k) run += part[k];
        for (int i = w0; i < w1; ++i) {
            pre[i] = (uint16_t)run;
            run += __popc(bm[i]);
        }
    }
    __device__ __forceinline__ int find(int32_t w, int32_t v) const {
        const uint32_t r = (uint32_t)(w - v - 1);
        const uint32_t word = bm[r >> 5];
        const uint32_t p0 = pre[r >> 5];
        const uint32_t bit = 1u << (r & 31);
        if (!(word & bit)) return -1;
        return (int)(p0 + __popc(word & (bit - 1u)));
    }
};

// One item per WPI waves; 4/WPI items per workgroup.  LOG2S: log2 of hash
// slots (rows up to 2^(LOG2S-1) out-neighbours).  Each wave is split into
// 64/G groups of G lanes; a group walks its own in-edges (static stride inside
// the item) and streams each suffix G elements at a time, loading the next
// chunk and the next in-edge descriptor ahead of use.  t(v,w) partial counts
// live in LDS as packed 16-bit halves (an item has at most 65535 in-edges, so
// a half cannot carry).
template <class Table, int MAXB, int WPI, int G>
__global__ __launch_bounds__(kThreads) void k_tc_items(const Item* __restrict__ all_items,
                                                       const int64_t* __restrict__ heads, int cls,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ adj,
                                                       const int2* __restrict__ in_ea,
                                                       int32_t* __restrict__ t) {
    constexpr int NI = 4 / WPI;
    constexpr int GPW = 64 / G;
    constexpr int NGI = WPI * GPW;  // groups per item
    __shared__ Table hash[NI];
    __shared__ uint32_t cnt[NI][MAXB / 2];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = wave / WPI;
    const int wsub = wave % WPI;
    const int tsub = threadIdx.x % (64 * WPI);
    const int gl = lane % G, gi = lane / G;
    const int gid = wsub * GPW + gi;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (gi * G));
    const Item* __restrict__ items = all_items + heads[2 * cls];
    const int64_t n_items = heads[2 * cls + 1];
    Table& H = hash[slot];

    for (int64_t base = (int64_t)blockIdx.x * NI; base < n_items; base += (int64_t)gridDim.x * NI) {
        const int64_t it = base + slot;
        const bool have = it < n_items;
        int64_t s = 0, b0 = 0;
        int32_t B = 0, len = 0, v = 0;
        if (have) {
            const Item I = items[it];
            s = I.s;
            len = I.len;
            v = I.v;
            b0 = off[v];
            B = (int32_t)(off[v + 1] - b0);
        }
        H.clear(tsub, 64 * WPI);
        for (int i = tsub; i < MAXB / 2; i += 64 * WPI) cnt[slot][i] = 0;
        __syncthreads();
        int32_t maxv = -1;
        if (have) {
            for (int j = tsub; j < B; j += 64 * WPI) H.insert(adj[b0 + j], v, j);
            maxv = adj[b0 + B - 1];
        }
        __syncthreads();
        H.prepare(tsub, 64 * WPI, maxv - v);  // window: rank range actually used
        __syncthreads();
        if (have) {
            const int64_t kend = s + len;
            int64_t k = s + gid;
            bool done = k >= kend;
            int2 cur = done ? make_int2(0, 0) : in_ea[k];
            int2 nxt = (k + NGI < kend) ? in_ea[k + NGI] : make_int2(0, 0);
            int64_t cursor = (int64_t)cur.x + 1, end = cursor + cur.y;
            int32_t wn = (!done && cursor + gl < end) ? adj[cursor + gl] : INT32_MAX;
            uint32_t c = 0;
            for (;;) {
                if (__ballot(!done) == 0) break;
                const int64_t i = cursor + gl;
                const bool valid = !done && i < end;
                const int32_t w = valid ? wn : INT32_MAX;
                cursor += G;
                // next chunk of this suffix, in flight while this one is probed
                wn = (!done && cursor + gl < end) ? adj[cursor + gl] : INT32_MAX;
                const bool cand = valid && w <= maxv;
                const uint64_t cb = __ballot(cand);
                bool hit = false;
                if (cand) {
                    const int p = H.find(w, v);
                    if (p >= 0) {
                        hit = true;
                        atomicAdd(&cnt[slot][p >> 1], 1u << ((p & 1) * 16));
                        add_relaxed(&t[i], 1);
                    }
                }
                c += (uint32_t)__popcll(__ballot(hit) & gmask);
                // suffix sorted ascending: once no lane of the group holds a
                // candidate, nothing later in this suffix can match
                const bool fin = !done && (cursor >= end || (cb & gmask) == 0);
                if (fin) {
                    if (gl == 0 && c) add_relaxed(&t[cur.x], (int32_t)c);
                    c = 0;
                    k += NGI;
                    if (k >= kend) {
                        done = true;
                    } else {
                        cur = nxt;
                        cursor = (int64_t)cur.x + 1;
                        end = cursor + cur.y;
                        wn = (cursor + gl < end) ? adj[cursor + gl] : INT32_MAX;
                        nxt = (k + NGI < kend) ? in_ea[k + NGI] : make_int2(0, 0);
                    }
                }
            }
        }
        __syncthreads();
        if (have) {
            for (int j = tsub; j < B; j += 64 * WPI) {
                const uint32_t x = (cnt[slot][j >> 1] >> ((j & 1) * 16)) & 0xffffu;
                if (x) add_relaxed(&t[b0 + j], (int32_t)x);
            }
        }
        __syncthreads();
    }
}

// Rank-window items, one item per workgroup of NT threads.  The wave is split
// into 64/G lane groups, each walking its own in-edges G suffix elements per
// step, and every group keeps the descriptor and first chunk of its next
// in-edge loaded ahead.  Group state lives in vector registers; the loop runs
// while any group has work.  Wide windows take large workgroups so that the
// LDS they need still leaves room for enough waves per CU.  (Measured on
// R-MAT: G = 64 is fastest; smaller groups put more rows in flight but cost
// more per element.)
template <int LOG2R, int NT, int G>
__global__ __launch_bounds__(NT) void k_tc_window_g(const Item* __restrict__ all_items,
                                                    const int64_t* __restrict__ heads, int cls,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ adj,
                                                    const int2* __restrict__ in_ea,
                                                    int32_t* __restrict__ t) {
    constexpr int NW = (1 << LOG2R) / 32;
    constexpr int MAXB = 4096;
    constexpr int NWAVES = NT / 64;
    constexpr int NG = 64 / G;
    __shared__ uint32_t bm[NW];
    __shared__ uint16_t pre[NW];
    __shared__ uint32_t part[NWAVES];
    __shared__ uint32_t cnt[MAXB / 2];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int gl = lane % G, gi = lane / G;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (gi * G));
    const Item* __restrict__ items = all_items + heads[2 * cls];
    const int64_t n_items = heads[2 * cls + 1];

    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item I = items[it];
        const int32_t v = I.v;
        const int32_t b0 = (int32_t)off[v];
        const int32_t B = (int32_t)(off[v + 1] - b0);
        for (int i = tid; i < NW; i += NT) bm[i] = 0;
        for (int i = tid; i < MAXB / 2; i += NT) cnt[i] = 0;
        __syncthreads();
        for (int j = tid; j < B; j += NT) {
            const uint32_t r = (uint32_t)(adj[b0 + j] - v - 1);
            atomicOr(&bm[r >> 5], 1u << (r & 31));
        }
        const int32_t maxv = adj[b0 + B - 1];
        __syncthreads();
        {  // exclusive prefix of popcounts over the words in use
            const int nw = (maxv - v + 31) >> 5;
            const int per = (nw + NT - 1) / NT;
            const int w0 = tid * per, w1 = min(nw, w0 + per);
            uint32_t sum = 0;
            for (int i = w0; i < w1; ++i) sum += __popc(bm[i]);
            uint32_t x = sum;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            if (lane == 63) part[wave] = x;
            __syncthreads();
            uint32_t run = x - sum;
            for (int k = 0; k < wave; ++k) run += part[k];
            for (int i = w0; i < w1; ++i) {
                pre[i] = (uint16_t)run;
                run += __popc(bm[i]);
            }
        }
        __syncthreads();

        const int32_t kend = (int32_t)I.s + I.len;
        constexpr int32_t kstride = NWAVES * NG;
        int32_t k = (int32_t)I.s + wave * NG + gi;
        // current in-edge of the group
        bool live = k < kend;
        int2 d = live ? in_ea[k] : make_int2(0, 0);
        int32_t e = d.x, cb = d.x + 1, a1 = d.x + 1 + d.y;
        int32_t w = (live && gl < d.y) ? adj[cb + gl] : INT32_MAX;
        // next in-edge, loaded ahead
        int32_t kn = k + kstride;
        int2 dn = kn < kend ? in_ea[kn] : make_int2(0, 0);
        int32_t wfirst = (kn < kend && gl < dn.y) ? adj[dn.x + 1 + gl] : INT32_MAX;
        uint32_t c = 0;
        while (__ballot(live) != 0) {
            const int32_t i = cb + gl;
            const int32_t nxt = i + G;
            const int32_t wn = (live && nxt < a1) ? adj[nxt] : INT32_MAX;
            const bool cand = live && i < a1 && w <= maxv;
            bool hit = false;
            if (cand) {
                const uint32_t r = (uint32_t)(w - v - 1);
                const uint32_t word = bm[r >> 5];
                const uint32_t bit = 1u << (r & 31);
                if (word & bit) {
                    const uint32_t p = (uint32_t)pre[r >> 5] + __popc(word & (bit - 1u));
                    hit = true;
                    atomicAdd(&cnt[p >> 1], 1u << ((p & 1u) * 16u));
                    add_relaxed(&t[i], 1);
                }
            }
            c += (uint32_t)__popcll(__ballot(hit) & gmask);
            const bool any = (__ballot(cand) & gmask) != 0;
            if (live) {
                if (any && cb + G < a1) {  // more of this suffix
                    cb += G;
                    w = wn;
                } else {  // in-edge done: credit t(u,v), move to the prefetched next one
                    if (gl == 0 && c) add_relaxed(&t[e], (int32_t)c);
                    c = 0;
                    k = kn;
                    live = k < kend;
                    e = dn.x;
                    cb = dn.x + 1;
                    a1 = dn.x + 1 + dn.y;
                    w = wfirst;
                    kn = k + kstride;
                    dn = kn < kend ? in_ea[kn] : make_int2(0, 0);
                    wfirst = (kn < kend && gl < dn.y) ? adj[dn.x + 1 + gl] : INT32_MAX;
                }
            }
        }
        __syncthreads();
        for (int j = tid; j < B; j += NT) {
            const uint32_t x = (cnt[j >> 1] >> ((j & 1) * 16)) & 0xffffu;
            if (x) add_relaxed(&t[b0 + j], (int32_t)x);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int64_t lower_bound(const int32_t* __restrict__ a, int64_t lo, int64_t hi,
                                               int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Rows too long for LDS: one thread per in-edge u->v, each suffix element of
// N+(u) searched in N+(v) (searches move right).
__global__ __launch_bounds__(kThreads) void k_tc_search(const Item* __restrict__ all_items,
                                                        const int64_t* __restrict__ heads, int cls,
                                                        const int64_t* __restrict__ off,
                                                        const int32_t* __restrict__ adj,
                                                        const int2* __restrict__ in_ea,
                                                        int32_t* __restrict__ t) {
    const Item* __restrict__ items = all_items + heads[2 * cls];
    const int64_t n_items = heads[2 * cls + 1];
    for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const Item I = items[it];
        const int64_t bb = off[I.v], be = off[I.v + 1];
        for (int64_t k = I.s + threadIdx.x; k < I.s + I.len; k += blockDim.x) {
            const int2 ea = in_ea[k];
            const int64_t e = ea.x;
            const int64_t a1 = e + 1 + ea.y;
            int64_t b = bb;
            int32_t c = 0;
            for (int64_t i = e + 1; i < a1 && b < be; ++i) {
                const int32_t w = adj[i];
                b = lower_bound(adj, b, be, w);
                if (b < be && adj[b] == w) {
                    add_relaxed(&t[i], 1);
                    add_relaxed(&t[b], 1);
                    ++c;
                    ++b;
                }
            }
            if (c) add_relaxed(&t[e], c);
        }
    }
}

// Work-item classes:
//   0..3  hash, packed entries (row within 2^20 ranks above v), by row length
//   4..7  hash, wide entries, by row length
//   8..10 rank window of 2^14, 2^16, 2^18 ranks (rows longer than 128)
//   11    binary search (rows longer than the LDS cap)
constexpr int kClasses = 12;
constexpr int kSearch = 11;
constexpr int kWindowLog2[3] = {14, 16, 18};

// In-edges per work item: at least the row length (the hash build is then at
// most half the item's cost) and at most 65535 (16-bit LDS counters).
__host__ __device__ inline int64_t item_size(int64_t chunk, int64_t B) {
    int64_t cs = chunk > B ? chunk : B;
    return cs > 65535 ? 65535 : cs;
}
constexpr int kMaxB[4] = {128, 512, 2048, 4096};

// Number of work items of vertex v in each class (one class is non-zero).
__global__ __launch_bounds__(kThreads) void k_item_count(const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ adj,
                                                         const int64_t* __restrict__ in_off, int64_t n,
                                                         int64_t chunk, int64_t lds_max,
                                                         int64_t packed_range, int64_t window_max,
                                                         int32_t* __restrict__ cnt) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t B = off[v + 1] - off[v];
        const int64_t I = in_off[v + 1] - in_off[v];
        int cls = -1;
        if (B > 0 && I > 0) {
            cls = kSearch;
            if (B <= lds_max) {
                for (int c = 3; c >= 0; --c)
                    if (B <= kMaxB[c]) cls = c;
                if (n - 1 - v > packed_range) cls += 4;
                // rank range of the row: its last (largest) element minus v
                const int64_t R = (int64_t)adj[off[v + 1] - 1] - v;
                if (B > kMaxB[0] && window_max > 0) {
                    for (int c = 2; c >= 0; --c)
                        if (R <= ((int64_t)1 << kWindowLog2[c]) && R <= window_max) cls = 8 + c;
                }
            }
        }
        const int64_t cs = item_size(chunk, B);
        const int32_t k = cls >= 0 ? (int32_t)((I + cs - 1) / cs) : 0;
        for (int c = 0; c < kClasses; ++c) cnt[(int64_t)c * n + v] = (c == cls) ? k : 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_item_fill(const int64_t* __restrict__ off,
                                                        const int64_t* __restrict__ in_off, int64_t n,
                                                        int64_t chunk, const int32_t* __restrict__ cnt,
                                                        const int64_t* __restrict__ base,
                                                        Item* __restrict__ items) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < kClasses; ++c) {
            const int32_t k = cnt[(int64_t)c * n + v];
            if (!k) continue;
            // class lists are laid out one after another: base of class c is
            // the total of the earlier classes
            int64_t b = base[(int64_t)c * (n + 1) + v];
            for (int cc = 0; cc < c; ++cc) b += base[(int64_t)cc * (n + 1) + n];
            const int64_t cs = item_size(chunk, off[v + 1] - off[v]);
            const int64_t i0 = in_off[v], i1 = in_off[v + 1];
            for (int32_t j = 0; j < k; ++j) {
                Item I;
                I.v = (int32_t)v;
                I.s = i0 + (int64_t)j * cs;
                I.len = (int32_t)min(cs, i1 - I.s);
                items[b + j] = I;
            }
        }
    }
}

// Offsets of the class lists and their lengths, on the device.
__global__ void k_item_heads(const int64_t* __restrict__ base, int64_t n, int64_t* __restrict__ heads) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    for (int c = 0; c < kClasses; ++c) {
        const int64_t len = base[(int64_t)c * (n + 1) + n];
        heads[2 * c] = acc;
        heads[2 * c + 1] = len;
        acc += len;
    }
}

inline unsigned grid_for(int64_t N, int64_t cap) {
    int64_t b = (N + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

struct TcLayout {
    int32_t* cnt;    // [kClasses][n]
    int64_t* base;   // [kClasses][n+1]
    Item* items;     // [max items]
    int64_t* heads;  // [2*kClasses]: start, length per class
    void* scan;
    size_t bytes;
};

TcLayout tc_layout(void* p, const mcd_graph* g, int64_t chunk) {
    Carve c{(char*)p, 0, 0};
    TcLayout L;
    const int64_t n = g->n;
    const int64_t max_items = n + g->m / item_size(chunk, 0) + 1;  // items hold >= item_size(chunk, 0) in-edges
    L.cnt = c.take<int32_t>((size_t)kClasses * n);
    L.base = c.take<int64_t>((size_t)kClasses * (n + 1));
    L.items = c.take<Item>((size_t)max_items);
    L.heads = c.take<int64_t>(2 * kClasses);
    L.scan = c.take<char>(scan_scratch_bytes(n));
    L.bytes = c.used;
    return L;
}

template <class Table, int MAXB, int WPI, int G>
void launch_class(const mcd_graph* g, const TcLayout& L, int c, int64_t chunk, int32_t* t, hipStream_t s) {
    constexpr int NI = 4 / WPI;
    // grid-stride over the class list; its length is read on the device
    const int64_t cap_items = g->n + g->m / item_size(chunk, 0) + 1;
    int64_t blocks = (cap_items + NI - 1) / NI;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL((k_tc_items<Table, MAXB, WPI, G>), dim3((unsigned)blocks), dim3(kThreads), 0, s,
                       L.items, L.heads, c, g->off, g->adj, g->in_ea, t);
}

template <int LOG2R, int NT, int G>
void launch_window_g(const mcd_graph* g, const TcLayout& L, int c, int64_t chunk, int32_t* t, hipStream_t s) {
    const int64_t cap_items = g->n + g->m / item_size(chunk, 0) + 1;
    int64_t blocks = cap_items < 16384 ? cap_items : 16384;
    hipLaunchKernelGGL((k_tc_window_g<LOG2R, NT, G>), dim3((unsigned)blocks), dim3(NT), 0, s, L.items, L.heads, c,
                       g->off, g->adj, g->in_ea, t);
}

}  // namespace

size_t tc_scratch_bytes(const mcd_graph* g, int64_t chunk) { return tc_layout(nullptr, g, chunk).bytes; }

void launch_triangles(const mcd_graph* g, int32_t* t, void* ws, int64_t chunk, int64_t lds_max,
                      int64_t packed_range, int64_t window_max, hipStream_t s) {
    fill_i32(t, g->m, 0, s);
    if (g->m <= 0 || g->n <= 0) return;
    if (chunk < 1) chunk = 1;
    TcLayout L = tc_layout(ws, g, chunk);
    const int64_t n = g->n;
    hipLaunchKernelGGL(k_item_count, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, g->off, g->adj, g->in_off,
                       n, chunk, lds_max, packed_range, window_max, L.cnt);
    for (int c = 0; c < kClasses; ++c)
        exclusive_scan_i32_i64(L.cnt + (int64_t)c * n, n, L.base + (int64_t)c * (n + 1), L.scan, s);
    hipLaunchKernelGGL(k_item_fill, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, g->off, g->in_off, n,
                       chunk, L.cnt, L.base, L.items);
    hipLaunchKernelGGL(k_item_heads, dim3(1), dim3(64), 0, s, L.base, n, L.heads);
    launch_class<RowHash<8, true>, 128, 1, 16>(g, L, 0, chunk, t, s);
    launch_class<RowHash<10, true>, 512, 2, 64>(g, L, 1, chunk, t, s);
    launch_class<RowHash<12, true>, 2048, 4, 64>(g, L, 2, chunk, t, s);
    launch_class<RowHash<13, true>, 4096, 4, 64>(g, L, 3, chunk, t, s);
    launch_class<RowHash<8, false>, 128, 1, 16>(g, L, 4, chunk, t, s);
    launch_class<RowHash<10, false>, 512, 2, 64>(g, L, 5, chunk, t, s);
    launch_class<RowHash<12, false>, 2048, 4, 64>(g, L, 6, chunk, t, s);
    launch_class<RowHash<13, false>, 4096, 4, 64>(g, L, 7, chunk, t, s);
    launch_window_g<14, 512, 64>(g, L, 8, chunk, t, s);
    launch_window_g<16, 1024, 64>(g, L, 9, chunk, t, s);
    launch_window_g<18, 1024, 64>(g, L, 10, chunk, t, s);
    hipLaunchKernelGGL(k_tc_search, dim3(4096), dim3(kThreads), 0, s, L.items, L.heads, kSearch, g->off,
                       g->adj, g->in_ea, t);
}

}  // namespace mcd
