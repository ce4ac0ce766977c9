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
// in coalesced chunks, probing each element.  A hit w credits
//     t(v,w) : an LDS counter of v's row, flushed once per work item;
//     t(u,v) and t(u,w): in the rank-window classes (almost all the work),
//              the wave's hit ballot of each chunk is stored as one 64-bit
//              word of the in-edge's hit bitmask, and a second pass over the
//              rows of u turns the bitmasks into counts (t(u,w) as column
//              sums, t(u,v) as popcounts) with plain stores; in the smaller
//              classes, global atomics (one per in-edge for t(u,v), one per
//              hit for t(u,w)).
// Device-scope atomics on a multi-XCD GPU are carried out at the memory side,
// one request per cache line touched, so the bitmasks replace about 10^10
// atomic requests by 8-byte stores.  The probe count is the sum over edges of
// |suffix of N+(u) after v|, the smallest list the intersection needs to
// scan.  Every count is an integer sum, so the result does not depend on
// scheduling.
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
                                                       int32_t* __restrict__ t, int ipart, int nparts) {
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

    // this launch takes the groups of NI items g = ipart (mod nparts)
    for (int64_t base = ((int64_t)blockIdx.x * nparts + ipart) * NI; base < n_items;
         base += (int64_t)gridDim.x * nparts * NI) {
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

// The chunks a wave streams for the rank-window kernel: `left` more in-edge
// descriptors at dp, dp + stride, ... of its item, and for the current one
// the suffix [pos, a1) of row u after v in chunks of 64 E consecutive
// elements (E per lane).  Descriptors are fetched 64 at a time, one per lane
// (bx, by), and read out lane by lane into scalar registers; every other
// field is wave-uniform.
template <int E>
struct ChunkGen {
    const int2* __restrict__ dp;
    const int64_t* __restrict__ wbase;  // first word of every edge's hit bitmask
    int32_t left, stride, e, pos, a1, bi;
    int32_t bx, by;  // per lane: a batch of descriptors
    int64_t bw;      // per lane: the bitmask base of the lane's descriptor
    int64_t wb;      // bitmask base of the current in-edge
    bool done;
    // move to the next non-empty chunk
    __device__ __forceinline__ void next(int lane) {
        pos += 64 * E;
        while (pos >= a1) {
            if (left == 0) {
                done = true;
                return;
            }
            if (bi == 64) {
                const int2 d = lane < left ? dp[lane * stride] : make_int2(0, 0);
                bx = d.x;
                by = d.y;
                bw = lane < left ? wbase[d.x] : 0;
                dp += 64 * stride;
                bi = 0;
                // wait for the batch here (vmcnt(0)), once per 64 in-edges:
                // the lane reads below then carry no wait, and the chunk
                // loads in flight in the ring are not drained at every
                // in-edge
                __builtin_amdgcn_s_waitcnt(0x0F70);
            }
            e = __builtin_amdgcn_readlane(bx, bi);
            const int32_t len = __builtin_amdgcn_readlane(by, bi);
            const uint32_t wlo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)bw, bi);
            const uint32_t whi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(bw >> 32), bi);
            wb = (int64_t)(((uint64_t)whi << 32) | wlo);
            ++bi;
            --left;
            pos = e + 1;
            a1 = e + 1 + len;
        }
    }
    // first bitmask word of the current chunk (one word per 64 elements)
    __device__ __forceinline__ int64_t word() const { return wb + ((pos - e - 1) >> 6); }
};

// v_writelane_b32: `old` with lane `lane` replaced by the wave-uniform `val`
// (the compiler's intrinsic; clang has no builtin name for it).
__device__ int32_t writelane(int32_t val, int32_t lane, int32_t old) __asm("llvm.amdgcn.writelane.i32");

// Element 64 k + lane of the generator's current chunk (lanes past its end
// repeat its last element), loaded from the chunk's first element `base` at
// byte offset min(ob, last) where ob = (64 k + lane) * sizeof(element) and
// last is the byte offset of the chunk's last element; a finished generator
// reads element 0 of the adjacency (the kernel runs only on graphs with
// edges), so that every slot of the ring below issues the same loads and the
// wait for a slot's data counts the loads issued after it.  T16: from the
// 16-bit copy of the adjacency (adj16[e] = adj[e] - top16 for the top 65,536
// ranks), for items whose suffixes lie entirely in that range; the element is
// returned as stored and the probe adds top16 with the rank offset.  (The
// compiler zero-extends the 16-bit ring at the top of the ring's loop, which
// waits there for the loads of all D slots: a wait per D chunks.  Variants
// without that wait read 4 bytes from a 2-byte boundary, or 32-bit elements,
// and were slower.)
template <bool T16>
__device__ __forceinline__ int32_t load_elem(const void* __restrict__ base, uint32_t last, uint32_t ob) {
    const uint32_t o = ob < last ? ob : last;
    const char* __restrict__ p = (const char*)base + o;
    if (T16) return (int32_t)*(const uint16_t*)p;
    return *(const int32_t*)p;
}

// Rows of N+(v) for the walking kernel below, held in LDS by the workgroup.
// build() enters them (the whole workgroup, ending with a barrier) and
// returns the per-item constants the probes need; probe() tells whether a
// suffix element is in the row, position() where (called for hits only).
//
// Rank window, for rows whose ranks all lie in (v, v + 2^LOG2R]: bit r of the
// bitmap marks rank v + 1 + r, beside each 32-bit word the number of set bits
// before it.  Up to 2^16 ranks a word and its prefix sit side by side (one
// address for both); the 2^18 window keeps 16-bit prefixes apart, so that two
// workgroups still fit a CU's LDS.  Word NW stays zero: lanes with nothing to
// probe look up rank offset 32 NW and miss.  T16: suffix elements come from
// the 16-bit copy of the adjacency (element + top16 is the rank).
template <int LOG2R, bool T16_>
struct WindowRow {
    static constexpr bool T16 = T16_;
    static constexpr int NW = (1 << LOG2R) / 32;
    static constexpr bool PAIR = LOG2R <= 16;
    static constexpr uint32_t ZR = 32u * NW;
    uint2 bp[PAIR ? NW + 1 : 1];
    uint32_t bw[PAIR ? 1 : NW + 1];
    uint16_t bpre[PAIR ? 1 : NW];
    uint32_t part[16];
    struct Key {
        int32_t roff;  // loaded element + roff = rank offset r
    };
    struct Hit {
        uint32_t word, rr;
    };
    __device__ __forceinline__ uint32_t& word_at(int i) {
        if constexpr (PAIR) return bp[i].x;
        else return bw[i];
    }
    template <int NT>
    __device__ __forceinline__ Key build(const int32_t* __restrict__ adj, int32_t b0, int32_t B, int32_t v,
                                         int32_t top16, int tid, int lane, int wave) {
        for (int i = tid; i <= NW; i += NT) word_at(i) = 0;
        __syncthreads();
        for (int j = tid; j < B; j += NT) {
            const uint32_t r = (uint32_t)(adj[b0 + j] - v - 1);
            atomicOr(&word_at(r >> 5), 1u << (r & 31));
        }
        const int32_t maxv = adj[b0 + B - 1];
        __syncthreads();
        {  // exclusive prefix of popcounts over the words in use
            const int nw = (maxv - v + 31) >> 5;
            const int per = (nw + NT - 1) / NT;
            const int w0 = tid * per, w1 = min(nw, w0 + per);
            uint32_t sum = 0;
            for (int i = w0; i < w1; ++i) sum += __popc(word_at(i));
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
                if constexpr (PAIR) bp[i].y = run;
                else bpre[i] = (uint16_t)run;
                run += __popc(word_at(i));
            }
        }
        __syncthreads();
        return Key{(T16 ? top16 : 0) - v - 1};
    }
    // branch-free up to the count itself: lanes outside the chunk look up the
    // zero word and miss, and so do elements outside the window (offsets of
    // 32 NW or more, negative ones included, clamp to it); inside the window
    // the words past the row's largest rank hold no bit
    __device__ __forceinline__ bool probe(const Key& k, int32_t x, bool valid, Hit& h) const {
        const uint32_t r = (uint32_t)(x + k.roff);
        h.rr = valid ? min(r, ZR) : ZR;
        if constexpr (PAIR) h.word = bp[h.rr >> 5].x;
        else h.word = bw[h.rr >> 5];
        // (the bit-field extract takes its offset and width mod 32)
        return __builtin_amdgcn_ubfe(h.word, h.rr, 1u) != 0u;
    }
    // position of the element in N+(v): the set bits below it
    __device__ __forceinline__ uint32_t position(const Key&, const Hit& h) const {
        const uint32_t pw = PAIR ? bp[h.rr >> 5].y : (uint32_t)bpre[h.rr >> 5];
        return pw + __popc(__builtin_amdgcn_ubfe(h.word, 0u, h.rr));
    }
};

// Hash of N+(v) (RowHash), for rows whose ranks span too much for a window.
// Suffix elements above the row's largest rank are not looked up.
template <int LOG2S, bool PACKED>
struct HashRow {
    static constexpr bool T16 = false;
    RowHash<LOG2S, PACKED> H;
    struct Key {
        int32_t v, maxv;
    };
    struct Hit {
        int32_t p;
    };
    template <int NT>
    __device__ __forceinline__ Key build(const int32_t* __restrict__ adj, int32_t b0, int32_t B, int32_t v,
                                         int32_t, int tid, int, int) {
        H.clear(tid, NT);
        __syncthreads();
        for (int j = tid; j < B; j += NT) H.insert(adj[b0 + j], v, j);
        __syncthreads();
        return Key{v, adj[b0 + B - 1]};
    }
    __device__ __forceinline__ bool probe(const Key& k, int32_t x, bool valid, Hit& h) const {
        h.p = valid && x <= k.maxv ? H.find(x, k.v) : -1;
        return h.p >= 0;
    }
    __device__ __forceinline__ uint32_t position(const Key&, const Hit& h) const { return (uint32_t)h.p; }
};

// Items of the rank-window classes and of the larger hash classes, one item
// per workgroup of NT threads.  Each wave walks its own in-edges of the item,
// one at a time, all 64 lanes on chunks of 64 E elements of the in-edge's
// suffix.  The walk (in-edge, chunk, loop control) is wave-uniform, so it
// runs on the scalar unit and the vector work per element is the probe alone;
// the scalar unit is shared by the CU's waves, so a chunk of several elements
// per lane spreads its cost.  Loads run D chunks ahead of their use in a ring
// of registers.  t(v,w) partial counts are 32-bit LDS counters, one per
// element of N+(v).  The hit ballot of every 64 elements is stored as a word
// of the in-edge's bitmask (bits, at wbase[e] + suffix offset / 64), for the
// credit passes.  Wide windows take large workgroups so that the LDS they
// need still leaves room for enough waves per CU.
template <class Row, int MAXB, int NT, int D, int MINW, int E>
__global__ __launch_bounds__(NT, MINW) void k_tc_walk(const Item* __restrict__ all_items,
                                                     const int64_t* __restrict__ heads, int cls,
                                                     const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ adj,
                                                     const uint16_t* __restrict__ adj16, int32_t top16,
                                                     const int2* __restrict__ in_ea,
                                                     const int64_t* __restrict__ wbase,
                                                     unsigned long long* __restrict__ bits,
                                                     int32_t* __restrict__ t, int ipart, int nparts) {
    constexpr bool T16 = Row::T16;
    constexpr int NWAVES = NT / 64;
    __shared__ Row row;
    __shared__ uint32_t cnt[MAXB];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const Item* __restrict__ items = all_items + heads[2 * cls];
    const int64_t n_items = heads[2 * cls + 1];

    // this launch takes the items it = ipart (mod nparts) of the class
    for (int64_t it = (int64_t)blockIdx.x * nparts + ipart; it < n_items; it += (int64_t)gridDim.x * nparts) {
        const Item I = items[it];
        const int32_t v = I.v;
        const int32_t b0 = (int32_t)off[v];
        const int32_t B = (int32_t)(off[v + 1] - b0);
        for (int i = tid; i < B; i += NT) cnt[i] = 0;
        const typename Row::Key key = row.template build<NT>(adj, b0, B, v, top16, tid, lane, wave);

        ChunkGen<E> gen{in_ea + I.s + wave, wbase, I.len > wave ? (I.len - wave + NWAVES - 1) / NWAVES : 0, NWAVES,
                        0, -64, 0, 64, 0, 0, 0, 0, false};  // pos = -64, bi = 64: next() fetches the first batch
        gen.next(lane);
        constexpr uint32_t SZ = T16 ? 2u : 4u;  // bytes per loaded element
        uint32_t ob[E];                          // byte offset of this lane's element k in a chunk
#pragma unroll
        for (int k = 0; k < E; ++k) ob[k] = (uint32_t)(64 * k + lane) * SZ;
        int32_t w[D][E], spos[D], sa1[D];
        int64_t sw[D];
        bool sv[D];
        // the ring's refill of slot q from the generator's current chunk
        auto refill = [&](int q) {
            sv[q] = !gen.done;
            spos[q] = gen.pos;
            sa1[q] = gen.a1;
            sw[q] = gen.word();
            const int64_t p = gen.done ? 0 : gen.pos;
            const uint32_t last = gen.done ? 0u : (uint32_t)(gen.a1 - gen.pos - 1) * SZ;
            const void* base = T16 ? (const void*)(adj16 + p) : (const void*)(adj + p);
#pragma unroll
            for (int k = 0; k < E; ++k) w[q][k] = load_elem<T16>(base, last, ob[k]);
            if (sv[q]) gen.next(lane);
        };
#pragma unroll
        for (int q = 0; q < D; ++q) refill(q);
        bool more = sv[0];
        while (more) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
                if (!sv[q]) {  // this and every later slot are empty
                    more = false;
                    break;
                }
                const int32_t pos = spos[q], nv = sa1[q] - pos;
                const uint32_t lastb = (uint32_t)(nv - 1) * SZ;
                // lane k of (xlo, xhi) collects the hit ballot of the chunk's
                // k-th 64 elements
                uint32_t xlo = 0u, xhi = 0u;
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    // a part of the chunk past the suffix's end is skipped
                    // (wave-uniform): short suffixes cost one probe, not E
                    if (64 * k >= nv) break;
                    typename Row::Hit h;
                    const bool hit = row.probe(key, w[q][k], ob[k] <= lastb, h);
                    const unsigned long long hb = __ballot(hit);
                    xlo = (uint32_t)writelane((int32_t)(uint32_t)hb, k, (int32_t)xlo);
                    xhi = (uint32_t)writelane((int32_t)(uint32_t)(hb >> 32), k, (int32_t)xhi);
                    if (hit) atomicAdd(&cnt[row.position(key, h)], 1u);
                }
                // this chunk's words of the in-edge's hit bitmask, one per 64
                // elements (lane k stores word k): every word of such an
                // in-edge is written, once
                const int nwords = (min(nv, 64 * E) + 63) >> 6;
                if (lane < nwords)
                    __builtin_nontemporal_store(((unsigned long long)xhi << 32) | xlo, &bits[sw[q] + lane]);
                // refill the slot with the chunk D ahead
                refill(q);
            }
        }
        __syncthreads();
        for (int j = tid; j < B; j += NT) {
            const uint32_t x = cnt[j];
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
//   0..3   hash, packed entries (row within 2^20 ranks above v), by row length
//   4..7   hash, wide entries, by row length
//   8..10  rank window of 2^14, 2^16, 2^18 ranks (rows longer than 128)
//   11     binary search (rows longer than the LDS cap)
//   12, 13 rank window of 2^14, 2^16 ranks for v among the top 65,536 ranks:
//          every suffix element then lies there too, and the suffixes are
//          read from the 16-bit copy of the adjacency
constexpr int kClasses = 14;
constexpr int kSearch = 11;
__host__ __device__ inline bool window_class(int c) { return (c >= 8 && c <= 10) || c == 12 || c == 13; }
// classes run by the walking kernel (hit bitmasks, no global atomics): the
// rank windows and the hash classes of rows longer than 128
__host__ __device__ inline bool walk_class(int c) { return window_class(c) || (c >= 1 && c <= 7 && c != 4); }
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
                                                         int64_t packed_range, int64_t window_max, int64_t top16,
                                                         int8_t* __restrict__ vcls, int32_t* __restrict__ vcnt,
                                                         uint8_t* __restrict__ wflag) {
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
                    if (top16 >= 0 && v >= top16 && (cls == 8 || cls == 9)) cls += 4;
                }
            }
        }
        const int64_t cs = item_size(chunk, B);
        const int32_t k = cls >= 0 ? (int32_t)((I + cs - 1) / cs) : 0;
        vcls[v] = (int8_t)(k > 0 ? cls : -1);
        vcnt[v] = k;
        wflag[v] = walk_class(cls) ? 1 : 0;  // in-edges credited through hit bitmasks
    }
}

// Words of every edge's hit bitmask: ceil(suffix length / 64) when its head
// is an item of the walking kernel (the only one that writes bitmasks), else 0.
__global__ __launch_bounds__(kThreads) void k_tc_words(const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ adj,
                                                       const uint8_t* __restrict__ wflag, int64_t m,
                                                       int32_t* __restrict__ words) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t L = off[src[e] + 1] - e - 1;
        words[e] = wflag[adj[e]] ? (int32_t)((L + 63) >> 6) : 0;
    }
}

// The credits of the hit bitmasks.  With d the length of row u and x_j the
// bitmask of its j-th edge u -> w_j (bit s: the suffix element w_(j+1+s) is a
// common neighbour, i.e. {u, w_j, w_(j+1+s)} is a triangle),
//     t(u, w_k) += #{ j < k : bit k - j - 1 of x_j }   (column sums)
//     t(u, w_j) += popcount(x_j)                       (the in-edge's count)
// Each position of t belongs to one row, so the additions are plain stores;
// the passes run after every other credit has landed.
//
// Rows of at most kShortRow edges (bitmasks of one word): edge-parallel, one
// lane per edge over 64-edge windows; the earlier edges of a lane's row lie
// within 63 positions, in its window or the previous one, so the column sum
// is a walk over the distances k = 1 .. 63 with two lane shuffles each.
constexpr int64_t kShortRow = 64;

__global__ __launch_bounds__(kThreads) void k_tc_credit_short(const int64_t* __restrict__ off,
                                                              const int32_t* __restrict__ src,
                                                              const int64_t* __restrict__ wbase,
                                                              const unsigned long long* __restrict__ bits,
                                                              int64_t m, int64_t per_wave,
                                                              int32_t* __restrict__ t) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t nwin = (m + 63) >> 6;
    const int64_t w_begin = wave * per_wave, w_end = min(nwin, w_begin + per_wave);
    if (w_begin >= w_end) return;
    // a lane's bitmask word (rows of at most kShortRow edges only) and its
    // position in its row; -1 for lanes outside such rows
    auto load = [&](int64_t win, unsigned long long& x, int32_t& j) {
        const int64_t e = win * 64 + lane;
        x = 0ull;
        j = -1;
        if (e < m) {
            const int64_t rs = off[src[e]], d = off[src[e] + 1] - rs;
            if (d <= kShortRow) {
                j = (int32_t)(e - rs);
                const int64_t w0 = wbase[e];
                if (wbase[e + 1] > w0) x = bits[w0];
            }
        }
    };
    unsigned long long xprev = 0ull, x;
    int32_t jprev, j;
    if (w_begin > 0) load(w_begin - 1, xprev, jprev);
    for (int64_t win = w_begin; win < w_end; ++win) {
        load(win, x, j);
        // distances that can reach an earlier edge of the same short row
        int kmax = j > 0 ? j : 0;
        for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
        int32_t col = 0;
        if (__ballot(x != 0ull || xprev != 0ull) != 0ull) {
            for (int k = 1; k <= kmax; ++k) {
                const int srcl = (lane - k) & 63;
                const unsigned long long a = __shfl(x, srcl), b = __shfl(xprev, srcl);
                const unsigned long long xs = lane >= k ? a : b;
                if (k <= j) col += (int32_t)((xs >> (k - 1)) & 1ull);
            }
        }
        const int32_t add = col + __popcll(x);
        if (j >= 0 && add) t[win * 64 + lane] += add;
        xprev = x;
    }
}

// Rows longer than kShortRow: the row is cut into tiles of 64 positions and
// the tiles into runs of kRun; one wave per run, the runs of all such rows
// dealt out over the grid (a hub row's runs spread over many waves).  For a
// run, the bitmasks of the row's edges are taken 64 at a time, lane j holding
// edge j's: the lane loads the kRun + 1 consecutive words of its bitmask that
// cover the run and realigns them to the tiles (one shift for all of them),
// then, tile by tile, the 64 x 64 bit block is transposed across the lanes and
// each lane's popcount is its column's sum, kept in registers until the run's
// end.  Each bitmask word is thus read once per run instead of once per tile.
constexpr int kRun = 16;

// 64 x 64 bit transpose across the wave: lane j holds row j on entry, lane i
// holds column i (bit j = bit i of row j) on exit.  Six stages swap the
// off-diagonal blocks of 32, 16, ..., 1 bits between lanes j and j ^ s.
__device__ __forceinline__ unsigned long long transpose64(unsigned long long x, int lane) {
    const unsigned long long masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                         0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int sh = 32 >> k;
        const unsigned long long m = masks[k];
        const unsigned long long y = __shfl_xor(x, sh);
        x = (lane & sh) ? ((x & ~m) | ((y & ~m) >> sh)) : ((x & m) | ((y & m) << sh));
    }
    return x;
}

__global__ __launch_bounds__(kThreads) void k_tc_credit_long(const int64_t* __restrict__ off,
                                                             const int64_t* __restrict__ wbase,
                                                             const unsigned long long* __restrict__ bits,
                                                             const int32_t* __restrict__ run_row,
                                                             const int64_t* __restrict__ rbase, int64_t n,
                                                             int32_t* __restrict__ t) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (kThreads / 64);
    const int64_t nr = rbase[n];
    for (int64_t q = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); q < nr; q += nwaves) {
        const int64_t u = run_row[q];
        const int64_t e0 = off[u], d = off[u + 1] - e0;
        const int64_t c0 = (q - rbase[u]) * kRun;  // first tile of the run
        const int64_t k0 = 64 * c0;                // its first position
        const int nc = (int)min((int64_t)kRun, ((d + 63) >> 6) - c0);
        // edges with a bit in the run: j < min(d - 1, k0 + 64 nc - 1)
        const int64_t jend = min(d - 1, k0 + 64 * (int64_t)nc - 1);
        int32_t col[kRun];
#pragma unroll
        for (int k = 0; k < kRun; ++k) col[k] = 0;
        for (int64_t jb = 0; jb < jend; jb += 64) {
            const int64_t j = jb + lane;
            // bit s of edge j's bitmask is position j + 1 + s; the run starts at
            // suffix offset s0 = k0 - j - 1, so tile k's bits are the bitmask's
            // bits s0 + 64 k ... s0 + 64 k + 63
            unsigned long long W[kRun + 1];
            int sh = 0;
            if (j < jend) {
                const int64_t w0 = wbase[e0 + j], nw = wbase[e0 + j + 1] - w0;
                const int64_t s0 = k0 - j - 1;
                const int64_t wi = s0 >> 6;  // floor
                sh = (int)(s0 & 63);
#pragma unroll
                for (int k = 0; k <= kRun; ++k) {
                    const int64_t i = wi + k;
                    W[k] = (i >= 0 && i < nw) ? bits[w0 + i] : 0ull;
                }
            } else {
#pragma unroll
                for (int k = 0; k <= kRun; ++k) W[k] = 0ull;
            }
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const unsigned long long x = sh ? ((W[k] >> sh) | (W[k + 1] << (64 - sh))) : W[k];
                if (__ballot(x != 0ull) == 0ull) continue;
                col[k] += __popcll(transpose64(x, lane));
            }
        }
        // popcounts of the run's own bitmasks (edge j credits t at its own
        // position with its hit count), then the column sums
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            if (k >= nc) break;
            const int64_t j = k0 + 64 * k + lane;
            int32_t pc = 0;
            if (j < d - 1) {
                const int64_t w1 = wbase[e0 + j + 1];
                for (int64_t wq = wbase[e0 + j]; wq < w1; ++wq) pc += __popcll(bits[wq]);
            }
            if (j < d && (col[k] | pc)) t[e0 + j] += col[k] + pc;
        }
    }
}

// Runs of every row longer than kShortRow that holds bitmask words:
// ceil(ceil(length / 64) / kRun), else 0.
__global__ __launch_bounds__(kThreads) void k_long_runs(const int64_t* __restrict__ off,
                                                        const int64_t* __restrict__ wbase, int64_t n,
                                                        int32_t* __restrict__ runs) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = off[u], b = off[u + 1];
        const int64_t tiles = (b - a + 63) >> 6;
        runs[u] = (b - a > kShortRow && wbase[b] > wbase[a]) ? (int32_t)((tiles + kRun - 1) / kRun) : 0;
    }
}

// The row of every run: run_row[rbase[u] + r] = u for r < runs[u].
__global__ __launch_bounds__(kThreads) void k_run_rows(const int32_t* __restrict__ runs,
                                                       const int64_t* __restrict__ rbase, int64_t n,
                                                       int32_t* __restrict__ run_row) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t k = runs[u];
        for (int32_t r = 0; r < k; ++r) run_row[rbase[u] + r] = (int32_t)u;
    }
}

// adj16[e] = adj[e] - top16 for ranks in the top 65,536 (others are never read
// through it).
__global__ __launch_bounds__(kThreads) void k_adj16(const int32_t* __restrict__ adj, int64_t m, int32_t top16,
                                                    uint16_t* __restrict__ adj16) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = adj[e];
        adj16[e] = a >= top16 ? (uint16_t)(a - top16) : (uint16_t)0xffff;
    }
}

// Work items grouped by class, each class's items in vertex order.  A block
// of kVB vertices sums its items per class (k_class_blocks); a workgroup per
// class scans those sums into every block's offset in that class's list
// (k_class_offsets), one thread lays out the lists (k_class_heads); each block
// then places its vertices' items (k_item_fill), one block-wide exclusive scan
// per class.
constexpr int kVB = 1024;               // vertices per block
constexpr int kVPT = kVB / kThreads;    // per thread

__global__ __launch_bounds__(kThreads) void k_class_blocks(const int8_t* __restrict__ vcls,
                                                           const int32_t* __restrict__ vcnt, int64_t n,
                                                           int64_t* __restrict__ bsum) {
    __shared__ unsigned long long cs[kClasses];
    const int tid = threadIdx.x;
    if (tid < kClasses) cs[tid] = 0;
    __syncthreads();
    const int64_t v0 = (int64_t)blockIdx.x * kVB;
    for (int i = 0; i < kVPT; ++i) {
        const int64_t v = v0 + (int64_t)i * kThreads + tid;
        if (v < n && vcls[v] >= 0) atomicAdd(&cs[vcls[v]], (unsigned long long)vcnt[v]);
    }
    __syncthreads();
    if (tid < kClasses) bsum[(int64_t)blockIdx.x * kClasses + tid] = (int64_t)cs[tid];
}

// One workgroup per class c: bsum[b][c] becomes the offset of block b's
// first item of class c within that class's list, ctot[c] the list's length.
__global__ __launch_bounds__(1024) void k_class_offsets(int64_t* __restrict__ bsum, int64_t nb,
                                                        int64_t* __restrict__ ctot) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x, c = blockIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = tid * per, b1 = min(nb, b0 + per);
    int64_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += bsum[b * kClasses + c];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t x = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int64_t b = b0; b < b1; ++b) {
        const int64_t x = bsum[b * kClasses + c];
        bsum[b * kClasses + c] = run;
        run += x;
    }
    if (tid == 1023) ctot[c] = part[1023];
}

// heads[2c], heads[2c+1]: start and length of class c's list (the lists are
// laid out one after another).
__global__ void k_class_heads(const int64_t* __restrict__ ctot, int64_t* __restrict__ heads) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t start = 0;
    for (int c = 0; c < kClasses; ++c) {
        heads[2 * c] = start;
        heads[2 * c + 1] = ctot[c];
        start += ctot[c];
    }
}

__global__ __launch_bounds__(kThreads) void k_item_fill(const int64_t* __restrict__ off,
                                                        const int64_t* __restrict__ in_off, int64_t n,
                                                        int64_t chunk, const int8_t* __restrict__ vcls,
                                                        const int32_t* __restrict__ vcnt,
                                                        const int64_t* __restrict__ bsum,
                                                        const int64_t* __restrict__ heads,
                                                        Item* __restrict__ items) {
    __shared__ int64_t wpart[kThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t v0 = (int64_t)blockIdx.x * kVB;
    // a thread's vertices are consecutive: v0 + tid * kVPT + i
    int8_t cl[kVPT];
    int32_t kk[kVPT];
    for (int i = 0; i < kVPT; ++i) {
        const int64_t v = v0 + (int64_t)tid * kVPT + i;
        cl[i] = v < n ? vcls[v] : (int8_t)-1;
        kk[i] = v < n ? vcnt[v] : 0;
    }
    for (int c = 0; c < kClasses; ++c) {
        int64_t mine = 0;
        for (int i = 0; i < kVPT; ++i) mine += cl[i] == c ? kk[i] : 0;
        // block-wide exclusive prefix of mine
        int64_t inc = mine;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wpart[w] = inc;
        __syncthreads();
        int64_t before = inc - mine;
        for (int ww = 0; ww < w; ++ww) before += wpart[ww];
        __syncthreads();
        if (mine == 0) continue;
        int64_t slot = heads[2 * c] + bsum[(int64_t)blockIdx.x * kClasses + c] + before;
        for (int i = 0; i < kVPT; ++i) {
            if (cl[i] != c) continue;
            const int64_t v = v0 + (int64_t)tid * kVPT + i;
            const int64_t cs = item_size(chunk, off[v + 1] - off[v]);
            const int64_t i0 = in_off[v], i1 = in_off[v + 1];
            for (int32_t j = 0; j < kk[i]; ++j) {
                Item I;
                I.v = (int32_t)v;
                I.s = i0 + (int64_t)j * cs;
                I.len = (int32_t)min(cs, i1 - I.s);
                items[slot + j] = I;
            }
            slot += kk[i];
        }
    }
}

// First rank of the 16-bit range (the top 65,536 ranks; every rank when n is
// smaller).
inline int64_t top16_of(int64_t n) { return n > 65536 ? n - 65536 : 0; }

inline unsigned grid_for(int64_t N, int64_t cap) {
    int64_t b = (N + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

struct TcLayout {
    int8_t* vcls;    // [n] class of each vertex's items (-1: none)
    int32_t* vcnt;   // [n] items of each vertex
    int64_t* bsum;   // [ceil(n / kVB)][kClasses] block sums, then block offsets within each class
    int64_t* ctot;   // [kClasses] items per class
    Item* items;     // [max items]
    int64_t* heads;  // [2*kClasses]: start, length per class
    uint8_t* wflag;  // [n] head of walking-kernel items
    int32_t* words;  // [m] bitmask words per edge
    int64_t* wbase;  // [m+1] first bitmask word per edge
    unsigned long long* bits;  // [bitmask words] hit bitmasks
    uint16_t* adj16;   // [m] 16-bit copy of the adjacency for the top 65,536 ranks
    int32_t* rruns;    // [n] runs of a row longer than kShortRow with bitmask words
    int64_t* rbase;    // [n+1] its first run
    int32_t* run_row;  // [m/32 + 1] row of every run
    void* scan;
    size_t bytes;
};

TcLayout tc_layout(void* p, const mcd_graph* g, int64_t chunk) {
    Carve c{(char*)p, 0, 0};
    TcLayout L;
    const int64_t n = g->n, m = g->m;
    const int64_t max_items = n + m / item_size(chunk, 0) + 1;  // items hold >= item_size(chunk, 0) in-edges
    L.vcls = c.take<int8_t>((size_t)n);
    L.vcnt = c.take<int32_t>((size_t)n);
    L.bsum = c.take<int64_t>((size_t)kClasses * (size_t)((n + kVB - 1) / kVB));
    L.ctot = c.take<int64_t>((size_t)kClasses);
    L.items = c.take<Item>((size_t)max_items);
    L.heads = c.take<int64_t>(2 * kClasses);
    L.wflag = c.take<uint8_t>((size_t)n);
    L.words = c.take<int32_t>((size_t)m);
    L.wbase = c.take<int64_t>((size_t)m + 1);
    L.bits = c.take<unsigned long long>((size_t)g->bitmask_words);
    L.adj16 = c.take<uint16_t>((size_t)m);
    L.rruns = c.take<int32_t>((size_t)n);
    L.rbase = c.take<int64_t>((size_t)n + 1);
    // rows longer than 64 hold at most length / 32 tiles (so runs) each
    L.run_row = c.take<int32_t>((size_t)(m / 32) + 1);
    L.scan = c.take<char>(scan_scratch_bytes(n > m ? n : m));
    L.bytes = c.used;
    return L;
}

template <class Table, int MAXB, int WPI, int G>
void launch_class(const mcd_graph* g, const TcLayout& L, int c, int64_t chunk, int32_t* t, hipStream_t s,
                  int ipart = 0, int nparts = 1) {
    constexpr int NI = 4 / WPI;
    // grid-stride over the class list; its length is read on the device
    const int64_t cap_items = g->n + g->m / item_size(chunk, 0) + 1;
    int64_t blocks = (cap_items + NI - 1) / NI;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL((k_tc_items<Table, MAXB, WPI, G>), dim3((unsigned)blocks), dim3(kThreads), 0, s,
                       L.items, L.heads, c, g->off, g->adj, g->in_ea, t, ipart, nparts);
}

// ipart / nparts: this launch takes every nparts-th item of the class.
// tc_window_occupancy = 1 (the default) takes the build of the kernel held to
// 8 waves per SIMD (some scalar registers spilled to vector lanes) instead of
// the compiler's own budget of 106 scalar registers, which allows 7: with
// 16-wave workgroups that is the difference between one and two resident
// workgroups per CU (R-MAT scale 26: 625 -> 513 ms for the whole count).
// Elements per lane of a rank-window chunk: 8, so that a wave's walk
// (in-edge, chunk, ring slot: scalar work, lane reads, the hit word store) is
// paid once per 512 suffix elements, while a chunk's probes past its
// suffix's end are skipped; 3 ring slots keep 24 loads of a wave in flight
// within 64 registers (8 waves per SIMD).  (R-MAT scale 26, whole count: 4
// elements per lane with 4 slots 363 ms, 5 354, 6 347, 8 with 3 slots 345,
// 8 with 2 slots 352; 10 or 12 elements spill and take 1.2 s.)
constexpr int kWindowE = 8;

template <class Row, int MAXB, int NT, int D>
void launch_walk(const mcd_graph* g, const TcLayout& L, int c, int64_t chunk, int32_t* t, hipStream_t s,
                 int ipart, int nparts) {
    const int64_t cap_items = g->n + g->m / item_size(chunk, 0) + 1;
    int64_t blocks = cap_items < 16384 ? cap_items : 16384;
    const int32_t top16 = (int32_t)top16_of(g->n);
    if (g->ctx->tc_window_occupancy)
        hipLaunchKernelGGL((k_tc_walk<Row, MAXB, NT, D, 8, kWindowE>), dim3((unsigned)blocks), dim3(NT), 0, s,
                           L.items, L.heads, c, g->off, g->adj, L.adj16, top16, g->in_ea, L.wbase, L.bits, t, ipart,
                           nparts);
    else
        hipLaunchKernelGGL((k_tc_walk<Row, MAXB, NT, D, 1, kWindowE>), dim3((unsigned)blocks), dim3(NT), 0, s,
                           L.items, L.heads, c, g->off, g->adj, L.adj16, top16, g->in_ea, L.wbase, L.bits, t, ipart,
                           nparts);
}

template <int LOG2R, int NT, int D, bool T16 = false>
void launch_window(const mcd_graph* g, const TcLayout& L, int c, int64_t chunk, int32_t* t, hipStream_t s,
                   int ipart = 0, int nparts = 1) {
    launch_walk<WindowRow<LOG2R, T16>, 4096, NT, D>(g, L, c, chunk, t, s, ipart, nparts);
}

// Hash class c of the walking kernel: rows of at most MAXB = kMaxB[c % 4]
// entries in a table of 2^LOG2S slots.  A probe of the wave runs as long as
// its longest linear-probe sequence, so the tables are kept sparse where the
// LDS allows (R-MAT scale 26, whole count with rows of up to 512 entries in
// 1024, 2048 and 4096 slots: 334, 307 and 300 ms).
template <int LOG2S, bool PACKED, int MAXB, int NT, int D>
void launch_hash_walk(const mcd_graph* g, const TcLayout& L, int c, int64_t chunk, int32_t* t, hipStream_t s,
                      int ipart = 0, int nparts = 1) {
    static_assert(2 * MAXB <= (1 << LOG2S), "hash tables at most half full");
    launch_walk<HashRow<LOG2S, PACKED>, MAXB, NT, D>(g, L, c, chunk, t, s, ipart, nparts);
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
                       n, chunk, lds_max, packed_range, window_max, top16_of(n), L.vcls, L.vcnt, L.wflag);
    hipLaunchKernelGGL(k_adj16, dim3(grid_for(g->m, 16384)), dim3(kThreads), 0, s, g->adj, g->m,
                       (int32_t)top16_of(n), L.adj16);
    // where the hit bitmask of every edge starts (edges whose head is not a
    // walking-kernel item get none)
    hipLaunchKernelGGL(k_tc_words, dim3(grid_for(g->m, 16384)), dim3(kThreads), 0, s, g->off, g->src, g->adj,
                       L.wflag, g->m, L.words);
    exclusive_scan_i32_i64(L.words, g->m, L.wbase, L.scan, s);
    {
        const int64_t nb = (n + kVB - 1) / kVB;
        hipLaunchKernelGGL(k_class_blocks, dim3((unsigned)nb), dim3(kThreads), 0, s, L.vcls, L.vcnt, n, L.bsum);
        hipLaunchKernelGGL(k_class_offsets, dim3(kClasses), dim3(1024), 0, s, L.bsum, nb, L.ctot);
        hipLaunchKernelGGL(k_class_heads, dim3(1), dim3(64), 0, s, L.ctot, L.heads);
        hipLaunchKernelGGL(k_item_fill, dim3((unsigned)nb), dim3(kThreads), 0, s, g->off, g->in_off, n, chunk,
                           L.vcls, L.vcnt, L.bsum, L.heads, L.items);
    }
    // The classes run on three streams at once (the context's and its two
    // side streams, forked here and joined at the end): each kernel's tail of
    // long items then overlaps the others' work.  The counts are integer
    // atomics, so the result does not depend on the interleaving.
    mcd_ctx* c = g->ctx;
    hipStream_t s1 = c->side[0], s2 = c->side[1];
    (void)hipEventRecord(c->fork, s);
    (void)hipStreamWaitEvent(s1, c->fork, 0);
    (void)hipStreamWaitEvent(s2, c->fork, 0);
    // Classes in launch order per stream, placed so that the three streams
    // end together (R-MAT scale 26, kernel times with three streams busy:
    // stream 0 about 66 + 106 + 9 + 11 + 37 ms, stream 1 170 + 11 + 12 + 24 + 3,
    // stream 2 68 + 134 + 37); the two largest window classes and the
    // largest hash class run as two halves of their item lists.
    launch_window<14, 512, 3, true>(g, L, 12, chunk, t, s, 0, 2);
    launch_window<14, 512, 3, true>(g, L, 12, chunk, t, s2, 1, 2);
    launch_window<16, 1024, 3, true>(g, L, 13, chunk, t, s1, 0, 2);
    launch_window<16, 1024, 3, true>(g, L, 13, chunk, t, s, 1, 2);
    launch_window<18, 1024, 3>(g, L, 10, chunk, t, s2);
    launch_window<14, 512, 3>(g, L, 8, chunk, t, s1);
    launch_window<16, 1024, 3>(g, L, 9, chunk, t, s1);
    launch_hash_walk<12, false, 512, 256, 3>(g, L, 5, chunk, t, s1);
    launch_hash_walk<13, true, 2048, 512, 3>(g, L, 2, chunk, t, s1);
    launch_class<RowHash<8, true>, 128, 1, 16>(g, L, 0, chunk, t, s1);
    launch_hash_walk<12, true, 512, 256, 3>(g, L, 1, chunk, t, s2, 1, 2);
    launch_class<RowHash<8, false>, 128, 1, 16>(g, L, 4, chunk, t, s);
    launch_hash_walk<13, true, 4096, 1024, 3>(g, L, 3, chunk, t, s);
    launch_hash_walk<13, false, 2048, 512, 3>(g, L, 6, chunk, t, s);
    launch_hash_walk<13, false, 4096, 1024, 3>(g, L, 7, chunk, t, s);
    launch_hash_walk<12, true, 512, 256, 3>(g, L, 1, chunk, t, s, 0, 2);
    hipLaunchKernelGGL(k_tc_search, dim3(4096), dim3(kThreads), 0, s, L.items, L.heads, kSearch, g->off,
                       g->adj, g->in_ea, t);
    (void)hipEventRecord(c->join[0], s1);
    (void)hipEventRecord(c->join[1], s2);
    (void)hipStreamWaitEvent(s, c->join[0], 0);
    (void)hipStreamWaitEvent(s, c->join[1], 0);
    // every class has finished: the bitmasks' credits, row by row
    {
        const int64_t m = g->m, nwin = (m + 63) >> 6;
        const int64_t waves = 65536, per_wave = (nwin + waves - 1) / waves;
        hipLaunchKernelGGL(k_tc_credit_short, dim3((unsigned)((waves + 3) / 4)), dim3(kThreads), 0, s, g->off, g->src,
                           L.wbase, L.bits, m, per_wave, t);
        hipLaunchKernelGGL(k_long_runs, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, g->off, L.wbase, n,
                           L.rruns);
        exclusive_scan_i32_i64(L.rruns, n, L.rbase, L.scan, s);
        hipLaunchKernelGGL(k_run_rows, dim3(grid_for(n, 8192)), dim3(kThreads), 0, s, L.rruns, L.rbase, n,
                           L.run_row);
        hipLaunchKernelGGL(k_tc_credit_long, dim3(8192), dim3(kThreads), 0, s, g->off, L.wbase, L.bits, L.run_row,
                           L.rbase, n, t);
    }
}

}  // namespace mcd
