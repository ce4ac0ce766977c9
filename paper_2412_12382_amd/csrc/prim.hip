// Device-wide primitives for gfx950: LSD radix sort of 64-bit keys, unique
// compaction of a sorted key array, exclusive scan, fills.
//
// All kernels use 256-thread workgroups (four 64-lane wavefronts).  Block-level
// work is split into contiguous ranges so that every pass is stable and
// deterministic, and per-block partial results go through a single-block scan.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kIters = 16;                   // 64-key rounds per wave and tile
constexpr int kTile = kThreads * kIters;     // 4096 keys per block iteration
constexpr int kMaxBlocks = 2048;
constexpr int kScanThreads = 1024;

__host__ __device__ inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int grid_blocks(int64_t tiles) {
    if (tiles < 1) return 1;
    return (int)(tiles < kMaxBlocks ? tiles : kMaxBlocks);
}

__device__ __forceinline__ uint64_t lane_lt_mask() { return __lanemask_lt(); }

// Digit histogram of block b's key range, stored digit-major: counts[d*NB + b].
// Keys are read 16 bytes per lane when the key array is 16-byte aligned (the
// block range starts on a tile); each wave keeps 4 sub-histograms, picked
// by lane, so that lanes with the same digit (skewed keys: hub vertices)
// collide 4 times less on one LDS address.
template <class K>
__global__ __launch_bounds__(kThreads) void k_rs_hist(const K* __restrict__ keys, int64_t N,
                                                      int shift, int64_t tpb, int NB,
                                                      int64_t* __restrict__ counts) {
    constexpr int kSub = 4;
    constexpr int kPer = 16 / (int)sizeof(K);  // keys per 16-byte load
    __shared__ uint32_t h[kWaves * kSub][256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    uint32_t* hh = h[w * kSub + (lane & (kSub - 1))];
    for (int i = tid; i < kWaves * kSub * 256; i += kThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * tpb * kTile;
    const int64_t end = min(N, beg + tpb * (int64_t)kTile);
    const int64_t nvec = ((uintptr_t)keys & 15u) == 0u ? (end - beg) / kPer : 0;
    const uint4* __restrict__ v4 = (const uint4*)(keys + beg);
    for (int64_t i = tid; i < nvec; i += kThreads) {
        union {
            uint4 v;
            K k[kPer];
        } u;
        u.v = v4[i];
#pragma unroll
        for (int j = 0; j < kPer; ++j) atomicAdd(&hh[(uint32_t)(u.k[j] >> shift) & 255u], 1u);
    }
    for (int64_t i = beg + nvec * kPer + tid; i < end; i += kThreads)
        atomicAdd(&hh[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int ww = 0; ww < kWaves * kSub; ++ww) s += h[ww][tid];
    counts[(int64_t)tid * NB + blockIdx.x] = s;
}

// In-place exclusive scan of a[0..len) by one workgroup; *total (if non-null)
// receives the sum.
__global__ __launch_bounds__(kScanThreads) void k_scan_single(int64_t* __restrict__ a, int64_t len,
                                                              int64_t* __restrict__ total) {
    __shared__ int64_t part[kScanThreads];
    const int tid = threadIdx.x;
    const int64_t per = (len + kScanThreads - 1) / kScanThreads;
    const int64_t b = tid * per, e = min(len, b + per);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += a[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - s;
    for (int64_t i = b; i < e; ++i) {
        int64_t v = a[i];
        a[i] = run;
        run += v;
    }
    if (total && tid == kScanThreads - 1) *total = part[tid];
}

// Per digit d (one workgroup each): exclusive scan, in place, of the block
// counts counts[d*NB .. d*NB+NB) and the digit total in tot[d].
__global__ __launch_bounds__(kThreads) void k_rs_rowscan(int64_t* __restrict__ counts, int NB,
                                                         int64_t* __restrict__ tot) {
    __shared__ int64_t part[kThreads];
    int64_t* row = counts + (int64_t)blockIdx.x * NB;
    const int tid = threadIdx.x;
    const int per = (NB + kThreads - 1) / kThreads;
    const int b = tid * per, e = min(NB, b + per);
    int64_t sum = 0;
    for (int i = b; i < e; ++i) sum += row[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int i = b; i < e; ++i) {
        const int64_t v = row[i];
        row[i] = run;
        run += v;
    }
    if (tid == kThreads - 1) tot[blockIdx.x] = part[tid];
}

// Exclusive prefix over the block's threads of x (one value per thread), and
// the total in *total.  Uses sh[kWaves].
template <class T>
__device__ __forceinline__ T block_excl_scan(T x, T* sh, T* total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) {
        if (ww < w) before += sh[ww];
        all += sh[ww];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

// Stable scatter of block b's key range by the digit at `shift` (KV: an
// int32 value travels with every key, vin -> vout).  Each wave
// ranks its own contiguous 1024-key slice of the tile with 64-lane ballots
// (lanes holding the same digit form a peer mask); slices are ordered wave by
// wave, so the rank order equals the input order.  The ranked tile is first
// placed in LDS grouped by digit, then written out so that consecutive
// threads store consecutive keys of a digit's run (coalesced writes).
template <class K, bool KV>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const K* __restrict__ in,
                                                         K* __restrict__ out, const int32_t* __restrict__ vin,
                                                         int32_t* __restrict__ vout, int64_t N,
                                                         int shift, int64_t tpb, int NB,
                                                         const int64_t* __restrict__ rowpre,
                                                         const int64_t* __restrict__ rowtot) {
    __shared__ int64_t run[256];
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t loff[256];
    __shared__ uint32_t tcnt[256];
    __shared__ K stage[kTile];
    __shared__ int32_t vstage[KV ? kTile : 1];
    __shared__ int64_t sh64[kWaves];
    __shared__ uint32_t sh32[kWaves];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    {
        int64_t all;
        const int64_t base = block_excl_scan<int64_t>(rowtot[tid], sh64, &all);
        run[tid] = base + rowpre[(int64_t)tid * NB + blockIdx.x];
    }
    const int64_t ntiles = div_up(N, kTile);
    const int64_t t0 = (int64_t)blockIdx.x * tpb;
    const int64_t t1 = min(ntiles, t0 + tpb);
    const uint64_t lt = lane_lt_mask();
    // keys of the next tile are loaded while the current one is written out
    K key[kIters];
    int32_t val[KV ? kIters : 1];
    auto load_tile = [&](int64_t tile) {
        const int64_t base = tile * kTile + (int64_t)w * (kTile / kWaves);
#pragma unroll
        for (int it = 0; it < kIters; ++it) {
            const int64_t i = base + it * 64 + lane;
            const bool ok = tile < t1 && i < N;
            key[it] = ok ? in[i] : (K)0;
            if (KV) val[KV ? it : 0] = ok ? vin[i] : 0;
        }
    };
    load_tile(t0);
    __syncthreads();
    for (int64_t tile = t0; tile < t1; ++tile) {
        for (int j = lane; j < 256; j += 64) wcnt[w][j] = 0;
        uint32_t rnk[kIters];
        const int64_t base = tile * kTile + (int64_t)w * (kTile / kWaves);
#pragma unroll
        for (int it = 0; it < kIters; ++it) {
            const int64_t i = base + it * 64 + lane;
            const bool valid = i < N;
            const K k = key[it];
            const uint32_t d = (uint32_t)(k >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const uint64_t bb = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? bb : ~bb;
            }
            const uint32_t before = valid ? wcnt[w][d] : 0u;
            rnk[it] = before + (uint32_t)__popcll(peers & lt);
            if (valid && (peers & lt) == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        {  // digit tid: tile count, tile-local start, and each wave's start within it
            uint32_t c[kWaves], sum = 0;
#pragma unroll
            for (int ww = 0; ww < kWaves; ++ww) {
                c[ww] = wcnt[ww][tid];
                sum += c[ww];
            }
            uint32_t total;
            const uint32_t start = block_excl_scan<uint32_t>(sum, sh32, &total);
            loff[tid] = start;
            tcnt[tid] = sum;
            uint32_t acc = start;
#pragma unroll
            for (int ww = 0; ww < kWaves; ++ww) {
                wcnt[ww][tid] = acc;
                acc += c[ww];
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kIters; ++it) {
            const int64_t i = base + it * 64 + lane;
            if (i < N) {
                const uint32_t d = (uint32_t)(key[it] >> shift) & 255u;
                stage[wcnt[w][d] + rnk[it]] = key[it];
                if (KV) vstage[wcnt[w][d] + rnk[it]] = val[KV ? it : 0];
            }
        }
        load_tile(tile + 1);
        __syncthreads();
        const int64_t tile_n = min((int64_t)kTile, N - tile * kTile);
        for (int j = tid; j < tile_n; j += kThreads) {
            const K k = stage[j];
            const uint32_t d = (uint32_t)(k >> shift) & 255u;
            out[run[d] + (j - (int64_t)loff[d])] = k;
            if (KV) vout[run[d] + (j - (int64_t)loff[d])] = vstage[j];
        }
        __syncthreads();
        run[tid] += tcnt[tid];
        __syncthreads();
    }
}

__device__ __forceinline__ bool uniq_flag(const uint64_t* __restrict__ in, int64_t i) {
    const uint64_t k = in[i];
    return k != MCD_SENTINEL && (i == 0 || in[i - 1] != k);
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* sh) {
    // sh: kWaves entries
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    int64_t s = 0;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) s += sh[ww];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kThreads) void k_uniq_count(const uint64_t* __restrict__ in, int64_t N,
                                                         int64_t tpb, int64_t* __restrict__ counts) {
    __shared__ int64_t sh[kWaves];
    const int64_t beg = (int64_t)blockIdx.x * tpb * kTile;
    const int64_t end = min(N, beg + tpb * (int64_t)kTile);
    int64_t c = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kThreads) c += uniq_flag(in, i) ? 1 : 0;
    const int64_t s = block_sum_i64(c, sh);
    if (threadIdx.x == 0) counts[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_uniq_scatter(const uint64_t* __restrict__ in, int64_t N,
                                                           int64_t tpb, const int64_t* __restrict__ offs,
                                                           uint64_t* __restrict__ out) {
    __shared__ uint32_t wc[kWaves];
    const int tid = threadIdx.x, w = tid >> 6;
    const int64_t beg = (int64_t)blockIdx.x * tpb * kTile;
    const int64_t end = min(N, beg + tpb * (int64_t)kTile);
    const uint64_t lt = lane_lt_mask();
    int64_t run = offs[blockIdx.x];
    for (int64_t c0 = beg; c0 < end; c0 += kThreads) {
        const int64_t i = c0 + tid;
        const bool f = (i < end) && uniq_flag(in, i);
        const uint64_t bal = __ballot(f);
        if ((tid & 63) == 0) wc[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t woff = 0, tot = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            woff += (ww < w) ? wc[ww] : 0u;
            tot += wc[ww];
        }
        if (f) out[run + woff + __popcll(bal & lt)] = in[i];
        run += tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_scan_count_i32(const int32_t* __restrict__ in, int64_t N,
                                                             int64_t tpb, int64_t* __restrict__ counts) {
    __shared__ int64_t sh[kWaves];
    const int64_t beg = (int64_t)blockIdx.x * tpb * kTile;
    const int64_t end = min(N, beg + tpb * (int64_t)kTile);
    int64_t c = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kThreads) c += in[i];
    const int64_t s = block_sum_i64(c, sh);
    if (threadIdx.x == 0) counts[blockIdx.x] = s;
}

// Block-local exclusive scan of 256 values per round, carried across rounds.
__global__ __launch_bounds__(kThreads) void k_scan_apply_i32(const int32_t* __restrict__ in, int64_t N,
                                                             int64_t tpb, const int64_t* __restrict__ offs,
                                                             int64_t* __restrict__ out) {
    __shared__ int64_t ws[kWaves];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t beg = (int64_t)blockIdx.x * tpb * kTile;
    const int64_t end = min(N, beg + tpb * (int64_t)kTile);
    int64_t run = offs[blockIdx.x];
    for (int64_t c0 = beg; c0 < end; c0 += kThreads) {
        const int64_t i = c0 + tid;
        const int64_t v = (i < end) ? (int64_t)in[i] : 0;
        int64_t x = v;  // inclusive wave scan
        for (int off = 1; off < 64; off <<= 1) {
            int64_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) ws[w] = x;
        __syncthreads();
        int64_t woff = 0, tot = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
            woff += (ww < w) ? ws[ww] : 0;
            tot += ws[ww];
        }
        if (i < end) out[i] = run + woff + x - v;
        run += tot;
        __syncthreads();
    }
}

template <class T>
__global__ void k_fill(T* __restrict__ p, int64_t N, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
void fill_any(T* p, int64_t N, T v, hipStream_t s) {
    if (N <= 0) return;
    int64_t blocks = div_up(N, kThreads);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, N, v);
}

}  // namespace

size_t radix_scratch_bytes(int64_t) { return mcd_align(sizeof(int64_t) * 256 * (kMaxBlocks + 1)); }

template <class K, bool KV>
K* radix_sort(K* a, K* b, int32_t* va, int32_t* vb, int32_t** vres, int64_t N, int nbits, void* scratch,
              hipStream_t s, int first_bit) {
    if (KV) *vres = va;
    if (N <= 1 || nbits <= 0) return a;
    const int64_t ntiles = div_up(N, kTile);
    const int NB = grid_blocks(ntiles);
    const int64_t tpb = div_up(ntiles, NB);
    int64_t* counts = (int64_t*)scratch;
    int64_t* tot = counts + (int64_t)256 * kMaxBlocks;
    const int passes = (nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = first_bit + 8 * p;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3(NB), dim3(kThreads), 0, s, a, N, shift, tpb, NB, counts);
        hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(kThreads), 0, s, counts, NB, tot);
        hipLaunchKernelGGL((k_rs_scatter<K, KV>), dim3(NB), dim3(kThreads), 0, s, a, b, va, vb, N, shift, tpb, NB,
                           counts, tot);
        K* t = a;
        a = b;
        b = t;
        int32_t* tv = va;
        va = vb;
        vb = tv;
    }
    if (KV) *vres = va;
    return a;
}

uint64_t* radix_sort_u64(uint64_t* a, uint64_t* b, int64_t N, int nbits, void* scratch, hipStream_t s,
                         int first_bit) {
    return radix_sort<uint64_t, false>(a, b, nullptr, nullptr, nullptr, N, nbits, scratch, s, first_bit);
}

uint64_t* radix_sort_u64_kv(uint64_t* a, uint64_t* b, int32_t* va, int32_t* vb, int32_t** vres, int64_t N,
                            int nbits, void* scratch, hipStream_t s, int first_bit) {
    return radix_sort<uint64_t, true>(a, b, va, vb, vres, N, nbits, scratch, s, first_bit);
}

uint32_t* radix_sort_u32(uint32_t* a, uint32_t* b, int64_t N, int nbits, void* scratch, hipStream_t s) {
    return radix_sort<uint32_t, false>(a, b, nullptr, nullptr, nullptr, N, nbits, scratch, s, 0);
}

size_t compact_scratch_bytes(int64_t) { return mcd_align(sizeof(int64_t) * (kMaxBlocks + 1)); }

void unique_sorted_u64(const uint64_t* in, int64_t N, uint64_t* out, int64_t* d_count,
                       void* scratch, hipStream_t s) {
    if (N <= 0) {
        fill_any<int64_t>(d_count, 1, 0, s);
        return;
    }
    const int64_t ntiles = div_up(N, kTile);
    const int NB = grid_blocks(ntiles);
    const int64_t tpb = div_up(ntiles, NB);
    int64_t* counts = (int64_t*)scratch;
    hipLaunchKernelGGL(k_uniq_count, dim3(NB), dim3(kThreads), 0, s, in, N, tpb, counts);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanThreads), 0, s, counts, (int64_t)NB, d_count);
    hipLaunchKernelGGL(k_uniq_scatter, dim3(NB), dim3(kThreads), 0, s, in, N, tpb, counts, out);
}

size_t scan_scratch_bytes(int64_t) { return mcd_align(sizeof(int64_t) * (kMaxBlocks + 1)); }

void exclusive_scan_i32_i64(const int32_t* in, int64_t N, int64_t* out, void* scratch,
                            hipStream_t s) {
    if (N <= 0) {
        fill_any<int64_t>(out, 1, 0, s);
        return;
    }
    const int64_t ntiles = div_up(N, kTile);
    const int NB = grid_blocks(ntiles);
    const int64_t tpb = div_up(ntiles, NB);
    int64_t* counts = (int64_t*)scratch;
    hipLaunchKernelGGL(k_scan_count_i32, dim3(NB), dim3(kThreads), 0, s, in, N, tpb, counts);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanThreads), 0, s, counts, (int64_t)NB, out + N);
    hipLaunchKernelGGL(k_scan_apply_i32, dim3(NB), dim3(kThreads), 0, s, in, N, tpb, counts, out);
}

void fill_i32(int32_t* p, int64_t N, int32_t v, hipStream_t s) { fill_any<int32_t>(p, N, v, s); }
void fill_i64(int64_t* p, int64_t N, int64_t v, hipStream_t s) { fill_any<int64_t>(p, N, v, s); }
void fill_u32(uint32_t* p, int64_t N, uint32_t v, hipStream_t s) { fill_any<uint32_t>(p, N, v, s); }

}  // namespace mcd
