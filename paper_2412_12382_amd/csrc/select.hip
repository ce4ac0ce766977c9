// Exact nearest-rank selection among the nonzero edge similarities.
//
// Every nonzero similarity gets a 32-bit key whose unsigned order agrees with
// the order of the exact values: for Tectonic and Jaccard the bit pattern of
// the positive quotient num/den rounded to fp32 through fp64 (the integers
// are exact in fp64, and each rounding is monotone, so exact order implies
// key order for any operands below 2^53, whereas converting a denominator of
// 2^24 or more to fp32 first would not be); for TW the int32 value with its
// sign bit flipped (exact).  A four-pass
// 8-bit radix select finds the key of the k-th smallest value.  For TW that is
// the answer; for Tectonic several distinct rationals may share one fp32 key,
// so the rationals inside that key are ordered exactly by cross-multiplying
// (minimum above a bound, then its multiplicity, repeated).
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;

inline unsigned grid_for(int64_t N, int64_t cap) {
    int64_t b = (N + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

struct Sim {
    int64_t num, den;
    uint32_t key;
    bool nonzero;
};

__device__ __forceinline__ Sim sim_of(const int32_t* __restrict__ dsum, const int32_t* __restrict__ t,
                                      int64_t e, int measure) {
    Sim s;
    const int64_t D = (uint32_t)dsum[e];
    const int32_t tt = t[e];
    if (measure == MCD_SIM_TW || measure == MCD_SIM_K3 || measure == MCD_SIM_K4) {  // integers: key = value
        const int32_t x = measure == MCD_SIM_TW ? (int32_t)(3 * (int64_t)tt - D + 2) : tt;
        s.num = x;
        s.den = 1;
        s.nonzero = x != 0;
        s.key = (uint32_t)x ^ 0x80000000u;
    } else {  // non-negative rationals: key = fp32 value (monotone in the exact value)
        s.num = tt;
        s.den = measure == MCD_SIM_JACCARD ? D - tt : D;
        s.nonzero = tt != 0;
        s.key = __float_as_uint((float)((double)tt / (double)s.den));
    }
    return s;
}

// sign(a/b - c/d), b, d > 0
__device__ __forceinline__ int rat_cmp(int64_t a, int64_t b, int64_t c, int64_t d) {
    const __int128 l = (__int128)a * d, r = (__int128)c * b;
    return (l > r) - (l < r);
}

__global__ __launch_bounds__(kThreads) void k_sel_hist(const int32_t* __restrict__ dsum,
                                                       const int32_t* __restrict__ t, int64_t m,
                                                       int measure, uint32_t prefix, uint32_t pmask,
                                                       int shift, unsigned long long* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const Sim s = sim_of(dsum, t, e, measure);
        if (s.nonzero && (s.key & pmask) == prefix) atomicAdd(&h[(s.key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// Per-block minimum rational strictly above lb (lb_valid = 0: no bound) among
// nonzero similarities whose key equals `key`.  out[2*b] = num, out[2*b+1] =
// den; den = 0 means none.
__global__ __launch_bounds__(kThreads) void k_sel_min(const int32_t* __restrict__ dsum,
                                                      const int32_t* __restrict__ t, int64_t m,
                                                      int measure, uint32_t key, int64_t lb_num,
                                                      int64_t lb_den, int lb_valid,
                                                      int64_t* __restrict__ out) {
    __shared__ int64_t sn[kThreads], sd[kThreads];
    int64_t bn = 0, bd = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const Sim s = sim_of(dsum, t, e, measure);
        if (!s.nonzero || s.key != key) continue;
        if (lb_valid && rat_cmp(s.num, s.den, lb_num, lb_den) <= 0) continue;
        if (bd == 0 || rat_cmp(s.num, s.den, bn, bd) < 0) {
            bn = s.num;
            bd = s.den;
        }
    }
    sn[threadIdx.x] = bn;
    sd[threadIdx.x] = bd;
    __syncthreads();
    for (int half = kThreads / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) {
            const int64_t on = sn[threadIdx.x + half], od = sd[threadIdx.x + half];
            if (od != 0 && (sd[threadIdx.x] == 0 || rat_cmp(on, od, sn[threadIdx.x], sd[threadIdx.x]) < 0)) {
                sn[threadIdx.x] = on;
                sd[threadIdx.x] = od;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = sn[0];
        out[2 * blockIdx.x + 1] = sd[0];
    }
}

__global__ __launch_bounds__(kThreads) void k_sel_min_final(int64_t* __restrict__ part, int nb,
                                                            int64_t* __restrict__ out) {
    if (threadIdx.x != 0) return;
    int64_t bn = 0, bd = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t on = part[2 * b], od = part[2 * b + 1];
        if (od != 0 && (bd == 0 || rat_cmp(on, od, bn, bd) < 0)) {
            bn = on;
            bd = od;
        }
    }
    out[0] = bn;
    out[1] = bd;
}

__global__ __launch_bounds__(kThreads) void k_sel_count_eq(const int32_t* __restrict__ dsum,
                                                           const int32_t* __restrict__ t, int64_t m,
                                                           int measure, uint32_t key, int64_t num,
                                                           int64_t den, unsigned long long* __restrict__ cnt) {
    unsigned long long c = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const Sim s = sim_of(dsum, t, e, measure);
        if (s.nonzero && s.key == key && rat_cmp(s.num, s.den, num, den) == 0) ++c;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

}  // namespace

constexpr int kSelBlocks = 1024;

size_t select_scratch_bytes(const mcd_graph*) {
    return mcd_align(sizeof(int64_t) * (256 + 2 * kSelBlocks + 8));
}

void sel_hist(const mcd_graph* g, int measure, const int32_t* t, uint32_t prefix, uint32_t pmask,
              int shift, int64_t* hist256, hipStream_t s) {
    fill_i64(hist256, 256, 0, s);
    if (g->m <= 0) return;
    hipLaunchKernelGGL(k_sel_hist, dim3(grid_for(g->m, kSelBlocks)), dim3(kThreads), 0, s, g->dsum, t, g->m, measure,
                       prefix, pmask, shift, (unsigned long long*)hist256);
}

void sel_min_above(const mcd_graph* g, int measure, const int32_t* t, uint32_t key, int64_t lb_num,
                   int64_t lb_den, int lb_valid, int64_t* part, int64_t* out2, hipStream_t s) {
    const unsigned nb = grid_for(g->m, kSelBlocks);
    hipLaunchKernelGGL(k_sel_min, dim3(nb), dim3(kThreads), 0, s, g->dsum, t, g->m, measure,
                       key, lb_num, lb_den, lb_valid, part);
    hipLaunchKernelGGL(k_sel_min_final, dim3(1), dim3(64), 0, s, part, (int)nb, out2);
}

void sel_count_eq(const mcd_graph* g, int measure, const int32_t* t, uint32_t key, int64_t num,
                  int64_t den, int64_t* cnt, hipStream_t s) {
    fill_i64(cnt, 1, 0, s);
    hipLaunchKernelGGL(k_sel_count_eq, dim3(grid_for(g->m, kSelBlocks)), dim3(kThreads), 0, s, g->dsum, t, g->m,
                       measure, key, num, den, (unsigned long long*)cnt);
}

}  // namespace mcd
