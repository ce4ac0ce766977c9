// Learned threshold picker: per-graph features of the Tectonic similarity
// distribution, an FP32 MLP 66 -> 64 -> 64 -> 1 (ReLU) with hand-written
// forward, backward (mean squared error) and Adam kernels, the snap of its
// output to a threshold grid, and the training targets from a sweep.
//
// Parameter layout (8513 floats): W1[64][66], b1[64], W2[64][64], b2[64],
// W3[64], b3.  Features are standardised inside the forward pass with the
// caller's mean/std vectors.  Gradients are summed over the batch in a fixed
// order (per-row partials, then a column reduction), so a training step is
// deterministic.
#include "common.hpp"

namespace mcd {
namespace {

constexpr int kThreads = 256;
constexpr int NI = MCD_MLP_IN, NH = MCD_MLP_HIDDEN;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPAR = OFF_B3 + 1;
static_assert(NPAR == MCD_MLP_PARAMS, "parameter count");

inline unsigned grid_for(int64_t N, int64_t cap) {
    int64_t b = (N + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

#define GRID_STRIDE(i, N)                                                              \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (N);          \
         i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_fill_ull(unsigned long long* __restrict__ p, int64_t N) {
    GRID_STRIDE(i, N) p[i] = 0ull;
}

// ---------------------------------------------------------------- features

// graph of every rank-numbered vertex (binary search of vbase on its id)
__device__ __forceinline__ int graph_of(const int64_t* __restrict__ vbase, int G, int64_t x) {
    int lo = 0, hi = G;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (vbase[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// hist[g][b] over edges, bin = floor(128 t / D) (integer division, < 64 since
// t <= min degree - 1); mdeg[g] = max degree
__global__ __launch_bounds__(kThreads) void k_feat_hist(const int32_t* __restrict__ src,
                                                        const int32_t* __restrict__ dsum,
                                                        const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ t, int64_t m,
                                                        const int64_t* __restrict__ vbase, int G,
                                                        unsigned long long* __restrict__ hist) {
    // one graph: 8 copies of the 64 bins per wave, picked by lane (stride 65
    // words: the copies sit in different banks), so lanes with equal bins
    // (t = 0 above all) collide at most 8 ways; batches: one (graph, bin)
    // table per block when it fits
    constexpr int kCopies = 8, kStride = 65;
    __shared__ uint32_t h[4096];
    const bool local = G * 64 <= 4096;
    const int nloc = G == 1 ? (kThreads / 64) * kCopies * kStride : G * 64;
    if (local)
        for (int i = threadIdx.x; i < nloc; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    GRID_STRIDE(e, m) {
        const uint32_t D = (uint32_t)dsum[e];
        const uint32_t tt = (uint32_t)t[e];
        // floor(128 t / D) without a 64-bit division: an fp32 estimate (off by
        // at most one near a bin edge), then one exact integer correction
        int b = (int)(128.0f * (float)tt * __frcp_rn((float)D));
        const uint64_t num = (uint64_t)tt << 7;
        if (b > 0 && num < (uint64_t)b * D) --b;
        else if (num >= (uint64_t)(b + 1) * D) ++b;
        if (b > 63) b = 63;
        if (G == 1) {
            atomicAdd(&h[((threadIdx.x >> 6) * kCopies + (lane & (kCopies - 1))) * kStride + b], 1u);
        } else {
            const int g = graph_of(vbase, G, perm[src[e]]);
            if (local) atomicAdd(&h[g * 64 + b], 1u);
            else atomicAdd(&hist[(int64_t)g * 64 + b], 1ull);
        }
    }
    __syncthreads();
    if (G == 1) {
        for (int i = threadIdx.x; i < 64; i += blockDim.x) {
            uint32_t c = 0;
            for (int k = 0; k < (kThreads / 64) * kCopies; ++k) c += h[k * kStride + i];
            if (c) atomicAdd(&hist[i], (unsigned long long)c);
        }
    } else if (local) {
        for (int i = threadIdx.x; i < G * 64; i += blockDim.x)
            if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
    }
}

// max degree per graph; lanes sharing lane 0's graph reduce before one atomic.
// One graph: each thread keeps its maximum over the grid-stride loop and the
// block reduces it, one atomic per block (one address would otherwise take an
// atomic from every wave and iteration, serialised at the memory).
__global__ __launch_bounds__(kThreads) void k_feat_maxdeg(const int32_t* __restrict__ deg,
                                                          const int32_t* __restrict__ perm, int64_t n,
                                                          const int64_t* __restrict__ vbase, int G,
                                                          unsigned long long* __restrict__ mdeg) {
    if (G == 1) {
        __shared__ unsigned long long wmax[kThreads / 64];
        unsigned long long x = 0;
        GRID_STRIDE(v, n) {
            const unsigned long long d = (unsigned long long)deg[v];
            x = d > x ? d : x;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long y = __shfl_xor(x, o);
            x = y > x ? y : x;
        }
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < kThreads / 64; ++i) x = wmax[i] > x ? wmax[i] : x;
            if (x) atomicMax(&mdeg[0], x);
        }
        return;
    }
    GRID_STRIDE(v, n) {
        const int g = G == 1 ? 0 : graph_of(vbase, G, perm[v]);
        const unsigned long long d = (unsigned long long)deg[v];
        const int g0 = __shfl(g, 0);
        unsigned long long x = g == g0 ? d : 0ull;
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long y = __shfl_xor(x, o);
            x = y > x ? y : x;
        }
        if ((threadIdx.x & 63) == 0 && x) atomicMax(&mdeg[g0], x);
        if (g != g0) atomicMax(&mdeg[g], d);
    }
}

// x[g] = (hist / m_g, log1p(2 m_g / n_g), log1p(max degree))
__global__ __launch_bounds__(64) void k_feat_finish(const unsigned long long* __restrict__ hist,
                                                    const unsigned long long* __restrict__ mdeg,
                                                    const int64_t* __restrict__ vbase, int G,
                                                    float* __restrict__ x) {
    const int g = blockIdx.x;
    if (g >= G) return;
    __shared__ unsigned long long msum;
    if (threadIdx.x == 0) msum = 0;
    __syncthreads();
    const unsigned long long c = hist[(int64_t)g * 64 + threadIdx.x];
    atomicAdd(&msum, c);
    __syncthreads();
    const double mg = (double)msum;
    const double ng = (double)(vbase[g + 1] - vbase[g]);
    x[(int64_t)g * NI + threadIdx.x] = mg > 0 ? (float)((double)c / mg) : 0.f;
    if (threadIdx.x == 0) {
        x[(int64_t)g * NI + 64] = (float)log1p(ng > 0 ? 2.0 * mg / ng : 0.0);
        x[(int64_t)g * NI + 65] = (float)log1p((double)mdeg[g]);
    }
}

// ------------------------------------------------------------------- MLP

// One workgroup of 64 threads per row; h1/h2 (after ReLU) and the
// standardised input are kept for the backward pass when `keep` is set.
__global__ __launch_bounds__(64) void k_mlp_fwd(const float* __restrict__ p, const float* __restrict__ mean,
                                                const float* __restrict__ stdv, const float* __restrict__ x,
                                                int B, float* __restrict__ y, float* __restrict__ keep_xs,
                                                float* __restrict__ keep_h1, float* __restrict__ keep_h2) {
    const int r = blockIdx.x, j = threadIdx.x;
    if (r >= B) return;
    __shared__ float xs[NI], h1[NH], h2[NH];
    for (int k = j; k < NI; k += 64) xs[k] = (x[(int64_t)r * NI + k] - mean[k]) / stdv[k];
    __syncthreads();
    float a = p[OFF_B1 + j];
    for (int k = 0; k < NI; ++k) a += p[OFF_W1 + j * NI + k] * xs[k];
    h1[j] = a > 0.f ? a : 0.f;
    __syncthreads();
    float b = p[OFF_B2 + j];
    for (int k = 0; k < NH; ++k) b += p[OFF_W2 + j * NH + k] * h1[k];
    h2[j] = b > 0.f ? b : 0.f;
    __syncthreads();
    float c = p[OFF_W3 + j] * h2[j];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (j == 0) y[r] = c + p[OFF_B3];
    if (keep_xs) {
        for (int k = j; k < NI; k += 64) keep_xs[(int64_t)r * NI + k] = xs[k];
        keep_h1[(int64_t)r * NH + j] = h1[j];
        keep_h2[(int64_t)r * NH + j] = h2[j];
    }
}

// The training loss of one row with output y (MlpLoss): mse_w (y - target)^2,
// minus, when the row's ARI curve a[0..K-1] is given, the ARI interpolated
// linearly at z = (K-1) y clamped to [0, K-1].  The segment index is decided
// in fp32.  Returns the loss; *dldy its derivative in y (the ARI term's slope
// is 0 outside 0 < z < K-1).
__device__ __forceinline__ float row_loss(const MlpLoss& L, int r, float y, float* dldy) {
    const float d = y - L.target[r];
    float loss = L.mse_w * d * d, g = 2.f * L.mse_w * d;
    if (L.ari) {
        const double* a = L.ari + (int64_t)r * L.K;
        const float zmax = (float)(L.K - 1);
        const float z = fminf(fmaxf(zmax * y, 0.f), zmax);
        int i0 = (int)floorf(z);
        if (i0 > L.K - 2) i0 = L.K - 2;
        const float a0 = (float)a[i0], a1 = (float)a[i0 + 1];
        loss -= a0 + (z - (float)i0) * (a1 - a0);
        const float zy = zmax * y;
        if (zy > 0.f && zy < zmax) g -= zmax * (a1 - a0);
    }
    *dldy = g;
    return loss;
}

// Per-row gradient of the mean of row_loss over the batch into part[r][NPAR].
__global__ __launch_bounds__(64) void k_mlp_bwd_row(const float* __restrict__ p, const float* __restrict__ xs_all,
                                                    const float* __restrict__ h1_all,
                                                    const float* __restrict__ h2_all,
                                                    const float* __restrict__ y, MlpLoss L,
                                                    int B, float* __restrict__ part) {
    const int r = blockIdx.x, j = threadIdx.x;
    if (r >= B) return;
    __shared__ float xs[NI], h1[NH], dh2[NH];
    for (int k = j; k < NI; k += 64) xs[k] = xs_all[(int64_t)r * NI + k];
    h1[j] = h1_all[(int64_t)r * NH + j];
    const float h2 = h2_all[(int64_t)r * NH + j];
    float dldy;
    row_loss(L, r, y[r], &dldy);
    const float dy = dldy / (float)B;
    float* g = part + (int64_t)r * NPAR;
    g[OFF_W3 + j] = dy * h2;
    if (j == 0) g[OFF_B3] = dy;
    dh2[j] = h2 > 0.f ? dy * p[OFF_W3 + j] : 0.f;
    __syncthreads();
    for (int k = 0; k < NH; ++k) g[OFF_W2 + j * NH + k] = dh2[j] * h1[k];
    g[OFF_B2 + j] = dh2[j];
    // dh1[j] = sum_i W2[i][j] dh2[i], masked by ReLU
    float s = 0.f;
    for (int i = 0; i < NH; ++i) s += p[OFF_W2 + i * NH + j] * dh2[i];
    const float dh1 = h1[j] > 0.f ? s : 0.f;
    for (int k = 0; k < NI; ++k) g[OFF_W1 + j * NI + k] = dh1 * xs[k];
    g[OFF_B1 + j] = dh1;
}

// grad[q] = sum over rows r = 0..B-1 (in order) of part[r][q]; loss likewise
__global__ __launch_bounds__(kThreads) void k_mlp_reduce(const float* __restrict__ part, int B,
                                                         const float* __restrict__ y, MlpLoss L,
                                                         float* __restrict__ grad, float* __restrict__ loss) {
    GRID_STRIDE(q, NPAR) {
        float s = 0.f;
        for (int r = 0; r < B; ++r) s += part[(int64_t)r * NPAR + q];
        grad[q] = s;
    }
    if (loss && blockIdx.x == 0 && threadIdx.x == 0) {
        float l = 0.f, unused;
        for (int r = 0; r < B; ++r) l += row_loss(L, r, y[r], &unused);
        *loss = l / (float)B;
    }
}

// Adam (Kingma & Ba) with bias correction; step counts from 1.  Weight decay
// is decoupled (Loshchilov & Hutter): p -= lr * wd * p before the Adam update.
__global__ __launch_bounds__(kThreads) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m1, float* __restrict__ m2, int step,
                                                   float lr, float wd, float beta1, float beta2, float eps) {
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    GRID_STRIDE(q, NPAR) {
        const float gq = g[q];
        const float a = beta1 * m1[q] + (1.f - beta1) * gq;
        const float b = beta2 * m2[q] + (1.f - beta2) * gq * gq;
        m1[q] = a;
        m2[q] = b;
        const float pq = p[q] - lr * wd * p[q];
        p[q] = pq - lr * (a / c1) / (sqrtf(b / c2) + eps);
    }
}

// index = clamp(round((K-1) y), 0, K-1); delta = (a + b index) / c
__global__ __launch_bounds__(kThreads) void k_select(const float* __restrict__ y, int B, int K, int64_t a,
                                                     int64_t b, int64_t c, int32_t* __restrict__ index,
                                                     int64_t* __restrict__ delta) {
    GRID_STRIDE(r, B) {
        float q = rintf((float)(K - 1) * y[r]);
        q = fminf(fmaxf(q, 0.f), (float)(K - 1));
        const int32_t i = (int32_t)q;
        if (index) index[r] = i;
        if (delta) {
            delta[2 * r] = a + b * i;
            delta[2 * r + 1] = c;
        }
    }
}

// Training target per graph: the centroid of the thresholds whose ARI is
// within a fraction of the best, i.e. ARI >= best - (1 - frac) |best|
// (frac = 1: the centroid of the exact maxima); index = round-half-down of the
// centroid, y = centroid / (K - 1).
__global__ __launch_bounds__(kThreads) void k_targets(const double* __restrict__ ari, int G, int K, double frac,
                                                      int32_t* __restrict__ index, float* __restrict__ y) {
    GRID_STRIDE(g, G) {
        const double* a = ari + (int64_t)g * K;
        double best = a[0];
        for (int i = 1; i < K; ++i) best = fmax(best, a[i]);
        const double cut = best - (1.0 - frac) * fabs(best);
        int64_t s = 0, c = 0;
        for (int i = 0; i < K; ++i)
            if (a[i] >= cut) {
                s += i;
                ++c;
            }
        // centroid = s / c; round half down in exact integer arithmetic
        const int32_t mid = (int32_t)((2 * s + c - 1) / (2 * c));
        if (index) index[g] = mid;
        if (y) y[g] = (float)((double)s / (double)c / (double)(K - 1));
    }
}

// column mean and standard deviation (population), the latter raised to at
// least min_std so near-constant columns are not blown up
__global__ __launch_bounds__(64) void k_feat_stats(const float* __restrict__ x, int B, float min_std,
                                                   float* __restrict__ mean, float* __restrict__ stdv) {
    for (int k = threadIdx.x; k < NI; k += 64) {
        double s = 0, ss = 0;
        for (int r = 0; r < B; ++r) {
            const double v = x[(int64_t)r * NI + k];
            s += v;
            ss += v * v;
        }
        const double mu = s / B;
        double var = ss / B - mu * mu;
        if (var < 0) var = 0;
        const double sd = sqrt(var);
        mean[k] = (float)mu;
        stdv[k] = (float)fmax(sd, (double)min_std);
    }
}

// column minimum and maximum
__global__ __launch_bounds__(64) void k_feat_range(const float* __restrict__ x, int B, float* __restrict__ lo,
                                                   float* __restrict__ hi) {
    for (int k = threadIdx.x; k < NI; k += 64) {
        float a = x[k], b = x[k];
        for (int r = 1; r < B; ++r) {
            const float v = x[(int64_t)r * NI + k];
            a = fminf(a, v);
            b = fmaxf(b, v);
        }
        lo[k] = a;
        hi[k] = b;
    }
}

// Graph g is outside the training range when some feature leaves
// [lo - margin (hi - lo), hi + margin (hi - lo)]; its threshold is then the
// fallback's.  The bounds are formed in fp32 with one rounding per operation
// (no fused multiply-add), as the oracle does.
__global__ __launch_bounds__(kThreads) void k_fallback(const float* __restrict__ x, int B,
                                                       const float* __restrict__ lo, const float* __restrict__ hi,
                                                       float margin, const int64_t* __restrict__ picked,
                                                       const int64_t* __restrict__ fallback,
                                                       int64_t* __restrict__ delta, int32_t* __restrict__ flags) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < B; g += gridDim.x * blockDim.x) {
        bool out = false;
        for (int k = 0; k < NI; ++k) {
            const float w = __fmul_rn(margin, __fsub_rn(hi[k], lo[k]));
            const float v = x[(int64_t)g * NI + k];
            out |= v < __fsub_rn(lo[k], w) || v > __fadd_rn(hi[k], w);
        }
        if (flags) flags[g] = out ? 1 : 0;
        if (delta) {
            const int64_t* src = out ? fallback : picked;
            const int64_t num = src[2 * g], den = src[2 * g + 1];
            delta[2 * g] = num;
            delta[2 * g + 1] = den;
        }
    }
}

}  // namespace

void launch_feature_range(const float* x, int B, float* lo, float* hi, hipStream_t s) {
    hipLaunchKernelGGL(k_feat_range, dim3(1), dim3(64), 0, s, x, B, lo, hi);
}

void launch_fallback(const float* x, int B, const float* lo, const float* hi, float margin, const int64_t* picked,
                     const int64_t* fallback, int64_t* delta, int32_t* flags, hipStream_t s) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_fallback, dim3(grid_for(B, 1024)), dim3(kThreads), 0, s, x, B, lo, hi, margin, picked,
                       fallback, delta, flags);
}

// One block: *any = whether some flag is set (the picker's decision to run
// the sweep, taken on the device).
__global__ __launch_bounds__(kThreads) void k_any_flag(const int32_t* __restrict__ flags, int B,
                                                       int32_t* __restrict__ any) {
    __shared__ int hit;
    if (threadIdx.x == 0) hit = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < B; i += blockDim.x)
        if (flags[i]) hit = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) *any = hit;
}

void launch_any_flag(const int32_t* flags, int B, int32_t* any, hipStream_t s) {
    hipLaunchKernelGGL(k_any_flag, dim3(1), dim3(kThreads), 0, s, flags, B, any);
}

size_t features_scratch_bytes(int G) { return mcd_align(sizeof(unsigned long long) * (size_t)G * 65); }

void launch_features(const mcd_graph* g, const int32_t* t, int G, const int64_t* vbase, float* x, void* ws,
                     hipStream_t s) {
    unsigned long long* hist = (unsigned long long*)ws;
    unsigned long long* mdeg = hist + (size_t)G * 64;
    hipLaunchKernelGGL((k_fill_ull), dim3(grid_for((int64_t)G * 65, 1024)), dim3(kThreads), 0, s, hist,
                       (int64_t)G * 65);
    if (g->m > 0)
        hipLaunchKernelGGL(k_feat_hist, dim3(grid_for(g->m, 4096)), dim3(kThreads), 0, s, g->src, g->dsum,
                           g->perm, t, g->m, vbase, G, hist);
    if (g->n > 0)
        hipLaunchKernelGGL(k_feat_maxdeg, dim3(grid_for(g->n, 4096)), dim3(kThreads), 0, s, g->deg, g->perm,
                           g->n, vbase, G, mdeg);
    hipLaunchKernelGGL(k_feat_finish, dim3(G), dim3(64), 0, s, hist, mdeg, vbase, G, x);
}

size_t mlp_scratch_bytes(int B) {
    return mcd_align(sizeof(float) * (size_t)B * (NI + 2 * NH + NPAR + 2) + sizeof(float) * NPAR);
}

struct MlpWs {
    float *xs, *h1, *h2, *part, *y, *grad;
};

static MlpWs mlp_ws(void* ws, int B) {
    MlpWs w;
    float* f = (float*)ws;
    w.xs = f;
    w.h1 = w.xs + (size_t)B * NI;
    w.h2 = w.h1 + (size_t)B * NH;
    w.part = w.h2 + (size_t)B * NH;
    w.y = w.part + (size_t)B * NPAR;
    w.grad = w.y + (size_t)B + 2;
    return w;
}

void launch_mlp_forward(const float* params, const float* mean, const float* stdv, const float* x, int B,
                        float* y, hipStream_t s) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, s, params, mean, stdv, x, B, y, (float*)nullptr,
                       (float*)nullptr, (float*)nullptr);
}

void launch_mlp_gradient(const float* params, const float* mean, const float* stdv, const float* x,
                         const MlpLoss& L, int B, float* grad, float* loss, void* ws, hipStream_t s) {
    MlpWs w = mlp_ws(ws, B);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, s, params, mean, stdv, x, B, w.y, w.xs, w.h1, w.h2);
    hipLaunchKernelGGL(k_mlp_bwd_row, dim3(B), dim3(64), 0, s, params, w.xs, w.h1, w.h2, w.y, L, B, w.part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(NPAR, 64)), dim3(kThreads), 0, s, w.part, B, w.y, L,
                       grad ? grad : w.grad, loss);
}

void launch_mlp_train_step(float* params, float* m1, float* m2, int step, float lr, float wd, const float* mean,
                           const float* stdv, const float* x, const MlpLoss& L, int B, float* loss, void* ws,
                           hipStream_t s) {
    MlpWs w = mlp_ws(ws, B);
    launch_mlp_gradient(params, mean, stdv, x, L, B, w.grad, loss, ws, s);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(NPAR, 64)), dim3(kThreads), 0, s, params, w.grad, m1, m2, step, lr,
                       wd, 0.9f, 0.999f, 1e-8f);
}

void launch_select(const float* y, int B, int K, int64_t a, int64_t b, int64_t c, int32_t* index,
                   int64_t* delta, hipStream_t s) {
    if (B <= 0) return;
    hipLaunchKernelGGL(k_select, dim3(grid_for(B, 1024)), dim3(kThreads), 0, s, y, B, K, a, b, c, index, delta);
}

void launch_targets(const double* ari, int G, int K, double frac, int32_t* index, float* y, hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(k_targets, dim3(grid_for(G, 1024)), dim3(kThreads), 0, s, ari, G, K, frac, index, y);
}

void launch_feature_stats(const float* x, int B, float min_std, float* mean, float* stdv, hipStream_t s) {
    hipLaunchKernelGGL(k_feat_stats, dim3(1), dim3(64), 0, s, x, B, min_std, mean, stdv);
}

}  // namespace mcd
