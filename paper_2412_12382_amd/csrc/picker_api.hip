// The learned threshold picker as a library object (mcd_picker_*): its device
// state, the He-uniform initialisation from a counter-based generator, the
// training loop, the pick sequence (features -> MLP -> grid snap -> range
// guard -> the sweep's rule of thumb where the guard fires -> prune and
// components) and a versioned checkpoint file with a CRC.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "common.hpp"

struct mcd_picker {
    mcd_ctx* ctx;
    float* block;  // one device allocation holding every array below
    float* params;
    float* adam_m;
    float* adam_v;
    float* mean;
    float* stdv;
    float* lo;
    float* hi;
    float margin;
    int32_t step;      // Adam steps taken since the last mcd_picker_prepare
    int32_t prepared;  // standardisation and training range are set
};

namespace {

#define REQUIRE(cond, code, msg)                 \
    do {                                         \
        if (!(cond)) return mcd_fail(code, msg); \
    } while (0)

constexpr int NI = MCD_MLP_IN, NH = MCD_MLP_HIDDEN, NPAR = MCD_MLP_PARAMS;
constexpr int kGridK = MCD_PICKER_GRID_K;
constexpr int64_t kGridA = MCD_PICKER_GRID_A, kGridB = MCD_PICKER_GRID_B, kGridC = MCD_PICKER_GRID_C;
constexpr uint32_t kInitTag = 0x4D4C5030u;  // "MLP0": stream of the initial weights
constexpr uint32_t kInitSub = 0x55u;

// Philox-4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): each round multiplies words 0 and 2
// by the two round constants, swaps the halves across, and xors in the key;
// the key is bumped by the golden-ratio Weyl increments between rounds.
void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * c[0];
        const uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t x0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
        const uint32_t x2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)b;
        c[3] = (uint32_t)a;
        c[0] = x0;
        c[2] = x2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform in (0, 1) of draw i of a stream: counter (i, sub, tag) under the
// 64-bit seed as key; 53 bits from the first two output words, shifted by
// half a step so 0 never occurs.
#pragma clang fp contract(off)
double uniform01(uint64_t seed, uint32_t tag, uint64_t i) {
    uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), kInitSub, tag};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t v = ((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6);
    return (double)v * (1.0 / 9007199254740992.0) + 0.5 / 9007199254740992.0;
}

// He-uniform initial parameters: every weight of a layer with fan-in f is
// (2 u - 1) sqrt(6 / f) for its own draw u (draw index = its position in the
// flat vector), rounded once to fp32; biases start at zero.
void he_uniform(uint64_t seed, float* p) {
    const int fan_out[3] = {NH, NH, 1}, fan_in[3] = {NI, NH, NH};
    int o = 0;
    for (int l = 0; l < 3; ++l) {
        const double bound = sqrt(6.0 / (double)fan_in[l]);
        const int k = fan_out[l] * fan_in[l];
        for (int i = 0; i < k; ++i) p[o + i] = (float)((2.0 * uniform01(seed, kInitTag, (uint64_t)(o + i)) - 1.0) * bound);
        o += k;
        for (int i = 0; i < fan_out[l]; ++i) p[o + i] = 0.f;
        o += fan_out[l];
    }
}
#pragma clang fp contract(on)

// CRC-32 of the checkpoint (the reflected IEEE 802.3 polynomial 0xEDB88320,
// initial value and final xor all ones), bit by bit.
uint32_t crc32(const unsigned char* d, size_t n) {
    uint32_t c = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; ++i) {
        c ^= d[i];
        for (int b = 0; b < 8; ++b) c = (c >> 1) ^ (0xEDB88320u & (0u - (c & 1u)));
    }
    return c ^ 0xFFFFFFFFu;
}

// Checkpoint file (little-endian), version 1:
//   0  char[8]  "MCDPICK\0"
//   8  uint32   version
//   12 uint32   inputs (66), hidden (64), parameters (8513)
//   24 int32    grid K, int32 zero
//   32 int64    grid a, b, c   (delta_i = (a + b i) / c)
//   56 float    margin of the range guard, uint32 zero
//   64 float    params[8513], mean[66], std[66], lo[66], hi[66]
//   .. uint32   CRC-32 of every byte before it
constexpr char kMagic[8] = {'M', 'C', 'D', 'P', 'I', 'C', 'K', 0};
constexpr uint32_t kVersion = 1;
constexpr size_t kHeader = 64;
constexpr size_t kFloats = (size_t)NPAR + 4 * NI;
constexpr size_t kFileBytes = kHeader + 4 * kFloats + 4;

template <class T>
void put(std::vector<unsigned char>& b, size_t off, T v) {
    memcpy(b.data() + off, &v, sizeof(T));
}
template <class T>
T get(const std::vector<unsigned char>& b, size_t off) {
    T v;
    memcpy(&v, b.data() + off, sizeof(T));
    return v;
}

mcd_status use_device(const mcd_ctx* ctx) {
    MCD_HIP(hipSetDevice(ctx->device));
    return MCD_OK;
}

// The picker's grid as sweep thresholds (ascending, so the order is the identity).
void grid_deltas(mcd::SweepDeltas* ds, int* order) {
    ds->K = kGridK;
    for (int i = 0; i < kGridK; ++i) {
        ds->num[i] = kGridA + kGridB * i;
        ds->den[i] = kGridC;
        order[i] = i;
    }
}

struct PickLayout {
    void* feat;
    float* x;
    float* y;
    int32_t* index;
    int64_t* deltas;
    int32_t* flags;
    void* sweep;
    mcd_sweep_stats* stats;
    double* q;
    int32_t* rule_index;
    int64_t* rule_deltas;
    int32_t* any;
    void* cc;
    size_t bytes;
};

PickLayout pick_layout(void* ws, const mcd_graph* g, int G) {
    Carve c{(char*)ws, 0, ~(size_t)0};
    PickLayout L;
    L.feat = c.take<char>(mcd::features_scratch_bytes(G));
    L.x = c.take<float>((size_t)G * NI);
    L.y = c.take<float>(G);
    L.index = c.take<int32_t>(G);
    L.deltas = c.take<int64_t>(2 * (size_t)G);
    L.flags = c.take<int32_t>(G);
    L.sweep = c.take<char>(mcd::sweep_scratch_bytes(g, G, kGridK, false));
    L.stats = c.take<mcd_sweep_stats>((size_t)G * kGridK);
    L.q = c.take<double>((size_t)G * kGridK);
    L.rule_index = c.take<int32_t>(G);
    L.rule_deltas = c.take<int64_t>(2 * (size_t)G);
    L.any = c.take<int32_t>(1);
    L.cc = c.take<char>(mcd::cc_scratch_bytes(g));
    L.bytes = c.used;
    return L;
}

bool finite_all(const float* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return false;
    return true;
}

// Reads and checks a checkpoint file into b: length, magic, version, CRC,
// network shape, grid, finite values, positive standard deviations.
mcd_status read_checkpoint(const char* path, std::vector<unsigned char>& b) {
    REQUIRE(path, MCD_ERR_INVALID_ARG, "path is NULL");
    FILE* fp = fopen(path, "rb");
    REQUIRE(fp, MCD_ERR_CHECKPOINT, std::string("cannot open ") + path);
    b.assign(kFileBytes + 1, 0);
    const size_t r = fread(b.data(), 1, b.size(), fp);
    fclose(fp);
    REQUIRE(r == kFileBytes, MCD_ERR_CHECKPOINT,
            std::string("checkpoint ") + path + " has the wrong length (truncated or trailing bytes)");
    b.resize(kFileBytes);
    REQUIRE(memcmp(b.data(), kMagic, 8) == 0, MCD_ERR_CHECKPOINT, "not a picker checkpoint (bad magic)");
    REQUIRE(get<uint32_t>(b, 8) == kVersion, MCD_ERR_CHECKPOINT, "unsupported checkpoint version");
    REQUIRE(crc32(b.data(), kFileBytes - 4) == get<uint32_t>(b, kFileBytes - 4), MCD_ERR_CHECKPOINT,
            "checkpoint CRC mismatch (corrupted file)");
    REQUIRE(get<uint32_t>(b, 12) == (uint32_t)NI && get<uint32_t>(b, 16) == (uint32_t)NH &&
                get<uint32_t>(b, 20) == (uint32_t)NPAR,
            MCD_ERR_CHECKPOINT, "checkpoint network shape differs from 66 -> 64 -> 64 -> 1");
    REQUIRE(get<int32_t>(b, 24) == kGridK && get<int64_t>(b, 32) == kGridA && get<int64_t>(b, 40) == kGridB &&
                get<int64_t>(b, 48) == kGridC,
            MCD_ERR_CHECKPOINT, "checkpoint threshold grid differs from (9 + 7 i) / 900, i < 64");
    const float margin = get<float>(b, 56);
    const float* f = (const float*)(b.data() + kHeader);
    REQUIRE(isfinite(margin) && margin >= 0.f && finite_all(f, kFloats), MCD_ERR_CHECKPOINT,
            "checkpoint holds non-finite values or a negative margin");
    for (int k = 0; k < NI; ++k)
        REQUIRE(f[NPAR + NI + k] > 0.f, MCD_ERR_CHECKPOINT, "checkpoint standard deviation not positive");
    return MCD_OK;
}

}  // namespace

// The library is built with hidden visibility; the C ABI below is exported.
#pragma GCC visibility push(default)
extern "C" {

mcd_status mcd_picker_create(mcd_ctx* ctx, uint64_t seed, mcd_picker** out) {
    REQUIRE(ctx && out, MCD_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    mcd_picker* p = new mcd_picker();
    p->ctx = ctx;
    const size_t per = (size_t)NPAR * 3 + 4 * (size_t)NI;
    if (hipMalloc((void**)&p->block, per * sizeof(float)) != hipSuccess) {
        delete p;
        return mcd_fail(MCD_ERR_DEVICE, "hipMalloc of the picker state failed");
    }
    p->params = p->block;
    p->adam_m = p->params + NPAR;
    p->adam_v = p->adam_m + NPAR;
    p->mean = p->adam_v + NPAR;
    p->stdv = p->mean + NI;
    p->lo = p->stdv + NI;
    p->hi = p->lo + NI;
    p->margin = MCD_PICKER_MARGIN;
    // host image: initial weights, zero moments, identity standardisation
    // and an empty training range (the picker is not prepared yet)
    std::vector<float> h(per, 0.f);
    he_uniform(seed, h.data());
    for (int k = 0; k < NI; ++k) h[3 * (size_t)NPAR + NI + k] = 1.f;
    hipError_t e = hipMemcpyAsync(p->block, h.data(), per * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(p->block);
        delete p;
        return mcd_fail(MCD_ERR_DEVICE, std::string("copying the initial picker state: ") + hipGetErrorString(e));
    }
    *out = p;
    return MCD_OK;
}

mcd_status mcd_picker_destroy(mcd_picker* p) {
    if (!p) return MCD_OK;
    // the stream may still use the state: wait for it before freeing
    hipError_t e = hipSetDevice(p->ctx->device);
    if (e == hipSuccess) e = hipStreamSynchronize(p->ctx->stream);
    const hipError_t f = hipFree(p->block);
    delete p;
    if (e != hipSuccess || f != hipSuccess)
        return mcd_fail(MCD_ERR_DEVICE, std::string("releasing the picker: ") + hipGetErrorString(e != hipSuccess ? e : f));
    return MCD_OK;
}

mcd_status mcd_picker_prepare(mcd_picker* p, const float* x, int32_t batch, float min_std, float margin) {
    REQUIRE(p && x && batch >= 1, MCD_ERR_INVALID_ARG, "NULL argument or empty batch");
    REQUIRE(min_std > 0.f, MCD_ERR_INVALID_ARG, "min_std must be positive");
    REQUIRE(margin >= 0.f && isfinite(margin), MCD_ERR_INVALID_ARG, "margin must be finite and non-negative");
    mcd_status st = use_device(p->ctx);
    if (st != MCD_OK) return st;
    hipStream_t s = p->ctx->stream;
    mcd::launch_feature_stats(x, batch, min_std, p->mean, p->stdv, s);
    mcd::launch_feature_range(x, batch, p->lo, p->hi, s);
    // fresh Adam moments (a fill kernel: the call stays capturable)
    mcd::fill_i32((int32_t*)p->adam_m, 2 * (int64_t)NPAR, 0, s);
    p->margin = margin;
    p->step = 0;
    p->prepared = 1;
    return MCD_OK;
}

mcd_status mcd_picker_train_step(mcd_picker* p, const float* x, const float* y, const double* ari, float mse_weight,
                                 int32_t batch, float lr, float weight_decay, float* loss, void* ws, size_t ws_bytes) {
    REQUIRE(p && x && y && ws && batch >= 1, MCD_ERR_INVALID_ARG, "NULL argument or empty batch");
    REQUIRE(mse_weight >= 0.f && mse_weight < 1e30f, MCD_ERR_INVALID_ARG, "mse_weight must be finite and >= 0");
    REQUIRE(((uintptr_t)ws & 255u) == 0u, MCD_ERR_INVALID_ARG, "ws must be 256-byte aligned");
    REQUIRE(p->prepared, MCD_ERR_INVALID_ARG, "mcd_picker_prepare must come before training");
    REQUIRE(ws_bytes >= mcd::mlp_scratch_bytes(batch), MCD_ERR_WORKSPACE, "MLP workspace too small");
    REQUIRE(p->step < INT32_MAX, MCD_ERR_RANGE, "too many Adam steps");
    mcd_status st = use_device(p->ctx);
    if (st != MCD_OK) return st;
    p->step += 1;
    const mcd::MlpLoss L{y, ari, kGridK, mse_weight};
    mcd::launch_mlp_train_step(p->params, p->adam_m, p->adam_v, p->step, lr, weight_decay, p->mean, p->stdv, x, L,
                               batch, loss, ws, p->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_picker_fit(mcd_picker* p, const float* x, const float* y, const double* ari, float mse_weight,
                          int32_t batch, int32_t steps, float lr, float weight_decay, float min_std, float margin,
                          float* losses, void* ws, size_t ws_bytes) {
    REQUIRE(p && steps >= 0, MCD_ERR_INVALID_ARG, "NULL picker or negative step count");
    mcd_status st = mcd_picker_prepare(p, x, batch, min_std, margin);
    if (st != MCD_OK) return st;
    for (int32_t k = 0; k < steps; ++k)
        if ((st = mcd_picker_train_step(p, x, y, ari, mse_weight, batch, lr, weight_decay,
                                        losses ? losses + k : nullptr, ws, ws_bytes)) != MCD_OK)
            return st;
    return MCD_OK;
}

mcd_status mcd_picker_forward(const mcd_picker* p, const float* x, int32_t batch, float* y) {
    REQUIRE(p && batch >= 0 && (batch == 0 || (x && y)), MCD_ERR_INVALID_ARG, "NULL argument");
    mcd_status st = use_device(p->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_mlp_forward(p->params, p->mean, p->stdv, x, batch, y, p->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_picker_pick_workspace_size(const mcd_graph* g, int32_t n_graphs, size_t* bytes) {
    REQUIRE(g && bytes && n_graphs >= 1, MCD_ERR_INVALID_ARG, "NULL argument or n_graphs < 1");
    *bytes = pick_layout(nullptr, g, n_graphs).bytes;
    return MCD_OK;
}

mcd_status mcd_picker_pick(const mcd_picker* p, const mcd_graph* g, mcd_measure measure, const int32_t* t,
                           int32_t n_graphs, const int64_t* vbase, int32_t mode, int32_t* index, int64_t* deltas,
                           int32_t* used_fallback, int32_t* labels, int64_t* n_components, void* ws,
                           size_t ws_bytes) {
    REQUIRE(p && g && vbase && ws && (g->m == 0 || t) && (g->n == 0 || labels), MCD_ERR_INVALID_ARG,
            "NULL argument");
    REQUIRE(((uintptr_t)ws & 255u) == 0u, MCD_ERR_INVALID_ARG, "ws must be 256-byte aligned");
    REQUIRE(n_graphs >= 1, MCD_ERR_INVALID_ARG, "need n_graphs >= 1");
    REQUIRE(p->ctx->device == g->ctx->device, MCD_ERR_INVALID_ARG, "picker and graph live on different devices");
    REQUIRE(p->prepared, MCD_ERR_INVALID_ARG, "the picker has no standardisation: prepare, fit or load it first");
    REQUIRE(measure == MCD_SIM_TECTONIC || measure == MCD_SIM_TW || measure == MCD_SIM_K3 ||
                measure == MCD_SIM_JACCARD || measure == MCD_SIM_K4,
            MCD_ERR_INVALID_ARG, "unknown measure");
    REQUIRE(mode == MCD_PICK_AUTO || mode == MCD_PICK_FORCE_SWEEP || mode == MCD_PICK_NETWORK,
            MCD_ERR_INVALID_ARG, "unknown pick mode");
    const PickLayout L = pick_layout(ws, g, n_graphs);
    REQUIRE(ws_bytes >= L.bytes, MCD_ERR_WORKSPACE, "pick workspace too small");
    const char* env = getenv("MCD_FORCE_SWEEP");
    if (env && env[0] && strcmp(env, "0") != 0) mode = MCD_PICK_FORCE_SWEEP;
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    hipStream_t s = g->ctx->stream;
    const int G = n_graphs;
    int32_t* idx = index ? index : L.index;
    int64_t* dl = deltas ? deltas : L.deltas;
    int32_t* flags = used_fallback ? used_fallback : L.flags;
    // the network's threshold per graph, and the range guard's verdict
    mcd::launch_features(g, t, G, vbase, L.x, L.feat, s);
    mcd::launch_mlp_forward(p->params, p->mean, p->stdv, L.x, G, L.y, s);
    mcd::launch_select(L.y, G, kGridK, kGridA, kGridB, kGridC, idx, dl, s);
    mcd::launch_fallback(L.x, G, p->lo, p->hi, p->margin, nullptr, nullptr, nullptr, flags, s);
    if (mode != MCD_PICK_NETWORK) {  // the full sweep with modularity, and its rule of thumb (jump 1/10)
        // automatic mode decides on the device whether any graph needs the
        // sweep: its kernels return at once otherwise
        const int32_t* gate = nullptr;
        if (mode == MCD_PICK_AUTO) {
            mcd::launch_any_flag(flags, G, L.any, s);
            gate = L.any;
        }
        mcd::SweepDeltas ds;
        int order[MCD_SWEEP_MAX];
        grid_deltas(&ds, order);
        mcd::launch_sweep(g, measure, t, ds, order, G, vbase, nullptr, L.stats, nullptr, L.q, nullptr, nullptr,
                          L.sweep, s, gate);
        mcd::launch_sweep_rule(ds, order, G, vbase, L.stats, L.q, 1, 10, L.rule_index, L.rule_deltas, s);
        if (mode == MCD_PICK_FORCE_SWEEP) {  // every graph takes the rule's threshold
            MCD_HIP(hipMemcpyAsync(dl, L.rule_deltas, sizeof(int64_t) * 2 * (size_t)G, hipMemcpyDeviceToDevice, s));
            mcd::fill_i32(flags, G, 1, s);
        } else {
            mcd::launch_fallback(L.x, G, p->lo, p->hi, p->margin, dl, L.rule_deltas, dl, flags, s);
        }
    } else {
        mcd::fill_i32(flags, G, 0, s);
    }
    int32_t* parent = mcd::launch_components_init(g, labels, n_components, L.cc, s);
    mcd::launch_weigh_prune(g, measure, t, 0, 1, G, vbase, dl, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                            s, g->n > 0 ? parent : nullptr);
    mcd::launch_components_finish(g, labels, n_components, L.cc, s);
    return MCD_OK;
}

mcd_status mcd_picker_export(const mcd_picker* p, float* params, float* mean, float* std, float* lo, float* hi,
                             float* host_margin) {
    REQUIRE(p, MCD_ERR_INVALID_ARG, "picker is NULL");
    mcd_status st = use_device(p->ctx);
    if (st != MCD_OK) return st;
    hipStream_t s = p->ctx->stream;
    const float* from[5] = {p->params, p->mean, p->stdv, p->lo, p->hi};
    float* to[5] = {params, mean, std, lo, hi};
    const size_t cnt[5] = {(size_t)NPAR, (size_t)NI, (size_t)NI, (size_t)NI, (size_t)NI};
    for (int i = 0; i < 5; ++i)
        if (to[i]) MCD_HIP(hipMemcpyAsync(to[i], from[i], cnt[i] * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (host_margin) *host_margin = p->margin;
    return MCD_OK;
}

mcd_status mcd_picker_import(mcd_picker* p, const float* params, const float* mean, const float* std,
                             const float* lo, const float* hi, float margin) {
    REQUIRE(p && params && mean && std && lo && hi, MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(margin >= 0.f && isfinite(margin), MCD_ERR_INVALID_ARG, "margin must be finite and non-negative");
    mcd_status st = use_device(p->ctx);
    if (st != MCD_OK) return st;
    hipStream_t s = p->ctx->stream;
    const float* from[5] = {params, mean, std, lo, hi};
    float* to[5] = {p->params, p->mean, p->stdv, p->lo, p->hi};
    const size_t cnt[5] = {(size_t)NPAR, (size_t)NI, (size_t)NI, (size_t)NI, (size_t)NI};
    for (int i = 0; i < 5; ++i)
        MCD_HIP(hipMemcpyAsync(to[i], from[i], cnt[i] * sizeof(float), hipMemcpyDeviceToDevice, s));
    mcd::fill_i32((int32_t*)p->adam_m, 2 * (int64_t)NPAR, 0, s);
    p->margin = margin;
    p->step = 0;
    p->prepared = 1;
    return MCD_OK;
}

mcd_status mcd_picker_save(const mcd_picker* p, const char* path) {
    REQUIRE(p && path, MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(p->prepared, MCD_ERR_INVALID_ARG, "the picker has no standardisation to save");
    mcd_status st = use_device(p->ctx);
    if (st != MCD_OK) return st;
    std::vector<unsigned char> b(kFileBytes, 0);
    memcpy(b.data(), kMagic, 8);
    put<uint32_t>(b, 8, kVersion);
    put<uint32_t>(b, 12, (uint32_t)NI);
    put<uint32_t>(b, 16, (uint32_t)NH);
    put<uint32_t>(b, 20, (uint32_t)NPAR);
    put<int32_t>(b, 24, kGridK);
    put<int64_t>(b, 32, kGridA);
    put<int64_t>(b, 40, kGridB);
    put<int64_t>(b, 48, kGridC);
    put<float>(b, 56, p->margin);
    hipStream_t s = p->ctx->stream;
    float* f = (float*)(b.data() + kHeader);
    MCD_HIP(hipMemcpyAsync(f, p->params, sizeof(float) * NPAR, hipMemcpyDeviceToHost, s));
    MCD_HIP(hipMemcpyAsync(f + NPAR, p->mean, sizeof(float) * 4 * NI, hipMemcpyDeviceToHost, s));
    MCD_HIP(hipStreamSynchronize(s));
    put<uint32_t>(b, kFileBytes - 4, crc32(b.data(), kFileBytes - 4));
    // write beside the target, then rename: a reader never sees half a file
    const std::string tmp = std::string(path) + ".tmp";
    FILE* fp = fopen(tmp.c_str(), "wb");
    REQUIRE(fp, MCD_ERR_CHECKPOINT, "cannot open " + tmp + " for writing");
    const size_t w = fwrite(b.data(), 1, b.size(), fp);
    const int c = fclose(fp);
    if (w != b.size() || c != 0) {
        remove(tmp.c_str());
        return mcd_fail(MCD_ERR_CHECKPOINT, "short write to " + tmp);
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return mcd_fail(MCD_ERR_CHECKPOINT, std::string("cannot rename the checkpoint to ") + path);
    }
    return MCD_OK;
}

mcd_status mcd_picker_check_file(const char* path) {
    std::vector<unsigned char> b;
    return read_checkpoint(path, b);
}

mcd_status mcd_picker_load(mcd_picker* p, const char* path) {
    REQUIRE(p, MCD_ERR_INVALID_ARG, "picker is NULL");
    std::vector<unsigned char> b;
    mcd_status st = read_checkpoint(path, b);
    if (st != MCD_OK) return st;
    const float margin = get<float>(b, 56);
    const float* f = (const float*)(b.data() + kHeader);
    if ((st = use_device(p->ctx)) != MCD_OK) return st;
    hipStream_t s = p->ctx->stream;
    MCD_HIP(hipMemcpyAsync(p->params, f, sizeof(float) * NPAR, hipMemcpyHostToDevice, s));
    MCD_HIP(hipMemcpyAsync(p->mean, f + NPAR, sizeof(float) * 4 * NI, hipMemcpyHostToDevice, s));
    mcd::fill_i32((int32_t*)p->adam_m, 2 * (int64_t)NPAR, 0, s);
    MCD_HIP(hipStreamSynchronize(s));
    p->margin = margin;
    p->step = 0;
    p->prepared = 1;
    return MCD_OK;
}

}  // extern "C"
#pragma GCC visibility pop
