// C ABI of the library: argument checks, workspace carving, orchestration of
// the kernels on the context stream, and scalar read-backs.
#include <limits.h>
#include <stdio.h>
#include <stdlib.h>

#include <string>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"

// The library is built with hidden visibility; the C ABI below is exported.
#pragma GCC visibility push(default)
#include "mcd.h"
#pragma GCC visibility pop

static thread_local std::string g_last_error;

mcd_status mcd_fail(mcd_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define REQUIRE(cond, code, msg)                \
    do {                                        \
        if (!(cond)) return mcd_fail(code, msg); \
    } while (0)

// Caller buffers that the library carves into typed arrays (graph storage,
// workspaces) must start on a 256-byte boundary; NULL passes.
#define REQUIRE_ALIGNED(p)                                                                          \
    REQUIRE(((uintptr_t)(p) & 255u) == 0u, MCD_ERR_INVALID_ARG, #p " must be 256-byte aligned")

// Scratch of the allocation-free entry point (mcd_prune_components_noalloc):
// the union-find parent array of a graph of at most MCD_NOALLOC_MAX_VERTICES
// vertices.  Each device holds its own copy, at its own address, from module
// load to process end.  Host code never passes `scratch` itself to a kernel
// (on the host it names a stand-in, not device memory): the device address is
// looked up once per device, with that device current, and kept.
static __device__ __align__(256) int32_t scratch[MCD_NOALLOC_MAX_VERTICES];

namespace {

int id_bits(int64_t n) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < n) ++b;
    return b;
}

mcd_status use_device(const mcd_ctx* ctx) {
    MCD_HIP(hipSetDevice(ctx->device));
    return MCD_OK;
}

bool valid_measure(int m) {
    return m == MCD_SIM_TECTONIC || m == MCD_SIM_TW || m == MCD_SIM_K3 || m == MCD_SIM_JACCARD || m == MCD_SIM_K4;
}

mcd_status check_delta(mcd_rational d) {
    REQUIRE(d.den > 0, MCD_ERR_INVALID_ARG, "threshold denominator must be positive");
    REQUIRE(d.den < ((int64_t)1 << 31) && d.num < ((int64_t)1 << 31) && d.num > -((int64_t)1 << 31),
            MCD_ERR_RANGE, "threshold numerator and denominator must lie below 2^31 in magnitude");
    return MCD_OK;
}

// Layout of the graph storage buffer.
struct StorageLayout {
    int64_t* off;
    int32_t* src;
    int32_t* adj;
    int32_t* dsum;
    int32_t* deg;
    int32_t* perm;
    int64_t* in_off;
    int2* in_ea;
    size_t bytes;
};

StorageLayout storage_layout(void* base, int64_t P, int64_t n) {
    Carve c{(char*)base, 0, 0};
    StorageLayout L;
    L.off = c.take<int64_t>((size_t)n + 1);
    L.src = c.take<int32_t>((size_t)P);
    L.adj = c.take<int32_t>((size_t)P + 4);  // +4: 16-byte loads may read past the last edge
    L.dsum = c.take<int32_t>((size_t)P);
    L.deg = c.take<int32_t>((size_t)n);
    L.perm = c.take<int32_t>((size_t)n);
    L.in_off = c.take<int64_t>((size_t)n + 1);
    L.in_ea = c.take<int2>((size_t)P);
    L.bytes = c.used;
    return L;
}

struct BuildLayout {
    uint64_t* k1;
    uint64_t* k2;
    uint64_t* uniq;
    int32_t* inv;
    int32_t* deg_orig;
    int32_t* outdeg;
    void* radix;
    void* compact;
    void* scan;
    size_t bytes;
};

BuildLayout build_layout(void* base, int64_t P, int64_t n) {
    Carve c{(char*)base, 0, 0};
    BuildLayout L;
    const int64_t K = P > n ? P : n;
    L.k1 = c.take<uint64_t>((size_t)K);
    L.k2 = c.take<uint64_t>((size_t)K);
    L.uniq = c.take<uint64_t>((size_t)P);
    L.inv = c.take<int32_t>((size_t)n);
    L.deg_orig = c.take<int32_t>((size_t)n);
    L.outdeg = c.take<int32_t>((size_t)n);
    L.radix = c.take<char>(mcd::radix_scratch_bytes(K));
    L.compact = c.take<char>(mcd::compact_scratch_bytes(K));
    L.scan = c.take<char>(mcd::scan_scratch_bytes(n));
    L.bytes = c.used;
    return L;
}

struct RunLayout {
    int32_t* t;
    int32_t* kept_pairs;
    int32_t* kept_counts;
    void* cc;
    void* tc;
    size_t bytes;
};

RunLayout run_layout(void* base, const mcd_graph* g) {
    Carve c{(char*)base, 0, 0};
    RunLayout L;
    L.t = c.take<int32_t>((size_t)g->m);
    L.kept_pairs = c.take<int32_t>((size_t)2 * MCD_KEPT_SEGMENTS * mcd::kept_segment_len(g->m));
    L.kept_counts = c.take<int32_t>((size_t)MCD_KEPT_SEGMENTS);
    L.cc = c.take<char>(mcd::cc_scratch_bytes(g));
    L.tc = c.take<char>(mcd::tc_scratch_bytes(g, g->ctx->tc_chunk));
    L.bytes = c.used;
    return L;
}

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // by device id; null until looked up

// Device address of `scratch` on the current device `device` (looked up on
// the first call for that device).
mcd_status scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        MCD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return mcd_fail(MCD_ERR_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return MCD_OK;
}

mcd_status sync_read(mcd_ctx* ctx, const int64_t* d, int64_t* h, int count) {
    MCD_HIP(hipMemcpyAsync(h, d, sizeof(int64_t) * count, hipMemcpyDeviceToHost, ctx->stream));
    MCD_HIP(hipStreamSynchronize(ctx->stream));
    return MCD_OK;
}

}  // namespace

#pragma GCC visibility push(default)
extern "C" {

const char* mcd_status_string(mcd_status s) {
    switch (s) {
        case MCD_OK: return "MCD_OK";
        case MCD_ERR_INVALID_ARG: return "MCD_ERR_INVALID_ARG";
        case MCD_ERR_INVALID_VERTEX: return "MCD_ERR_INVALID_VERTEX";
        case MCD_ERR_RANGE: return "MCD_ERR_RANGE";
        case MCD_ERR_WORKSPACE: return "MCD_ERR_WORKSPACE";
        case MCD_ERR_NO_DEVICE: return "MCD_ERR_NO_DEVICE";
        case MCD_ERR_DEVICE: return "MCD_ERR_DEVICE";
        case MCD_ERR_NOT_CONVERGED: return "MCD_ERR_NOT_CONVERGED";
        case MCD_ERR_EMPTY: return "MCD_ERR_EMPTY";
        case MCD_ERR_CHECKPOINT: return "MCD_ERR_CHECKPOINT";
        default: return "MCD_ERR_UNKNOWN";
    }
}

const char* mcd_last_error(void) { return g_last_error.c_str(); }

mcd_status mcd_ctx_create(int device, void* stream, mcd_ctx** out) {
    REQUIRE(out, MCD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return mcd_fail(MCD_ERR_NO_DEVICE, "no HIP device available");
    REQUIRE(device >= 0 && device < count, MCD_ERR_NO_DEVICE, "device id out of range");
    MCD_HIP(hipSetDevice(device));
    mcd_ctx* c = new mcd_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->tc_chunk = 512;
    c->tc_lds_max = MCD_TC_LDS_LIMIT;
    c->tc_packed_range = MCD_TC_PACKED_LIMIT;
    c->tc_window_max = MCD_TC_WINDOW_LIMIT;
    c->k4_row_cache = 1;
    c->sweep_shape = 0;
    c->tc_window_occupancy = 1;
    if (hipMalloc((void**)&c->d_ctrl, sizeof(int64_t) * MCD_CTRL_WORDS) != hipSuccess) {
        delete c;
        return mcd_fail(MCD_ERR_DEVICE, "hipMalloc of the control block failed");
    }
    if (hipHostMalloc((void**)&c->h_ctrl, sizeof(int64_t) * MCD_CTRL_WORDS, hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipFree(c->d_ctrl);
        delete c;
        return mcd_fail(MCD_ERR_DEVICE, "hipHostMalloc of the read-back block failed");
    }
    void* scr = nullptr;  // the allocation-free entry point's scratch, looked up once per device
    if (scratch_address(device, &scr) != MCD_OK) {
        (void)hipFree(c->d_ctrl);
        (void)hipHostFree(c->h_ctrl);
        delete c;
        return MCD_ERR_DEVICE;  // message set by scratch_address
    }
    bool ok = true;
    for (int i = 0; i < 2; ++i) {
        ok = ok && hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming) == hipSuccess;
    }
    ok = ok && hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipFree(c->d_ctrl);
        (void)hipHostFree(c->h_ctrl);
        delete c;
        return mcd_fail(MCD_ERR_DEVICE, "creating the side streams failed");
    }
    *out = c;
    return MCD_OK;
}

mcd_status mcd_ctx_set_stream(mcd_ctx* ctx, void* stream) {
    REQUIRE(ctx, MCD_ERR_INVALID_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)stream;
    return MCD_OK;
}

mcd_status mcd_ctx_set_param(mcd_ctx* ctx, const char* name, int64_t value) {
    REQUIRE(ctx && name, MCD_ERR_INVALID_ARG, "NULL argument");
    const std::string k(name);
    if (k == "tc_chunk") {
        REQUIRE(value >= 1 && value <= (1 << 24), MCD_ERR_RANGE, "tc_chunk must lie in [1, 2^24]");
        ctx->tc_chunk = value;
    } else if (k == "tc_lds_max") {
        REQUIRE(value >= 0 && value <= MCD_TC_LDS_LIMIT, MCD_ERR_RANGE, "tc_lds_max must lie in [0, 4096]");
        ctx->tc_lds_max = value;
    } else if (k == "tc_window_max") {
        REQUIRE(value >= 0 && value <= MCD_TC_WINDOW_LIMIT, MCD_ERR_RANGE, "tc_window_max must lie in [0, 2^18]");
        ctx->tc_window_max = value;
    } else if (k == "tc_packed_range") {
        REQUIRE(value >= 0 && value <= MCD_TC_PACKED_LIMIT, MCD_ERR_RANGE,
                "tc_packed_range must lie in [0, 2^20 - 2]");
        ctx->tc_packed_range = value;
    } else if (k == "k4_row_cache") {
        REQUIRE(value == 0 || value == 1, MCD_ERR_RANGE, "k4_row_cache must be 0 or 1");
        ctx->k4_row_cache = value;
    } else if (k == "sweep_shape") {
        REQUIRE(value >= 0 && value <= 2, MCD_ERR_RANGE, "sweep_shape must be 0, 1 or 2");
        ctx->sweep_shape = value;
    } else if (k == "tc_window_occupancy") {
        REQUIRE(value == 0 || value == 1, MCD_ERR_RANGE, "tc_window_occupancy must be 0 or 1");
        ctx->tc_window_occupancy = value;
    } else {
        return mcd_fail(MCD_ERR_INVALID_ARG, "unknown parameter " + k);
    }
    return MCD_OK;
}

mcd_status mcd_ctx_get_param(const mcd_ctx* ctx, const char* name, int64_t* value) {
    REQUIRE(ctx && name && value, MCD_ERR_INVALID_ARG, "NULL argument");
    const std::string k(name);
    if (k == "tc_chunk") *value = ctx->tc_chunk;
    else if (k == "tc_lds_max") *value = ctx->tc_lds_max;
    else if (k == "tc_packed_range") *value = ctx->tc_packed_range;
    else if (k == "tc_window_max") *value = ctx->tc_window_max;
    else if (k == "k4_row_cache") *value = ctx->k4_row_cache;
    else if (k == "sweep_shape") *value = ctx->sweep_shape;
    else if (k == "tc_window_occupancy") *value = ctx->tc_window_occupancy;
    else return mcd_fail(MCD_ERR_INVALID_ARG, "unknown parameter " + k);
    return MCD_OK;
}

mcd_status mcd_ctx_destroy(mcd_ctx* ctx) {
    if (!ctx) return MCD_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < 2; ++i) {
        (void)hipStreamSynchronize(ctx->side[i]);
        (void)hipStreamDestroy(ctx->side[i]);
        (void)hipEventDestroy(ctx->join[i]);
    }
    (void)hipEventDestroy(ctx->fork);
    (void)hipFree(ctx->d_ctrl);
    (void)hipHostFree(ctx->h_ctrl);
    delete ctx;
    return MCD_OK;
}

mcd_status mcd_graph_build_sizes(int64_t n_pairs, int64_t n_vertices, size_t* storage_bytes,
                                 size_t* ws_bytes) {
    REQUIRE(n_pairs >= 0 && n_vertices >= 0, MCD_ERR_INVALID_ARG, "negative size");
    REQUIRE(n_vertices < ((int64_t)1 << 31) - 1, MCD_ERR_RANGE, "n_vertices must be below 2^31 - 1");
    REQUIRE(n_pairs < ((int64_t)1 << 31), MCD_ERR_RANGE, "n_pairs must be below 2^31");
    if (storage_bytes) *storage_bytes = storage_layout(nullptr, n_pairs, n_vertices).bytes;
    if (ws_bytes) *ws_bytes = build_layout(nullptr, n_pairs, n_vertices).bytes;
    return MCD_OK;
}

mcd_status mcd_graph_build(mcd_ctx* ctx, const int32_t* src, const int32_t* dst, int64_t n_pairs,
                           int64_t n_vertices, void* storage, size_t storage_bytes, void* ws,
                           size_t ws_bytes, mcd_graph** out) {
    REQUIRE_ALIGNED(storage);
    REQUIRE_ALIGNED(ws);
    REQUIRE(ctx && out, MCD_ERR_INVALID_ARG, "ctx or out is NULL");
    *out = nullptr;
    size_t need_st = 0, need_ws = 0;
    mcd_status st = mcd_graph_build_sizes(n_pairs, n_vertices, &need_st, &need_ws);
    if (st != MCD_OK) return st;
    REQUIRE(n_pairs == 0 || (src && dst), MCD_ERR_INVALID_ARG, "src or dst is NULL");
    REQUIRE(storage && ws, MCD_ERR_INVALID_ARG, "storage or workspace is NULL");
    REQUIRE(storage_bytes >= need_st, MCD_ERR_WORKSPACE, "graph storage too small");
    REQUIRE(ws_bytes >= need_ws, MCD_ERR_WORKSPACE, "build workspace too small");
    if ((st = use_device(ctx)) != MCD_OK) return st;

    hipStream_t s = ctx->stream;
    const int64_t P = n_pairs, n = n_vertices;
    const int bits = id_bits(n);
    StorageLayout G = storage_layout(storage, P, n);
    BuildLayout B = build_layout(ws, P, n);
    int64_t* ctrl = ctx->d_ctrl;  // [0] bad id flag, [1] m, [2] max out-degree, [3] max degree, [4] bitmask words
    mcd::fill_i64(ctrl, 5, 0, s);

    // Canonical simple graph: sort + dedup of packed (min, max) pairs.
    mcd::launch_canon(src, dst, P, n, bits, B.k1, ctrl + 0, s);
    uint64_t* sorted = mcd::radix_sort_u64(B.k1, B.k2, P, 2 * bits, B.radix, s);
    mcd::unique_sorted_u64(sorted, P, B.uniq, ctrl + 1, B.compact, s);
    if ((st = sync_read(ctx, ctrl, ctx->h_ctrl, 2)) != MCD_OK) return st;
    if (ctx->h_ctrl[0]) return mcd_fail(MCD_ERR_INVALID_VERTEX, "a pair has an id outside [0, n)");
    const int64_t m = ctx->h_ctrl[1];

    // Degrees, rank by (degree, id), orientation low -> high rank, CSR.
    mcd::fill_i32(B.deg_orig, n, 0, s);
    mcd::launch_degree(B.uniq, m, bits, B.deg_orig, s);
    {  // upper endpoints: sorted as 32-bit keys, then counted by runs (no random atomics)
        uint32_t* h1 = (uint32_t*)B.k1;
        uint32_t* h2 = (uint32_t*)B.k2;
        mcd::launch_upper_ends(B.uniq, m, bits, h1, s);
        const uint32_t* sorted_hi = mcd::radix_sort_u32(h1, h2, m, bits, B.radix, s);
        mcd::launch_count_runs(sorted_hi, m, B.deg_orig, s);
    }
    mcd::launch_rank_keys(B.deg_orig, n, bits, B.k1, s);
    uint64_t* ranked = mcd::radix_sort_u64(B.k1, B.k2, n, 2 * bits, B.radix, s);
    mcd::launch_rank_apply(ranked, n, bits, B.deg_orig, G.perm, B.inv, G.deg, s);
    mcd::launch_orient_keys(B.uniq, m, bits, B.inv, B.k1, s);
    uint64_t* oriented = mcd::radix_sort_u64(B.k1, B.k2, m, 2 * bits, B.radix, s);
    mcd::fill_i32(B.outdeg, n, 0, s);
    mcd::launch_csr_fill(oriented, m, bits, G.src, G.adj, B.outdeg, s);
    mcd::exclusive_scan_i32_i64(B.outdeg, n, G.off, B.scan, s);
    mcd::launch_edge_dsum(G.src, G.adj, G.deg, m, G.dsum, s);
    mcd::launch_max_i32(B.outdeg, n, ctrl + 2, s);
    mcd::launch_max_i32(G.deg, n, ctrl + 3, s);
    mcd::launch_bitmask_words(B.outdeg, n, ctrl + 4, s);
    // in-edge lists (edges grouped by head), in-degree = degree - out-degree
    mcd::launch_in_count(G.deg, B.outdeg, n, B.inv, s);
    mcd::exclusive_scan_i32_i64(B.inv, n, G.in_off, B.scan, s);
    // the suffix lengths ride along with the sort (two int32[m] buffers in
    // the unique keys' uint64[P] space, consumed by now)
    int32_t* suf = (int32_t*)B.uniq;
    int32_t* suf2 = suf + m;
    int32_t* suf_sorted = suf;
    mcd::launch_in_keys(G.src, G.adj, G.off, m, B.k1, suf, s);
    uint64_t* by_head = mcd::radix_sort_u64_kv(B.k1, B.k2, suf, suf2, &suf_sorted, m, bits, B.radix, s, 32);
    mcd::launch_in_fill(by_head, suf_sorted, m, G.in_ea, s);
    if ((st = sync_read(ctx, ctrl, ctx->h_ctrl, 5)) != MCD_OK) return st;

    mcd_graph* g = new mcd_graph();
    g->ctx = ctx;
    g->n = n;
    g->m = m;
    g->cap = P;
    g->bits = bits;
    g->max_outdeg = (int32_t)ctx->h_ctrl[2];
    g->max_deg = (int32_t)ctx->h_ctrl[3];
    g->bitmask_words = ctx->h_ctrl[4];
    g->off = G.off;
    g->src = G.src;
    g->adj = G.adj;
    g->dsum = G.dsum;
    g->deg = G.deg;
    g->perm = G.perm;
    g->in_off = G.in_off;
    g->in_ea = G.in_ea;
    *out = g;
    return MCD_OK;
}

mcd_status mcd_graph_info(const mcd_graph* g, int64_t* n, int64_t* m, int32_t* max_deg,
                          int32_t* max_outdeg) {
    REQUIRE(g, MCD_ERR_INVALID_ARG, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_deg) *max_deg = g->max_deg;
    if (max_outdeg) *max_outdeg = g->max_outdeg;
    return MCD_OK;
}

mcd_status mcd_graph_edges(const mcd_graph* g, int32_t* u, int32_t* v) {
    REQUIRE(g && (g->m == 0 || (u && v)), MCD_ERR_INVALID_ARG, "NULL argument");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_edges_orig(g->src, g->adj, g->perm, g->m, u, v, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_graph_degrees(const mcd_graph* g, int32_t* deg) {
    REQUIRE(g && (g->n == 0 || deg), MCD_ERR_INVALID_ARG, "NULL argument");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_scatter_by_perm(g->deg, g->perm, g->n, deg, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_graph_perm(const mcd_graph* g, int32_t* perm) {
    REQUIRE(g && (g->n == 0 || perm), MCD_ERR_INVALID_ARG, "NULL argument");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    if (g->n > 0)
        MCD_HIP(hipMemcpyAsync(perm, g->perm, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToDevice,
                               g->ctx->stream));
    return MCD_OK;
}

mcd_status mcd_graph_destroy(mcd_graph* g) {
    delete g;
    return MCD_OK;
}

mcd_status mcd_triangles_workspace_size(const mcd_graph* g, size_t* bytes) {
    REQUIRE(g && bytes, MCD_ERR_INVALID_ARG, "NULL argument");
    *bytes = mcd::tc_scratch_bytes(g, g->ctx->tc_chunk);
    return MCD_OK;
}

mcd_status mcd_triangles(const mcd_graph* g, int32_t* t, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && (g->m == 0 || (t && ws)), MCD_ERR_INVALID_ARG, "NULL argument");
    size_t need = 0;
    mcd_triangles_workspace_size(g, &need);
    REQUIRE(g->m == 0 || ws_bytes >= need, MCD_ERR_WORKSPACE, "triangle workspace too small");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_triangles(g, t, ws, g->ctx->tc_chunk, g->ctx->tc_lds_max, g->ctx->tc_packed_range,
                          g->ctx->tc_window_max, g->ctx->stream);
    return MCD_OK;
}

// ---- autotuner for the triangle-count launch parameters ----
namespace {
constexpr int64_t kTuneChunks[] = {256, 512, 1024, 2048};
constexpr int64_t kTuneWindows[] = {0, 1 << 14, 1 << 16, 1 << 18};
constexpr int64_t kTunePacked[] = {0, MCD_TC_PACKED_LIMIT};
constexpr int64_t kTuneLds[] = {1024, 2048, 4096};

// Smallest time over reps of one triangle count with the given parameters.
mcd_status time_triangles(const mcd_graph* g, int32_t* t, void* ws, const int64_t p[4], int reps, float* ms) {
    hipStream_t s = g->ctx->stream;
    hipEvent_t e0, e1;
    MCD_HIP(hipEventCreate(&e0));
    MCD_HIP(hipEventCreate(&e1));
    float best = 3.4e38f;
    for (int r = 0; r < reps; ++r) {
        MCD_HIP(hipEventRecord(e0, s));
        mcd::launch_triangles(g, t, ws, p[0], p[1], p[2], p[3], s);
        MCD_HIP(hipEventRecord(e1, s));
        MCD_HIP(hipEventSynchronize(e1));
        float x = 0.f;
        MCD_HIP(hipEventElapsedTime(&x, e0, e1));
        if (x < best) best = x;
    }
    MCD_HIP(hipEventDestroy(e0));
    MCD_HIP(hipEventDestroy(e1));
    *ms = best;
    return MCD_OK;
}
}  // namespace

mcd_status mcd_tune_triangles_workspace_size(const mcd_graph* g, size_t* bytes) {
    REQUIRE(g && bytes, MCD_ERR_INVALID_ARG, "NULL argument");
    size_t need = 0;
    for (int64_t c : kTuneChunks) need = std::max(need, mcd::tc_scratch_bytes(g, c));
    need = std::max(need, mcd::tc_scratch_bytes(g, g->ctx->tc_chunk));
    *bytes = need;
    return MCD_OK;
}

mcd_status mcd_tune_triangles(const mcd_graph* g, int32_t* t, void* ws, size_t ws_bytes, int32_t reps,
                              int64_t* host_best, float* host_ms) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && (g->m == 0 || (t && ws)), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(reps >= 1 && reps <= 100, MCD_ERR_RANGE, "reps must lie in [1, 100]");
    size_t need = 0;
    mcd_tune_triangles_workspace_size(g, &need);
    REQUIRE(g->m == 0 || ws_bytes >= need, MCD_ERR_WORKSPACE, "tuning workspace too small");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd_ctx* ctx = g->ctx;
    int64_t best[4] = {ctx->tc_chunk, ctx->tc_lds_max, ctx->tc_packed_range, ctx->tc_window_max};
    float best_ms = 0.f;
    if (g->m > 0) {
        if ((st = time_triangles(g, t, ws, best, 1, &best_ms)) != MCD_OK) return st;  // warm-up
        if ((st = time_triangles(g, t, ws, best, reps, &best_ms)) != MCD_OK) return st;
        // one coordinate at a time: item chunk, window cutoff, packed range, LDS cap
        const int64_t* cand[4] = {kTuneChunks, kTuneLds, kTunePacked, kTuneWindows};
        const int ncand[4] = {4, 3, 2, 4};
        const int order[4] = {0, 3, 2, 1};
        for (int oi = 0; oi < 4; ++oi) {
            const int k = order[oi];
            for (int j = 0; j < ncand[k]; ++j) {
                if (cand[k][j] == best[k]) continue;
                int64_t p[4] = {best[0], best[1], best[2], best[3]};
                p[k] = cand[k][j];
                float ms = 0.f;
                if ((st = time_triangles(g, t, ws, p, reps, &ms)) != MCD_OK) return st;
                if (ms < best_ms) {
                    best_ms = ms;
                    best[k] = p[k];
                }
            }
        }
        ctx->tc_chunk = best[0];
        ctx->tc_lds_max = best[1];
        ctx->tc_packed_range = best[2];
        ctx->tc_window_max = best[3];
        // leave t holding the counts of the chosen setting
        mcd::launch_triangles(g, t, ws, best[0], best[1], best[2], best[3], ctx->stream);
        MCD_HIP(hipStreamSynchronize(ctx->stream));
    }
    if (host_best)
        for (int i = 0; i < 4; ++i) host_best[i] = best[i];
    if (host_ms) *host_ms = best_ms;
    return MCD_OK;
}

mcd_status mcd_k4(const mcd_graph* g, int32_t* k4) {
    REQUIRE(g && (g->m == 0 || k4), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(g->max_outdeg <= MCD_K4_MAX_COMMON, MCD_ERR_RANGE,
            "4-clique counts need every row of the oriented graph to hold at most 4096 edges");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_k4(g, k4, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_weights(const mcd_graph* g, mcd_measure measure, const int32_t* t, float* w_f32,
                       int32_t* w_i32) {
    REQUIRE(g && (g->m == 0 || t), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    REQUIRE(!w_i32 || measure == MCD_SIM_TW || measure == MCD_SIM_K3 || measure == MCD_SIM_K4,
            MCD_ERR_INVALID_ARG, "integer weights exist for TW, K3 and K4 only");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_weights(g, measure, t, w_f32, w_i32, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_prune(const mcd_graph* g, mcd_measure measure, const int32_t* t, mcd_rational delta,
                     uint32_t* keep_bits, int64_t* n_kept) {
    REQUIRE(g && (g->m == 0 || (t && keep_bits)), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    mcd_status st = check_delta(delta);
    if (st != MCD_OK) return st;
    if ((st = use_device(g->ctx)) != MCD_OK) return st;
    mcd::launch_prune(g, measure, t, delta.num, delta.den, keep_bits, n_kept, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_components_workspace_size(const mcd_graph* g, size_t* bytes) {
    REQUIRE(g && bytes, MCD_ERR_INVALID_ARG, "NULL argument");
    *bytes = mcd::cc_scratch_bytes(g);
    return MCD_OK;
}

mcd_status mcd_components(const mcd_graph* g, const uint32_t* keep_bits, int32_t* labels,
                          int64_t* n_components, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && (g->n == 0 || (labels && ws)), MCD_ERR_INVALID_ARG, "NULL argument");
    size_t need = 0;
    mcd_components_workspace_size(g, &need);
    REQUIRE(ws_bytes >= need, MCD_ERR_WORKSPACE, "components workspace too small");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_components(g, keep_bits, labels, n_components, ws, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_kept_segment_len(const mcd_graph* g, int64_t* len) {
    REQUIRE(g && len, MCD_ERR_INVALID_ARG, "NULL argument");
    *len = mcd::kept_segment_len(g->m);
    return MCD_OK;
}

mcd_status mcd_weigh_prune(const mcd_graph* g, mcd_measure measure, const int32_t* t, mcd_rational delta,
                           int32_t n_graphs, const int64_t* vbase, const int64_t* deltas, float* w_f32,
                           int32_t* w_i32, uint32_t* keep_bits, int32_t* kept_pairs, int32_t* kept_counts,
                           int64_t* n_kept) {
    REQUIRE(g, MCD_ERR_INVALID_ARG, "graph is NULL");
    REQUIRE(g->m == 0 || t, MCD_ERR_INVALID_ARG, "t is NULL");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    REQUIRE(!w_i32 || measure == MCD_SIM_TW || measure == MCD_SIM_K3 || measure == MCD_SIM_K4,
            MCD_ERR_INVALID_ARG, "integer weights exist for TW, K3 and K4 only");
    REQUIRE((kept_pairs == nullptr) == (kept_counts == nullptr), MCD_ERR_INVALID_ARG,
            "kept_pairs and kept_counts go together");
    mcd_status st;
    if (deltas) {
        REQUIRE(n_graphs >= 1, MCD_ERR_INVALID_ARG, "n_graphs must be at least 1");
        REQUIRE(n_graphs == 1 || vbase, MCD_ERR_INVALID_ARG, "vbase is NULL");
    } else if ((st = check_delta(delta)) != MCD_OK) {
        return st;
    }
    if ((st = use_device(g->ctx)) != MCD_OK) return st;
    mcd::launch_weigh_prune(g, measure, t, delta.num, delta.den, deltas ? n_graphs : 1, vbase, deltas, w_f32, w_i32,
                            keep_bits, kept_pairs, kept_counts, n_kept, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_prune_components(const mcd_graph* g, mcd_measure measure, const int32_t* t, mcd_rational delta,
                                int32_t n_graphs, const int64_t* vbase, const int64_t* deltas, float* w_f32,
                                int32_t* w_i32, uint32_t* keep_bits, int64_t* n_kept, int32_t* labels,
                                int64_t* n_components, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && (g->n == 0 || (labels && ws)), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(g->m == 0 || t, MCD_ERR_INVALID_ARG, "t is NULL");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    REQUIRE(!w_i32 || measure == MCD_SIM_TW || measure == MCD_SIM_K3 || measure == MCD_SIM_K4,
            MCD_ERR_INVALID_ARG, "integer weights exist for TW, K3 and K4 only");
    REQUIRE(ws_bytes >= mcd::cc_scratch_bytes(g), MCD_ERR_WORKSPACE, "components workspace too small");
    mcd_status st;
    if (deltas) {
        REQUIRE(n_graphs >= 1, MCD_ERR_INVALID_ARG, "n_graphs must be at least 1");
        REQUIRE(n_graphs == 1 || vbase, MCD_ERR_INVALID_ARG, "vbase is NULL");
    } else if ((st = check_delta(delta)) != MCD_OK) {
        return st;
    }
    if ((st = use_device(g->ctx)) != MCD_OK) return st;
    hipStream_t s = g->ctx->stream;
    // with no vertex there is no edge either: the pass only zeroes n_kept
    int32_t* parent = mcd::launch_components_init(g, labels, n_components, ws, s);
    // A threshold of at most 0 keeps every edge of a measure that is never
    // negative: the pass then writes weights and keep bits only, and the
    // components come from the vertex-by-vertex union of every edge.
    const bool nonnegative = measure != MCD_SIM_TW;
    if (!deltas && nonnegative && delta.num <= 0 && g->n > 0 && g->m > 0) {
        mcd::launch_weigh_prune(g, measure, t, delta.num, delta.den, 1, nullptr, nullptr, w_f32, w_i32, keep_bits,
                                nullptr, nullptr, n_kept, s, nullptr);
        mcd::launch_components_all_edges(g, parent, parent + g->n, s);
    } else {
        mcd::launch_weigh_prune(g, measure, t, delta.num, delta.den, deltas ? n_graphs : 1, vbase, deltas, w_f32,
                                w_i32, keep_bits, nullptr, nullptr, n_kept, s, g->n > 0 ? parent : nullptr);
    }
    mcd::launch_components_finish(g, labels, n_components, ws, s);
    return MCD_OK;
}

mcd_status mcd_prune_components_noalloc(const mcd_graph* g, mcd_measure measure, const int32_t* t,
                                        mcd_rational delta, int32_t n_graphs, const int64_t* vbase,
                                        const int64_t* deltas, float* w_f32, int32_t* w_i32, uint32_t* keep_bits,
                                        int64_t* n_kept, int32_t* labels, int64_t* n_components) {
    REQUIRE(g && (g->n == 0 || labels), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(g->n <= MCD_NOALLOC_MAX_VERTICES, MCD_ERR_RANGE,
            "mcd_prune_components_noalloc takes graphs of at most 2^24 vertices");
    REQUIRE(g->m == 0 || t, MCD_ERR_INVALID_ARG, "t is NULL");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    REQUIRE(!w_i32 || measure == MCD_SIM_TW || measure == MCD_SIM_K3 || measure == MCD_SIM_K4,
            MCD_ERR_INVALID_ARG, "integer weights exist for TW, K3 and K4 only");
    mcd_status st;
    if (deltas) {
        REQUIRE(n_graphs >= 1, MCD_ERR_INVALID_ARG, "n_graphs must be at least 1");
        REQUIRE(n_graphs == 1 || vbase, MCD_ERR_INVALID_ARG, "vbase is NULL");
    } else if ((st = check_delta(delta)) != MCD_OK) {
        return st;
    }
    if ((st = use_device(g->ctx)) != MCD_OK) return st;
    void* ws = nullptr;  // looked up when the context was created: no allocation here
    if ((st = scratch_address(g->ctx->device, &ws)) != MCD_OK) return st;
    hipStream_t s = g->ctx->stream;
    // the same kernels as mcd_prune_components; the init kernel sets every
    // parent of this graph's vertices, so nothing left by an earlier call matters
    int32_t* parent = mcd::launch_components_init(g, labels, n_components, ws, s);
    mcd::launch_weigh_prune(g, measure, t, delta.num, delta.den, deltas ? n_graphs : 1, vbase, deltas, w_f32, w_i32,
                            keep_bits, nullptr, nullptr, n_kept, s, g->n > 0 ? parent : nullptr);
    mcd::launch_components_finish(g, labels, n_components, ws, s);
    return MCD_OK;
}

mcd_status mcd_components_kept(const mcd_graph* g, const int32_t* kept_pairs, const int32_t* kept_counts,
                               int32_t* labels, int64_t* n_components, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && (g->n == 0 || (labels && ws)), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(g->m == 0 || (kept_pairs && kept_counts), MCD_ERR_INVALID_ARG, "kept list is NULL");
    REQUIRE(ws_bytes >= mcd::cc_scratch_bytes(g), MCD_ERR_WORKSPACE, "components workspace too small");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_components_kept(g, kept_pairs, kept_counts, labels, n_components, ws, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_run_workspace_size(const mcd_graph* g, size_t* bytes) {
    REQUIRE(g && bytes, MCD_ERR_INVALID_ARG, "NULL argument");
    *bytes = run_layout(nullptr, g).bytes;
    return MCD_OK;
}

mcd_status mcd_run(const mcd_graph* g, mcd_measure measure, mcd_rational delta, int32_t* labels,
                   int64_t* n_components, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && (g->n == 0 || (labels && ws)), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    mcd_status st = check_delta(delta);
    if (st != MCD_OK) return st;
    size_t need = 0;
    mcd_run_workspace_size(g, &need);
    REQUIRE(ws_bytes >= need, MCD_ERR_WORKSPACE, "run workspace too small");
    if ((st = use_device(g->ctx)) != MCD_OK) return st;
    RunLayout L = run_layout(ws, g);
    hipStream_t s = g->ctx->stream;
    mcd::launch_triangles(g, L.t, L.tc, g->ctx->tc_chunk, g->ctx->tc_lds_max, g->ctx->tc_packed_range,
                          g->ctx->tc_window_max, s);
    mcd::launch_weigh_prune(g, measure, L.t, delta.num, delta.den, 1, nullptr, nullptr, nullptr, nullptr, nullptr,
                            L.kept_pairs, L.kept_counts, nullptr, s);
    mcd::launch_components_kept(g, L.kept_pairs, L.kept_counts, labels, n_components, L.cc, s);
    return MCD_OK;
}

mcd_status mcd_sweep_workspace_size(const mcd_graph* g, int32_t n_graphs, int32_t n_thresholds,
                                    int32_t has_truth, size_t* bytes) {
    REQUIRE(g && bytes, MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(n_graphs >= 1 && n_thresholds >= 1 && n_thresholds <= MCD_SWEEP_MAX_THRESHOLDS,
            MCD_ERR_INVALID_ARG, "need n_graphs >= 1 and 1 <= n_thresholds <= 64");
    *bytes = mcd::sweep_scratch_bytes(g, n_graphs, n_thresholds, has_truth != 0);
    return MCD_OK;
}

// Thresholds of a sweep sorted by exact value (equal ones keep the caller's
// order): order[i] = caller slot of the i-th smallest.
mcd_status sort_thresholds(const mcd_rational* host_deltas, int K, int* order, mcd::SweepDeltas* ds) {
    REQUIRE(K >= 1 && K <= MCD_SWEEP_MAX_THRESHOLDS, MCD_ERR_RANGE, "1 to 64 thresholds per sweep");
    mcd_status st;
    for (int i = 0; i < K; ++i) {
        if ((st = check_delta(host_deltas[i])) != MCD_OK) return st;
        order[i] = i;
    }
    for (int i = 1; i < K; ++i) {  // insertion sort by exact value
        const int x = order[i];
        int j = i - 1;
        while (j >= 0) {
            const mcd_rational& a = host_deltas[order[j]];
            const mcd_rational& b = host_deltas[x];
            if ((__int128)a.num * b.den <= (__int128)b.num * a.den) break;
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = x;
    }
    ds->K = K;
    for (int i = 0; i < K; ++i) {
        ds->num[i] = host_deltas[order[i]].num;
        ds->den[i] = host_deltas[order[i]].den;
    }
    return MCD_OK;
}

mcd_status mcd_sweep(const mcd_graph* g, mcd_measure measure, const int32_t* t,
                     const mcd_rational* host_deltas, int32_t n_thresholds, int32_t n_graphs,
                     const int64_t* vbase, const int32_t* truth, mcd_sweep_stats* stats, double* ari,
                     double* modularity, double* prf, int32_t* labels, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && host_deltas && vbase && stats && ws, MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(g->m == 0 || t, MCD_ERR_INVALID_ARG, "t is NULL");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    size_t need = 0;
    mcd_status st = mcd_sweep_workspace_size(g, n_graphs, n_thresholds, truth != nullptr, &need);
    if (st != MCD_OK) return st;
    REQUIRE(ws_bytes >= need, MCD_ERR_WORKSPACE, "sweep workspace too small");
    int order[MCD_SWEEP_MAX_THRESHOLDS];
    mcd::SweepDeltas ds;
    if ((st = sort_thresholds(host_deltas, n_thresholds, order, &ds)) != MCD_OK) return st;
    if ((st = use_device(g->ctx)) != MCD_OK) return st;
    mcd::launch_sweep(g, measure, t, ds, order, n_graphs, vbase, truth, stats, ari, modularity, prf, labels, ws,
                      g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_sweep_rule(mcd_ctx* ctx, const mcd_rational* host_deltas, int32_t n_thresholds, int32_t n_graphs,
                          const int64_t* vbase, const mcd_sweep_stats* stats, const double* modularity,
                          int64_t jump_num, int64_t jump_den, int32_t* index, int64_t* deltas) {
    REQUIRE(ctx && host_deltas && vbase && stats && index, MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(n_graphs >= 1, MCD_ERR_INVALID_ARG, "n_graphs must be at least 1");
    REQUIRE(jump_den > 0 && jump_num >= 0 && jump_num < ((int64_t)1 << 31) && jump_den < ((int64_t)1 << 31),
            MCD_ERR_RANGE, "jump fraction must be num/den with 0 <= num, 0 < den < 2^31");
    int order[MCD_SWEEP_MAX_THRESHOLDS];
    mcd::SweepDeltas ds;
    mcd_status st = sort_thresholds(host_deltas, n_thresholds, order, &ds);
    if (st != MCD_OK) return st;
    if ((st = use_device(ctx)) != MCD_OK) return st;
    mcd::launch_sweep_rule(ds, order, n_graphs, vbase, stats, modularity, jump_num, jump_den, index, deltas,
                           ctx->stream);
    return MCD_OK;
}

mcd_status mcd_features_workspace_size(int32_t n_graphs, size_t* bytes) {
    REQUIRE(bytes && n_graphs >= 1, MCD_ERR_INVALID_ARG, "need n_graphs >= 1");
    *bytes = mcd::features_scratch_bytes(n_graphs);
    return MCD_OK;
}

mcd_status mcd_features(const mcd_graph* g, const int32_t* t, int32_t n_graphs, const int64_t* vbase,
                        float* x, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && vbase && x && ws && (g->m == 0 || t), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(n_graphs >= 1, MCD_ERR_INVALID_ARG, "need n_graphs >= 1");
    REQUIRE(ws_bytes >= mcd::features_scratch_bytes(n_graphs), MCD_ERR_WORKSPACE, "features workspace too small");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_features(g, t, n_graphs, vbase, x, ws, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_feature_stats(mcd_ctx* ctx, const float* x, int32_t batch, float min_std, float* mean,
                             float* std) {
    REQUIRE(ctx && x && mean && std && batch >= 1, MCD_ERR_INVALID_ARG, "NULL argument or empty batch");
    REQUIRE(min_std > 0.f, MCD_ERR_INVALID_ARG, "min_std must be positive");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    mcd::launch_feature_stats(x, batch, min_std, mean, std, ctx->stream);
    return MCD_OK;
}

mcd_status mcd_feature_range(mcd_ctx* ctx, const float* x, int32_t batch, float* lo, float* hi) {
    REQUIRE(ctx && x && lo && hi && batch >= 1, MCD_ERR_INVALID_ARG, "NULL argument or empty batch");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    mcd::launch_feature_range(x, batch, lo, hi, ctx->stream);
    return MCD_OK;
}

mcd_status mcd_picker_fallback(mcd_ctx* ctx, const float* x, int32_t batch, const float* lo, const float* hi,
                               float margin, const int64_t* picked, const int64_t* fallback, int64_t* delta,
                               int32_t* flags) {
    REQUIRE(ctx && lo && hi && batch >= 0 && (batch == 0 || x), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(!delta || (picked && fallback), MCD_ERR_INVALID_ARG, "delta needs picked and fallback");
    REQUIRE(margin >= 0.f, MCD_ERR_INVALID_ARG, "margin must be non-negative");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    mcd::launch_fallback(x, batch, lo, hi, margin, picked, fallback, delta, flags, ctx->stream);
    return MCD_OK;
}

mcd_status mcd_mlp_forward(mcd_ctx* ctx, const float* params, const float* mean, const float* std,
                           const float* x, int32_t batch, float* y) {
    REQUIRE(ctx && params && mean && std && batch >= 0 && (batch == 0 || (x && y)), MCD_ERR_INVALID_ARG,
            "NULL argument");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    mcd::launch_mlp_forward(params, mean, std, x, batch, y, ctx->stream);
    return MCD_OK;
}

mcd_status mcd_mlp_workspace_size(int32_t batch, size_t* bytes) {
    REQUIRE(bytes && batch >= 1, MCD_ERR_INVALID_ARG, "need batch >= 1");
    *bytes = mcd::mlp_scratch_bytes(batch);
    return MCD_OK;
}

mcd_status mcd_mlp_gradient(mcd_ctx* ctx, const float* params, const float* mean, const float* std,
                            const float* x, const float* target, const double* ari, int32_t K, float mse_weight,
                            int32_t batch, float* grad, float* loss, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(ctx && params && mean && std && x && target && grad && ws && batch >= 1, MCD_ERR_INVALID_ARG,
            "NULL argument or empty batch");
    REQUIRE(!ari || K >= 2, MCD_ERR_INVALID_ARG, "an ARI table needs K >= 2");
    REQUIRE(mse_weight >= 0.f && mse_weight < 1e30f, MCD_ERR_INVALID_ARG, "mse_weight must be finite and >= 0");
    REQUIRE(ws_bytes >= mcd::mlp_scratch_bytes(batch), MCD_ERR_WORKSPACE, "MLP workspace too small");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    const mcd::MlpLoss L{target, ari, K, mse_weight};
    mcd::launch_mlp_gradient(params, mean, std, x, L, batch, grad, loss, ws, ctx->stream);
    return MCD_OK;
}

mcd_status mcd_mlp_train_step(mcd_ctx* ctx, float* params, float* adam_m, float* adam_v, int32_t step,
                              float lr, float weight_decay, const float* mean, const float* std, const float* x,
                              const float* target, const double* ari, int32_t K, float mse_weight, int32_t batch,
                              float* loss, void* ws, size_t ws_bytes) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(ctx && params && adam_m && adam_v && mean && std && x && target && ws && batch >= 1,
            MCD_ERR_INVALID_ARG, "NULL argument or empty batch");
    REQUIRE(step >= 1, MCD_ERR_INVALID_ARG, "Adam steps count from 1");
    REQUIRE(!ari || K >= 2, MCD_ERR_INVALID_ARG, "an ARI table needs K >= 2");
    REQUIRE(mse_weight >= 0.f && mse_weight < 1e30f, MCD_ERR_INVALID_ARG, "mse_weight must be finite and >= 0");
    REQUIRE(ws_bytes >= mcd::mlp_scratch_bytes(batch), MCD_ERR_WORKSPACE, "MLP workspace too small");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    const mcd::MlpLoss L{target, ari, K, mse_weight};
    mcd::launch_mlp_train_step(params, adam_m, adam_v, step, lr, weight_decay, mean, std, x, L, batch, loss, ws,
                               ctx->stream);
    return MCD_OK;
}

mcd_status mcd_grid_select(mcd_ctx* ctx, const float* y, int32_t batch, int32_t K, int64_t a, int64_t b,
                           int64_t c, int32_t* index, int64_t* delta) {
    REQUIRE(ctx && batch >= 0 && (batch == 0 || y), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(K >= 1 && c > 0, MCD_ERR_INVALID_ARG, "need K >= 1 and c > 0");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    mcd::launch_select(y, batch, K, a, b, c, index, delta, ctx->stream);
    return MCD_OK;
}

mcd_status mcd_sweep_targets(mcd_ctx* ctx, const double* ari, int32_t n_graphs, int32_t K, double frac,
                             int32_t* index, float* y) {
    REQUIRE(ctx && ari && n_graphs >= 1 && K >= 2, MCD_ERR_INVALID_ARG, "NULL argument or table under 2 columns");
    REQUIRE(frac > 0.0 && frac <= 1.0, MCD_ERR_INVALID_ARG, "frac must lie in (0, 1]");
    mcd_status st = use_device(ctx);
    if (st != MCD_OK) return st;
    mcd::launch_targets(ari, n_graphs, K, frac, index, y, ctx->stream);
    return MCD_OK;
}

mcd_status mcd_prune_graphs(const mcd_graph* g, mcd_measure measure, const int32_t* t, int32_t n_graphs,
                            const int64_t* vbase, const int64_t* deltas, uint32_t* keep_bits,
                            int64_t* n_kept) {
    REQUIRE(g && vbase && deltas && (g->m == 0 || (t && keep_bits)), MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(n_graphs >= 1, MCD_ERR_INVALID_ARG, "need n_graphs >= 1");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    mcd::launch_prune_graphs(g, measure, t, n_graphs, vbase, deltas, keep_bits, n_kept, g->ctx->stream);
    return MCD_OK;
}

mcd_status mcd_percentile_workspace_size(const mcd_graph* g, size_t* bytes) {
    REQUIRE(g && bytes, MCD_ERR_INVALID_ARG, "NULL argument");
    *bytes = mcd::select_scratch_bytes(g);
    return MCD_OK;
}

mcd_status mcd_percentile_threshold(const mcd_graph* g, mcd_measure measure, const int32_t* t,
                                    int64_t pct_num, int64_t pct_den, void* ws, size_t ws_bytes,
                                    mcd_rational* host_out) {
    REQUIRE_ALIGNED(ws);
    REQUIRE(g && t && ws && host_out, MCD_ERR_INVALID_ARG, "NULL argument");
    REQUIRE(valid_measure(measure), MCD_ERR_INVALID_ARG, "unknown measure");
    REQUIRE(pct_den > 0 && pct_num >= 0 && pct_num <= pct_den && pct_den < ((int64_t)1 << 31),
            MCD_ERR_INVALID_ARG, "percentile must be a fraction in [0, 1] with den below 2^31");
    size_t need = 0;
    mcd_percentile_workspace_size(g, &need);
    REQUIRE(ws_bytes >= need, MCD_ERR_WORKSPACE, "percentile workspace too small");
    mcd_status st = use_device(g->ctx);
    if (st != MCD_OK) return st;
    hipStream_t s = g->ctx->stream;
    mcd_ctx* ctx = g->ctx;
    int64_t* hist = (int64_t*)ws;
    int64_t* res = hist + 256;
    int64_t* part = hist + 264;
    int64_t hh[256];
    uint32_t prefix = 0, pmask = 0;
    int64_t k = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        mcd::sel_hist(g, measure, t, prefix, pmask, shift, hist, s);
        MCD_HIP(hipMemcpyAsync(hh, hist, sizeof(hh), hipMemcpyDeviceToHost, s));
        MCD_HIP(hipStreamSynchronize(s));
        if (shift == 24) {
            int64_t K = 0;
            for (int d = 0; d < 256; ++d) K += hh[d];
            if (K == 0) return mcd_fail(MCD_ERR_EMPTY, "every similarity is zero");
            k = (pct_num * K + pct_den - 1) / pct_den - 1;
            if (k < 0) k = 0;
        }
        int d = 0;
        while (d < 255 && k >= hh[d]) {
            k -= hh[d];
            ++d;
        }
        prefix |= (uint32_t)d << shift;
        pmask |= 255u << shift;
    }
    if (measure == MCD_SIM_TW || measure == MCD_SIM_K3 || measure == MCD_SIM_K4) {  // integers: key = value
        host_out->num = (int64_t)(int32_t)(prefix ^ 0x80000000u);
        host_out->den = 1;
        return MCD_OK;
    }
    // Distinct rationals sharing one fp32 key: walk them in exact order.
    int64_t lb_num = 0, lb_den = 1;
    int lb_valid = 0;
    for (int guard = 0; guard < 1 << 20; ++guard) {
        mcd::sel_min_above(g, measure, t, prefix, lb_num, lb_den, lb_valid, part, res, s);
        MCD_HIP(hipMemcpyAsync(ctx->h_ctrl, res, sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s));
        MCD_HIP(hipStreamSynchronize(s));
        const int64_t num = ctx->h_ctrl[0], den = ctx->h_ctrl[1];
        if (den == 0) return mcd_fail(MCD_ERR_DEVICE, "percentile selection lost its bucket");
        mcd::sel_count_eq(g, measure, t, prefix, num, den, res + 2, s);
        MCD_HIP(hipMemcpyAsync(ctx->h_ctrl + 2, res + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        MCD_HIP(hipStreamSynchronize(s));
        const int64_t c = ctx->h_ctrl[2];
        if (k < c) {
            int64_t x = num < 0 ? -num : num, y = den;
            while (y) {
                const int64_t r = x % y;
                x = y;
                y = r;
            }
            host_out->num = num / x;
            host_out->den = den / x;
            return MCD_OK;
        }
        k -= c;
        lb_num = num;
        lb_den = den;
        lb_valid = 1;
    }
    return mcd_fail(MCD_ERR_NOT_CONVERGED, "percentile tie resolution did not finish");
}

}  // extern "C"
#pragma GCC visibility pop
