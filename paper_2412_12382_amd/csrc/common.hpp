// Internal declarations shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "mcd.h"

// Sort key that marks a dropped pair (self-loop or invalid id): all ones, so it
// sorts after every valid packed key.
#define MCD_SENTINEL 0xffffffffffffffffull

struct mcd_ctx {
    int device;
    hipStream_t stream;
    int64_t* d_ctrl;   // device control block: flags and counters (MCD_CTRL_WORDS int64)
    int64_t* h_ctrl;   // pinned host mirror for scalar read-backs
    // tunable launch parameters (mcd_ctx_set_param)
    int64_t tc_chunk;    // in-edges per triangle work item
    int64_t tc_lds_max;  // longest row hashed in LDS; longer rows use binary search
    int64_t tc_packed_range;  // widest rank range (w - v - 1) of a packed LDS table
    int64_t tc_window_max;    // widest rank range of a row held as an LDS rank window
    int64_t k4_row_cache;     // 4-cliques: keep the row offsets of L in LDS when they fit
    int64_t sweep_shape;      // launch shape of the sweep's level loop (0, 1, 2)
    int64_t tc_window_occupancy;  // rank-window kernels built for 8 waves per SIMD (1) or not (0)
    // side streams (default priority) and events on which the triangle
    // count runs its work-item classes concurrently, forked from and joined
    // back into `stream`
    hipStream_t side[2];
    hipEvent_t fork, join[2];
};
#define MCD_TC_WINDOW_LIMIT (1 << 18)
#define MCD_TC_LDS_LIMIT 4096
#define MCD_TC_PACKED_LIMIT ((1 << 20) - 2)
#define MCD_CTRL_WORDS 64
// longest common higher neighbourhood the 4-clique kernel holds in LDS
#define MCD_K4_MAX_COMMON 4096

struct mcd_graph {
    mcd_ctx* ctx;
    int64_t n;         // vertices
    int64_t m;         // undirected edges
    int64_t cap;       // capacity of the per-edge arrays (= n_pairs of the build)
    int bits;          // bits of a vertex id in packed keys (>= 1)
    int32_t max_deg;
    int32_t max_outdeg;
    int64_t bitmask_words;  // sum over edges of ceil(suffix length / 64)
    // Borrowed from the caller's storage buffer.  Vertices are renumbered by
    // rank (degree, original id); "new id" below means that rank.
    int64_t* off;      // [n+1] CSR row offsets of the oriented graph (rows = new ids)
    int32_t* src;      // [cap] row (new id) of every edge
    int32_t* adj;      // [cap] head (new id) of every edge; rows sorted ascending
    int32_t* dsum;     // [cap] deg u + deg v of every edge (read as uint32)
    int32_t* deg;      // [n]   degree by new id (non-decreasing)
    int32_t* perm;     // [n]   original id of every new id
    int64_t* in_off;   // [n+1] offsets of the in-edge lists
    int2* in_ea;       // [cap] (edge id e of x->v, length of row x after v), grouped by head v, by e within
};

// Thread-local error reporting used by the ABI layer.
mcd_status mcd_fail(mcd_status s, const std::string& msg);

#define MCD_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return mcd_fail(MCD_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

static inline size_t mcd_align(size_t x) { return (x + 255) & ~(size_t)255; }

// Bump allocator over a caller-provided buffer.
struct Carve {
    char* base;
    size_t used;
    size_t cap;
    template <class T>
    T* take(size_t count) {
        size_t bytes = mcd_align(count * sizeof(T) + 1);
        T* p = (T*)(base ? base + used : nullptr);
        used += bytes;
        return p;
    }
    bool ok() const { return used <= cap; }
};

namespace mcd {

// ---- device-wide primitives (prim.hip) ----
// Stable LSD radix sort of N keys on bits [first_bit, first_bit + nbits):
// ping-pongs between a and b and returns the buffer holding the result.
// scratch: radix_scratch_bytes(N).
size_t radix_scratch_bytes(int64_t N);
uint64_t* radix_sort_u64(uint64_t* a, uint64_t* b, int64_t N, int nbits, void* scratch,
                         hipStream_t s, int first_bit = 0);
// The same for 32-bit keys on bits [0, nbits).
uint32_t* radix_sort_u32(uint32_t* a, uint32_t* b, int64_t N, int nbits, void* scratch, hipStream_t s);
// radix_sort_u64 carrying an int32 value with every key (va, vb: the value
// buffers, like a, b); *vres receives the buffer holding the sorted values.
uint64_t* radix_sort_u64_kv(uint64_t* a, uint64_t* b, int32_t* va, int32_t* vb, int32_t** vres, int64_t N,
                            int nbits, void* scratch, hipStream_t s, int first_bit = 0);
// Distinct keys of a sorted array, MCD_SENTINEL excluded, into out; the count
// goes to *d_count (device).  scratch: compact_scratch_bytes(N).
size_t compact_scratch_bytes(int64_t N);
void unique_sorted_u64(const uint64_t* in, int64_t N, uint64_t* out, int64_t* d_count,
                       void* scratch, hipStream_t s);
// out[0..N] = exclusive prefix sums of in[0..N) (out[N] = total).
size_t scan_scratch_bytes(int64_t N);
void exclusive_scan_i32_i64(const int32_t* in, int64_t N, int64_t* out, void* scratch,
                            hipStream_t s);
void fill_i32(int32_t* p, int64_t N, int32_t v, hipStream_t s);
void fill_i64(int64_t* p, int64_t N, int64_t v, hipStream_t s);
void fill_u32(uint32_t* p, int64_t N, uint32_t v, hipStream_t s);

// ---- graph construction (build.hip) ----
void launch_canon(const int32_t* src, const int32_t* dst, int64_t P, int64_t n, int bits,
                  uint64_t* keys, int64_t* d_err, hipStream_t s);
// deg[x] += occurrences of x as the lower endpoint of the sorted unique keys
void launch_degree(const uint64_t* uniq, int64_t m, int bits, int32_t* deg_orig, hipStream_t s);
// hi[e] = upper endpoint of key e (to be sorted), then deg[x] += its run length
void launch_upper_ends(const uint64_t* uniq, int64_t m, int bits, uint32_t* hi, hipStream_t s);
void launch_count_runs(const uint32_t* sorted, int64_t m, int32_t* deg, hipStream_t s);
void launch_rank_keys(const int32_t* deg_orig, int64_t n, int bits, uint64_t* keys, hipStream_t s);
void launch_rank_apply(const uint64_t* sorted, int64_t n, int bits, const int32_t* deg_orig,
                       int32_t* perm, int32_t* inv, int32_t* deg_new, hipStream_t s);
void launch_edge_dsum(const int32_t* src, const int32_t* adj, const int32_t* deg, int64_t m, int32_t* dsum,
                      hipStream_t s);
void launch_orient_keys(const uint64_t* uniq, int64_t m, int bits, const int32_t* inv,
                        uint64_t* keys, hipStream_t s);
void launch_csr_fill(const uint64_t* sorted, int64_t m, int bits, int32_t* src, int32_t* adj,
                     int32_t* outdeg, hipStream_t s);
void launch_max_i32(const int32_t* a, int64_t N, int64_t* d_out, hipStream_t s);
// *d_out = the words of the triangle count's hit bitmasks over all rows
void launch_bitmask_words(const int32_t* outdeg, int64_t n, int64_t* d_out, hipStream_t s);
void launch_edges_orig(const int32_t* src, const int32_t* adj, const int32_t* perm, int64_t m,
                       int32_t* u, int32_t* v, hipStream_t s);
void launch_scatter_by_perm(const int32_t* val_new, const int32_t* perm, int64_t n,
                            int32_t* out_orig, hipStream_t s);
// in_cnt[v] = deg[v] - outdeg[v]
void launch_in_count(const int32_t* deg, const int32_t* outdeg, int64_t n, int32_t* in_cnt,
                     hipStream_t s);
// keys[e] = (head of e) << 32 | e, to be sorted on the head bits, and
// suf[e] = off[src[e]+1] - e - 1
void launch_in_keys(const int32_t* src, const int32_t* adj, const int64_t* off, int64_t m, uint64_t* keys,
                    int32_t* suf, hipStream_t s);
// in_ea[i] = (e, suf[e]) for the edges e of the head-sorted keys
// sorted: (head, edge id) keys; suf: the suffix lengths in the same order
void launch_in_fill(const uint64_t* sorted, const int32_t* suf, int64_t m, int2* in_ea, hipStream_t s);

// ---- triangles (tc.hip) ----
size_t tc_scratch_bytes(const mcd_graph* g, int64_t chunk);
void launch_triangles(const mcd_graph* g, int32_t* t, void* ws, int64_t chunk, int64_t lds_max,
                      int64_t packed_range, int64_t window_max, hipStream_t s);

// ---- weights / prune (weight.hip) ----
void launch_weights(const mcd_graph* g, int measure, const int32_t* t, float* wf, int32_t* wi,
                    hipStream_t s);
void launch_prune(const mcd_graph* g, int measure, const int32_t* t, int64_t num, int64_t den,
                  uint32_t* keep_bits, int64_t* n_kept, hipStream_t s);
void launch_prune_graphs(const mcd_graph* g, int measure, const int32_t* t, int G, const int64_t* vbase,
                         const int64_t* deltas, uint32_t* keep_bits, int64_t* n_kept, hipStream_t s);

// Edges per segment of a kept-edge list (multiple of 64).
int64_t kept_segment_len(int64_t m);
// Weights and prune in one pass; deltas (device, per graph) overrides num/den
// when non-NULL.  Every output may be NULL.
void launch_weigh_prune(const mcd_graph* g, int measure, const int32_t* t, int64_t num, int64_t den, int G,
                        const int64_t* vbase, const int64_t* deltas, float* wf, int32_t* wi, uint32_t* keep_bits,
                        int32_t* kept_pairs, int32_t* kept_counts, int64_t* n_kept, hipStream_t s,
                        int32_t* parent = nullptr);  // non-NULL: unite every kept edge in that union-find

// ---- 4-clique participation (k4.hip) ----
void launch_k4(const mcd_graph* g, int32_t* k4, hipStream_t s);

// ---- components (cc.hip) ----
size_t cc_scratch_bytes(const mcd_graph* g);
void launch_components(const mcd_graph* g, const uint32_t* keep_bits, int32_t* labels,
                       int64_t* n_components, void* ws, hipStream_t s);
void launch_components_kept(const mcd_graph* g, const int32_t* kept_pairs, const int32_t* kept_counts,
                            int32_t* labels, int64_t* n_components, void* ws, hipStream_t s);
// The two halves of a components step around unions made elsewhere: the
// union-find in ws set to singletons (its parent array returned), then the
// labels and the count.
int32_t* launch_components_init(const mcd_graph* g, int32_t* labels, int64_t* n_components, void* ws,
                                hipStream_t s);
void launch_components_finish(const mcd_graph* g, int32_t* labels, int64_t* n_components, void* ws,
                              hipStream_t s);
// Unions of every edge of the graph into the union-find `parent` (after
// launch_components_init), vertex by vertex around a sampled large
// component; `giant`: one device int32 of scratch.
void launch_components_all_edges(const mcd_graph* g, int32_t* parent, int32_t* giant, hipStream_t s);

// ---- percentile (select.hip) ----
size_t select_scratch_bytes(const mcd_graph* g);
// Histogram (256 int64) of the digit at `shift` of the keys of nonzero
// similarities whose key matches prefix under pmask.
void sel_hist(const mcd_graph* g, int measure, const int32_t* t, uint32_t prefix, uint32_t pmask,
              int shift, int64_t* hist256, hipStream_t s);
// Minimum rational (out2[0] / out2[1], den 0 = none) strictly above lb among
// nonzero similarities with the given key; part holds 2 int64 per block.
void sel_min_above(const mcd_graph* g, int measure, const int32_t* t, uint32_t key, int64_t lb_num,
                   int64_t lb_den, int lb_valid, int64_t* part, int64_t* out2, hipStream_t s);
// Number of nonzero similarities with the given key equal to num/den.
void sel_count_eq(const mcd_graph* g, int measure, const int32_t* t, uint32_t key, int64_t num,
                  int64_t den, int64_t* cnt, hipStream_t s);

// ---- threshold sweep (sweep.hip) ----
#define MCD_SWEEP_MAX 64
struct SweepDeltas {  // thresholds sorted ascending, passed by value to kernels
    int K;
    int64_t num[MCD_SWEEP_MAX];
    int64_t den[MCD_SWEEP_MAX];
};
size_t sweep_scratch_bytes(const mcd_graph* g, int G, int K, bool truth);
// out_index[i]: caller's slot of the i-th smallest threshold
void launch_sweep(const mcd_graph* g, int measure, const int32_t* t, const SweepDeltas& ds,
                  const int* out_index, int G, const int64_t* vbase, const int32_t* truth,
                  mcd_sweep_stats* stats, double* ari, double* modularity, double* prf, int32_t* labels,
                  void* ws, hipStream_t s, const int32_t* gate = nullptr);

// the threshold rule of thumb over a sweep's statistics (order as for launch_sweep)
void launch_sweep_rule(const SweepDeltas& ds, const int* order, int G, const int64_t* vbase,
                       const mcd_sweep_stats* stats, const double* modularity, int64_t jump_num, int64_t jump_den,
                       int32_t* index, int64_t* deltas, hipStream_t s);

// ---- picker (picker.hip) ----
size_t features_scratch_bytes(int G);
void launch_features(const mcd_graph* g, const int32_t* t, int G, const int64_t* vbase, float* x, void* ws,
                     hipStream_t s);
size_t mlp_scratch_bytes(int B);
void launch_mlp_forward(const float* params, const float* mean, const float* stdv, const float* x, int B,
                        float* y, hipStream_t s);
// Training loss per row: mse_w (y - target)^2, minus (when ari, the row's
// ARI curve of K thresholds, is given) the ARI interpolated at (K-1) y.
struct MlpLoss {
    const float* target;
    const double* ari;  // [B][K] or null
    int K;
    float mse_w;
};
void launch_mlp_gradient(const float* params, const float* mean, const float* stdv, const float* x,
                         const MlpLoss& L, int B, float* grad, float* loss, void* ws, hipStream_t s);
void launch_mlp_train_step(float* params, float* m1, float* m2, int step, float lr, float wd, const float* mean,
                           const float* stdv, const float* x, const MlpLoss& L, int B, float* loss, void* ws,
                           hipStream_t s);
void launch_select(const float* y, int B, int K, int64_t a, int64_t b, int64_t c, int32_t* index,
                   int64_t* delta, hipStream_t s);
void launch_targets(const double* ari, int G, int K, double frac, int32_t* index, float* y, hipStream_t s);
void launch_feature_stats(const float* x, int B, float min_std, float* mean, float* stdv, hipStream_t s);
void launch_feature_range(const float* x, int B, float* lo, float* hi, hipStream_t s);
void launch_fallback(const float* x, int B, const float* lo, const float* hi, float margin, const int64_t* picked,
                     const int64_t* fallback, int64_t* delta, int32_t* flags, hipStream_t s);
// *any = 1 if some flags[0..B) is nonzero, else 0
void launch_any_flag(const int32_t* flags, int B, int32_t* any, hipStream_t s);

}  // namespace mcd
