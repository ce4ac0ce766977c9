/*
 * mcd.h - C ABI of the MI355X (gfx950) motif-based community detection library.
 *
 * The library computes Algorithm 1 of Chen & Tsourakakis, "Parallel
 * Motif-Based Community Detection" (arXiv 2412.12382): weight every edge of an
 * undirected simple graph by a triangle-based similarity, remove the edges
 * whose similarity is below a threshold, and return the connected components
 * of what remains.  Definitions follow the paper's notation paragraph (Sec. 1)
 * and Table "tab:simfunctions":
 *     t(u,v)      = |N(u) n N(v)|                    (triangles on the edge)
 *     wedge(u,v)  = |N(u) u N(v)| - |N(u) n N(v)| - 2
 *     Tectonic    = t(u,v) / (deg u + deg v)
 *     TW          = t(u,v) - wedge(u,v) = 3 t - deg u - deg v + 2   (Eq. eq:tw)
 *     K3          = t(u,v)
 *     Jaccard     = t(u,v) / (deg u + deg v - t(u,v))
 *     K4          = number of 4-cliques containing {u,v}
 *
 * Conventions
 *   - Every call returns mcd_status: MCD_OK (0) or a negative error.  Nothing
 *     aborts or throws across the ABI.  mcd_last_error() gives a message for
 *     the calling thread's most recent failure.
 *   - Array arguments are DEVICE pointers owned by the caller unless the name
 *     says host_.  The library never allocates device memory except a small
 *     control block in mcd_ctx_create (and the fixed scratch array of
 *     mcd_prune_components_noalloc, held per device from load to process
 *     end).  Calls that need scratch memory take a
 *     workspace (ws, ws_bytes) sized by the matching *_workspace_size query;
 *     a smaller workspace gives MCD_ERR_WORKSPACE.  Workspaces and the graph
 *     storage buffer must start on a 256-byte boundary (the library carves
 *     them into typed arrays); another start gives MCD_ERR_INVALID_ARG.
 *   - Work is enqueued on the context's stream.  Calls documented as
 *     "synchronous" wait for that stream before returning (they return host
 *     scalars); all others are asynchronous and their outputs are valid once
 *     the stream reaches them.
 *   - Handles (mcd_ctx, mcd_graph) are host objects created and freed by the
 *     library.  A graph handle BORROWS the caller's storage buffer, which must
 *     outlive it.  One context per host thread.
 *   - Vertex ids are int32 in [0, n); n < 2^31 - 1.  The build takes fewer
 *     than 2^31 raw pairs (n_pairs < 2^31, so m < 2^31 undirected edges);
 *     edge offsets and counts are int64 beyond that point.
 *   - Per-edge arrays are in LIBRARY EDGE ORDER: the order of mcd_graph_edges,
 *     fixed for a graph handle.  Vertex arrays are indexed by original id.
 */
#ifndef MCD_H
#define MCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mcd_status;
#define MCD_OK 0
#define MCD_ERR_INVALID_ARG (-1)    /* NULL pointer, negative size, den <= 0 ...    */
#define MCD_ERR_INVALID_VERTEX (-2) /* an input id outside [0, n)                    */
#define MCD_ERR_RANGE (-3)          /* a size beyond the supported range             */
#define MCD_ERR_WORKSPACE (-4)      /* workspace or storage smaller than required    */
#define MCD_ERR_NO_DEVICE (-5)      /* no HIP device, or the device id is invalid    */
#define MCD_ERR_DEVICE (-6)         /* a HIP runtime call failed                     */
#define MCD_ERR_NOT_CONVERGED (-7)  /* an iterative step hit its iteration cap       */
#define MCD_ERR_EMPTY (-8)          /* the requested statistic has no data           */
#define MCD_ERR_CHECKPOINT (-9)     /* a picker checkpoint or autotune cache file is
                                       unreadable or corrupt                          */

typedef struct mcd_ctx mcd_ctx;
typedef struct mcd_graph mcd_graph;

/* A threshold delta = num / den, den > 0, |num| and den below 2^31. */
typedef struct {
    int64_t num;
    int64_t den;
} mcd_rational;

/* Similarity measures of Table tab:simfunctions that the library evaluates. */
typedef enum {
    MCD_SIM_TECTONIC = 0, /* t / (deg u + deg v)                      */
    MCD_SIM_TW = 1,       /* t - wedge = 3t - deg u - deg v + 2       */
    MCD_SIM_K3 = 2,       /* t, the number of triangles on the edge   */
    MCD_SIM_JACCARD = 3,  /* t / (deg u + deg v - t) = |N(u) n N(v)| / |N(u) u N(v)|;
                             Prop. 1: pruning it at p/q equals pruning Tectonic at p/(p+q) */
    MCD_SIM_K4 = 4        /* kappa-clique participation, kappa = 4: the per-edge count of
                             mcd_k4, passed where the other measures take t */
} mcd_measure;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device` whose work goes to `stream` (a
 * hipStream_t, NULL = the default stream).  Allocates a small device control
 * block and pinned host memory for scalar read-backs.
 * Errors: MCD_ERR_NO_DEVICE, MCD_ERR_DEVICE, MCD_ERR_INVALID_ARG (out NULL). */
mcd_status mcd_ctx_create(int device, void* stream, mcd_ctx** out);
/* Replaces the stream of a context. */
mcd_status mcd_ctx_set_stream(mcd_ctx* ctx, void* stream);
/* Launch parameters of later calls on this context (results never depend on
 * them; the autotuner sets them):
 *   "tc_chunk"   in-edges per triangle-count work item, [1, 2^24], default 512;
 *   "tc_lds_max" longest out-neighbour row hashed in LDS, [0, 4096], default
 *                4096; longer rows use the binary-search path;
 *   "tc_packed_range" widest rank range of a row stored in the one-word LDS
 *                table, [0, 2^20 - 2], default 2^20 - 2; wider rows use the
 *                two-array table;
 *   "tc_window_max" widest rank range of a row held as an LDS rank bitmap,
 *                [0, 2^18], default 2^18 (0 disables the bitmap path);
 *   "k4_row_cache" mcd_k4 keeps the row offsets of the common neighbours
 *                of a long row in LDS when they fit, 0 or 1, default 1
 *                (0: read them per pair);
 *   "sweep_shape" launch shape of mcd_sweep's level loop (one persistent
 *                launch): 0 = 1024 threads per block, 1 = 512, 2 = 256
 *                threads per block, default 0;
 *   "tc_window_occupancy" the rank-bitmap triangle kernels built for 8
 *                waves per SIMD (1) or with the compiler's register budget
 *                (0), default 1.  Counts are identical either way.
 * Errors: MCD_ERR_INVALID_ARG (unknown name), MCD_ERR_RANGE (bad value). */
mcd_status mcd_ctx_set_param(mcd_ctx* ctx, const char* name, int64_t value);
mcd_status mcd_ctx_get_param(const mcd_ctx* ctx, const char* name, int64_t* value);
mcd_status mcd_ctx_destroy(mcd_ctx* ctx);

/* Name of a status code (static string). */
const char* mcd_status_string(mcd_status s);
/* Message of the calling thread's last failure ("" if none). */
const char* mcd_last_error(void);

/* ------------------------------------------------------------ graph build */

/* Sizes for mcd_graph_build on n_pairs raw pairs over n_vertices vertices:
 *   storage_bytes: the persistent graph storage the handle borrows;
 *   ws_bytes:      scratch needed only during the build.
 * Errors: MCD_ERR_INVALID_ARG, MCD_ERR_RANGE (n_vertices >= 2^31 - 1 or
 * n_pairs >= 2^31: the largest input is 2^31 - 1 raw pairs). */
mcd_status mcd_graph_build_sizes(int64_t n_pairs, int64_t n_vertices, size_t* storage_bytes,
                                 size_t* ws_bytes);

/* Builds the simple undirected graph G of the paper's notation paragraph
 * (Sec. 1) from raw pairs (src[i], dst[i]), i < n_pairs: every pair with
 * src != dst is the undirected edge {src, dst}; self-loops are dropped and
 * duplicates (in either direction) collapse to one edge.
 * Internally vertices are ranked by (degree, id) and each edge is oriented
 * from its lower- to its higher-ranked endpoint (the degree ordering that
 * Sec. 2 cites for triangle counting); the result is a CSR of out-neighbours
 * sorted by rank, plus the row of every edge.
 *   src, dst:  device int32[n_pairs], read only.
 *   storage:   device buffer of at least storage_bytes (mcd_graph_build_sizes),
 *              borrowed by the handle until mcd_graph_destroy.
 *   ws:        device scratch of at least ws_bytes, free again on return.
 * Synchronous (returns the handle with m known on the host).
 * Errors: MCD_ERR_INVALID_VERTEX (an id outside [0, n_vertices); no handle is
 * returned), MCD_ERR_WORKSPACE, MCD_ERR_INVALID_ARG, MCD_ERR_RANGE, MCD_ERR_DEVICE. */
mcd_status mcd_graph_build(mcd_ctx* ctx, const int32_t* src, const int32_t* dst, int64_t n_pairs,
                           int64_t n_vertices, void* storage, size_t storage_bytes, void* ws,
                           size_t ws_bytes, mcd_graph** out);

/* Host-side facts of a built graph: n, m (undirected edges), max degree and
 * max out-degree of the orientation.  Any output pointer may be NULL. */
mcd_status mcd_graph_info(const mcd_graph* g, int64_t* n, int64_t* m, int32_t* max_deg,
                          int32_t* max_outdeg);

/* Endpoints (original ids) of every edge in library edge order: u[e] is the
 * lower-ranked endpoint, v[e] the higher-ranked one.  u, v: device int32[m]. */
mcd_status mcd_graph_edges(const mcd_graph* g, int32_t* u, int32_t* v);

/* deg(x) = |N(x)| for every original id x.  deg: device int32[n]. */
mcd_status mcd_graph_degrees(const mcd_graph* g, int32_t* deg);

/* The library's internal vertex numbering (rank by (degree, original id)):
 * perm[r] is the original id of internal vertex r.  perm: device int32[n].
 * Kept-edge lists (mcd_weigh_prune) hold internal numbers. */
mcd_status mcd_graph_perm(const mcd_graph* g, int32_t* perm);

mcd_status mcd_graph_destroy(mcd_graph* g);

/* ----------------------------------------------------------------- steps */

/* Scratch for mcd_triangles with the context's current parameters. */
mcd_status mcd_triangles_workspace_size(const mcd_graph* g, size_t* bytes);

/* t(e) = |N(u) n N(v)| for every edge e = {u,v} (Sec. 1 notation; Sec. 3.3
 * names this the dominant cost).  Each triangle is found once, from its
 * lowest-ranked edge, and credited to its three edges.  t: device int32[m];
 * ws: device scratch of mcd_triangles_workspace_size bytes. */
mcd_status mcd_triangles(const mcd_graph* g, int32_t* t, void* ws, size_t ws_bytes);

/* Autotuner of the triangle-count launch parameters (item chunk, rank-window
 * cutoff, packed-hash range, LDS row cap) on this graph: a coordinate search
 * over a fixed candidate grid, each setting timed with HIP events on the
 * context's stream (smallest of `reps` runs, after a warm-up).  The fastest
 * setting is stored in the context (mcd_ctx_get_param reads it back) and
 * returned in host_best[4] = {tc_chunk, tc_lds_max, tc_packed_range,
 * tc_window_max} (may be NULL) with its time in *host_ms (may be NULL).  The
 * counts never depend on the parameters; t (device int32[m]) ends holding
 * them.  ws: mcd_tune_triangles_workspace_size bytes.  Synchronous. */
mcd_status mcd_tune_triangles_workspace_size(const mcd_graph* g, size_t* bytes);
mcd_status mcd_tune_triangles(const mcd_graph* g, int32_t* t, void* ws, size_t ws_bytes, int32_t reps,
                              int64_t* host_best, float* host_ms);

/* Autotune cache: the tuned launch parameters of a context kept in a JSON
 * text file at `path`, one entry per (device architecture name, floor(log2 n),
 * floor(log2 m), tuning version of this library).  The parameters kept are
 * tc_chunk, tc_lds_max, tc_packed_range, tc_window_max, tc_window_occupancy
 * and sweep_shape (see mcd_ctx_set_param).
 *   mcd_tune_cache_load:  on an entry for g's key, every value passes the
 *     checks of mcd_ctx_set_param and is set on ctx (all or none), *hit = 1;
 *     otherwise ctx is unchanged and *hit = 0.  A missing file is a miss.
 *   mcd_tune_cache_store: records ctx's current parameters (and ms, the tuned
 *     time, for information) as g's entry, replacing an entry of the same
 *     key and keeping the others; the file is written beside `path` and then
 *     renamed over it.  Calls that write one file concurrently race.
 *   mcd_tune_cache_check_file: the file checks alone, on the host (no device
 *     needed): MCD_OK for a sound or missing file.
 * g must belong to ctx.  Synchronous, host only (no device work).  Errors:
 * MCD_ERR_CHECKPOINT (the file is unreadable, malformed, or holds a value
 * the context refuses; the file is left as it was), MCD_ERR_INVALID_ARG,
 * MCD_ERR_DEVICE (the device's properties could not be read). */
mcd_status mcd_tune_cache_load(mcd_ctx* ctx, const mcd_graph* g, const char* path, int32_t* hit);
mcd_status mcd_tune_cache_store(const mcd_ctx* ctx, const mcd_graph* g, const char* path, float ms);
mcd_status mcd_tune_cache_check_file(const char* path);

/* kappa-clique participation for kappa = 4 (Table tab:simfunctions):
 * k4[e] = the number of 4-cliques containing edge e (library edge order),
 * device int32[m].  Each 4-clique is found once, from its lowest edge in the
 * degree order, and credits its six edges with atomics.  The result feeds
 * mcd_weights / mcd_prune / mcd_weigh_prune / mcd_sweep with MCD_SIM_K4 in
 * place of t.  Work for rows longer than 256 edges runs on a side stream of
 * the context, forked from and joined back into the context's stream (so the
 * call can be captured into a graph like any other).  Errors: MCD_ERR_RANGE
 * when a row of the oriented graph holds more than 4096 edges.  Asynchronous. */
mcd_status mcd_k4(const mcd_graph* g, int32_t* k4);

/* Edge similarity of Table tab:simfunctions from t (as produced by
 * mcd_triangles).  w_f32 (device float[m], may be NULL): the measure in IEEE
 * fp32; Tectonic and Jaccard as the correctly rounded quotient.
 * w_i32 (device int32[m], may be NULL; TW, K3 and K4 only): the exact integer. */
mcd_status mcd_weights(const mcd_graph* g, mcd_measure measure, const int32_t* t, float* w_f32,
                       int32_t* w_i32);

/* Algorithm 1, first step: edge e is removed iff sim(e) < delta, so it is
 * kept iff NOT (sim(e) < delta); ties are kept.  The decision is exact
 * integer arithmetic on sim = sn / sd: Tectonic keeps iff t den >= num (deg u
 * + deg v), TW iff TW den >= num, K3 iff t den >= num, Jaccard iff t den >=
 * num (deg u + deg v - t).
 *   keep_bits: device uint32[ceil(m/32)], bit (e % 32) of word e / 32.
 *   n_kept:    device int64[1] (may be NULL), the number of kept edges. */
mcd_status mcd_prune(const mcd_graph* g, mcd_measure measure, const int32_t* t, mcd_rational delta,
                     uint32_t* keep_bits, int64_t* n_kept);

/* Number of segments of a compacted kept-edge list (see mcd_weigh_prune). */
#define MCD_KEPT_SEGMENTS 16384

/* Weights and prune in ONE pass over the edges: the two read the same data
 * (t, both endpoints, both degrees), so Algorithm 1's first step costs one
 * stream of the edge arrays.  The decision is mcd_prune's (ties kept, exact
 * integer cross-multiplication); the weights are mcd_weights'.
 *   delta:      the threshold when deltas is NULL;
 *   deltas:     NULL, or device int64[2 n_graphs]: graph k's threshold is
 *               deltas[2k] / deltas[2k+1] (den > 0; the comparison is exact in
 *               128-bit arithmetic); graph k owns the original ids
 *               [vbase[k], vbase[k+1]) (vbase: device int64[n_graphs+1]).
 *   w_f32, w_i32: as mcd_weights (each may be NULL; w_i32 for TW and K3 only).
 *   keep_bits:  as mcd_prune (may be NULL).
 *   kept_pairs, kept_counts: the kept edges as a segmented list, the input of
 *               mcd_components_kept (both NULL, or both given).  The edges,
 *               in library edge order, are cut into S = MCD_KEPT_SEGMENTS runs
 *               of L = mcd_kept_segment_len edges; segment s writes the kept
 *               edges of run s, in edge order, as pairs of INTERNAL vertex
 *               numbers (mcd_graph_perm) to kept_pairs[2 s L ...] and their
 *               number to kept_counts[s].  kept_pairs: device int32[2 S L];
 *               kept_counts: device int32[MCD_KEPT_SEGMENTS].
 *   n_kept:     device int64[1] (may be NULL), the number of kept edges.
 * Asynchronous. */
mcd_status mcd_weigh_prune(const mcd_graph* g, mcd_measure measure, const int32_t* t, mcd_rational delta,
                           int32_t n_graphs, const int64_t* vbase, const int64_t* deltas, float* w_f32,
                           int32_t* w_i32, uint32_t* keep_bits, int32_t* kept_pairs, int32_t* kept_counts,
                           int64_t* n_kept);

/* Edges per run (and pair capacity per segment) of a kept-edge list of this
 * graph: L = 64 ceil(ceil(m / 64) / MCD_KEPT_SEGMENTS). */
mcd_status mcd_kept_segment_len(const mcd_graph* g, int64_t* len);

/* Scratch for mcd_components / mcd_components_kept / mcd_run on this graph. */
mcd_status mcd_components_workspace_size(const mcd_graph* g, size_t* bytes);
mcd_status mcd_run_workspace_size(const mcd_graph* g, size_t* bytes);

/* Algorithm 1, second step: connected components of (V, kept edges).
 * labels[x] (device int32[n], by original id) is the smallest original id in
 * x's component, so isolated vertices label themselves.  keep_bits may be
 * NULL (every edge kept).  n_components: device int64[1] (may be NULL).
 * Lock-free union-find (roots hook under the higher-ranked root, finds halve
 * paths), then every component takes the smallest original id among its
 * vertices as its label. */
mcd_status mcd_components(const mcd_graph* g, const uint32_t* keep_bits, int32_t* labels,
                          int64_t* n_components, void* ws, size_t ws_bytes);

/* mcd_components over a kept-edge list written by mcd_weigh_prune on the
 * same graph (kept_pairs, kept_counts as described there).  Same labels and
 * count as mcd_components on the equivalent keep_bits.  Asynchronous. */
mcd_status mcd_components_kept(const mcd_graph* g, const int32_t* kept_pairs, const int32_t* kept_counts,
                               int32_t* labels, int64_t* n_components, void* ws, size_t ws_bytes);

/* Algorithm 1's two steps fused into one pass over the edges, from given
 * similarity inputs t: the weights and keep decisions of mcd_weigh_prune
 * (delta, or per-graph deltas with vbase; w_f32, w_i32, keep_bits and n_kept
 * may each be NULL), with every kept edge united in the components' union-find
 * as soon as it is decided, then labels and n_components as mcd_components.
 * A single delta <= 0 with a measure that is never negative (all but TW)
 * keeps every edge: the pass then writes the weights and keep bits only, and
 * every edge is united vertex by vertex around a sampled large component
 * (same labels and count).  No kept-edge list is written.  labels: device
 * int32[n]; ws: mcd_components_workspace_size bytes.  Asynchronous. */
mcd_status mcd_prune_components(const mcd_graph* g, mcd_measure measure, const int32_t* t, mcd_rational delta,
                                int32_t n_graphs, const int64_t* vbase, const int64_t* deltas, float* w_f32,
                                int32_t* w_i32, uint32_t* keep_bits, int64_t* n_kept, int32_t* labels,
                                int64_t* n_components, void* ws, size_t ws_bytes);

/* Most vertices of a graph given to mcd_prune_components_noalloc: the size of
 * its device scratch array (int32 each, 64 MiB per device). */
#define MCD_NOALLOC_MAX_VERTICES (1 << 24)

/* mcd_prune_components without a workspace, for callers that cannot allocate
 * device memory or pass a workspace (code under HIP graph capture, tight
 * serving loops, hosts that forbid allocation).  Same arguments, kernels and
 * results as mcd_prune_components, minus ws / ws_bytes: the components'
 * union-find parent array lives in a device array of the library, sized for
 * MCD_NOALLOC_MAX_VERTICES vertices, that each device holds from the
 * library's load until the process ends.  The call allocates nothing and
 * calls no allocating routine; the caller still passes every output buffer.
 * Every call on one device shares that device's array and leaves its contents
 * behind (each call first resets the part it uses), so calls that overlap on
 * one device, on any streams or contexts, race and give wrong labels: order
 * them.  Errors: MCD_ERR_RANGE when the graph has more than
 * MCD_NOALLOC_MAX_VERTICES vertices; otherwise those of mcd_prune_components.
 * Asynchronous. */
mcd_status mcd_prune_components_noalloc(const mcd_graph* g, mcd_measure measure, const int32_t* t,
                                        mcd_rational delta, int32_t n_graphs, const int64_t* vbase,
                                        const int64_t* deltas, float* w_f32, int32_t* w_i32, uint32_t* keep_bits,
                                        int64_t* n_kept, int32_t* labels, int64_t* n_components);

/* Algorithm 1 in one call: triangles, weights, prune at delta, components.
 * labels / n_components as in mcd_components.  Asynchronous. */
mcd_status mcd_run(const mcd_graph* g, mcd_measure measure, mcd_rational delta, int32_t* labels,
                   int64_t* n_components, void* ws, size_t ws_bytes);

/* Per graph and threshold results of mcd_sweep. */
typedef struct {
    int64_t m_kept;            /* edges kept (NOT sim < delta)                       */
    int64_t n_components;      /* connected components, singletons included          */
    int64_t largest_component; /* vertices in the largest component                  */
    int64_t pairs_cluster;     /* A: vertex pairs that share a component             */
    int64_t pairs_class;       /* B: vertex pairs that share a planted class (or 0)  */
    int64_t pairs_both;        /* S: vertex pairs that share both (or 0)             */
    int64_t pairs_total;       /* N = n_g (n_g - 1) / 2                               */
    int64_t intra_edges;       /* input edges inside one component (with modularity) */
    int64_t volume_sq;         /* sum over components of (sum of input degrees)^2,
                                  exact while 2m < 2^31.5 (with modularity)          */
} mcd_sweep_stats;

/* Most thresholds one mcd_sweep call evaluates. */
#define MCD_SWEEP_MAX_THRESHOLDS 64

/* Scratch for mcd_sweep. */
mcd_status mcd_sweep_workspace_size(const mcd_graph* g, int32_t n_graphs, int32_t n_thresholds,
                                    int32_t has_truth, size_t* bytes);

/* Algorithm 1 at K thresholds at once, over one graph or a batch of disjoint
 * graphs packed into g (graph k owns the original ids [vbase[k], vbase[k+1])).
 * Every edge's level (how many of the thresholds it survives) fixes all K prune
 * masks; one union-find then absorbs the edges level by level from the
 * highest threshold down, and after each level per-graph statistics are taken
 * (the selection statistics of Sec. 4.4: kept edges, number of components,
 * largest component).  With planted labels `truth`, the adjusted Rand index
 * ARI = (S - A B / N) / ((A + B) / 2 - A B / N) (1 when the denominator is 0)
 * is evaluated in fp64 from the exact pair counts.  With `modularity`, each
 * partition's modularity on the input graph (Sec. 2), Q = intra / m -
 * volume_sq / (4 m^2) in fp64 from the exact integers of the stats, m the
 * graph's edges (0 for a graph without edges); this adds a pass over the
 * edges per threshold.
 *   host_deltas: K thresholds (any order, duplicates allowed), K <= 64.
 *   vbase:       device int64[n_graphs + 1], vbase[0] = 0, vbase[n_graphs] = n,
 *                non-decreasing (n_graphs = 1, vbase = {0, n}: a single graph).
 *   truth:       device int32[n] class of every original id, ids in [0, n); a
 *                class may not span two graphs.  NULL: no ARI (pairs_class,
 *                pairs_both and ari are 0).
 *   stats:       device mcd_sweep_stats[n_graphs][K] (slot k = caller's k-th threshold).
 *   ari:         device double[n_graphs][K], may be NULL.
 *   modularity:  device double[n_graphs][K], may be NULL (then intra_edges and
 *                volume_sq are 0).
 *   prf:         device double[n_graphs][K][3], may be NULL; with truth: the
 *                evaluation of Sec. 4 (Setup, Evaluation): every component is
 *                matched to the planted class of largest Jaccard overlap (ties:
 *                smaller class id) and precision, recall and F1 are averaged
 *                over components weighted by size (fp64 sums; the summation
 *                order is not fixed, so the last bits may vary run to run).
 *   labels:      device int32[K][n] min-original-id labels per threshold, may be NULL.
 * Asynchronous; no host synchronisation or memset inside, so the call can be
 * captured in a HIP graph. */
mcd_status mcd_sweep(const mcd_graph* g, mcd_measure measure, const int32_t* t,
                     const mcd_rational* host_deltas, int32_t n_thresholds, int32_t n_graphs,
                     const int64_t* vbase, const int32_t* truth, mcd_sweep_stats* stats, double* ari,
                     double* modularity, double* prf, int32_t* labels, void* ws, size_t ws_bytes);

/* The paper's rule of thumb for the threshold (Sec. 4.4, Fig. tab:selection),
 * per graph, from a sweep's statistics: walking the thresholds downwards, the
 * largest single increase of the largest component (between consecutive
 * thresholds, in vertices) marks where dense regions stop being split; if
 * that jump is at least jump_num/jump_den of the graph's vertices the rule
 * picks the threshold just above it.  Otherwise it picks the threshold of
 * maximum modularity (ties: the highest threshold), or, when modularity is
 * NULL, the highest threshold.
 *   host_deltas, n_thresholds: the thresholds given to mcd_sweep (same order).
 *   stats, modularity: mcd_sweep's outputs [n_graphs][K] (modularity may be NULL).
 *   vbase: as for mcd_sweep.  index: device int32[n_graphs], the picked slot;
 *   deltas: device int64[2 n_graphs] (may be NULL), the picked num, den.
 * Asynchronous. */
mcd_status mcd_sweep_rule(mcd_ctx* ctx, const mcd_rational* host_deltas, int32_t n_thresholds, int32_t n_graphs,
                          const int64_t* vbase, const mcd_sweep_stats* stats, const double* modularity,
                          int64_t jump_num, int64_t jump_den, int32_t* index, int64_t* deltas);

/* -------------------------------------------------- learned threshold picker */

#define MCD_MLP_IN 66      /* 64 histogram bins, log1p mean degree, log1p max degree */
#define MCD_MLP_HIDDEN 64
#define MCD_MLP_PARAMS 8513 /* W1[64][66] b1[64] W2[64][64] b2[64] W3[64] b3 */

/* Per-graph input features of the picker (one graph, or a batch as in
 * mcd_sweep): x[k][0..63] = fraction of graph k's edges whose Tectonic value
 * t / D falls in bin floor(128 t / D) (the values lie in [0, 1/2)),
 * x[k][64] = log1p(2 m_k / n_k), x[k][65] = log1p(max degree).
 * x: device float[n_graphs][66]. */
mcd_status mcd_features_workspace_size(int32_t n_graphs, size_t* bytes);
mcd_status mcd_features(const mcd_graph* g, const int32_t* t, int32_t n_graphs, const int64_t* vbase,
                        float* x, void* ws, size_t ws_bytes);

/* Column mean and population standard deviation, raised to at least min_std
 * (> 0) so near-constant columns are not amplified, of a feature matrix x
 * (device float[batch][66]) into mean, std (device float[66]). */
mcd_status mcd_feature_stats(mcd_ctx* ctx, const float* x, int32_t batch, float min_std, float* mean,
                             float* std);

/* Column minimum and maximum of a feature matrix x (device float[batch][66],
 * batch >= 1) into lo, hi (device float[66]): the training range that
 * mcd_picker_fallback checks against. */
mcd_status mcd_feature_range(mcd_ctx* ctx, const float* x, int32_t batch, float* lo, float* hi);

/* The learned threshold's guard (the full sweep is the picker's fallback):
 * graph g is out of the training range when some feature x[g][k] lies
 * outside [lo[k] - margin w_k, hi[k] + margin w_k], w_k = hi[k] - lo[k] (each
 * bound formed in fp32, one rounding per operation); flags[g] = 1 then, else
 * 0 (flags: device int32[batch], may be NULL).  delta[g] (device
 * int64[batch][2], may be NULL) = fallback[g] for flagged graphs, else
 * picked[g] (delta may alias picked or fallback).  margin >= 0. */
mcd_status mcd_picker_fallback(mcd_ctx* ctx, const float* x, int32_t batch, const float* lo, const float* hi,
                               float margin, const int64_t* picked, const int64_t* fallback, int64_t* delta,
                               int32_t* flags);

/* FP32 MLP 66 -> 64 -> 64 -> 1 with ReLU on the hidden layers, applied to
 * (x - mean) / std.  params: device float[MCD_MLP_PARAMS]; y: device float[batch]. */
mcd_status mcd_mlp_forward(mcd_ctx* ctx, const float* params, const float* mean, const float* std,
                           const float* x, int32_t batch, float* y);

/* Scratch for mcd_mlp_gradient / mcd_mlp_train_step at this batch size. */
mcd_status mcd_mlp_workspace_size(int32_t batch, size_t* bytes);

/* Gradient of the training loss L = (1/batch) sum over rows of
 *     mse_weight (y - target)^2 - ARI_r((K - 1) y)
 * with respect to params (device float[MCD_MLP_PARAMS]), and L itself (device
 * float[1], may be NULL), summed over the batch in a fixed order.  ari (device
 * double[batch][K], K >= 2, may be NULL: no ARI term) is each row's ARI at
 * the K grid thresholds; ARI_r(z) interpolates it linearly at z clamped to
 * [0, K - 1] (segment chosen in fp32), with slope 0 outside 0 < z < K - 1.
 * mse_weight >= 0 (1 with no ARI table: the plain squared error).  The ARI
 * term makes the network's snapped threshold score well under the sweep's own
 * judge, the ARI against the planted partition. */
mcd_status mcd_mlp_gradient(mcd_ctx* ctx, const float* params, const float* mean, const float* std,
                            const float* x, const float* target, const double* ari, int32_t K, float mse_weight,
                            int32_t batch, float* grad, float* loss, void* ws, size_t ws_bytes);

/* One full-batch Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected,
 * step counted from 1) on params with moment buffers adam_m, adam_v (device
 * float[MCD_MLP_PARAMS], zero before step 1), with decoupled weight decay
 * (p -= lr * weight_decay * p first; 0 = plain Adam), on the loss of
 * mcd_mlp_gradient.  loss: the pre-step loss. */
mcd_status mcd_mlp_train_step(mcd_ctx* ctx, float* params, float* adam_m, float* adam_v, int32_t step,
                              float lr, float weight_decay, const float* mean, const float* std, const float* x,
                              const float* target, const double* ari, int32_t K, float mse_weight, int32_t batch,
                              float* loss, void* ws, size_t ws_bytes);

/* The picker as a library object.  mcd_picker_create allocates its device
 * state (parameters, Adam moments, standardisation, training range: 103 KB)
 * on the context's device; mcd_picker_destroy frees it.  The network maps a
 * graph's features (mcd_features) to y in [0, 1], snapped to the grid
 * delta_i = (MCD_PICKER_GRID_A + MCD_PICKER_GRID_B i) / MCD_PICKER_GRID_C,
 * i < MCD_PICKER_GRID_K (64 evenly spaced values in [0.01, 0.5]).  The
 * threshold sweep over the same grid is both its fallback and its judge:
 * graphs whose features leave the training range (widened by the picker's
 * margin) take the sweep's rule of thumb instead (mcd_sweep_rule). */
typedef struct mcd_picker mcd_picker;
#define MCD_PICKER_GRID_K 64
#define MCD_PICKER_GRID_A 9
#define MCD_PICKER_GRID_B 7
#define MCD_PICKER_GRID_C 900
#define MCD_PICKER_MARGIN 0.25f /* default margin of the range guard, of each feature's width */

/* Creates a picker whose weights are He-uniform, drawn from `seed`: weight
 * number i of the flat vector (a layer of fan-in f) is (2 u_i - 1) sqrt(6/f)
 * rounded to fp32, u_i the uniform in (0,1) of Philox-4x32-10 (Salmon et al.,
 * SC'11) at counter (i, 0x55, 0x4D4C5030) under key `seed`, built from the
 * first two output words (53 bits, plus half a step); biases are zero.  The
 * picker cannot pick until prepared, fitted or loaded.  Synchronous.
 * Errors: MCD_ERR_INVALID_ARG, MCD_ERR_DEVICE. */
mcd_status mcd_picker_create(mcd_ctx* ctx, uint64_t seed, mcd_picker** out);
mcd_status mcd_picker_destroy(mcd_picker* p);

/* Sets the standardisation (mcd_feature_stats with min_std) and the training
 * range (mcd_feature_range) from training features x (device
 * float[batch][66]), the guard's margin (>= 0), and restarts Adam. */
mcd_status mcd_picker_prepare(mcd_picker* p, const float* x, int32_t batch, float min_std, float margin);

/* One Adam step as mcd_mlp_train_step on the picker's own parameters and
 * moments (its step counter advances), K = MCD_PICKER_GRID_K: ari (device
 * double[batch][64], the rows' ARI over the picker's grid, may be NULL) and
 * mse_weight as there.  loss (device float[1]) may be NULL.
 * ws: mcd_mlp_workspace_size(batch). */
mcd_status mcd_picker_train_step(mcd_picker* p, const float* x, const float* y, const double* ari, float mse_weight,
                                 int32_t batch, float lr, float weight_decay, float* loss, void* ws, size_t ws_bytes);

/* mcd_picker_prepare, then `steps` train steps on (x, y, ari): full-batch
 * training on the sweep's targets (mcd_sweep_targets) and ARI table
 * (mcd_sweep).  losses: device float[steps], each step's pre-step loss, may
 * be NULL.  Asynchronous. */
mcd_status mcd_picker_fit(mcd_picker* p, const float* x, const float* y, const double* ari, float mse_weight,
                          int32_t batch, int32_t steps, float lr, float weight_decay, float min_std, float margin,
                          float* losses, void* ws, size_t ws_bytes);

/* The network's output y (device float[batch]) for features x. */
mcd_status mcd_picker_forward(const mcd_picker* p, const float* x, int32_t batch, float* y);

/* Scratch for mcd_picker_pick on this graph (or batch of n_graphs). */
mcd_status mcd_picker_pick_workspace_size(const mcd_graph* g, int32_t n_graphs, size_t* bytes);

#define MCD_PICK_AUTO 0        /* the network, the sweep's rule where the guard fires */
#define MCD_PICK_FORCE_SWEEP 1 /* the sweep's rule of thumb for every graph          */
#define MCD_PICK_NETWORK 2     /* the network for every graph, no guard               */

/* Algorithm 1 with a learned threshold, per graph of a batch (vbase as in
 * mcd_sweep): features -> network -> grid snap -> range guard -> (where the
 * guard fires, or in MCD_PICK_FORCE_SWEEP mode, or when the environment sets
 * MCD_FORCE_SWEEP to anything but "0": the grid sweep with modularity and its
 * rule of thumb, jump 1/10) -> prune at each graph's threshold and components.
 *   index:         device int32[n_graphs], the network's grid index (may be NULL);
 *   deltas:        device int64[n_graphs][2], the threshold each graph used (may be NULL);
 *   used_fallback: device int32[n_graphs], 1 where the sweep's threshold was used (may be NULL);
 *   labels, n_components: as for mcd_components over the whole batch.
 * Asynchronous in every mode (the call can be captured in a HIP graph):
 * MCD_PICK_AUTO decides on the device whether any graph needs the sweep, whose
 * kernels otherwise return at once.
 * The work goes to the graph's context stream; picker and graph must be on
 * one device.  Errors: MCD_ERR_INVALID_ARG (unprepared picker, another
 * device), MCD_ERR_WORKSPACE. */
mcd_status mcd_picker_pick(const mcd_picker* p, const mcd_graph* g, mcd_measure measure, const int32_t* t,
                           int32_t n_graphs, const int64_t* vbase, int32_t mode, int32_t* index, int64_t* deltas,
                           int32_t* used_fallback, int32_t* labels, int64_t* n_components, void* ws,
                           size_t ws_bytes);

/* Copies the picker's state out to (export) or in from (import) caller
 * device buffers: params float[MCD_MLP_PARAMS], mean, std, lo, hi float[66];
 * export skips NULL outputs and returns the margin in *host_margin (may be
 * NULL); import restarts Adam and marks the picker prepared. */
mcd_status mcd_picker_export(const mcd_picker* p, float* params, float* mean, float* std, float* lo, float* hi,
                             float* host_margin);
mcd_status mcd_picker_import(mcd_picker* p, const float* params, const float* mean, const float* std,
                             const float* lo, const float* hi, float margin);

/* Checkpoint of a prepared picker (network, standardisation, training range,
 * margin) as a little-endian file: "MCDPICK\0", version 1, the network shape,
 * the grid, the margin, the arrays, and a CRC-32 (IEEE) of everything before
 * it.  save writes `path`.tmp and renames it; load checks length, magic,
 * version, CRC, shape, grid, finiteness and positive std before touching the
 * picker.  Both synchronous.  Errors: MCD_ERR_CHECKPOINT (I/O or any check). */
mcd_status mcd_picker_save(const mcd_picker* p, const char* path);
mcd_status mcd_picker_load(mcd_picker* p, const char* path);
/* The checks of mcd_picker_load alone, on the host (no device needed):
 * MCD_OK for a sound checkpoint, MCD_ERR_CHECKPOINT otherwise. */
mcd_status mcd_picker_check_file(const char* path);

/* Snaps picker outputs to the grid delta_i = (a + b i) / c, i = 0..K-1:
 * i = clamp(round((K - 1) y), 0, K - 1).  index: device int32[batch] (may be
 * NULL); delta: device int64[batch][2] = (num, den) (may be NULL).  c > 0. */
mcd_status mcd_grid_select(mcd_ctx* ctx, const float* y, int32_t batch, int32_t K, int64_t a, int64_t b,
                           int64_t c, int32_t* index, int64_t* delta);

/* Training targets from a sweep's ARI table (device double[n_graphs][K], K >= 2):
 * the centroid c of the thresholds whose ARI is at least
 * best - (1 - frac) |best|, 0 < frac <= 1 (1: the exact maxima only), as the
 * index round-half-down(c) (index, device int32[n_graphs], may be NULL) and as
 * c / (K - 1) (y, device float[n_graphs], may be NULL). */
mcd_status mcd_sweep_targets(mcd_ctx* ctx, const double* ari, int32_t n_graphs, int32_t K, double frac,
                             int32_t* index, float* y);

/* mcd_prune with one threshold per graph of a batch, read from device memory:
 * deltas[2k] / deltas[2k+1] (den > 0) is graph k's threshold. */
mcd_status mcd_prune_graphs(const mcd_graph* g, mcd_measure measure, const int32_t* t, int32_t n_graphs,
                            const int64_t* vbase, const int64_t* deltas, uint32_t* keep_bits,
                            int64_t* n_kept);

/* Scratch for mcd_percentile_threshold. */
mcd_status mcd_percentile_workspace_size(const mcd_graph* g, size_t* bytes);

/* Nearest-rank percentile pct_num/pct_den of the NONZERO similarities: with
 * the K nonzero values in exact ascending order, the value at 0-based index
 * ceil(pct_num K / pct_den) - 1 (at least 0), returned exactly as a reduced
 * fraction (TW: den = 1) in *host_out.
 * Synchronous.  Errors: MCD_ERR_EMPTY if every similarity is zero. */
mcd_status mcd_percentile_threshold(const mcd_graph* g, mcd_measure measure, const int32_t* t,
                                    int64_t pct_num, int64_t pct_den, void* ws, size_t ws_bytes,
                                    mcd_rational* host_out);

#ifdef __cplusplus
}
#endif
#endif /* MCD_H */
