/*
 * CPU oracle for motif-based community detection (Chen & Tsourakakis,
 * "Parallel Motif-Based Community Detection", arXiv 2412.12382).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or table with the GPU library.
 *
 * Every routine is the plain definition of what the method computes, written
 * for clarity rather than speed: sorting with qsort, bitmap marking, BFS,
 * exact integer/rational comparisons, fp64 where the value is real-valued.
 *
 * Passages followed (section / algorithm / equation / table of the paper):
 *   - Notation paragraph of Sec. 1: simple undirected graph, N(u), deg(u),
 *     t(u,v) = |N(u) n N(v)|, wedge(u,v) = |N(u) u N(v)| - |N(u) n N(v)| - 2.
 *   - Algorithm 1 (motif-based community detection): drop every edge with
 *     sim(e) < delta, return the connected components of what remains.
 *   - Table "tab:simfunctions": Tectonic t/(deg u + deg v); TW = t - wedge
 *     (Eq. "eq:tw").
 *   - Sec. 3.3 (parallel implementation): similarities are computed once on
 *     the input graph, then components of the sparsified graph.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_VERTEX -2
#define OR_ERR_EMPTY -3

/* ------------------------------------------------------------- graph */

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/* Ascending sort of k 64-bit keys.  Large arrays are cut into one run per
 * thread, each run sorted by qsort, and neighbouring runs merged pairwise
 * until one remains: the output is the same sorted array that a single qsort
 * gives, in less wall time on many cores. */
static void merge_u64(const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb, uint64_t* out) {
    int64_t i = 0, j = 0, o = 0;
    while (i < na && j < nb) out[o++] = (b[j] < a[i]) ? b[j++] : a[i++];
    while (i < na) out[o++] = a[i++];
    while (j < nb) out[o++] = b[j++];
}

static void sort_u64(uint64_t* a, int64_t k) {
    int T = 1;
#ifdef _OPENMP
    T = omp_get_max_threads();
#endif
    if (T < 2 || k < (1 << 20)) {
        qsort(a, (size_t)k, sizeof(uint64_t), cmp_u64);
        return;
    }
    int64_t* bnd = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T + 1));
    for (int i = 0; i <= T; ++i) bnd[i] = k * i / T;
#pragma omp parallel for schedule(static, 1)
    for (int i = 0; i < T; ++i) qsort(a + bnd[i], (size_t)(bnd[i + 1] - bnd[i]), sizeof(uint64_t), cmp_u64);
    uint64_t* buf = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)k);
    uint64_t *from = a, *to = buf;
    for (int w = 1; w < T; w *= 2) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < T; i += 2 * w) {
            const int i1 = (i + w < T) ? i + w : T, i2 = (i + 2 * w < T) ? i + 2 * w : T;
            merge_u64(from + bnd[i], bnd[i1] - bnd[i], from + bnd[i1], bnd[i2] - bnd[i1], to + bnd[i]);
        }
        uint64_t* x = from;
        from = to;
        to = x;
    }
    if (from != a) memcpy(a, from, sizeof(uint64_t) * (size_t)k);
    free(buf);
    free(bnd);
}

/* Simple undirected graph from raw pairs (Sec. 1 notation: undirected,
 * unweighted, no self-loops, no multi-edges).  Each pair (u,v), u != v, is the
 * edge {min,max}; self-loops are dropped; duplicates collapse.  Output: the m
 * edges as sorted (lo,hi) with lo < hi.  lo/hi must hold n_pairs entries.
 * Returns OR_ERR_VERTEX if any id lies outside [0,n). */
int or_canon(int64_t n, int64_t n_pairs, const int32_t* src, const int32_t* dst,
             int64_t* m_out, int32_t* lo, int32_t* hi) {
    if (n < 0 || n_pairs < 0) return OR_ERR_ARG;
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n_pairs > 0 ? n_pairs : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < n_pairs; ++i) {
        int64_t u = src[i], v = dst[i];
        if (u < 0 || u >= n || v < 0 || v >= n) {
            free(keys);
            return OR_ERR_VERTEX;
        }
        if (u == v) continue;
        uint64_t a = (uint64_t)(u < v ? u : v), b = (uint64_t)(u < v ? v : u);
        keys[k++] = (a << 32) | b;
    }
    sort_u64(keys, k);
    int64_t m = 0;
    for (int64_t i = 0; i < k; ++i) {
        if (i > 0 && keys[i] == keys[i - 1]) continue;
        lo[m] = (int32_t)(keys[i] >> 32);
        hi[m] = (int32_t)(keys[i] & 0xffffffffu);
        ++m;
    }
    free(keys);
    *m_out = m;
    return OR_OK;
}

/* deg(u) = |N(u)| (Sec. 1 notation). */
void or_degrees(int64_t n, int64_t m, const int32_t* lo, const int32_t* hi, int32_t* deg) {
    memset(deg, 0, sizeof(int32_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e) {
        deg[lo[e]]++;
        deg[hi[e]]++;
    }
}

typedef struct {
    int32_t nb;
    int32_t eid;
} nbr_t;

static int cmp_nbr(const void* a, const void* b) {
    int32_t x = ((const nbr_t*)a)->nb, y = ((const nbr_t*)b)->nb;
    return (x > y) - (x < y);
}

/* Symmetric adjacency: row u lists N(u) in increasing id order, each entry
 * with the index of its edge.  off has n+1 entries; adj/eid have 2m. */
void or_adjacency(int64_t n, int64_t m, const int32_t* lo, const int32_t* hi,
                  int64_t* off, int32_t* adj, int32_t* eid) {
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    memset(off, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m; ++e) {
        off[lo[e] + 1]++;
        off[hi[e] + 1]++;
    }
    for (int64_t u = 0; u < n; ++u) off[u + 1] += off[u];
    nbr_t* tmp = (nbr_t*)malloc(sizeof(nbr_t) * (size_t)(2 * m > 0 ? 2 * m : 1));
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = lo[e], b = hi[e];
        tmp[off[a] + fill[a]].nb = b;
        tmp[off[a] + fill[a]].eid = (int32_t)e;
        fill[a]++;
        tmp[off[b] + fill[b]].nb = a;
        tmp[off[b] + fill[b]].eid = (int32_t)e;
        fill[b]++;
    }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; ++u)
        qsort(tmp + off[u], (size_t)(off[u + 1] - off[u]), sizeof(nbr_t), cmp_nbr);
    for (int64_t i = 0; i < 2 * m; ++i) {
        adj[i] = tmp[i].nb;
        eid[i] = tmp[i].eid;
    }
    free(tmp);
    free(fill);
}

/* t(u,v) = |N(u) n N(v)| for every edge (Sec. 1 notation).
 * Each edge is handled by one endpoint u: u marks N(u) in a private bitmap and
 * counts how many w in N(v) are marked.  The endpoint that does the marking
 * is the one whose (deg, id) is larger, so the scanned list is the shorter
 * one; this only chooses which of the two equal counts is evaluated. */
void or_triangles(int64_t n, const int64_t* off, const int32_t* adj, const int32_t* eid,
                  int32_t* t) {
#pragma omp parallel
    {
        unsigned char* mark = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
#pragma omp for schedule(dynamic, 64)
        for (int64_t u = 0; u < n; ++u) {
            int64_t du = off[u + 1] - off[u];
            for (int64_t i = off[u]; i < off[u + 1]; ++i) mark[adj[i]] = 1;
            for (int64_t i = off[u]; i < off[u + 1]; ++i) {
                int64_t v = adj[i];
                int64_t dv = off[v + 1] - off[v];
                int v_smaller = (dv < du) || (dv == du && v < u);
                if (!v_smaller) continue;
                int32_t c = 0;
                for (int64_t j = off[v]; j < off[v + 1]; ++j) c += mark[adj[j]];
                t[eid[i]] = c;
            }
            for (int64_t i = off[u]; i < off[u + 1]; ++i) mark[adj[i]] = 0;
        }
        free(mark);
    }
}

/* kappa-clique participation for kappa = 4 (Table tab:simfunctions): the
 * number of 4-cliques containing edge {u,v} equals the number of adjacent
 * pairs {x,y} inside N(u) n N(v).  Plain definition: mark N(u) n N(v), then
 * for every marked x count the marked y > x in N(x).  off/adj/eid as built by
 * or_adjacency (symmetric CSR); k4 indexed by edge id. */
void or_k4(int64_t n, const int64_t* off, const int32_t* adj, const int32_t* eid, int32_t* k4) {
#pragma omp parallel
    {
        unsigned char* inu = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
        unsigned char* com = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
        int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t u = 0; u < n; ++u) {
            for (int64_t i = off[u]; i < off[u + 1]; ++i) inu[adj[i]] = 1;
            for (int64_t i = off[u]; i < off[u + 1]; ++i) {
                const int64_t v = adj[i];
                if (v <= u) continue;  /* each edge once, from its smaller end */
                int64_t L = 0;
                for (int64_t j = off[v]; j < off[v + 1]; ++j)
                    if (inu[adj[j]]) {
                        com[adj[j]] = 1;
                        list[L++] = adj[j];
                    }
                int64_t c = 0;
                for (int64_t a = 0; a < L; ++a) {
                    const int32_t x = list[a];
                    for (int64_t j = off[x]; j < off[x + 1]; ++j) c += (adj[j] > x && com[adj[j]]);
                }
                for (int64_t a = 0; a < L; ++a) com[list[a]] = 0;
                k4[eid[i]] = (int32_t)c;
            }
            for (int64_t i = off[u]; i < off[u + 1]; ++i) inu[adj[i]] = 0;
        }
        free(inu);
        free(com);
        free(list);
    }
}

/* Tectonic similarity t(u,v) / (deg(u) + deg(v))  (Table tab:simfunctions),
 * in fp64. */
void or_tectonic(int64_t m, const int32_t* lo, const int32_t* hi, const int32_t* t,
                 const int32_t* deg, double* w) {
    for (int64_t e = 0; e < m; ++e) w[e] = (double)t[e] / ((double)deg[lo[e]] + (double)deg[hi[e]]);
}

/* wedge(u,v) = |N(u) u N(v)| - |N(u) n N(v)| - 2 (Sec. 1 notation), with the
 * union size from inclusion-exclusion |A u B| = |A| + |B| - |A n B|. */
void or_wedges(int64_t m, const int32_t* lo, const int32_t* hi, const int32_t* t,
               const int32_t* deg, int64_t* wedge) {
    for (int64_t e = 0; e < m; ++e) {
        int64_t uni = (int64_t)deg[lo[e]] + (int64_t)deg[hi[e]] - (int64_t)t[e];
        wedge[e] = uni - (int64_t)t[e] - 2;
    }
}

/* TW(e) = t(e) - wedge(e)  (Eq. eq:tw). */
void or_tw(int64_t m, const int32_t* lo, const int32_t* hi, const int32_t* t,
           const int32_t* deg, int64_t* tw) {
    int64_t* wedge = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    or_wedges(m, lo, hi, t, deg, wedge);
    for (int64_t e = 0; e < m; ++e) tw[e] = (int64_t)t[e] - wedge[e];
    free(wedge);
}

/* Jaccard coefficient of the neighbourhoods, t / (deg u + deg v - t)
 * (Table tab:simfunctions; |N(u) u N(v)| by inclusion-exclusion), in fp64. */
void or_jaccard(int64_t m, const int32_t* lo, const int32_t* hi, const int32_t* t, const int32_t* deg,
                double* w) {
    for (int64_t e = 0; e < m; ++e)
        w[e] = (double)t[e] / ((double)deg[lo[e]] + (double)deg[hi[e]] - (double)t[e]);
}

/* Exact sign of a/b - c/d for b,d > 0: sign(a d - c b). */
static int rat_cmp(int64_t a, int64_t b, int64_t c, int64_t d) {
    __int128 l = (__int128)a * d, r = (__int128)c * b;
    return (l > r) - (l < r);
}

/* sim(e) of Table tab:simfunctions as an exact rational num : den, den > 0.
 * measure 0 Tectonic: t : (deg u + deg v);  1 TW: tw : 1 (tw = t - wedge,
 * precomputed);  2 K3 (triangles on the edge): t : 1;  3 Jaccard:
 * t : (deg u + deg v - t);  4 K4 (4-cliques on the edge): the count, passed
 * in place of t, : 1. */
static void sim_rat(int measure, int64_t t, int64_t du, int64_t dv, int64_t tw, int64_t* num, int64_t* den) {
    switch (measure) {
        case 0: *num = t; *den = du + dv; break;
        case 1: *num = tw; *den = 1; break;
        case 2:
        case 4: *num = t; *den = 1; break;
        default: *num = t; *den = du + dv - t; break;
    }
}

/* Algorithm 1, first step: edge e is removed iff sim(e) < delta, so it is kept
 * iff NOT (sim(e) < delta).  delta = num/den with den > 0 is compared exactly
 * with the rational form of sim (sim_rat). */
int or_prune(int64_t m, int measure, const int32_t* lo, const int32_t* hi, const int32_t* t,
             const int32_t* deg, int64_t num, int64_t den, unsigned char* keep, int64_t* n_kept) {
    if (den <= 0 || measure < 0 || measure > 4) return OR_ERR_ARG;
    int64_t* tw = NULL;
    if (measure == 1) {
        tw = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
        or_tw(m, lo, hi, t, deg, tw);
    }
    int64_t k = 0;
    for (int64_t e = 0; e < m; ++e) {
        int64_t sn, sd;
        sim_rat(measure, t[e], deg[lo[e]], deg[hi[e]], tw ? tw[e] : 0, &sn, &sd);
        const int below = rat_cmp(sn, sd, num, den) < 0;
        keep[e] = below ? 0 : 1;
        k += keep[e];
    }
    free(tw);
    *n_kept = k;
    return OR_OK;
}

/* Algorithm 1, second step: connected components of (V, kept edges).
 * BFS started from s = 0,1,...,n-1 whenever s is unvisited; every vertex
 * reached gets label s, which is therefore the smallest id in its component.
 * keep may be NULL (all edges).  Returns the number of components. */
int64_t or_components(int64_t n, int64_t m, const int32_t* lo, const int32_t* hi,
                      const unsigned char* keep, int32_t* label) {
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e)
        if (!keep || keep[e]) {
            off[lo[e] + 1]++;
            off[hi[e] + 1]++;
        }
    for (int64_t u = 0; u < n; ++u) off[u + 1] += off[u];
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
    int64_t* fill = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e)
        if (!keep || keep[e]) {
            adj[off[lo[e]] + fill[lo[e]]++] = hi[e];
            adj[off[hi[e]] + fill[hi[e]]++] = lo[e];
        }
    free(fill);
    for (int64_t v = 0; v < n; ++v) label[v] = -1;
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t ncc = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        ++ncc;
        int64_t qh = 0, qt = 0;
        queue[qt++] = (int32_t)s;
        label[s] = (int32_t)s;
        while (qh < qt) {
            int32_t x = queue[qh++];
            for (int64_t i = off[x]; i < off[x + 1]; ++i) {
                int32_t y = adj[i];
                if (label[y] < 0) {
                    label[y] = (int32_t)s;
                    queue[qt++] = y;
                }
            }
        }
    }
    free(queue);
    free(adj);
    free(off);
    return ncc;
}

/* ------------------------------------------------- threshold selection */

typedef struct {
    int64_t num, den;
} rat_t;

static int cmp_rat(const void* a, const void* b) {
    const rat_t* x = (const rat_t*)a;
    const rat_t* y = (const rat_t*)b;
    return rat_cmp(x->num, x->den, y->num, y->den);
}

/* Nearest-rank percentile pn/pd of the nonzero similarity values: with K of
 * them sorted ascending (exact rational order), the value at 0-based index
 * ceil(pn K / pd) - 1 (clamped to 0).  Returned as num/den (den = 1 for TW
 * and K3).
 * Returns OR_ERR_EMPTY when every value is zero. */
int or_percentile(int64_t m, int measure, const int32_t* lo, const int32_t* hi,
                  const int32_t* t, const int32_t* deg, int64_t pn, int64_t pd,
                  int64_t* out_num, int64_t* out_den) {
    if (pd <= 0 || pn < 0 || pn > pd || measure < 0 || measure > 4) return OR_ERR_ARG;
    rat_t* v = (rat_t*)malloc(sizeof(rat_t) * (size_t)(m > 0 ? m : 1));
    int64_t* tw = NULL;
    if (measure == 1) {
        tw = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
        or_tw(m, lo, hi, t, deg, tw);
    }
    int64_t K = 0;
    for (int64_t e = 0; e < m; ++e) {
        rat_t r;
        sim_rat(measure, t[e], deg[lo[e]], deg[hi[e]], tw ? tw[e] : 0, &r.num, &r.den);
        if (r.num != 0) v[K++] = r;
    }
    free(tw);
    if (K == 0) {
        free(v);
        return OR_ERR_EMPTY;
    }
    qsort(v, (size_t)K, sizeof(rat_t), cmp_rat);
    int64_t k = (pn * K + pd - 1) / pd - 1;
    if (k < 0) k = 0;
    *out_num = v[k].num;
    *out_den = v[k].den;
    free(v);
    return OR_OK;
}

/* 64-bin histogram of the Tectonic similarity on [0, 1/2): bin = floor(128 t /
 * (deg u + deg v)) by integer division (t <= min(deg) - 1 keeps it below 64). */
void or_histogram(int64_t m, const int32_t* lo, const int32_t* hi, const int32_t* t,
                  const int32_t* deg, int64_t* hist) {
    memset(hist, 0, sizeof(int64_t) * 64);
    for (int64_t e = 0; e < m; ++e) {
        int64_t D = (int64_t)deg[lo[e]] + deg[hi[e]];
        int64_t b = (128 * (int64_t)t[e]) / D;
        if (b > 63) b = 63;
        hist[b]++;
    }
}

/* -------------------------------------------------------------- ARI */

static int64_t choose2(int64_t x) { return x * (x - 1) / 2; }

/* Adjusted Rand index (Hubert & Arabie 1985) of two labelings of n items.
 * sums[0] = sum_ij C(n_ij,2), sums[1] = sum_i C(a_i,2), sums[2] = sum_j
 * C(b_j,2), sums[3] = C(n,2), exact in int64; the index is
 * (S - A B / N) / ((A + B)/2 - A B / N), and 1 when the denominator is 0. */
double or_ari(int64_t n, const int32_t* x, const int32_t* y, int64_t* sums) {
    uint64_t* k = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    uint64_t* kx = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    uint64_t* ky = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        k[i] = ((uint64_t)(uint32_t)x[i] << 32) | (uint32_t)y[i];
        kx[i] = (uint32_t)x[i];
        ky[i] = (uint32_t)y[i];
    }
    qsort(k, (size_t)n, sizeof(uint64_t), cmp_u64);
    qsort(kx, (size_t)n, sizeof(uint64_t), cmp_u64);
    qsort(ky, (size_t)n, sizeof(uint64_t), cmp_u64);
    int64_t S = 0, A = 0, B = 0;
    uint64_t* arrs[3] = {k, kx, ky};
    int64_t* acc[3] = {&S, &A, &B};
    for (int a = 0; a < 3; ++a) {
        int64_t run = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (i > 0 && arrs[a][i] != arrs[a][i - 1]) {
                *acc[a] += choose2(run);
                run = 0;
            }
            ++run;
        }
        *acc[a] += choose2(run);
    }
    free(k);
    free(kx);
    free(ky);
    int64_t N = choose2(n);
    sums[0] = S;
    sums[1] = A;
    sums[2] = B;
    sums[3] = N;
    double prod = ((double)A * (double)B) / (double)N;
    double den = 0.5 * ((double)A + (double)B) - prod;
    if (N == 0 || den == 0.0) return 1.0;
    return ((double)S - prod) / den;
}

/* ------------------------------------------- sampled checks on raw pairs */

/* For query edges (qu[k], qv[k]) computes, straight from the raw pairs,
 * whether {qu,qv} is an edge of the simple graph, deg(qu), deg(qv) and
 * t(qu,qv) = |N(qu) n N(qv)| (Sec. 1 notation).  Neighbour lists of the query
 * vertices are gathered by one scan over the pairs, sorted and deduplicated.
 * For large graphs where the full oracle would be too slow. */
int or_query_edges(int64_t n, int64_t n_pairs, const int32_t* src, const int32_t* dst,
                   int64_t K, const int32_t* qu, const int32_t* qv, int32_t* is_edge,
                   int32_t* deg_u, int32_t* deg_v, int32_t* t) {
    /* slot[v] = index of v among the distinct query vertices, or -1 */
    int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) slot[v] = -1;
    int64_t nq = 0;
    for (int64_t k = 0; k < K; ++k) {
        if (qu[k] < 0 || qu[k] >= n || qv[k] < 0 || qv[k] >= n) {
            free(slot);
            return OR_ERR_VERTEX;
        }
        if (slot[qu[k]] < 0) slot[qu[k]] = (int32_t)nq++;
        if (slot[qv[k]] < 0) slot[qv[k]] = (int32_t)nq++;
    }
    int64_t* cnt = (int64_t*)calloc((size_t)nq + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n_pairs; ++i) {
        int32_t a = src[i], b = dst[i];
        if (a == b) continue;
        if (slot[a] >= 0) cnt[slot[a] + 1]++;
        if (slot[b] >= 0) cnt[slot[b] + 1]++;
    }
    for (int64_t s = 0; s < nq; ++s) cnt[s + 1] += cnt[s];
    int32_t* lst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt[nq] > 0 ? cnt[nq] : 1));
    int64_t* fill = (int64_t*)calloc((size_t)nq + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n_pairs; ++i) {
        int32_t a = src[i], b = dst[i];
        if (a == b) continue;
        if (slot[a] >= 0) lst[cnt[slot[a]] + fill[slot[a]]++] = b;
        if (slot[b] >= 0) lst[cnt[slot[b]] + fill[slot[b]]++] = a;
    }
    free(fill);
    /* sort + dedup each list in place; len[s] = distinct neighbours */
    int64_t* len = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
    for (int64_t s = 0; s < nq; ++s) {
        int32_t* L = lst + cnt[s];
        int64_t l = cnt[s + 1] - cnt[s];
        uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(l > 0 ? l : 1));
        for (int64_t i = 0; i < l; ++i) tmp[i] = (uint32_t)L[i];
        qsort(tmp, (size_t)l, sizeof(uint64_t), cmp_u64);
        int64_t d = 0;
        for (int64_t i = 0; i < l; ++i)
            if (i == 0 || tmp[i] != tmp[i - 1]) L[d++] = (int32_t)tmp[i];
        len[s] = d;
        free(tmp);
    }
    for (int64_t k = 0; k < K; ++k) {
        int32_t su = slot[qu[k]], sv = slot[qv[k]];
        const int32_t* A = lst + cnt[su];
        const int32_t* B = lst + cnt[sv];
        int64_t la = len[su], lb = len[sv];
        deg_u[k] = (int32_t)la;
        deg_v[k] = (int32_t)lb;
        int32_t common = 0, adjacent = 0;
        int64_t i = 0, j = 0;
        while (i < la && j < lb) {
            if (A[i] < B[j]) ++i;
            else if (A[i] > B[j]) ++j;
            else {
                ++common;
                ++i;
                ++j;
            }
        }
        for (int64_t x = 0; x < la; ++x)
            if (A[x] == qv[k]) adjacent = 1;
        is_edge[k] = adjacent;
        t[k] = common;
    }
    free(len);
    free(lst);
    free(cnt);
    free(slot);
    return OR_OK;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
