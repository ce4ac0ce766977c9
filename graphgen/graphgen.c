/*
 * Seeded synthetic input graphs for the motif-based community-detection path.
 *
 * This module only draws random graphs.  It holds none of the method's
 * arithmetic (no triangle, weight, threshold or component logic), so both the
 * CPU oracle and the GPU library may read what it produces.
 *
 * Every random number is a Philox-4x32-10 output (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11) keyed by the seed and
 * indexed by a counter that names the item being drawn, so the bytes produced
 * do not depend on the number of threads.
 *
 * Generators:
 *   R-MAT (Chakrabarti, Zhan, Faloutsos, SDM'04): recursive quadrant choice per
 *     directed sample, followed by a seeded vertex permutation.
 *   Planted-partition SBM: Bernoulli(p_in) inside blocks, Bernoulli(p_out)
 *     across, either per pair (small n) or by geometric skipping (large n).
 *   Degree-corrected SBM: power-law expected degrees and community sizes,
 *     Poisson edge counts, endpoints proportional to the degree parameter.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_TAG_RMAT 0x524d4154u   /* "RMAT" */
#define GG_TAG_PERM 0x5045524du   /* "PERM" */
#define GG_TAG_SBM 0x53424d30u    /* "SBM0" */
#define GG_TAG_SKIP 0x534b4950u   /* "SKIP" */
#define GG_TAG_DCSBM 0x44435342u  /* "DCSB" */

/* ---------------------------------------------------------------- Philox */

static inline void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

/* Philox-4x32 with 10 rounds; the key is bumped by the Weyl constants
 * between rounds. */
void gg_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

static inline void draw4(uint64_t seed, uint32_t tag, uint64_t idx, uint32_t sub, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), sub, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    gg_philox4x32_10(ctr, key, out);
}

/* Uniform double in the open interval (0,1) from one 32-bit draw. */
static inline double u01_open(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

/* Uniform double in [0,1) with 53 bits from two 32-bit draws. */
static inline double u01_53(uint32_t hi, uint32_t lo) {
    uint64_t v = ((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6);
    return (double)v * (1.0 / 9007199254740992.0);
}

/* Probability p in [0,1] as a 32-bit cut-point: an event fires iff draw < cut. */
static inline uint64_t prob_cut(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 4294967296ull;
    return (uint64_t)floor(p * 4294967296.0);
}

/* Generic draw exported for parameter sampling in the Python layer. */
void gg_draw4(uint64_t seed, uint32_t tag, uint64_t idx, uint32_t sub, uint32_t* out) {
    draw4(seed, tag, idx, sub, out);
}

/* ------------------------------------------------------ vertex permutation */

/* Balanced Feistel network on 2*h bits, 4 rounds, round function from Philox.
 * It is a bijection of [0, 2^(2h)); cycle-walking restricts it to [0, 2^s). */
static inline uint64_t feistel(uint64_t x, int h, uint64_t seed) {
    uint64_t mask = (h >= 32) ? 0xffffffffull : ((1ull << h) - 1);
    uint64_t L = (x >> h) & mask, R = x & mask;
    for (uint32_t r = 0; r < 4; ++r) {
        uint32_t o[4];
        draw4(seed, GG_TAG_PERM, R, r, o);
        uint64_t F = ((uint64_t)o[1] << 32 | o[0]) & mask;
        uint64_t nL = R, nR = L ^ F;
        L = nL;
        R = nR;
    }
    return (L << h) | R;
}

/* perm[v] for v in [0, 2^scale): a seeded bijection of [0, 2^scale). */
void gg_perm_table(int scale, uint64_t seed, int32_t* perm) {
    int h = (scale + 1) / 2;
    uint64_t n = 1ull << scale;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < (int64_t)n; ++v) {
        uint64_t y = feistel((uint64_t)v, h, seed);
        while (y >= n) y = feistel(y, h, seed);
        perm[v] = (int32_t)y;
    }
}

/* ------------------------------------------------------------------ R-MAT */

/* Directed R-MAT samples i in [0, n_pairs): at each of `scale` levels a 32-bit
 * draw r picks quadrant (0,0) if r < A, (0,1) if r < A+B, (1,0) if r < A+B+C,
 * else (1,1), with cut-points A = floor(a 2^32) etc.  No per-level noise.  If
 * perm is non-NULL both endpoints are mapped through it. */
int gg_rmat(int scale, int64_t n_pairs, double a, double b, double c, uint64_t seed,
            const int32_t* perm, int32_t* src, int32_t* dst) {
    if (scale < 1 || scale > 31 || n_pairs < 0) return -1;
    uint64_t cA = prob_cut(a), cAB = prob_cut(a + b), cABC = prob_cut(a + b + c);
    int words = (scale + 3) / 4;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_pairs; ++i) {
        uint32_t u = 0, v = 0;
        int lvl = 0;
        for (int w = 0; w < words; ++w) {
            uint32_t o[4];
            draw4(seed, GG_TAG_RMAT, (uint64_t)i, (uint32_t)w, o);
            for (int j = 0; j < 4 && lvl < scale; ++j, ++lvl) {
                uint64_t r = o[j];
                uint32_t rb, cb;
                if (r < cA) {
                    rb = 0; cb = 0;
                } else if (r < cAB) {
                    rb = 0; cb = 1;
                } else if (r < cABC) {
                    rb = 1; cb = 0;
                } else {
                    rb = 1; cb = 1;
                }
                u = (u << 1) | rb;
                v = (v << 1) | cb;
            }
        }
        if (perm) {
            u = (uint32_t)perm[u];
            v = (uint32_t)perm[v];
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
    return 0;
}

/* ---------------------------------------------------- planted partition */

/* Per-pair Bernoulli SBM over all i<j: pair (i,j) is drawn with counter i*n+j
 * and kept iff the draw is below the cut-point of p_in (same block) or p_out.
 * block_of[v] is the planted block.  Returns the number of edges written, or
 * the number needed (negative) if cap is too small; src/dst may be NULL to
 * count only. */
int64_t gg_sbm_pairs(int32_t n, const int32_t* block_of, double p_in, double p_out, uint64_t seed,
                     int32_t* src, int32_t* dst, int64_t cap) {
    uint64_t cin = prob_cut(p_in), cout = prob_cut(p_out);
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            uint32_t o[4];
            draw4(seed, GG_TAG_SBM, (uint64_t)(i * (int64_t)n + j), 0, o);
            uint64_t cut = (block_of[i] == block_of[j]) ? cin : cout;
            if ((uint64_t)o[0] < cut) {
                if (src && cnt < cap) {
                    src[cnt] = (int32_t)i;
                    dst[cnt] = (int32_t)j;
                }
                ++cnt;
            }
        }
    }
    if (src && cnt > cap) return -cnt;
    return cnt;
}

/* Number of candidate pairs of block pair (a,b), a<=b. */
static inline int64_t bp_count(const int64_t* bs, int a, int b) {
    int64_t sa = bs[a + 1] - bs[a], sb = bs[b + 1] - bs[b];
    return (a == b) ? sa * (sa - 1) / 2 : sa * sb;
}

/* Map a linear index to the pair (i,j) of block pair (a,b). */
static inline void bp_pair(const int64_t* bs, int a, int b, int64_t idx, int64_t* i, int64_t* j) {
    if (a != b) {
        int64_t sb = bs[b + 1] - bs[b];
        *i = bs[a] + idx / sb;
        *j = bs[b] + idx % sb;
        return;
    }
    /* Row r of the strict upper triangle holds s-1-r pairs. */
    int64_t s = bs[a + 1] - bs[a];
    double fs = (double)s;
    int64_t r = (int64_t)floor(((2.0 * fs - 1.0) - sqrt((2.0 * fs - 1.0) * (2.0 * fs - 1.0) - 8.0 * (double)idx)) / 2.0);
    if (r < 0) r = 0;
    while (r > 0 && r * (2 * s - r - 1) / 2 > idx) --r;
    while ((r + 1) * (2 * s - r - 2) / 2 <= idx) ++r;
    int64_t before = r * (2 * s - r - 1) / 2;
    *i = bs[a] + r;
    *j = bs[a] + r + 1 + (idx - before);
}

/* Enumerate the Bernoulli(p) subset of a block pair's candidates by geometric
 * skipping (Batagelj & Brandes 2005); draw d of block pair `bp` uses counter
 * (bp, d).  If out is NULL only counts. */
static int64_t bp_sample(const int64_t* bs, int a, int b, int bp, double p, uint64_t seed,
                         int32_t* src, int32_t* dst) {
    int64_t total = bp_count(bs, a, b);
    if (total <= 0 || !(p > 0.0)) return 0;
    int64_t cnt = 0;
    if (p >= 1.0) {
        for (int64_t idx = 0; idx < total; ++idx) {
            if (src) {
                int64_t i, j;
                bp_pair(bs, a, b, idx, &i, &j);
                src[cnt] = (int32_t)i;
                dst[cnt] = (int32_t)j;
            }
            ++cnt;
        }
        return cnt;
    }
    double lq = log1p(-p);
    int64_t pos = -1;
    uint64_t d = 0;
    for (;;) {
        uint32_t o[4];
        draw4(seed, GG_TAG_SKIP, (uint64_t)bp, (uint32_t)d, o);
        ++d;
        double skip = floor(log(u01_open(o[0])) / lq);
        if (skip > (double)total) break;
        pos += 1 + (int64_t)skip;
        if (pos >= total) break;
        if (src) {
            int64_t i, j;
            bp_pair(bs, a, b, pos, &i, &j);
            src[cnt] = (int32_t)i;
            dst[cnt] = (int32_t)j;
        }
        ++cnt;
    }
    return cnt;
}

/* SBM with contiguous blocks [bs[k], bs[k+1]) by geometric skipping, p_in inside
 * a block and p_out across.  Two phases: counts per block pair, then fill at
 * prefix offsets, so the output order is independent of the thread count.
 * Returns the edge count, or -needed if cap is too small (src NULL: count). */
int64_t gg_sbm_skip(int32_t k, const int64_t* bs, double p_in, double p_out, uint64_t seed,
                    int32_t* src, int32_t* dst, int64_t cap) {
    int64_t npairs = (int64_t)k * (k + 1) / 2;
    int64_t* cnt = (int64_t*)calloc((size_t)npairs + 1, sizeof(int64_t));
    int* pa = (int*)malloc(sizeof(int) * (size_t)npairs);
    int* pb = (int*)malloc(sizeof(int) * (size_t)npairs);
    int64_t q = 0;
    for (int a = 0; a < k; ++a)
        for (int b = a; b < k; ++b) {
            pa[q] = a;
            pb[q] = b;
            ++q;
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t x = 0; x < npairs; ++x) {
        double p = (pa[x] == pb[x]) ? p_in : p_out;
        cnt[x + 1] = bp_sample(bs, pa[x], pb[x], (int)x, p, seed, NULL, NULL);
    }
    for (int64_t x = 0; x < npairs; ++x) cnt[x + 1] += cnt[x];
    int64_t total = cnt[npairs];
    if (src && total <= cap) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t x = 0; x < npairs; ++x) {
            double p = (pa[x] == pb[x]) ? p_in : p_out;
            bp_sample(bs, pa[x], pb[x], (int)x, p, seed, src + cnt[x], dst + cnt[x]);
        }
    }
    free(cnt);
    free(pa);
    free(pb);
    if (src && total > cap) return -total;
    return total;
}

/* ------------------------------------------------- degree-corrected SBM */

/* Smallest index i with cum[i] > x, over cum[0..len). */
static inline int64_t upper_idx(const double* cum, int64_t len, double x) {
    int64_t lo = 0, hi = len - 1;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cum[mid] > x) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

/* Poisson(lambda) draw: inversion for means up to 64 (exp(-lambda) stays far
 * from underflow there), rounded normal approximation above. */
static int64_t poisson_draw(double lam, uint64_t seed, uint64_t idx) {
    uint32_t o[4];
    draw4(seed, GG_TAG_DCSBM, idx, 0xfffffff0u, o);
    if (lam <= 0) return 0;
    if (lam > 64.0) {
        double u1 = u01_open(o[0]), u2 = u01_open(o[1]);
        double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        double v = floor(lam + sqrt(lam) * z + 0.5);
        return v < 0 ? 0 : (int64_t)v;
    }
    double u = u01_53(o[0], o[1]);
    double pk = exp(-lam), cdf = pk;
    int64_t kk = 0;
    while (u > cdf && kk < 100000000) {
        ++kk;
        pk *= lam / (double)kk;
        cdf += pk;
    }
    return kk;
}

/* Degree-corrected SBM.
 *   theta[v]: expected-degree parameters (caller draws them);
 *   comm[v]: community of v, community c holds the vertices listed in
 *            members[cstart[c] .. cstart[c+1]).
 * Community c gets Poisson((1-mu) vol_c / 2) internal edges with endpoints
 * drawn proportional to theta inside c; the graph gets Poisson(mu vol / 2)
 * external edges with endpoints proportional to theta over all vertices,
 * re-drawing pairs that fall in one community.  Raw pairs may repeat or be
 * self-loops; the consumer simplifies.  Returns the number of pairs, or
 * -needed if cap is too small (src NULL: count). */
int64_t gg_dcsbm(int32_t n, const double* theta, int32_t ncomm, const int64_t* cstart,
                 const int32_t* members, const int32_t* comm, double mu, uint64_t seed,
                 int32_t* src, int32_t* dst, int64_t cap) {
    int64_t* ecount = (int64_t*)calloc((size_t)ncomm + 2, sizeof(int64_t));
    double vol = 0;
    for (int32_t v = 0; v < n; ++v) vol += theta[v];
    for (int32_t c = 0; c < ncomm; ++c) {
        double vc = 0;
        for (int64_t x = cstart[c]; x < cstart[c + 1]; ++x) vc += theta[members[x]];
        ecount[c + 1] = poisson_draw((1.0 - mu) * vc / 2.0, seed, (uint64_t)c);
    }
    int64_t ext = poisson_draw(mu * vol / 2.0, seed, (uint64_t)ncomm);
    for (int32_t c = 0; c < ncomm; ++c) ecount[c + 1] += ecount[c];
    int64_t total = ecount[ncomm] + ext;
    if (!src || total > cap) {
        free(ecount);
        return (src && total > cap) ? -total : total;
    }
    /* internal edges, one stream per community */
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t c = 0; c < ncomm; ++c) {
        int64_t s = cstart[c + 1] - cstart[c];
        if (s <= 0) continue;
        double* cum = (double*)malloc(sizeof(double) * (size_t)s);
        double acc = 0;
        for (int64_t x = 0; x < s; ++x) {
            acc += theta[members[cstart[c] + x]];
            cum[x] = acc;
        }
        int64_t base = ecount[c];
        int64_t ne = ecount[c + 1] - ecount[c];
        for (int64_t e = 0; e < ne; ++e) {
            uint32_t o[4];
            draw4(seed ^ 0x1111111111111111ull, GG_TAG_DCSBM, (uint64_t)c, (uint32_t)e, o);
            double x1 = u01_53(o[0], o[1]) * acc, x2 = u01_53(o[2], o[3]) * acc;
            src[base + e] = members[cstart[c] + upper_idx(cum, s, x1)];
            dst[base + e] = members[cstart[c] + upper_idx(cum, s, x2)];
        }
        free(cum);
    }
    /* external edges over the whole vertex set */
    double* gcum = (double*)malloc(sizeof(double) * (size_t)n);
    double acc = 0;
    for (int32_t v = 0; v < n; ++v) {
        acc += theta[v];
        gcum[v] = acc;
    }
    int64_t base = ecount[ncomm];
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ext; ++e) {
        int32_t a = 0, b = 0;
        for (uint32_t tries = 0; tries < 1000; ++tries) {
            uint32_t o[4];
            draw4(seed ^ 0x2222222222222222ull, GG_TAG_DCSBM, (uint64_t)e, tries, o);
            double x1 = u01_53(o[0], o[1]) * acc, x2 = u01_53(o[2], o[3]) * acc;
            a = (int32_t)upper_idx(gcum, n, x1);
            b = (int32_t)upper_idx(gcum, n, x2);
            if (comm[a] != comm[b]) break;
        }
        src[base + e] = a;
        dst[base + e] = b;
    }
    free(gcum);
    free(ecount);
    return total;
}

/* Fill out[i] = uniform (0,1) double of counter (idx0 + i) under (seed, tag). */
void gg_uniform(uint64_t seed, uint32_t tag, uint64_t idx0, int64_t count, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint32_t o[4];
        draw4(seed, tag, idx0 + (uint64_t)i, 0x55u, o);
        /* 53-bit uniform shifted by half an ulp so it lies in (0,1). */
        out[i] = u01_53(o[0], o[1]) + (0.5 / 9007199254740992.0);
    }
}
