// Lock-free union-find over rank-numbered vertices, shared by the components
// step, the fused prune + components pass and the threshold sweep.
//
// Parents only ever point to higher ranks (a root hooks under the higher-ranked
// root by compare-and-swap), so chains are acyclic and every walk ends.  Finds
// halve paths (pointer jumping to the grandparent); parent reads and halving
// writes are device-scope atomics so that no wave spins on a stale per-CU
// cache line.  A halving store only ever replaces a parent by one of its own
// ancestors, so concurrent finds never lose a link.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcd {

__device__ __forceinline__ int32_t uf_load(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void uf_store(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t uf_find(int32_t* parent, int32_t x) {
    for (;;) {
        const int32_t p = uf_load(&parent[x]);
        if (p == x) return x;
        const int32_t gp = uf_load(&parent[p]);
        if (gp != p) uf_store(&parent[x], gp);
        x = gp;
    }
}

// Unite the sets of a and b.  The two walks to the roots advance in lockstep
// (their loads are issued together) with path halving, and stop as soon as
// the two sides meet: equal parents, or one side's parent is the other
// vertex.  Every parent read is an ancestor of the vertex read, so a meeting
// proves one set; an edge whose endpoints already share a parent (most edges
// of a dense core once it has formed) costs one round trip.  Two distinct
// roots are joined by hooking the lower-ranked under the higher-ranked by
// compare-and-swap; a lost race re-reads both sides.  (Measured against two
// finds in turn: 1.3x faster on the kept edges of a pruned R-MAT, 4.5x on all
// edges under a keep mask, on par for the threshold sweep's level unions.)
__device__ __forceinline__ void uf_unite(int32_t* parent, int32_t a, int32_t b) {
    int32_t pa = uf_load(&parent[a]), pb = uf_load(&parent[b]);
    for (;;) {
        if (a == b || pa == pb || pa == b || pb == a) return;
        const bool ra = pa == a, rb = pb == b;
        if (ra && rb) {
            const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
            int32_t expected = lo;
            if (__hip_atomic_compare_exchange_strong(&parent[lo], &expected, hi, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                return;
            pa = uf_load(&parent[a]);
            pb = uf_load(&parent[b]);
            continue;
        }
        // one halving step on each side that is not at a root
        const int32_t ga = ra ? a : uf_load(&parent[pa]);
        const int32_t gb = rb ? b : uf_load(&parent[pb]);
        if (!ra) {
            if (ga != pa) {
                uf_store(&parent[a], ga);
                a = ga;
                pa = uf_load(&parent[ga]);
            } else {  // pa is a root
                a = pa;
            }
        }
        if (!rb) {
            if (gb != pb) {
                uf_store(&parent[b], gb);
                b = gb;
                pb = uf_load(&parent[gb]);
            } else {
                b = pb;
            }
        }
    }
}

}  // namespace mcd
