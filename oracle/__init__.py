"""CPU oracle for motif-based community detection (arXiv 2412.12382).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links
or runs anything here, and nothing here imports the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, gcc -O2 -fopenmp); this module
marshals numpy arrays.  See the C file's header for the passages followed.
Edges are reported in canonical order: sorted (lo, hi), lo < hi.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None

TECTONIC, TW, K3, JACCARD, K4 = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.or_canon.argtypes = [I64, I64, P, P, P, P, P]
        L.or_degrees.argtypes = [I64, I64, P, P, P]
        L.or_adjacency.argtypes = [I64, I64, P, P, P, P, P]
        L.or_triangles.argtypes = [I64, P, P, P, P]
        L.or_k4.argtypes = [I64, P, P, P, P]
        L.or_tectonic.argtypes = [I64, P, P, P, P, P]
        L.or_jaccard.argtypes = [I64, P, P, P, P, P]
        L.or_wedges.argtypes = [I64, P, P, P, P, P]
        L.or_tw.argtypes = [I64, P, P, P, P, P]
        L.or_prune.argtypes = [I64, ctypes.c_int, P, P, P, P, I64, I64, P, P]
        L.or_components.argtypes = [I64, I64, P, P, P, P]
        L.or_components.restype = I64
        L.or_percentile.argtypes = [I64, ctypes.c_int, P, P, P, P, I64, I64, P, P]
        L.or_histogram.argtypes = [I64, P, P, P, P, P]
        L.or_ari.argtypes = [I64, P, P, P]
        L.or_ari.restype = ctypes.c_double
        L.or_query_edges.argtypes = [I64, I64, P, P, I64, P, P, P, P, P, P]
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return lib().or_num_threads()


class OracleError(RuntimeError):
    pass


def canon(n: int, src, dst):
    """Sorted unique (lo, hi) edges of the simple graph on the raw pairs."""
    src, dst = _c(src, np.int32), _c(dst, np.int32)
    P = len(src)
    lo = np.empty(max(P, 1), np.int32)
    hi = np.empty(max(P, 1), np.int32)
    m = ctypes.c_int64(0)
    rc = lib().or_canon(n, P, _p(src), _p(dst), ctypes.byref(m), _p(lo), _p(hi))
    if rc == -2:
        raise OracleError("vertex id out of range")
    if rc != 0:
        raise OracleError(f"or_canon failed ({rc})")
    # views of the full-length buffers: no second copy of a billion-edge list
    return lo[:m.value], hi[:m.value]


def degrees(n: int, lo, hi):
    deg = np.empty(max(n, 1), np.int32)
    lib().or_degrees(n, len(lo), _p(lo), _p(hi), _p(deg))
    return deg[:n]


def adjacency(n: int, lo, hi):
    m = len(lo)
    off = np.empty(n + 1, np.int64)
    adj = np.empty(max(2 * m, 1), np.int32)
    eid = np.empty(max(2 * m, 1), np.int32)
    lib().or_adjacency(n, m, _p(lo), _p(hi), _p(off), _p(adj), _p(eid))
    return off, adj[:2 * m], eid[:2 * m]


def triangles(n: int, lo, hi):
    """t(e) = |N(lo) n N(hi)| per canonical edge."""
    off, adj, eid = adjacency(n, lo, hi)
    t = np.zeros(max(len(lo), 1), np.int32)
    lib().or_triangles(n, _p(off), _p(adj), _p(eid), _p(t))
    return t[:len(lo)]


def k4(n: int, lo, hi):
    """Number of 4-cliques containing each canonical edge."""
    off, adj, eid = adjacency(n, lo, hi)
    c = np.zeros(max(len(lo), 1), np.int32)
    lib().or_k4(n, _p(off), _p(adj), _p(eid), _p(c))
    return c[:len(lo)]


def tectonic(lo, hi, t, deg):
    w = np.empty(max(len(lo), 1), np.float64)
    lib().or_tectonic(len(lo), _p(lo), _p(hi), _p(t), _p(deg), _p(w))
    return w[:len(lo)]


def jaccard(lo, hi, t, deg):
    w = np.empty(max(len(lo), 1), np.float64)
    lib().or_jaccard(len(lo), _p(lo), _p(hi), _p(t), _p(deg), _p(w))
    return w[:len(lo)]


def wedges(lo, hi, t, deg):
    w = np.empty(max(len(lo), 1), np.int64)
    lib().or_wedges(len(lo), _p(lo), _p(hi), _p(t), _p(deg), _p(w))
    return w[:len(lo)]


def tw(lo, hi, t, deg):
    w = np.empty(max(len(lo), 1), np.int64)
    lib().or_tw(len(lo), _p(lo), _p(hi), _p(t), _p(deg), _p(w))
    return w[:len(lo)]


def prune(measure: int, lo, hi, t, deg, num: int, den: int):
    """keep[e] = NOT (sim(e) < num/den)  (Algorithm 1), as uint8."""
    keep = np.empty(max(len(lo), 1), np.uint8)
    k = ctypes.c_int64(0)
    rc = lib().or_prune(len(lo), measure, _p(lo), _p(hi), _p(t), _p(deg), num, den, _p(keep),
                        ctypes.byref(k))
    if rc != 0:
        raise OracleError(f"or_prune failed ({rc})")
    return keep[:len(lo)]


def components(n: int, lo, hi, keep=None):
    """Min-vertex labels of the components of (V, kept edges) and their count."""
    label = np.empty(max(n, 1), np.int32)
    kp = None if keep is None else _c(keep, np.uint8)
    ncc = lib().or_components(n, len(lo), _p(lo), _p(hi), _p(kp), _p(label))
    return label[:n], int(ncc)


def percentile(measure: int, lo, hi, t, deg, pn: int, pd: int):
    num, den = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib().or_percentile(len(lo), measure, _p(lo), _p(hi), _p(t), _p(deg), pn, pd,
                             ctypes.byref(num), ctypes.byref(den))
    if rc != 0:
        raise OracleError(f"or_percentile failed ({rc})")
    return num.value, den.value


def histogram(lo, hi, t, deg):
    h = np.zeros(64, np.int64)
    lib().or_histogram(len(lo), _p(lo), _p(hi), _p(t), _p(deg), _p(h))
    return h


def ari(x, y):
    """(ARI, [S, A, B, N]) of two labelings."""
    x, y = _c(x, np.int32), _c(y, np.int32)
    sums = np.zeros(4, np.int64)
    v = lib().or_ari(len(x), _p(x), _p(y), _p(sums))
    return v, sums


def query_edges(n: int, src, dst, qu, qv):
    """From raw pairs: (is_edge, deg_u, deg_v, t) for each query pair."""
    src, dst = _c(src, np.int32), _c(dst, np.int32)
    qu, qv = _c(qu, np.int32), _c(qv, np.int32)
    K = len(qu)
    out = [np.zeros(max(K, 1), np.int32) for _ in range(4)]
    rc = lib().or_query_edges(n, len(src), _p(src), _p(dst), K, _p(qu), _p(qv),
                              *[_p(a) for a in out])
    if rc != 0:
        raise OracleError(f"or_query_edges failed ({rc})")
    return tuple(a[:K] for a in out)


def run(n: int, src, dst, measure: int, num: int, den: int, timings: dict | None = None):
    """Algorithm 1 end to end on raw pairs; returns a dict of every product."""
    tm = {} if timings is None else timings
    t0 = time.perf_counter()
    lo, hi = canon(n, src, dst)
    deg = degrees(n, lo, hi)
    t1 = time.perf_counter()
    t = triangles(n, lo, hi)
    t2 = time.perf_counter()
    keep = prune(measure, lo, hi, t, deg, num, den)
    w = {TECTONIC: lambda: tectonic(lo, hi, t, deg), TW: lambda: tw(lo, hi, t, deg),
         K3: lambda: t.astype(np.int64), JACCARD: lambda: jaccard(lo, hi, t, deg),
         K4: lambda: t.astype(np.int64)}[measure]()
    t3 = time.perf_counter()
    labels, ncc = components(n, lo, hi, keep)
    t4 = time.perf_counter()
    tm.update(canon=t1 - t0, triangles=t2 - t1, weight_prune=t3 - t2, components=t4 - t3)
    return dict(lo=lo, hi=hi, deg=deg, t=t, w=w, keep=keep, labels=labels, ncc=ncc)


def sweep(n: int, lo, hi, t, deg, measure: int, deltas, truth=None, vbase=None, modularity=False, workers=1):
    """Algorithm 1 at every threshold of `deltas`, one graph or a batch of
    disjoint graphs (graph k owns ids [vbase[k], vbase[k+1])).

    Returns (stats[G][K][9], ari[G][K] or None, labels[K][n]) with the fields
    m_kept, n_components, largest_component, pairs_cluster (A), pairs_class
    (B), pairs_both (S), pairs_total (N), intra_edges, volume_sq; ARI from
    or_ari on each graph.  With modularity=True a fourth item, modularity
    [G][K]: Q = intra / m - volume_sq / (4 m^2) of each partition on the input
    graph (the modularity definition of Sec. 2 summed per community), where
    intra counts input edges inside one component and volume_sq sums the
    squared degree totals of the components.  workers > 1 evaluates the
    thresholds' prune and components in that many threads at once (each
    threshold on its own, as with one worker)."""
    if vbase is None:
        vbase = np.array([0, n], np.int64)
    vbase = np.asarray(vbase, np.int64)
    G, K = len(vbase) - 1, len(deltas)
    stats = np.zeros((G, K, 9), np.int64)
    ari_out = np.zeros((G, K)) if truth is not None else None
    q_out = np.zeros((G, K)) if modularity else None
    labels_all = np.zeros((K, n), np.int32)
    egraph = np.searchsorted(vbase, lo, side="right") - 1
    m_graph = np.bincount(egraph, minlength=G).astype(np.int64)
    def one(i):
        num, den = deltas[i]
        keep = prune(measure, lo, hi, t, deg, num, den)
        labels_all[i], _ = components(n, lo, hi, keep)
        return keep

    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            keeps = list(ex.map(one, range(K)))
    else:
        keeps = None
    for i in range(K):
        keep = keeps[i] if keeps is not None else one(i)
        labels = labels_all[i]
        kept_per_graph = np.bincount(egraph, weights=keep, minlength=G).astype(np.int64)
        if modularity:
            same = (labels[lo] == labels[hi]).astype(np.int64)
            intra = np.bincount(egraph, weights=same, minlength=G).astype(np.int64)
            vol = np.zeros(n, np.int64)
            np.add.at(vol, labels, deg.astype(np.int64))
        for gk in range(G):
            a, b = vbase[gk], vbase[gk + 1]
            lab = labels[a:b]
            nv = b - a
            roots = np.count_nonzero(lab == np.arange(a, b))
            sizes = np.bincount(lab - a, minlength=max(nv, 1)) if nv else np.zeros(1, np.int64)
            row = [int(kept_per_graph[gk]), roots, int(sizes.max()) if nv else 0]
            if truth is not None and nv:
                v, sums = ari(lab, truth[a:b])
                row += [int(sums[1]), int(sums[2]), int(sums[0]), int(sums[3])]
                ari_out[gk, i] = v
            else:
                A = int((sizes * (sizes - 1) // 2).sum()) if nv else 0
                row += [A, 0, 0, nv * (nv - 1) // 2]
                if truth is not None:
                    ari_out[gk, i] = 1.0
            if modularity:
                vsq = int(sum(int(x) * int(x) for x in vol[a:b] if x))
                mg = int(m_graph[gk])
                row += [int(intra[gk]), vsq]
                q_out[gk, i] = 0.0 if mg == 0 else float(intra[gk]) / float(mg) - float(vsq) / (4.0 * mg * mg)
            else:
                row += [0, 0]
            stats[gk, i] = row
    if modularity:
        return stats, ari_out, labels_all, q_out
    return stats, ari_out, labels_all


def rule_of_thumb(stats, deltas, vbase, modularity=None, jump=(1, 10)):
    """The threshold rule of thumb of Sec. 4.4 per graph, in this reading:
    with the thresholds in increasing exact order (ties in the given order),
    take the largest increase of the largest component between consecutive
    thresholds, the first maximum met walking downwards; if it is at least
    jump[0]/jump[1] of the graph's vertices, pick the threshold just above it,
    else the threshold of maximum modularity (the highest among equal maxima),
    else (no modularity) the highest threshold.  Returns caller slot indices."""
    from fractions import Fraction
    K = len(deltas)
    order = sorted(range(K), key=lambda k: (Fraction(int(deltas[k][0]), int(deltas[k][1])), k))
    vbase = np.asarray(vbase, np.int64)
    out = []
    for g in range(stats.shape[0]):
        nv = int(vbase[g + 1] - vbase[g])
        largest = [int(stats[g, order[i], 2]) for i in range(K)]
        best, at = 0, -1
        for i in range(K - 2, -1, -1):
            d = largest[i] - largest[i + 1]
            if d > best:
                best, at = d, i
        pick = K - 1
        if at >= 0 and best * jump[1] >= jump[0] * nv:
            pick = at + 1
        elif modularity is not None:
            bq = modularity[g, order[K - 1]]
            for i in range(K - 2, -1, -1):
                if modularity[g, order[i]] > bq:
                    bq, pick = modularity[g, order[i]], i
        out.append(order[pick])
    return np.array(out, np.int64)


def precision_recall_f1(labels, truth):
    """Evaluation of Sec. 4 (Setup): each output community S (same label) is
    matched to the planted class C of largest Jaccard overlap |C n S| / |C u S|
    (compared exactly; ties to the smaller class id); p = |C n S| / |S|,
    r = |C n S| / |C|; precision, recall and F1 = 2 p r / (p + r) are averaged
    over the communities weighted by |S|.  Returns (precision, recall, F1)."""
    labels = np.asarray(labels, np.int64)
    truth = np.asarray(truth, np.int64)
    n = len(labels)
    if n == 0:
        return 0.0, 0.0, 0.0
    T = int(truth.max()) + 1
    cells, x = np.unique(labels * T + truth, return_counts=True)
    lab, cls = cells // T, cells % T
    lsize = dict(zip(*np.unique(labels, return_counts=True)))
    csize = dict(zip(*np.unique(truth, return_counts=True)))
    best = {}
    for L, C, X in zip(lab.tolist(), cls.tolist(), x.tolist()):
        S, B = int(lsize[L]), int(csize[C])
        if L in best:
            X2, C2, B2 = best[L]
            a, b = X * (S + B2 - X2), X2 * (S + B - X)
            if a < b or (a == b and C > C2):
                continue
        best[L] = (X, C, B)
    P = R = F = 0.0
    for L, (X, C, B) in best.items():
        S = float(lsize[L])
        P += X
        R += X * S / B
        F += 2.0 * X * S / (S + B)
    return P / n, R / n, F / n
