"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

Nothing here compares the oracle with itself.  Each check uses an independent
route: hand-derived closed forms (tests/golden), brute force with Python sets,
dense matrix products, networkx / scipy / sklearn routines, the paper's
Proposition 1, exact Fractions, invariants and the SBM expectations of the
paper's Table "tab:expected".
"""
import os
import subprocess
import sys
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def edges_of(n, pairs):
    src = np.array([p[0] for p in pairs], np.int32)
    dst = np.array([p[1] for p in pairs], np.int32)
    return oracle.canon(n, src, dst)


def full(n, pairs):
    lo, hi = edges_of(n, pairs)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    return lo, hi, deg, t


# ---------------------------------------------------------------- generator

def test_philox_known_answers():
    # Published known-answer vectors of Philox-4x32-10 (Random123 distribution).
    assert list(gg.philox4x32_10([0, 0, 0, 0], [0, 0])) == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert list(gg.philox4x32_10([0xffffffff] * 4, [0xffffffff] * 2)) == [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert list(gg.philox4x32_10([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344],
                                 [0xa4093822, 0x299f31d0])) == [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


def test_generator_thread_count_independent():
    code = ("import graphgen as gg, hashlib;s,d,n=gg.rmat(14,seed=7);"
            "print(hashlib.sha1(s.tobytes()+d.tobytes()).hexdigest())")
    outs = []
    for th in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=th,
                   PYTHONPATH=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert outs[0] == outs[1]


def test_rmat_quadrant_frequencies():
    # Without the permutation, the top bit of (u, v) follows (a, b, c, d).
    s, d, n = gg.rmat(10, seed=3, permute=False)
    top_u = (s >> 9) & 1
    top_v = (d >> 9) & 1
    P = len(s)
    freq = [np.mean((top_u == 0) & (top_v == 0)), np.mean((top_u == 0) & (top_v == 1)),
            np.mean((top_u == 1) & (top_v == 0)), np.mean((top_u == 1) & (top_v == 1))]
    for f, want in zip(freq, [0.57, 0.19, 0.19, 0.05]):
        assert abs(f - want) < 5 * np.sqrt(want * (1 - want) / P)


def test_permutation_is_bijection():
    for s in (1, 2, 7, 10, 13):
        p = gg.perm_table(s, 11)
        assert np.array_equal(np.sort(p), np.arange(1 << s))


# ------------------------------------------------------------- closed forms

def load_golden():
    graphs = []
    cur = None
    with open(os.path.join(GOLDEN, "closed_forms.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "graph":
                cur = dict(name=parts[1], n=int(parts[2]), edges=[])
                graphs.append(cur)
            else:
                kv = dict(p.split("=") for p in parts[3:])
                num, den = kv["tec"].split("/")
                cur["edges"].append((int(parts[1]), int(parts[2]), int(kv["t"]), int(kv["wedge"]),
                                     int(kv["tw"]), Fraction(int(num), int(den))))
    return graphs


@pytest.mark.parametrize("g", load_golden(), ids=lambda g: g["name"])
def test_golden_closed_forms(g):
    n = g["n"]
    lo, hi, deg, t = full(n, [(a, b) for a, b, *_ in g["edges"]])
    w = oracle.tectonic(lo, hi, t, deg)
    wedge = oracle.wedges(lo, hi, t, deg)
    tw = oracle.tw(lo, hi, t, deg)
    idx = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(lo, hi))}
    assert len(idx) == len(g["edges"])
    for a, b, tt, wd, twv, tec in g["edges"]:
        i = idx[(a, b)]
        assert t[i] == tt and wedge[i] == wd and tw[i] == twv
        assert w[i] == float(tec)


def complete(n):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


@pytest.mark.parametrize("k", [3, 4, 5, 8, 13])
def test_complete_graph(k):
    lo, hi, deg, t = full(k, complete(k))
    assert np.all(t == k - 2)
    assert np.all(oracle.wedges(lo, hi, t, deg) == 0)
    assert np.all(oracle.tw(lo, hi, t, deg) == k - 2)
    assert np.all(oracle.tectonic(lo, hi, t, deg) == (k - 2) / (2 * k - 2))


def test_triangle_free_families():
    star = [(0, i) for i in range(1, 9)]
    cycle = [(i, (i + 1) % 9) for i in range(9)]
    kab = [(i, 4 + j) for i in range(4) for j in range(5)]
    for n, pairs in ((9, star), (9, cycle), (9, kab)):
        lo, hi, deg, t = full(n, pairs)
        assert np.all(t == 0)


@pytest.mark.parametrize("k", [4, 5, 9])
def test_wheel_and_windmill(k):
    pairs = [(0, i) for i in range(1, k + 1)] + [(i, i % k + 1) for i in range(1, k + 1)]
    lo, hi, deg, t = full(k + 1, pairs)
    assert np.all(t[lo == 0] == 2) and np.all(t[lo != 0] == 1)
    wind = []
    for j in range(k):
        a, b = 1 + 2 * j, 2 + 2 * j
        wind += [(0, a), (0, b), (a, b)]
    lo, hi, deg, t = full(2 * k + 1, wind)
    assert np.all(t == 1)


def test_two_cliques_bridge_two_components():
    k = 6
    pairs = complete(k) + [(k + a, k + b) for a, b in complete(k)] + [(2, k + 3)]
    n = 2 * k
    lo, hi, deg, t = full(n, pairs)
    bridge = np.nonzero((lo == 2) & (hi == k + 3))[0][0]
    assert t[bridge] == 0
    keep = oracle.prune(oracle.TECTONIC, lo, hi, t, deg, 1, 1000)
    assert keep.sum() == len(lo) - 1 and keep[bridge] == 0
    labels, ncc = oracle.components(n, lo, hi, keep)
    assert ncc == 2 and set(labels[:k]) == {0} and set(labels[k:]) == {k}


# ------------------------------------------------------------- brute force

def brute(n, pairs):
    N = [set() for _ in range(n)]
    for a, b in pairs:
        if a != b:
            N[a].add(b)
            N[b].add(a)
    E = sorted({(min(a, b), max(a, b)) for a, b in pairs if a != b})
    t = [len(N[a] & N[b]) for a, b in E]
    wedge = [len(N[a] | N[b]) - len(N[a] & N[b]) - 2 for a, b in E]
    tec = [Fraction(len(N[a] & N[b]), len(N[a]) + len(N[b])) for a, b in E]
    return E, N, t, wedge, tec


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_small_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    P = int(rng.integers(0, 4 * n + 1))
    src = rng.integers(0, n, P).astype(np.int32)
    dst = rng.integers(0, n, P).astype(np.int32)
    pairs = list(zip(src.tolist(), dst.tolist()))
    E, N, t_b, wedge_b, tec_b = brute(n, pairs)
    lo, hi = oracle.canon(n, src, dst)
    assert list(zip(lo.tolist(), hi.tolist())) == E
    deg = oracle.degrees(n, lo, hi)
    assert deg.tolist() == [len(x) for x in N]
    t = oracle.triangles(n, lo, hi)
    assert t.tolist() == t_b
    assert oracle.wedges(lo, hi, t, deg).tolist() == wedge_b
    assert oracle.tw(lo, hi, t, deg).tolist() == [a - b for a, b in zip(t_b, wedge_b)]
    assert oracle.tectonic(lo, hi, t, deg).tolist() == [float(x) for x in tec_b]
    # prune at a few rationals against exact Fractions (Algorithm 1: drop iff sim < delta)
    for num, den in ((0, 1), (1, 7), (1, 4), (3, 10), (1, 2)):
        keep = oracle.prune(oracle.TECTONIC, lo, hi, t, deg, num, den)
        assert keep.tolist() == [0 if x < Fraction(num, den) else 1 for x in tec_b]
    for num, den in ((-3, 1), (0, 1), (1, 2), (-5, 2)):
        keep = oracle.prune(oracle.TW, lo, hi, t, deg, num, den)
        assert keep.tolist() == [0 if (a - b) < Fraction(num, den) else 1 for a, b in zip(t_b, wedge_b)]


def test_invalid_vertex_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.canon(4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(oracle.OracleError):
        oracle.canon(4, np.array([-1], np.int32), np.array([1], np.int32))


def test_c1_dense_matrix_route():
    c1 = gg.sbm_c1()
    n = c1["n"]
    lo, hi = oracle.canon(n, c1["src"], c1["dst"])
    t = oracle.triangles(n, lo, hi)
    A = np.zeros((n, n), np.int64)
    A[lo, hi] = 1
    A[hi, lo] = 1
    A2 = A @ A
    assert np.array_equal(t, A2[lo, hi])
    # every triangle is counted on each of its 3 edges: sum t = 3T = trace(A^3)/2
    assert t.sum() == np.trace(A2 @ A) // 2


def test_networkx_triangles_rmat():
    import networkx as nx
    s, d, n = gg.rmat(11, seed=5)
    lo, hi = oracle.canon(n, s, d)
    t = oracle.triangles(n, lo, hi)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(lo.tolist(), hi.tolist()))
    tri = nx.triangles(G)
    per_v = np.zeros(n, np.int64)
    np.add.at(per_v, lo, t)
    np.add.at(per_v, hi, t)
    assert all(per_v[v] == 2 * tri[v] for v in range(n))
    deg = oracle.degrees(n, lo, hi)
    assert np.all(t <= np.minimum(deg[lo], deg[hi]) - 1)


# ------------------------------------------------------------------ prune

def test_prop1_jaccard_reparameterisation():
    # Proposition 1: Jaccard < d  <=>  Tectonic < d/(1+d); with d = p/q the
    # Tectonic threshold is p/(p+q).  Jaccard is evaluated here with Fractions.
    s, d, n = gg.rmat(10, seed=9)
    lo, hi = oracle.canon(n, s, d)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    D = deg[lo].astype(np.int64) + deg[hi]
    for p, q in ((1, 20), (1, 9), (1, 3), (2, 5), (1, 1)):
        jac_keep = np.array([0 if Fraction(int(a), int(b) - int(a)) < Fraction(p, q) else 1
                             for a, b in zip(t, D)], np.uint8)
        tec_keep = oracle.prune(oracle.TECTONIC, lo, hi, t, deg, p, p + q)
        assert np.array_equal(jac_keep, tec_keep)


def test_prune_ties_are_kept():
    # Algorithm 1 removes only edges with sim < delta: sim == delta stays.
    lo, hi, deg, t = full(3, complete(3))
    assert oracle.prune(oracle.TECTONIC, lo, hi, t, deg, 1, 4).tolist() == [1, 1, 1]
    assert oracle.prune(oracle.TECTONIC, lo, hi, t, deg, 25, 101).tolist() == [1, 1, 1]
    assert oracle.prune(oracle.TECTONIC, lo, hi, t, deg, 25, 100).tolist() == [1, 1, 1]
    assert oracle.prune(oracle.TECTONIC, lo, hi, t, deg, 25, 99).tolist() == [0, 0, 0]
    assert oracle.prune(oracle.TW, lo, hi, t, deg, 1, 1).tolist() == [1, 1, 1]
    assert oracle.prune(oracle.TW, lo, hi, t, deg, 3, 2).tolist() == [0, 0, 0]


def test_prune_monotone_and_refining():
    c1 = gg.sbm_c1()
    n = c1["n"]
    lo, hi = oracle.canon(n, c1["src"], c1["dst"])
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    prev_keep, prev_ncc, prev_lab = None, 0, None
    for k in range(16):  # the paper's Tectonic grid (0, 0.3, 0.02)
        keep = oracle.prune(oracle.TECTONIC, lo, hi, t, deg, k, 50)
        lab, ncc = oracle.components(n, lo, hi, keep)
        if prev_keep is not None:
            assert np.all(keep <= prev_keep)
            assert ncc >= prev_ncc
            # finer partition: same label now => same label before
            pairs = {}
            for v in range(n):
                pairs.setdefault(lab[v], set()).add(prev_lab[v])
            assert all(len(s) == 1 for s in pairs.values())
        prev_keep, prev_ncc, prev_lab = keep, ncc, lab
    assert prev_keep is not None


# ------------------------------------------------------------- components

@pytest.mark.parametrize("seed", range(4))
def test_components_vs_scipy(seed):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(50, 3000))
    P = int(rng.integers(0, n))
    src = rng.integers(0, n, P).astype(np.int32)
    dst = rng.integers(0, n, P).astype(np.int32)
    lo, hi = oracle.canon(n, src, dst)
    keep = (rng.random(len(lo)) < 0.7).astype(np.uint8)
    lab, ncc = oracle.components(n, lo, hi, keep)
    k = keep.astype(bool)
    M = coo_matrix((np.ones(k.sum()), (lo[k], hi[k])), shape=(n, n))
    nc, cl = connected_components(M, directed=False)
    assert nc == ncc
    # canonical labels = min vertex per scipy component
    mins = np.full(nc, n)
    np.minimum.at(mins, cl, np.arange(n))
    assert np.array_equal(lab, mins[cl])
    # invariants
    assert np.all(lab <= np.arange(n)) and np.all(lab[lab] == lab)
    assert np.all(lab[lo[k]] == lab[hi[k]])
    assert ncc == np.sum(lab == np.arange(n))


def test_components_relabel_invariant():
    s, d, n = gg.rmat(10, seed=2)
    lo, hi = oracle.canon(n, s, d)
    lab, ncc = oracle.components(n, lo, hi)
    perm = np.random.default_rng(0).permutation(n).astype(np.int32)
    lo2, hi2 = oracle.canon(n, perm[lo], perm[hi])
    lab2, ncc2 = oracle.components(n, lo2, hi2)
    assert ncc == ncc2
    # same partition: v ~ w  <=>  perm[v] ~ perm[w]
    a = lab
    b = lab2[perm]
    assert len(set(zip(a.tolist(), b.tolist()))) == ncc


# -------------------------------------------------------------------- ARI

def ari_fraction(x, y):
    from collections import Counter
    n = len(x)
    c2 = lambda v: Fraction(v * (v - 1), 2)
    S = sum(c2(v) for v in Counter(zip(x, y)).values())
    A = sum(c2(v) for v in Counter(x).values())
    B = sum(c2(v) for v in Counter(y).values())
    N = c2(n)
    exp = A * B / N
    den = (A + B) / 2 - exp
    return Fraction(1) if den == 0 else (S - exp) / den


@pytest.mark.parametrize("seed", range(6))
def test_ari_vs_sklearn_and_exact(seed):
    from sklearn.metrics import adjusted_rand_score
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    x = rng.integers(0, int(rng.integers(1, 20)), n).astype(np.int32)
    y = rng.integers(0, int(rng.integers(1, 20)), n).astype(np.int32)
    v, sums = oracle.ari(x, y)
    assert abs(v - adjusted_rand_score(y, x)) < 1e-12
    assert abs(v - float(ari_fraction(x.tolist(), y.tolist()))) < 1e-12
    assert oracle.ari(x, x)[0] == 1.0
    assert abs(oracle.ari(y, x)[0] - v) < 1e-15


# ------------------------------------------------- percentile / histogram

def test_percentile_exact_fractions():
    s, d, n = gg.rmat(10, seed=4)
    lo, hi = oracle.canon(n, s, d)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    vals = sorted(Fraction(int(a), int(deg[u]) + int(deg[v])) for a, u, v in zip(t, lo, hi) if a != 0)
    K = len(vals)
    for pn, pd in ((3, 10), (1, 2), (1, 1), (1, 1000)):
        k = max(0, -(-pn * K // pd) - 1)
        num, den = oracle.percentile(oracle.TECTONIC, lo, hi, t, deg, pn, pd)
        assert Fraction(num, den) == vals[k]
    tws = sorted(int(3 * a - deg[u] - deg[v] + 2) for a, u, v in zip(t, lo, hi))
    tws = [x for x in tws if x != 0]
    num, den = oracle.percentile(oracle.TW, lo, hi, t, deg, 3, 10)
    assert den == 1 and num == tws[max(0, -(-3 * len(tws) // 10) - 1)]


def test_histogram_bins():
    s, d, n = gg.rmat(10, seed=6)
    lo, hi = oracle.canon(n, s, d)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    h = oracle.histogram(lo, hi, t, deg)
    bins = [int(Fraction(128 * int(a), int(deg[u]) + int(deg[v]))) for a, u, v in zip(t, lo, hi)]
    assert max(bins) <= 63
    assert h.tolist() == np.bincount(bins, minlength=64).tolist()


# ------------------------------------------------------- sampled queries

def test_query_edges_matches_brute():
    s, d, n = gg.rmat(9, seed=8)
    pairs = list(zip(s.tolist(), d.tolist()))
    E, N, t_b, _, _ = brute(n, pairs)
    rng = np.random.default_rng(1)
    pick = rng.integers(0, len(E), 50)
    qu = np.array([E[i][0] for i in pick] + [0, 1], np.int32)
    qv = np.array([E[i][1] for i in pick] + [0, 2], np.int32)
    is_e, du, dv, t = oracle.query_edges(n, s, d, qu, qv)
    for k in range(len(qu)):
        a, b = int(qu[k]), int(qv[k])
        assert is_e[k] == (b in N[a])
        assert du[k] == len(N[a]) and dv[k] == len(N[b])
        assert t[k] == len(N[a] & N[b])


# ----------------------------------------- SBM expectations (tab:expected)

def test_expected_table_two_block_sbm():
    # Table tab:expected: per-edge expectations normalised by the block size n.
    # Inside B1: t ~ p1^2+q^2, wedge ~ 2(p1(1-p1)+q(1-q)), d_u+d_v ~ 2(p1+q).
    # Across:    t ~ p1 q + p2 q, d_u+d_v ~ p1+p2+2q.
    nb, p1, p2, q = 1500, 0.04, 0.12, 0.02
    n = 2 * nb
    # two blocks with different densities: draw them with the per-pair generator
    # at p_in = p1 for block 0 and p2 for block 1 by sampling the two blocks
    # separately and the cross edges at q.
    s1, d1, _ = gg.sbm_pairs(nb, 1, p1, 0.0, 21)
    s2, d2, _ = gg.sbm_pairs(nb, 1, p2, 0.0, 22)
    rng = np.random.default_rng(23)
    cross = rng.random((nb, nb)) < q
    cu, cv = np.nonzero(cross)
    src = np.concatenate([s1, s2 + nb, cu]).astype(np.int32)
    dst = np.concatenate([d1, d2 + nb, cv + nb]).astype(np.int32)
    lo, hi = oracle.canon(n, src, dst)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    wedge = oracle.wedges(lo, hi, t, deg)
    D = deg[lo] + deg[hi]
    inside1 = hi < nb
    across = (lo < nb) & (hi >= nb)
    rel = lambda a, b: abs(a - b) / b
    assert rel(t[inside1].mean() / nb, p1 ** 2 + q ** 2) < 0.05
    assert rel(wedge[inside1].mean() / nb, 2 * (p1 * (1 - p1) + q * (1 - q))) < 0.05
    assert rel(D[inside1].mean() / nb, 2 * (p1 + q)) < 0.05
    assert rel(t[across].mean() / nb, p1 * q + p2 * q) < 0.05
    assert rel(D[across].mean() / nb, p1 + p2 + 2 * q) < 0.05
    tw = oracle.tw(lo, hi, t, deg)
    assert rel(tw[inside1].mean() / nb, 3 * p1 ** 2 - 2 * p1 + 3 * q ** 2 - 2 * q) < 0.05


def test_prop1_jaccard_measure_equals_reparameterised_tectonic():
    # Proposition 1 between two of the oracle's own measures: Jaccard-prune at
    # p/q keeps exactly the edges Tectonic-prune keeps at p/(p+q); and the
    # Jaccard weight w_J relates to Tectonic w_T by w_J = w_T / (1 - w_T).
    s, d, n = gg.rmat(11, seed=12)
    lo, hi = oracle.canon(n, s, d)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    for p, q in ((1, 20), (1, 9), (1, 3), (2, 5), (1, 1), (0, 1)):
        assert np.array_equal(oracle.prune(oracle.JACCARD, lo, hi, t, deg, p, q),
                              oracle.prune(oracle.TECTONIC, lo, hi, t, deg, p, p + q))
    wt = oracle.tectonic(lo, hi, t, deg)
    assert np.allclose(oracle.jaccard(lo, hi, t, deg), wt / (1 - wt), rtol=1e-12)


def test_k3_measure_closed_forms():
    # K_n: every edge lies in n - 2 triangles; K3-prune at n - 2 keeps all
    # edges, at n - 1 none (ties kept).  A path has no triangles.
    for k in (4, 6):
        lo, hi, deg, t = full(k, complete(k))
        assert oracle.prune(oracle.K3, lo, hi, t, deg, k - 2, 1).all()
        assert not oracle.prune(oracle.K3, lo, hi, t, deg, k - 1, 1).any()
        assert oracle.prune(oracle.K3, lo, hi, t, deg, 2 * k - 5, 2).all()  # (k-2.5) < k-2
    lo, hi, deg, t = full(4, [(0, 1), (1, 2), (2, 3)])
    assert oracle.prune(oracle.K3, lo, hi, t, deg, 0, 1).all()
    assert not oracle.prune(oracle.K3, lo, hi, t, deg, 1, 3).any()


def test_sweep_modularity_matches_networkx():
    # Modularity of each threshold's partition on the input graph equals
    # networkx's modularity of those communities (Sec. 2 definition).
    import networkx as nx
    from networkx.algorithms.community import modularity as nx_modularity
    for seed in range(3):
        rng = np.random.default_rng(40 + seed)
        n = int(rng.integers(30, 120))
        P = int(rng.integers(n, 5 * n))
        s = rng.integers(0, n, P).astype(np.int32)
        d = rng.integers(0, n, P).astype(np.int32)
        lo, hi = oracle.canon(n, s, d)
        if len(lo) == 0:
            continue
        deg = oracle.degrees(n, lo, hi)
        t = oracle.triangles(n, lo, hi)
        deltas = [(0, 1), (1, 10), (1, 5), (1, 3)]
        st, _, labels, q = oracle.sweep(n, lo, hi, t, deg, oracle.TECTONIC, deltas, modularity=True)
        Gx = nx.Graph()
        Gx.add_nodes_from(range(n))
        Gx.add_edges_from(zip(lo.tolist(), hi.tolist()))
        for i in range(len(deltas)):
            comms = {}
            for v, c in enumerate(labels[i]):
                comms.setdefault(int(c), set()).add(v)
            assert abs(q[0, i] - nx_modularity(Gx, list(comms.values()))) <= 1e-12
            # intra edges: every kept edge is inside a component
            assert st[0, i, 7] >= st[0, i, 0]


def test_rule_of_thumb_cases():
    # thresholds given out of order; largest component (field 2) per slot
    deltas = [(3, 10), (1, 10), (2, 10), (4, 10)]   # ascending order of slots: 1, 2, 0, 3
    vbase = [0, 100]
    st = np.zeros((1, 4, 9), np.int64)
    # walking down 4/10 -> 3/10 -> 2/10 -> 1/10: largest 5, 8, 60, 70: jump 52 at 3/10 -> 2/10
    for slot, L in ((3, 5), (0, 8), (2, 60), (1, 70)):
        st[0, slot, 2] = L
    assert oracle.rule_of_thumb(st, deltas, vbase).tolist() == [0]  # 3/10, just above the jump
    # no jump of 10% of n: falls back to the maximum modularity
    st2 = st.copy()
    for slot, L in ((3, 5), (0, 8), (2, 12), (1, 14)):
        st2[0, slot, 2] = L
    q = np.array([[0.1, 0.3, 0.5, 0.2]])
    assert oracle.rule_of_thumb(st2, deltas, vbase, q).tolist() == [2]
    assert oracle.rule_of_thumb(st2, deltas, vbase).tolist() == [3]  # no modularity: highest threshold


def test_precision_recall_f1_hand_examples():
    # S1 = {0,1,2}, S2 = {3,4}; C1 = {0,1}, C2 = {2,3,4}: S1 -> C1 (J 2/3 vs 1/5),
    # S2 -> C2 (J 2/3): P = 4/5, R = 13/15, F1 = (12/5 + 8/5) / 5 = 4/5
    p, r, f = oracle.precision_recall_f1([0, 0, 0, 3, 3], [1, 1, 2, 2, 2])
    assert abs(p - 0.8) < 1e-15 and abs(r - 13 / 15) < 1e-15 and abs(f - 0.8) < 1e-15
    # identical partitions
    assert oracle.precision_recall_f1([5, 5, 7, 7, 7], [0, 0, 1, 1, 1]) == (1.0, 1.0, 1.0)
    # all singletons against one class of size n: P = 1, R = 1/n, F1 = 2/(n+1)
    n = 9
    p, r, f = oracle.precision_recall_f1(list(range(n)), [0] * n)
    assert p == 1.0 and abs(r - 1 / n) < 1e-15 and abs(f - 2 / (n + 1)) < 1e-15
    # a Jaccard tie goes to the smaller class: S = {0,1}, C0 = {0,2}, C1 = {1,3}
    p, r, f = oracle.precision_recall_f1([0, 0, 2, 3], [0, 1, 0, 1])
    # S={0,1} -> C0 (x=1,b=2); S={2} -> C0 (x=1,b=2); S={3} -> C1 (x=1,b=2)
    assert abs(p - (1 + 1 + 1) / 4) < 1e-15
    assert abs(r - (1 * 2 / 2 + 1 * 1 / 2 + 1 * 1 / 2) / 4) < 1e-15


def test_k4_participation_pins():
    # brute force over all 4-subsets on tiny graphs; K_n closed form C(n-2, 2)
    import itertools
    for k in (4, 5, 7):
        lo, hi, deg, t = full(k, complete(k))
        assert np.all(oracle.k4(k, lo, hi) == (k - 2) * (k - 3) // 2)
    for seed in range(5):
        rng = np.random.default_rng(60 + seed)
        n = int(rng.integers(5, 14))
        A = np.triu(rng.random((n, n)) < 0.6, 1)
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if A[i, j]]
        if not pairs:
            continue
        lo, hi = edges_of(n, pairs)
        S = set(zip(lo.tolist(), hi.tolist()))
        want = {e: 0 for e in S}
        for q in itertools.combinations(range(n), 4):
            es = list(itertools.combinations(q, 2))
            if all(e in S for e in es):
                for e in es:
                    want[e] += 1
        got = oracle.k4(n, lo, hi)
        assert [want[e] for e in zip(lo.tolist(), hi.tolist())] == got.tolist()
        # K4-prune at c keeps exactly the edges in at least c 4-cliques
        keep = oracle.prune(oracle.K4, lo, hi, got, oracle.degrees(n, lo, hi), 2, 1)
        assert np.array_equal(keep, (got >= 2).astype(np.uint8))


def test_complete_multipartite_closed_forms():
    # complete multipartite graph with parts of sizes p_1..p_k: a 4-clique
    # takes one vertex from each of four distinct parts, so an edge between
    # parts i and j lies in the sum over pairs {k, l} of the other parts of
    # p_k p_l 4-cliques (and K4 participation is 0 with fewer than four parts)
    import itertools
    for sizes in ((1, 1, 1, 1), (2, 2, 2), (3, 1, 4, 2), (2, 3, 1, 2, 4), (5, 5)):
        part = np.repeat(np.arange(len(sizes)), sizes)
        n = len(part)
        pairs = [(u, v) for u in range(n) for v in range(u + 1, n) if part[u] != part[v]]
        lo, hi = edges_of(n, pairs)
        got = oracle.k4(n, lo, hi)
        for e, (u, v) in enumerate(zip(lo.tolist(), hi.tolist())):
            rest = [sizes[q] for q in range(len(sizes)) if q not in (part[u], part[v])]
            want = sum(a * b for a, b in itertools.combinations(rest, 2))
            assert got[e] == want, (sizes, u, v)
        # the same graphs pin t, the degrees and the weights: an edge between
        # parts i and j has t = n - p_i - p_j, deg u = n - p_i, deg v = n - p_j
        deg = oracle.degrees(n, lo, hi)
        t = oracle.triangles(n, lo, hi)
        pu, pv = np.array(sizes)[part[lo]], np.array(sizes)[part[hi]]
        assert np.array_equal(deg[lo], n - pu) and np.array_equal(deg[hi], n - pv)
        assert np.array_equal(t, n - pu - pv)
        assert np.array_equal(oracle.tw(lo, hi, t, deg), 3 * (n - pu - pv) - (n - pu) - (n - pv) + 2)
        assert np.array_equal(oracle.tectonic(lo, hi, t, deg), (n - pu - pv) / ((n - pu) + (n - pv)))


def test_imbalanced_sbm_tw_recovers_tectonic_does_not():
    # Sec. 3's two-block analysis in the paper's visualised setting (blocks of
    # 50, p1 = 0.1, p2 = 0.8, q = 0.05), 20 seeds: across-block edges score
    # above the sparse block's own edges under Tectonic but far below them
    # under TW, so TW's best threshold recovers the blocks (nearly always
    # exactly) and Tectonic's does not; per graph TW's best ARI is never lower
    b = gg.sbm_two_blocks_batch(20)
    n, vb = b["n"], b["vbase"]
    lo, hi = oracle.canon(n, b["src"], b["dst"])
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    blk = np.asarray(b["truth"])
    in_b1 = (blk[lo] == blk[hi]) & (blk[lo] % 2 == 0)
    across = blk[lo] != blk[hi]
    w = oracle.tectonic(lo, hi, t, deg)
    tw = oracle.tw(lo, hi, t, deg)
    assert w[across].mean() > w[in_b1].mean()
    assert tw[in_b1].mean() > tw[across].mean() + 20
    _, a_tw, _ = oracle.sweep(n, lo, hi, t, deg, oracle.TW, [(k, 1) for k in range(-50, 14)], b["truth"], vb)
    _, a_te, _ = oracle.sweep(n, lo, hi, t, deg, oracle.TECTONIC, [(9 + 7 * i, 900) for i in range(64)],
                              b["truth"], vb)
    best_tw, best_te = a_tw.max(1), a_te.max(1)
    assert np.all(best_tw >= best_te)
    assert best_tw.mean() > 0.95 and (best_tw == 1.0).sum() >= 12
    assert best_te.mean() < 0.8 and not np.any(best_te == 1.0)
