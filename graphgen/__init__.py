"""Seeded synthetic input graphs (shared by the oracle and the GPU library).

Only random-graph drawing lives here; nothing in this package computes any
part of the community-detection method.  All randomness is Philox-4x32-10
(Salmon et al., SC'11), counter-indexed, so outputs are identical for any
thread count.

Workloads (sizes from the paper's setting and the scalability table's R-MAT
family; the R-MAT seed matrix here is the Graph500 one):

* ``sbm_c1``      planted partition, 1000 vertices, 4 equal blocks,
                  p_in = 0.10, p_out = 0.005, seed 0.
* ``rmat``        R-MAT scale s, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05),
                  seeded vertex permutation; raw directed samples (the library
                  symmetrises, deduplicates and drops self-loops).
* ``dcsbm``       degree-corrected SBM, power-law degrees and community sizes.
* ``sbm_batch``   many planted-partition SBMs of uneven sizes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "graphgen.c")
_lib = None

TAG_PARAMS = 0x50415241  # "PARA": parameter draws made from Python


def build(force: bool = True) -> str:
    """Compile the generator library with gcc/OpenMP (CPU only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.gg_philox4x32_10.argtypes = [P, P, P]
        L.gg_draw4.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, P]
        L.gg_perm_table.argtypes = [ctypes.c_int, ctypes.c_uint64, P]
        L.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_uint64, P, P, P]
        L.gg_rmat.restype = ctypes.c_int
        L.gg_sbm_pairs.argtypes = [ctypes.c_int32, P, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_uint64, P, P, ctypes.c_int64]
        L.gg_sbm_pairs.restype = ctypes.c_int64
        L.gg_sbm_skip.argtypes = [ctypes.c_int32, P, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_uint64, P, P, ctypes.c_int64]
        L.gg_sbm_skip.restype = ctypes.c_int64
        L.gg_dcsbm.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, P, P, ctypes.c_double,
                               ctypes.c_uint64, P, P, ctypes.c_int64]
        L.gg_dcsbm.restype = ctypes.c_int64
        L.gg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_int64, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().gg_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def uniforms(seed: int, tag: int, count: int, idx0: int = 0) -> np.ndarray:
    """count uniforms in (0,1), counter idx0.. under (seed, tag)."""
    out = np.empty(int(count), dtype=np.float64)
    if count:
        lib().gg_uniform(seed, tag, idx0, int(count), _p(out))
    return out


def perm_table(scale: int, seed: int) -> np.ndarray:
    perm = np.empty(1 << scale, dtype=np.int32)
    lib().gg_perm_table(scale, seed, _p(perm))
    return perm


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 1, permute: bool = True):
    """Raw directed R-MAT samples: returns (src, dst, n).

    16*2^scale samples with 32-bit integer cut-points per level; duplicates and
    self-loops are left in (the consumer canonicalises)."""
    n = 1 << scale
    P = edge_factor * n
    src = np.empty(P, dtype=np.int32)
    dst = np.empty(P, dtype=np.int32)
    perm = perm_table(scale, seed ^ 0x5A5A5A5A) if permute else None
    rc = lib().gg_rmat(scale, P, a, b, c, seed, _p(perm) if perm is not None else None,
                       _p(src), _p(dst))
    if rc != 0:
        raise ValueError("bad R-MAT arguments")
    return src, dst, n


def block_starts(n: int, k: int) -> np.ndarray:
    """Contiguous, near-equal blocks: block j is [floor(j n / k), floor((j+1) n / k))."""
    return np.array([(j * n) // k for j in range(k + 1)], dtype=np.int64)


def sbm_pairs(n: int, k: int, p_in: float, p_out: float, seed: int):
    """Per-pair Bernoulli planted partition (small n): (src, dst, labels)."""
    bs = block_starts(n, k)
    labels = np.zeros(n, dtype=np.int32)
    for j in range(k):
        labels[bs[j]:bs[j + 1]] = j
    L = lib()
    cnt = L.gg_sbm_pairs(n, _p(labels), p_in, p_out, seed, None, None, 0)
    src = np.empty(cnt, dtype=np.int32)
    dst = np.empty(cnt, dtype=np.int32)
    got = L.gg_sbm_pairs(n, _p(labels), p_in, p_out, seed, _p(src), _p(dst), cnt)
    assert got == cnt
    return src, dst, labels


def sbm_skip(n: int, k: int, p_in: float, p_out: float, seed: int):
    """Planted partition by geometric skipping (any n): (src, dst, labels)."""
    bs = block_starts(n, k)
    labels = np.zeros(n, dtype=np.int32)
    for j in range(k):
        labels[bs[j]:bs[j + 1]] = j
    L = lib()
    cnt = L.gg_sbm_skip(k, _p(bs), p_in, p_out, seed, None, None, 0)
    src = np.empty(cnt, dtype=np.int32)
    dst = np.empty(cnt, dtype=np.int32)
    got = L.gg_sbm_skip(k, _p(bs), p_in, p_out, seed, _p(src), _p(dst), cnt)
    assert got == cnt
    return src, dst, labels


def sbm_c1(seed: int = 0):
    """1000 vertices, 4 blocks of 250, p_in 0.10, p_out 0.005."""
    src, dst, labels = sbm_pairs(1000, 4, 0.10, 0.005, seed)
    return dict(name="sbm1k", n=1000, src=src, dst=dst, truth=labels)


def _powerlaw_cont(u: np.ndarray, lo: float, hi: float, gamma: float) -> np.ndarray:
    """Inverse CDF of the continuous power law x^-gamma on [lo, hi]."""
    e = 1.0 - gamma
    return (lo ** e + u * (hi ** e - lo ** e)) ** (1.0 / e)


def _powerlaw_mean(lo: float, hi: float, gamma: float) -> float:
    e1, e2 = 1.0 - gamma, 2.0 - gamma
    return (e1 / e2) * (hi ** e2 - lo ** e2) / (hi ** e1 - lo ** e1)


def dcsbm(n: int = 1_000_000, gamma_deg: float = 2.5, mean_deg: float = 20.0,
          max_deg: float = 2000.0, gamma_comm: float = 1.5, comm_min: int = 20,
          comm_max: int = 5000, mu: float = 0.3, seed: int = 2):
    """Degree-corrected SBM with planted communities: dict(src, dst, n, truth).

    theta ~ continuous power law (exponent gamma_deg) on [k_min, max_deg] with
    k_min solved so E[theta] = mean_deg; community sizes ~ power law (exponent
    gamma_comm) on [comm_min, comm_max], drawn until they cover n (the last one
    is trimmed); vertices are assigned to communities by a seeded shuffle."""
    lo, hi = 1.0, max_deg
    for _ in range(200):  # bisection on k_min for the requested mean
        mid = 0.5 * (lo + hi)
        if _powerlaw_mean(mid, max_deg, gamma_deg) < mean_deg:
            lo = mid
        else:
            hi = mid
    kmin = 0.5 * (lo + hi)
    theta = _powerlaw_cont(uniforms(seed, TAG_PARAMS, n, 0), kmin, max_deg, gamma_deg)
    sizes = []
    tot = 0
    i = 0
    while tot < n:
        u = uniforms(seed, TAG_PARAMS + 1, 1, i)[0]
        s = int(math.floor(_powerlaw_cont(np.array([u]), comm_min, comm_max + 1, gamma_comm)[0]))
        s = min(max(s, comm_min), comm_max)
        s = min(s, n - tot)
        sizes.append(s)
        tot += s
        i += 1
    sizes = np.array(sizes, dtype=np.int64)
    order = np.argsort(uniforms(seed, TAG_PARAMS + 2, n, 0), kind="stable").astype(np.int32)
    cstart = np.zeros(len(sizes) + 1, dtype=np.int64)
    cstart[1:] = np.cumsum(sizes)
    comm = np.empty(n, dtype=np.int32)
    for c in range(len(sizes)):
        comm[order[cstart[c]:cstart[c + 1]]] = c
    members = order
    L = lib()
    cnt = L.gg_dcsbm(n, _p(theta), len(sizes), _p(cstart), _p(members), _p(comm), mu, seed,
                     None, None, 0)
    src = np.empty(cnt, dtype=np.int32)
    dst = np.empty(cnt, dtype=np.int32)
    got = L.gg_dcsbm(n, _p(theta), len(sizes), _p(cstart), _p(members), _p(comm), mu, seed,
                     _p(src), _p(dst), cnt)
    assert got == cnt
    return dict(name="dcsbm", n=n, src=src, dst=dst, truth=comm, kmin=kmin)


def sbm_batch_params(g: int):
    """Parameters of batch graph g (seed 1000+g): n log-uniform in [1e3, 1e5],
    blocks log-uniform in [4, 64], intra degree U[8,30] (re-drawn while
    p_in > 0.5), mixing mu ~ U[0.05, 0.45]."""
    seed = 1000 + g
    u = uniforms(seed, TAG_PARAMS, 4, 0)
    n = int(round(math.exp(math.log(1e3) + u[0] * (math.log(1e5) - math.log(1e3)))))
    k = int(round(math.exp(math.log(4) + u[1] * (math.log(64) - math.log(4)))))
    k = max(2, min(k, n // 4))
    s = n / k
    mu = 0.05 + 0.40 * u[3]
    d_in = 8.0 + 22.0 * u[2]
    j = 0
    while d_in / (s - 1.0) > 0.5 and j < 64:
        j += 1
        d_in = 8.0 + 22.0 * uniforms(seed, TAG_PARAMS, 1, 16 + j)[0]
    p_in = min(d_in / (s - 1.0), 0.5)
    d_in = p_in * (s - 1.0)
    p_out = mu * d_in / ((1.0 - mu) * (n - s))
    return dict(seed=seed, n=n, k=k, p_in=p_in, p_out=p_out, mu=mu, d_in=d_in)


def sbm_batch_graph(g: int):
    pr = sbm_batch_params(g)
    src, dst, labels = sbm_skip(pr["n"], pr["k"], pr["p_in"], pr["p_out"], pr["seed"])
    return dict(name=f"sbm_batch_{g}", n=pr["n"], src=src, dst=dst, truth=labels, params=pr)


def sbm_batch(G: int = 256, n_max: int | None = None, first: int = 0):
    """Graphs first .. first+G-1 of the planted-partition batch as one disjoint
    union: dict(src, dst, n, vbase[G+1], truth (class ids unique across
    graphs), params).  n_max caps each graph's vertex count (smaller test
    batches); the other parameters keep their draws."""
    srcs, dsts, truths, params = [], [], [], []
    vbase = [0]
    cbase = 0
    for g in range(first, first + G):
        pr = dict(sbm_batch_params(g))
        if n_max is not None and pr["n"] > n_max:
            n = n_max
            k = max(2, min(pr["k"], n // 4))
            s = n / k
            p_in = min(pr["d_in"] / (s - 1.0), 0.5)
            d_in = p_in * (s - 1.0)
            p_out = pr["mu"] * d_in / ((1.0 - pr["mu"]) * (n - s))
            pr.update(n=n, k=k, p_in=p_in, p_out=p_out, d_in=d_in)
        src, dst, lab = sbm_skip(pr["n"], pr["k"], pr["p_in"], pr["p_out"], pr["seed"])
        srcs.append(src + vbase[-1])
        dsts.append(dst + vbase[-1])
        truths.append(lab + cbase)
        cbase += pr["k"]
        vbase.append(vbase[-1] + pr["n"])
        params.append(pr)
    return dict(src=np.concatenate(srcs).astype(np.int32), dst=np.concatenate(dsts).astype(np.int32),
                n=vbase[-1], vbase=np.array(vbase, np.int64),
                truth=np.concatenate(truths).astype(np.int32), params=params)


def sbm_two_blocks(n: int, p1: float, p2: float, q: float, seed: int):
    """The imbalanced two-block SBM of the paper's Sec. 3 analysis: blocks B1
    = [0, n) and B2 = [n, 2n), pairs inside B_i joined with probability p_i,
    pairs across with probability q, every pair an independent draw (three
    per-pair Bernoulli streams of distinct seeds).  (src, dst, labels)."""
    s1, d1, _ = sbm_pairs(n, 1, p1, 0.0, 3 * seed)
    s2, d2, _ = sbm_pairs(n, 1, p2, 0.0, 3 * seed + 1)
    sx, dx, labels = sbm_pairs(2 * n, 2, 0.0, q, 3 * seed + 2)  # across pairs only
    src = np.concatenate([s1, s2 + n, sx]).astype(np.int32)
    dst = np.concatenate([d1, d2 + n, dx]).astype(np.int32)
    return src, dst, labels


def sbm_two_blocks_batch(G: int, n: int = 50, p1: float = 0.1, p2: float = 0.8, q: float = 0.05, seed0: int = 0):
    """G independent imbalanced two-block SBMs (seeds seed0 .. seed0+G-1; the
    defaults are the paper's visualised setting) as one disjoint union:
    dict(src, dst, n, vbase[G+1], truth (block ids unique across graphs))."""
    srcs, dsts, truths = [], [], []
    for g in range(G):
        src, dst, lab = sbm_two_blocks(n, p1, p2, q, seed0 + g)
        srcs.append(src + 2 * n * g)
        dsts.append(dst + 2 * n * g)
        truths.append(lab + 2 * g)
    return dict(src=np.concatenate(srcs).astype(np.int32), dst=np.concatenate(dsts).astype(np.int32),
                n=2 * n * G, vbase=np.arange(G + 1, dtype=np.int64) * 2 * n,
                truth=np.concatenate(truths).astype(np.int32))
