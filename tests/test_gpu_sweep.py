"""GPU parity of the batched threshold sweep (levels + incremental
union-find + per-graph statistics + ARI) against the oracle."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2412_12382_amd.mcd")

GRID64 = [(9 + 7 * i, 900) for i in range(64)]
GRID16 = [(k, 50) for k in range(16)]


def gpu_sweep(src, dst, n, measure, deltas, truth=None, vbase=None, want_labels=True):
    from gpu_util import build
    g = build(src, dst, n)
    t = M.mcd_triangles(g)
    vb = None if vbase is None else torch.from_numpy(np.asarray(vbase, np.int64)).cuda()
    tr = None if truth is None else torch.from_numpy(np.asarray(truth, np.int32)).cuda()
    stats, ari, labels = M.mcd_sweep(g, measure, t, deltas, vbase=vb, truth=tr, want_labels=want_labels)
    torch.cuda.synchronize()
    return (stats.cpu().numpy(), None if ari is None else ari.cpu().numpy(),
            None if labels is None else labels.cpu().numpy()[:, :n])


def oracle_sweep(src, dst, n, measure, deltas, truth=None, vbase=None):
    lo, hi = oracle.canon(n, src, dst)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    return oracle.sweep(n, lo, hi, t, deg, measure, deltas, truth, vbase)


def compare(got, want):
    gs, ga, gl = got
    ws, wa, wl = want
    if gl is not None:
        assert np.array_equal(gl, wl)
    bad = np.argwhere(gs != ws)
    assert len(bad) == 0, [(tuple(b), int(gs[tuple(b)]), int(ws[tuple(b)])) for b in bad[:10]]
    if wa is not None:
        assert np.all(np.abs(ga - wa) <= 1e-12)


def test_sweep_rmat_grid16():
    s, d, n = gg.rmat(14, seed=31)
    compare(gpu_sweep(s, d, n, oracle.TECTONIC, GRID16), oracle_sweep(s, d, n, oracle.TECTONIC, GRID16))


def test_sweep_dense_level_two_large_components():
    """One graph made of two R-MAT graphs side by side: the lowest
    thresholds hold most edges and two large components form, only one of
    which the dense-level union may pass over; isolated vertices too."""
    s1, d1, n1 = gg.rmat(13, seed=51)
    s2, d2, n2 = gg.rmat(14, seed=52)
    s = np.concatenate([s1, s2 + n1]).astype(np.int32)
    d = np.concatenate([d1, d2 + n1]).astype(np.int32)
    n = n1 + n2 + 100  # 100 isolated vertices at the end
    compare(gpu_sweep(s, d, n, oracle.TECTONIC, GRID16), oracle_sweep(s, d, n, oracle.TECTONIC, GRID16))
    deltas = [(-40, 3), (-10, 1), (-1, 1), (0, 1), (2, 1)]
    compare(gpu_sweep(s, d, n, oracle.TW, deltas), oracle_sweep(s, d, n, oracle.TW, deltas))


def test_sweep_statistics_without_labels():
    """Without label output, thresholds that add no edge copy the previous
    threshold's statistics: duplicated thresholds, an empty top of the grid,
    planted classes (ARI) and a batch."""
    s, d, n = gg.rmat(14, seed=31)
    compare(gpu_sweep(s, d, n, oracle.TECTONIC, GRID16, want_labels=False),
            oracle_sweep(s, d, n, oracle.TECTONIC, GRID16))
    s, d, n = gg.rmat(12, seed=32)
    deltas = [(0, 1), (-10, 1), (3, 2), (-10, 1), (-40, 3), (7, 1), (-1, 1), (7, 1), (50, 1)]
    compare(gpu_sweep(s, d, n, oracle.TW, deltas, want_labels=False), oracle_sweep(s, d, n, oracle.TW, deltas))
    c1 = gg.sbm_c1()
    args = (c1["src"], c1["dst"], c1["n"], oracle.TECTONIC, GRID64[:60] + [(1, 1), (1, 1), (2, 1)], c1["truth"])
    compare(gpu_sweep(*args, want_labels=False), oracle_sweep(*args))
    src, dst, N, truth, vbase = small_sbm_batch()
    args = (src, dst, N, oracle.TECTONIC, GRID16 + [(15, 50)], truth, vbase)
    compare(gpu_sweep(*args, want_labels=False), oracle_sweep(*args))


def test_sweep_tw_unsorted_duplicates():
    s, d, n = gg.rmat(12, seed=32)
    deltas = [(0, 1), (-10, 1), (3, 2), (-10, 1), (-40, 3), (7, 1), (-1, 1)]
    compare(gpu_sweep(s, d, n, oracle.TW, deltas), oracle_sweep(s, d, n, oracle.TW, deltas))


def test_sweep_sbm_planted_ari():
    c1 = gg.sbm_c1()
    args = (c1["src"], c1["dst"], c1["n"], oracle.TECTONIC, GRID64, c1["truth"])
    compare(gpu_sweep(*args), oracle_sweep(*args))


def small_sbm_batch():
    """Six planted-partition graphs of the batch distribution (at most 3000
    vertices each) as one disjoint union: src, dst, n, truth, vbase."""
    graphs = []
    for g in range(6):
        pr = gg.sbm_batch_params(g)
        n = min(pr["n"], 3000)
        k = min(pr["k"], n // 4)
        src, dst, lab = gg.sbm_skip(n, k, min(pr["d_in"] / (n / k - 1), 0.5),
                                    pr["mu"] * pr["d_in"] / ((1 - pr["mu"]) * n), 1000 + g)
        graphs.append((n, src, dst, lab))
    vbase = np.zeros(len(graphs) + 1, np.int64)
    srcs, dsts, truths = [], [], []
    cbase = 0
    for i, (n, src, dst, lab) in enumerate(graphs):
        vbase[i + 1] = vbase[i] + n
        srcs.append(src + vbase[i])
        dsts.append(dst + vbase[i])
        truths.append(lab + cbase)
        cbase += int(lab.max()) + 1
    N = int(vbase[-1])
    src = np.concatenate(srcs).astype(np.int32)
    dst = np.concatenate(dsts).astype(np.int32)
    truth = np.concatenate(truths).astype(np.int32)
    return src, dst, N, truth, vbase


def test_sweep_batch_of_sbms():
    src, dst, N, truth, vbase = small_sbm_batch()
    args = (src, dst, N, oracle.TECTONIC, GRID64, truth, vbase)
    want = oracle_sweep(*args)
    for _ in range(3):  # repeated runs must agree exactly (surfaces races)
        compare(gpu_sweep(*args), want)


def test_sweep_matches_single_threshold_pipeline():
    # every sweep slot equals prune + components at that threshold alone
    from gpu_util import build
    s, d, n = gg.rmat(13, seed=33)
    g = build(s, d, n)
    t = M.mcd_triangles(g)
    stats, _, labels = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, GRID16, want_labels=True)
    for k, delta in enumerate(GRID16):
        keep, nk = M.mcd_prune(g, M.MCD_SIM_TECTONIC, t, delta)
        lab, ncc = M.mcd_components(g, keep)
        torch.cuda.synchronize()
        assert torch.equal(lab, labels[k, :n])
        assert int(ncc.item()) == int(stats[0, k, 1].item())
        assert int(nk.item()) == int(stats[0, k, 0].item())


def test_sweep_k3_and_jaccard():
    s, d, n = gg.rmat(13, seed=34)
    k3 = [(k, 1) for k in (0, 1, 2, 3, 5, 8, 13, 40)]
    compare(gpu_sweep(s, d, n, oracle.K3, k3), oracle_sweep(s, d, n, oracle.K3, k3))
    jac = [(k, 100) for k in range(0, 60, 4)]
    compare(gpu_sweep(s, d, n, oracle.JACCARD, jac), oracle_sweep(s, d, n, oracle.JACCARD, jac))


def test_sweep_modularity_and_rule_of_thumb():
    # modularity per threshold bit-exact in its integers and within 1e-12 in Q,
    # then the rule of thumb picks the same slots as the oracle's
    from gpu_util import build
    graphs = []
    for g in range(5):
        pr = gg.sbm_batch_params(g + 20)
        n = min(pr["n"], 2500)
        k = min(pr["k"], n // 4)
        src, dst, lab = gg.sbm_skip(n, k, min(pr["d_in"] / (n / k - 1), 0.5),
                                    pr["mu"] * pr["d_in"] / ((1 - pr["mu"]) * n), 2000 + g)
        graphs.append((n, src, dst, lab))
    vbase = np.zeros(len(graphs) + 1, np.int64)
    srcs, dsts, truths, cb = [], [], [], 0
    for i, (n, src, dst, lab) in enumerate(graphs):
        vbase[i + 1] = vbase[i] + n
        srcs.append(src + vbase[i])
        dsts.append(dst + vbase[i])
        truths.append(lab + cb)
        cb += int(lab.max()) + 1
    N = int(vbase[-1])
    src = np.concatenate(srcs).astype(np.int32)
    dst = np.concatenate(dsts).astype(np.int32)
    truth = np.concatenate(truths).astype(np.int32)
    deltas = GRID64[::3] + [(1, 2), (0, 1)]  # unsorted tail, a zero threshold
    g = build(src, dst, N)
    t = M.mcd_triangles(g)
    vb = torch.from_numpy(vbase).cuda()
    stats, ari, _, q = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, deltas, vbase=vb,
                                   truth=torch.from_numpy(truth).cuda(), want_modularity=True)
    lo, hi = oracle.canon(N, src, dst)
    deg = oracle.degrees(N, lo, hi)
    to = oracle.triangles(N, lo, hi)
    st_o, ari_o, _, q_o = oracle.sweep(N, lo, hi, to, deg, oracle.TECTONIC, deltas, truth, vbase, modularity=True)
    assert np.array_equal(stats.cpu().numpy(), st_o)
    assert np.all(np.abs(q.cpu().numpy() - q_o) <= 1e-12)
    for jump in ((1, 10), (1, 2), (1, 1000)):
        for with_q in (True, False):
            idx, dl = M.mcd_sweep_rule(g.ctx, deltas, stats, q if with_q else None, vbase=vb, jump=jump)
            want = oracle.rule_of_thumb(st_o, deltas, vbase, q_o if with_q else None, jump)
            assert np.array_equal(idx.cpu().numpy(), want), (jump, with_q)
            assert np.array_equal(dl.cpu().numpy(), np.array([deltas[k] for k in want], np.int64))


def test_sweep_precision_recall_f1():
    from gpu_util import build
    graphs = []
    for g in range(4):
        pr = gg.sbm_batch_params(g + 40)
        n = min(pr["n"], 2000)
        k = min(pr["k"], n // 4)
        src, dst, lab = gg.sbm_skip(n, k, min(pr["d_in"] / (n / k - 1), 0.5),
                                    pr["mu"] * pr["d_in"] / ((1 - pr["mu"]) * n), 3000 + g)
        graphs.append((n, src, dst, lab))
    vbase = np.zeros(len(graphs) + 1, np.int64)
    srcs, dsts, truths, cb = [], [], [], 0
    for i, (n, src, dst, lab) in enumerate(graphs):
        vbase[i + 1] = vbase[i] + n
        srcs.append(src + vbase[i])
        dsts.append(dst + vbase[i])
        truths.append(lab + cb)
        cb += int(lab.max()) + 1
    N = int(vbase[-1])
    src = np.concatenate(srcs).astype(np.int32)
    dst = np.concatenate(dsts).astype(np.int32)
    truth = np.concatenate(truths).astype(np.int32)
    deltas = GRID64[::5]
    g = build(src, dst, N)
    t = M.mcd_triangles(g)
    stats, ari, labels, _, prf = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, deltas, vbase=torch.from_numpy(vbase).cuda(),
                                             truth=torch.from_numpy(truth).cuda(), want_labels=True, want_prf=True)
    labels, prf = labels.cpu().numpy()[:, :N], prf.cpu().numpy()
    lo, hi = oracle.canon(N, src, dst)
    deg = oracle.degrees(N, lo, hi)
    to = oracle.triangles(N, lo, hi)
    _, _, labels_o = oracle.sweep(N, lo, hi, to, deg, oracle.TECTONIC, deltas, truth, vbase)
    assert np.array_equal(labels, labels_o)
    for i in range(len(deltas)):
        for gk in range(len(graphs)):
            a, b = vbase[gk], vbase[gk + 1]
            want = oracle.precision_recall_f1(labels_o[i, a:b], truth[a:b])
            assert np.all(np.abs(prf[gk, i] - np.array(want)) <= 1e-12 * np.maximum(1.0, np.abs(want))), (i, gk)


def test_imbalanced_sbm_tw_vs_tectonic():
    # the two-block study on the GPU: both sweeps equal the oracle's, and the
    # GPU's ARIs show the paper's outcome (TW recovers the blocks, Tectonic not)
    b = gg.sbm_two_blocks_batch(20)
    tw_grid = [(k, 1) for k in range(-50, 14)]
    got_tw = gpu_sweep(b["src"], b["dst"], b["n"], M.MCD_SIM_TW, tw_grid, b["truth"], b["vbase"])
    compare(got_tw, oracle_sweep(b["src"], b["dst"], b["n"], oracle.TW, tw_grid, b["truth"], b["vbase"]))
    got_te = gpu_sweep(b["src"], b["dst"], b["n"], M.MCD_SIM_TECTONIC, GRID64, b["truth"], b["vbase"])
    compare(got_te, oracle_sweep(b["src"], b["dst"], b["n"], oracle.TECTONIC, GRID64, b["truth"], b["vbase"]))
    best_tw, best_te = got_tw[1].max(1), got_te[1].max(1)
    assert np.all(best_tw >= best_te) and best_tw.mean() > 0.95 and best_te.mean() < 0.8
