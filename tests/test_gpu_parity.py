"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer products (edges, degrees, triangle counts, TW, keep masks, labels,
component counts, percentile thresholds) must be bit-exact; fp32 Tectonic
weights must be the oracle's fp64 value rounded to fp32, bit for bit (the
target's bound is 1e-6 relative).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

M = pytest.importorskip("paper_2412_12382_amd.mcd")


def check_all(src, dst, n, measure, delta):
    from gpu_util import gpu_all
    r = gpu_all(src, dst, n, measure, delta)
    lo, hi = oracle.canon(n, src, dst)
    assert r["g"].m == len(lo)
    assert np.array_equal(r["lo"], lo) and np.array_equal(r["hi"], hi)
    deg = oracle.degrees(n, lo, hi)
    assert np.array_equal(r["deg"], deg)
    if len(lo):
        assert r["g"].max_deg == deg.max()
    t = oracle.triangles(n, lo, hi)
    assert np.array_equal(r["t"], t)
    if measure in (oracle.TECTONIC, oracle.JACCARD):
        w = (oracle.tectonic if measure == oracle.TECTONIC else oracle.jaccard)(lo, hi, t, deg)
        # the bound is 1e-6 relative; both sides form the same rounding of the
        # exact quotient (fp32 division of 24-bit integers, equal to the fp64
        # quotient rounded to fp32), so the values must be identical
        assert np.all(np.abs(r["w"].astype(np.float64) - w) <= 1e-6 * np.abs(w))
        assert np.array_equal(r["w"].view(np.int32), w.astype(np.float32).view(np.int32))
    else:
        tw = oracle.tw(lo, hi, t, deg) if measure == oracle.TW else t.astype(np.int64)
        assert np.array_equal(r["tw"].astype(np.int64), tw)
        assert np.array_equal(r["w"].astype(np.float64), tw.astype(np.float64))
    keep = oracle.prune(measure, lo, hi, t, deg, *delta)
    assert np.array_equal(r["keep"], keep)
    assert r["n_kept"] == int(keep.sum())
    labels, ncc = oracle.components(n, lo, hi, keep)
    assert np.array_equal(r["labels"], labels) and r["ncc"] == ncc
    assert np.array_equal(r["labels_run"], labels) and r["ncc_run"] == ncc
    f = r["fused"]  # one-pass weights + prune, kept list, components over it
    assert np.array_equal(f["w"].view(np.int32), r["w"].view(np.int32))
    if measure in (oracle.TW, oracle.K3):
        assert np.array_equal(f["tw"], r["tw"])
    assert np.array_equal(f["keep"], keep) and f["n_kept"] == int(keep.sum())
    assert np.array_equal(f["kept_u"], f["want_u"]) and np.array_equal(f["kept_v"], f["want_v"])
    assert np.array_equal(f["labels"], labels) and f["ncc"] == ncc
    p = r["pc"]  # weights + prune + components in one pass
    assert np.array_equal(p["w"].view(np.int32), r["w"].view(np.int32))
    if measure in (oracle.TW, oracle.K3):
        assert np.array_equal(p["tw"], r["tw"])
    assert np.array_equal(p["keep"], keep) and p["n_kept"] == int(keep.sum())
    assert np.array_equal(p["labels"], labels) and p["ncc"] == ncc
    return r


def test_c1_sbm_tectonic():
    c1 = gg.sbm_c1()
    check_all(c1["src"], c1["dst"], c1["n"], oracle.TECTONIC, (3, 50))


def test_c1_sbm_tw():
    c1 = gg.sbm_c1()
    check_all(c1["src"], c1["dst"], c1["n"], oracle.TW, (-20, 1))


@pytest.mark.parametrize("seed", range(6))
def test_small_random_graphs(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 300))
    P = int(rng.integers(0, 6 * n))
    src = rng.integers(0, n, P).astype(np.int32)
    dst = rng.integers(0, n, P).astype(np.int32)
    check_all(src, dst, n, seed % 2, (1, 7) if seed % 2 == 0 else (-3, 2))


def test_degenerate_inputs():
    # no pairs; only self-loops; a single edge; duplicates in both directions
    check_all(np.zeros(0, np.int32), np.zeros(0, np.int32), 5, oracle.TECTONIC, (0, 1))
    check_all(np.arange(4, dtype=np.int32), np.arange(4, dtype=np.int32), 4, oracle.TECTONIC, (1, 3))
    check_all(np.array([1], np.int32), np.array([0], np.int32), 2, oracle.TW, (0, 1))
    s = np.array([0, 1, 1, 2, 0, 2, 2], np.int32)
    d = np.array([1, 0, 2, 1, 2, 0, 0], np.int32)
    check_all(s, d, 3, oracle.TECTONIC, (1, 4))
    check_all(s, d, 1 << 12, oracle.TECTONIC, (1, 4))  # mostly isolated vertices


def test_every_edge_kept_components():
    """A threshold of at most 0 keeps every edge of the nonnegative measures;
    mcd_prune_components then unites vertex by vertex around a sampled large
    component: two R-MAT graphs side by side (two large components, only one
    passed over), isolated vertices, K3/Jaccard/Tectonic, thresholds 0 and
    below; and a graph whose vertices all have degree 1 or 0."""
    s1, d1, n1 = gg.rmat(12, seed=61)
    s2, d2, n2 = gg.rmat(13, seed=62)
    s = np.concatenate([s1, s2 + n1]).astype(np.int32)
    d = np.concatenate([d1, d2 + n1]).astype(np.int32)
    n = n1 + n2 + 50
    check_all(s, d, n, oracle.TECTONIC, (0, 1))
    check_all(s, d, n, oracle.K3, (-3, 2))
    check_all(s, d, n, oracle.JACCARD, (0, 7))
    m = np.arange(0, 2000, 2, dtype=np.int32)
    check_all(m, m + 1, 2001, oracle.TECTONIC, (0, 1))


def test_invalid_vertex_rejected():
    from gpu_util import build
    with pytest.raises(M.MCDError) as ei:
        build(np.array([0, 5], np.int32), np.array([1, 2], np.int32), 5)
    assert ei.value.status == -2
    with pytest.raises(M.MCDError) as ei:
        build(np.array([0, -1], np.int32), np.array([1, 2], np.int32), 5)
    assert ei.value.status == -2


@pytest.mark.parametrize("scale", [12, 16])
def test_rmat_both_measures(scale):
    s, d, n = gg.rmat(scale, seed=scale)
    check_all(s, d, n, oracle.TECTONIC, (1, 20))
    check_all(s, d, n, oracle.TW, (-10, 1))


def test_rmat_percentile_thresholds():
    from gpu_util import build
    s, d, n = gg.rmat(14, seed=1)
    lo, hi = oracle.canon(n, s, d)
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    g = build(s, d, n)
    tg = M.mcd_triangles(g)
    for measure in (oracle.TECTONIC, oracle.TW, oracle.K3, oracle.JACCARD):
        for pn, pd in ((3, 10), (1, 2), (1, 1), (1, 1000), (0, 1)):
            want = Fraction(*oracle.percentile(measure, lo, hi, t, deg, pn, pd))
            num, den = M.mcd_percentile_threshold(g, measure, tg, pn, pd)
            assert Fraction(num, den) == want, (measure, pn, pd, num, den, want)
            assert math.gcd(num, den) == 1 and den > 0


def test_percentile_empty():
    from gpu_util import build
    s = np.array([0, 2, 4], np.int32)
    d = np.array([1, 3, 5], np.int32)  # a matching: every t = 0
    g = build(s, d, 6)
    t = M.mcd_triangles(g)
    with pytest.raises(M.MCDError) as ei:
        M.mcd_percentile_threshold(g, oracle.TECTONIC, t, 3, 10)
    assert ei.value.status == -8


def test_repeat_runs_bit_identical():
    from gpu_util import build, unpack_bits
    s, d, n = gg.rmat(15, seed=4)
    g = build(s, d, n)
    outs = []
    for _ in range(3):
        t = M.mcd_triangles(g)
        keep, _ = M.mcd_prune(g, oracle.TECTONIC, t, (1, 25))
        lab, ncc = M.mcd_components(g, keep)
        pc = M.mcd_prune_components(g, oracle.TECTONIC, t, delta=(1, 25), want_f32=False)
        k4 = M.mcd_k4(g)
        torch.cuda.synchronize()
        outs.append((t.cpu().numpy().copy(), unpack_bits(keep, g.m), lab.cpu().numpy().copy(),
                     pc["labels"].cpu().numpy().copy(), k4.cpu().numpy().copy()))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("chunk,lds_max,packed,window,occ", [(512, 4096, 1048574, 262144, 0), (1, 4096, 1048574, 0, 0),
                                                             (7, 100, 0, 0, 0), (64, 0, 1048574, 262144, 0),
                                                             (3, 600, 5000, 5000, 0), (100000, 2048, 0, 0, 0),
                                                             (512, 4096, 0, 0, 0), (5, 4096, 1048574, 16384, 0),
                                                             (9, 4096, 1048574, 65536, 0),
                                                             (512, 4096, 1048574, 262144, 1),
                                                             (5, 4096, 1048574, 16384, 1),
                                                             (9, 4096, 1048574, 65536, 1)])
def test_triangle_paths_and_chunks(chunk, lds_max, packed, window, occ):
    # every launch configuration (work-item size, LDS classes vs binary search,
    # the rank-window kernels' register budget) must give the oracle's counts
    from gpu_util import ctx, build
    s, d, n = gg.rmat(15, seed=21)
    lo, hi = oracle.canon(n, s, d)
    t_o = oracle.triangles(n, lo, hi)
    c = ctx()
    names = ("tc_chunk", "tc_lds_max", "tc_packed_range", "tc_window_max", "tc_window_occupancy")
    old = [M.mcd_ctx_get_param(c, k) for k in names]
    try:
        for k, val in zip(names, (chunk, lds_max, packed, window, occ)):
            M.mcd_ctx_set_param(c, k, val)
        from gpu_util import canonical_order
        g = build(s, d, n)
        _, _, order = canonical_order(g)
        t = M.mcd_triangles(g).cpu().numpy()[order]
        assert np.array_equal(t, t_o)
    finally:
        for k, val in zip(names, old):
            M.mcd_ctx_set_param(c, k, val)


@pytest.mark.parametrize("occ", [1, 0])
def test_triangles_past_the_16_bit_rank_range(occ):
    # with more than 65,536 vertices the rank-window items of the top 65,536
    # ranks read their suffixes from the 16-bit copy of the adjacency and the
    # others from the 32-bit one: both must give the oracle's counts
    from gpu_util import ctx, build, canonical_order
    s, d, n = gg.rmat(17, seed=5)
    assert n > 65536
    lo, hi = oracle.canon(n, s, d)
    t_o = oracle.triangles(n, lo, hi)
    c = ctx()
    old = M.mcd_ctx_get_param(c, "tc_window_occupancy")
    try:
        M.mcd_ctx_set_param(c, "tc_window_occupancy", occ)
        g = build(s, d, n)
        _, _, order = canonical_order(g)
        t = M.mcd_triangles(g).cpu().numpy()[order]
        assert np.array_equal(t, t_o)
    finally:
        M.mcd_ctx_set_param(c, "tc_window_occupancy", old)


def test_triangles_rank_windows_below_the_top_ranks():
    # two dense random blocks, the lighter one ranked entirely below the top
    # 65,536 ranks: its vertices are rank-window items read through the 32-bit
    # adjacency (windows of 2^16 and 2^18 ranks), the heavier block's top part
    # through the 16-bit copy
    from gpu_util import build, canonical_order
    rng = np.random.default_rng(1234)
    na, nb = 40000, 70000
    ea, eb = na * 300 // 2, nb * 400 // 2
    s = np.concatenate([rng.integers(0, na, ea), na + rng.integers(0, nb, eb)]).astype(np.int32)
    d = np.concatenate([rng.integers(0, na, ea), na + rng.integers(0, nb, eb)]).astype(np.int32)
    n = na + nb
    lo, hi = oracle.canon(n, s, d)
    t_o = oracle.triangles(n, lo, hi)
    g = build(s, d, n)
    _, _, order = canonical_order(g)
    t = M.mcd_triangles(g).cpu().numpy()[order]
    assert np.array_equal(t, t_o)


@pytest.mark.parametrize("measure,delta", [(oracle.TECTONIC, (1, 20)), (oracle.TW, (-5, 1))])
def test_prune_components_aligned_and_unaligned_inputs(measure, delta):
    # the fused pass with a host and with a device threshold (separate
    # kernel builds), on inputs and outputs at and off 16-byte boundaries,
    # must give the oracle's results
    from gpu_util import build, canonical_order, unpack_bits
    s, d, n = gg.rmat(14, seed=31)
    lo, hi = oracle.canon(n, s, d)
    t_o = oracle.triangles(n, lo, hi)
    deg = oracle.degrees(n, lo, hi)
    keep_o = oracle.prune(measure, lo, hi, t_o, deg, *delta)
    labels_o, ncc_o = oracle.components(n, lo, hi, keep_o)
    g = build(s, d, n)
    _, _, order = canonical_order(g)
    t = M.mcd_triangles(g)
    tw = measure == oracle.TW
    dev_delta = torch.tensor([list(delta)], dtype=torch.int64, device="cuda")
    for shift in (0, 1):
        buf = torch.zeros(g.m + 4, dtype=torch.int32, device="cuda")
        tt = buf[shift:shift + g.m]
        tt.copy_(t)
        wbuf = torch.zeros(g.m + 4, dtype=torch.int32 if tw else torch.float32, device="cuda")
        wout = wbuf[shift:shift + g.m]
        for kw in (dict(delta=delta), dict(deltas=dev_delta)):
            r = M.mcd_prune_components(g, measure, tt, w_i32=wout if tw else None, w_f32=None if tw else wout,
                                       want_f32=not tw, want_i32=tw, **kw)
            keep = unpack_bits(r["keep_bits"], g.m)[order]
            assert np.array_equal(keep, keep_o), (shift, kw)
            assert int(r["n_kept"].item()) == int(keep_o.sum())
            assert np.array_equal(r["labels"].cpu().numpy(), labels_o) and int(r["n_components"].item()) == ncc_o
            w = wout.cpu().numpy()[order]
            if tw:
                assert np.array_equal(w.astype(np.int64), oracle.tw(lo, hi, t_o, deg))
            else:
                w_o = oracle.tectonic(lo, hi, t_o, deg)
                assert np.array_equal(w.view(np.int32), w_o.astype(np.float32).view(np.int32))


def test_triangles_at_odd_word_offset():
    # t need only be 4-byte aligned: an output array starting 4 bytes into
    # an 8-byte word gives the same counts and nothing outside it is written
    from gpu_util import build, canonical_order
    s, d, n = gg.rmat(15, seed=22)
    lo, hi = oracle.canon(n, s, d)
    t_o = oracle.triangles(n, lo, hi)
    g = build(s, d, n)
    _, _, order = canonical_order(g)
    for shift in (0, 1):
        buf = torch.full((g.m + 2,), -5, dtype=torch.int32, device="cuda")
        t = M.mcd_triangles(g, buf[shift:])
        assert np.array_equal(t.cpu().numpy()[order], t_o), shift
        rest = buf.cpu().numpy()
        assert np.all(rest[:shift] == -5) and np.all(rest[shift + g.m:] == -5), shift  # nothing outside t


def test_param_validation():
    from gpu_util import ctx
    c = ctx()
    for name, bad in (("tc_chunk", 0), ("tc_lds_max", 5000), ("tc_lds_max", -1),
                      ("tc_packed_range", 1 << 20), ("tc_window_max", (1 << 18) + 1), ("k4_row_cache", 2),
                      ("tc_window_occupancy", 2), ("sweep_shape", 3)):
        with pytest.raises(M.MCDError) as ei:
            M.mcd_ctx_set_param(c, name, bad)
        assert ei.value.status == -3
    with pytest.raises(M.MCDError) as ei:
        M.mcd_ctx_set_param(c, "no_such_param", 1)
    assert ei.value.status == -1


def test_workspace_alignment_checked():
    # a workspace or storage buffer off a 256-byte boundary is refused before
    # any work is enqueued; the aligned buffer still works
    from gpu_util import build
    s, d, n = gg.rmat(10, seed=5)
    g = build(s, d, n)
    ws = torch.empty(M.mcd_triangles_workspace_size(g) + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MCDError) as ei:
        M.mcd_triangles(g, ws=ws[8:])
    assert ei.value.status == -1 and "aligned" in M.mcd_last_error()
    t = M.mcd_triangles(g, ws=ws)
    wc = torch.empty(M.mcd_components_workspace_size(g) + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MCDError):
        M.mcd_prune_components(g, M.MCD_SIM_TECTONIC, t, delta=(1, 10), ws=wc[64:])
    st_b, ws_b = M.mcd_graph_build_sizes(len(s), n)
    storage = torch.empty(st_b + 256, dtype=torch.uint8, device="cuda")
    wsb = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MCDError):
        M.mcd_graph_build(g.ctx, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), n, storage=storage[4:],
                          ws=wsb)


@pytest.mark.parametrize("k", [5, 130, 700])
def test_complete_graph_closed_form(k):
    # K_k: every edge lies in k-2 triangles (rows longer than the small LDS classes)
    from gpu_util import build
    i, j = np.triu_indices(k, 1)
    g = build(i.astype(np.int32), j.astype(np.int32), k)
    t = M.mcd_triangles(g).cpu().numpy()
    assert g.m == k * (k - 1) // 2 and np.all(t == k - 2)
    assert g.max_outdeg == k - 1


@pytest.mark.parametrize("packed,occ", [(1048574, 1), (0, 1), (1048574, 0), (0, 0)])
def test_triangles_long_hash_rows(packed, occ):
    """Rows of 129 to 4096 entries in LDS hash tables (the rank windows
    switched off), packed and wide entries, both register budgets: a 1500-
    clique (rows of up to 1499: k - 2 triangles on every edge) beside an
    R-MAT graph (oracle counts), in one graph."""
    from gpu_util import ctx, build, canonical_order
    k = 1500
    i, j = np.triu_indices(k, 1)
    s2, d2, n2 = gg.rmat(12, seed=91)
    s = np.concatenate([i, s2 + k]).astype(np.int32)
    d = np.concatenate([j, d2 + k]).astype(np.int32)
    n = k + n2
    lo2, hi2 = oracle.canon(n2, s2, d2)
    want = np.concatenate([np.full(k * (k - 1) // 2, k - 2, np.int32), oracle.triangles(n2, lo2, hi2)])
    c = ctx()
    names = ("tc_chunk", "tc_lds_max", "tc_packed_range", "tc_window_max", "tc_window_occupancy")
    old = [M.mcd_ctx_get_param(c, x) for x in names]
    try:
        for x, val in zip(names, (300, 4096, packed, 0, occ)):
            M.mcd_ctx_set_param(c, x, val)
        g = build(s, d, n)
        assert g.max_outdeg >= k - 1
        _, _, order = canonical_order(g)
        t = M.mcd_triangles(g).cpu().numpy()[order]
        assert np.array_equal(t, want)
    finally:
        for x, val in zip(names, old):
            M.mcd_ctx_set_param(c, x, val)


def test_autotuner_sets_params_and_keeps_counts():
    from gpu_util import build, canonical_order
    s, d, n = gg.rmat(14, seed=41)
    g = build(s, d, n)
    t0 = M.mcd_triangles(g).clone()
    best, ms = M.mcd_tune_triangles(g, reps=1)
    assert ms > 0
    assert best["tc_chunk"] in (256, 512, 1024, 2048)
    assert best["tc_lds_max"] in (1024, 2048, 4096)
    assert best["tc_window_max"] in (0, 1 << 14, 1 << 16, 1 << 18)
    for k, v in best.items():
        assert M.mcd_ctx_get_param(g.ctx, k) == v
    t1 = M.mcd_triangles(g)
    assert torch.equal(t0, t1)
    lo, hi, order = canonical_order(g)
    assert np.array_equal(t1.cpu().numpy()[order], oracle.triangles(n, lo, hi))
    # restore the defaults for later tests sharing the context
    for k, v in (("tc_chunk", 512), ("tc_lds_max", 4096), ("tc_packed_range", (1 << 20) - 2),
                 ("tc_window_max", 1 << 18)):
        M.mcd_ctx_set_param(g.ctx, k, v)


def test_tune_cache_round_trip(tmp_path):
    """Parameters stored for a graph come back on a graph of the same size
    bucket, not on another; a corrupt file is refused and changes nothing."""
    from gpu_util import build
    import json
    path = str(tmp_path / "tune.json")
    s, d, n = gg.rmat(12, seed=43)
    g = build(s, d, n)
    names = ("tc_chunk", "tc_lds_max", "tc_packed_range", "tc_window_max", "tc_window_occupancy", "sweep_shape")
    saved = {k: M.mcd_ctx_get_param(g.ctx, k) for k in names}
    chosen = {"tc_chunk": 300, "tc_lds_max": 2048, "tc_packed_range": 5000, "tc_window_max": 1 << 16,
              "tc_window_occupancy": 0, "sweep_shape": 2}
    try:
        assert not M.mcd_tune_cache_load(g, path)  # no file yet: a miss
        for k, v in chosen.items():
            M.mcd_ctx_set_param(g.ctx, k, v)
        M.mcd_tune_cache_store(g, path, 1.5)
        s2, d2, n2 = gg.rmat(15, seed=44)
        g2 = build(s2, d2, n2)
        M.mcd_ctx_set_param(g.ctx, "tc_chunk", 700)
        M.mcd_tune_cache_store(g2, path, 2.5)  # a second entry, other size bucket
        M.mcd_tune_cache_check_file(path)
        doc = json.load(open(path))
        assert len(doc["entries"]) == 2
        for k, v in saved.items():
            M.mcd_ctx_set_param(g.ctx, k, v)
        assert M.mcd_tune_cache_load(g, path)
        assert {k: M.mcd_ctx_get_param(g.ctx, k) for k in names} == chosen
        assert M.mcd_tune_cache_load(g2, path)
        assert M.mcd_ctx_get_param(g.ctx, "tc_chunk") == 700
        s3, d3, n3 = gg.rmat(10, seed=45)
        assert not M.mcd_tune_cache_load(build(s3, d3, n3), path)
        # a refused value: nothing is set
        doc["entries"][0]["params"]["tc_window_max"] = 1 << 20
        json.dump(doc, open(path, "w"))
        before = {k: M.mcd_ctx_get_param(g.ctx, k) for k in names}
        with pytest.raises(M.MCDError) as ei:
            M.mcd_tune_cache_load(g, path)
        assert ei.value.status == -9
        assert {k: M.mcd_ctx_get_param(g.ctx, k) for k in names} == before
    finally:
        for k, v in saved.items():
            M.mcd_ctx_set_param(g.ctx, k, v)


@pytest.mark.parametrize("scale", [12, 15])
def test_rmat_k3_and_jaccard(scale):
    s, d, n = gg.rmat(scale, seed=100 + scale)
    check_all(s, d, n, oracle.K3, (2, 1))
    check_all(s, d, n, oracle.JACCARD, (1, 20))


def test_c1_sbm_k3_and_jaccard():
    c1 = gg.sbm_c1()
    check_all(c1["src"], c1["dst"], c1["n"], oracle.K3, (4, 1))
    check_all(c1["src"], c1["dst"], c1["n"], oracle.JACCARD, (3, 47))


def test_prop1_on_the_gpu():
    # Proposition 1: the GPU's Jaccard-prune at p/q and Tectonic-prune at
    # p/(p+q) produce the same keep bits
    from gpu_util import build
    s, d, n = gg.rmat(14, seed=77)
    g = build(s, d, n)
    t = M.mcd_triangles(g)
    words = (g.m + 31) // 32
    for p, q in ((1, 20), (1, 9), (1, 3), (2, 5), (1, 1), (0, 1), (7, 93)):
        kj, nj = M.mcd_prune(g, M.MCD_SIM_JACCARD, t, (p, q))
        kt, nt = M.mcd_prune(g, M.MCD_SIM_TECTONIC, t, (p, p + q))
        assert torch.equal(kj[:words], kt[:words]) and int(nj.item()) == int(nt.item())


@pytest.mark.parametrize("case", ["c1", "rmat12", "rmat14", "rmat16", "k9", "random", "k300_rmat12"])
def test_k4_participation_and_prune(case):
    from gpu_util import build, canonical_order, unpack_bits
    if case == "c1":
        c1 = gg.sbm_c1()
        s, d, n = c1["src"], c1["dst"], c1["n"]
    elif case.startswith("rmat"):
        s, d, n = gg.rmat(int(case[4:]), seed=70)
    elif case == "k300_rmat12":
        # a 300-clique (rows of up to 299 edges: the LDS path) beside an
        # R-MAT graph, joined by random cross pairs
        k = 300
        pairs = [(i, j) for i in range(k) for j in range(i + 1, k)]
        s2, d2, n2 = gg.rmat(12, seed=5)
        rng = np.random.default_rng(3)
        s = np.concatenate([np.array([p[0] for p in pairs], np.int32), s2 + k,
                            rng.integers(0, k, 3000).astype(np.int32)])
        d = np.concatenate([np.array([p[1] for p in pairs], np.int32), d2 + k,
                            (k + rng.integers(0, n2, 3000)).astype(np.int32)])
        n = k + n2
    elif case == "k9":
        pairs = [(i, j) for i in range(9) for j in range(i + 1, 9)]
        s = np.array([p[0] for p in pairs], np.int32)
        d = np.array([p[1] for p in pairs], np.int32)
        n = 9
    else:
        rng = np.random.default_rng(71)
        n = 400
        s = rng.integers(0, n, 12000).astype(np.int32)
        d = rng.integers(0, n, 12000).astype(np.int32)
    g = build(s, d, n)
    lo, hi, order = canonical_order(g)
    k4 = M.mcd_k4(g)
    want = oracle.k4(n, lo, hi)
    assert np.array_equal(k4.cpu().numpy()[order], want)
    if M.mcd_graph_info(g)["max_outdeg"] > 256:
        # the long-row kernel also without the row offsets kept in LDS
        from gpu_util import ctx
        c = ctx()
        M.mcd_ctx_set_param(c, "k4_row_cache", 0)
        try:
            assert np.array_equal(M.mcd_k4(g).cpu().numpy()[order], want)
        finally:
            M.mcd_ctx_set_param(c, "k4_row_cache", 1)
    if case == "k9":
        assert np.all(want == 21)  # C(7, 2)
    deg = oracle.degrees(n, lo, hi)
    thr = (max(1, int(np.median(want))), 1)
    keep, nk = M.mcd_prune(g, M.MCD_SIM_K4, k4, thr)
    keep_o = oracle.prune(oracle.K4, lo, hi, want, deg, *thr)
    assert np.array_equal(unpack_bits(keep, g.m)[order], keep_o)
    lab, ncc = M.mcd_components(g, keep)
    lab_o, ncc_o = oracle.components(n, lo, hi, keep_o)
    assert np.array_equal(lab.cpu().numpy(), lab_o) and int(ncc.item()) == ncc_o
    pc = M.mcd_prune_components(g, M.MCD_SIM_K4, k4, delta=thr, want_i32=True)
    assert np.array_equal(pc["w_i32"].cpu().numpy()[order], want)
    assert np.array_equal(unpack_bits(pc["keep_bits"], g.m)[order], keep_o)
    assert np.array_equal(pc["labels"].cpu().numpy(), lab_o) and int(pc["n_components"].item()) == ncc_o


def test_device_threshold_one_graph_any_width():
    # a device threshold for a single graph, with terms that need the 128-bit
    # comparison and with small ones, decides exactly as the host threshold
    from gpu_util import build
    s, d, n = gg.rmat(14, seed=78)
    g = build(s, d, n)
    t = M.mcd_triangles(g)
    words = (g.m + 31) // 32
    for measure, (p, q) in ((M.MCD_SIM_TECTONIC, (3, 50)), (M.MCD_SIM_TW, (-7, 1)), (M.MCD_SIM_JACCARD, (1, 9))):
        want = M.mcd_weigh_prune(g, measure, t, delta=(p, q), want_kept=False)
        wk = want["keep_bits"][:words]
        for scale in (1, 1 << 40):
            dev = torch.tensor([[p * scale, q * scale]], dtype=torch.int64, device="cuda")
            got = M.mcd_weigh_prune(g, measure, t, deltas=dev, want_kept=False)
            assert torch.equal(got["keep_bits"][:words], wk), (measure, scale)
            assert int(got["n_kept"].item()) == int(want["n_kept"].item())
            pc = M.mcd_prune_components(g, measure, t, deltas=dev)
            assert torch.equal(pc["keep_bits"][:words], wk), (measure, scale)
