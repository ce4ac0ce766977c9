"""GPU parity of the learned threshold picker kernels against the float64
reference (oracle.mlp) and the oracle's histogram, prune and components."""
import numpy as np
import pytest
import torch

import graphgen as gg
import mlp_bound as mb
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2412_12382_amd.mcd")


def rand_problem(seed, B):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.NPAR).astype(np.float32)
    x = rng.normal(0, 1, (B, mlp.NI)).astype(np.float32)
    mean = rng.normal(0, 0.1, mlp.NI).astype(np.float32)
    std = rng.uniform(0.5, 2.0, mlp.NI).astype(np.float32)
    target = rng.uniform(0, 1, B).astype(np.float32)
    return p, mean, std, x, target


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_mlp_forward_and_gradient():
    from gpu_util import ctx
    for B in (1, 7, 192):
        p, mean, std, x, target = rand_problem(B, B)
        y = M.mcd_mlp_forward(ctx(), cuda(p), cuda(mean), cuda(std), cuda(x)).cpu().numpy()
        yo, _ = mlp.forward(p.astype(np.float64), mean.astype(np.float64), std.astype(np.float64), x)
        assert np.all(np.abs(y - yo) <= 1e-5 * np.maximum(np.abs(yo), 1.0))
        assert np.all(np.abs(y - yo) <= mb.forward_bound(p, mean, std, x))
        # the gradient on the rows whose ReLU masks are certain on both sides
        # (all but two of the 192): within the a priori bound and within the
        # much tighter empirical tolerance
        keep = mb.rows_with_clear_masks(p, mean, std, x)
        assert keep.sum() >= max(1, B - 2)
        x, target = x[keep], target[keep]
        g, loss = M.mcd_mlp_gradient(ctx(), cuda(p), cuda(mean), cuda(std), cuda(x), cuda(target))
        go, lo = mlp.gradient(p.astype(np.float64), mean.astype(np.float64), std.astype(np.float64), x,
                              target.astype(np.float64))
        g = g.cpu().numpy()
        assert np.all(np.abs(g - go) <= mb.gradient_bound(p, mean, std, x, target))
        tol = mb.empirical_tolerance(go, mb.row_abs_mean(p, mean, std, x, target), len(x))
        assert np.all(np.abs(g - go) <= tol), np.max(np.abs(g - go) / tol)
        assert abs(float(loss.item()) - lo) <= 1e-5 * max(lo, 1.0)


def test_mlp_gradient_with_ari_term():
    # the training loss with the sweep's ARI table: mse_w (y - t)^2 minus the
    # ARI interpolated at 63 y; rows whose 63 y lies within its error bound of
    # a grid point or an end (where the fp32 segment choice could differ), or
    # whose ReLU masks are uncertain, are left out of the batch
    from gpu_util import ctx
    B = 40
    p, mean, std, x, target = rand_problem(9, B)
    p[8448:8512] *= 0.02
    yo, _ = mlp.forward(p.astype(np.float64), mean.astype(np.float64), std.astype(np.float64), x)
    p[8512] += np.float32(0.5 - np.median(yo))
    yo, _ = mlp.forward(p.astype(np.float64), mean.astype(np.float64), std.astype(np.float64), x)
    z, zb = 63 * yo, mb.grid_position_bound(p, mean, std, x, 64)
    keep = (z > zb) & (z < 63 - zb) & (np.abs(z - np.round(z)) > zb)
    keep &= mb.rows_with_clear_masks(p, mean, std, x)
    x, target = x[keep], target[keep]
    assert len(x) >= 10
    ari = np.random.default_rng(10).uniform(-0.1, 1.0, (len(x), 64))
    g, loss = M.mcd_mlp_gradient(ctx(), cuda(p), cuda(mean), cuda(std), cuda(x), cuda(target), ari=cuda(ari),
                                 mse_weight=0.1)
    P64, m64, s64 = p.astype(np.float64), mean.astype(np.float64), std.astype(np.float64)
    go, lo = mlp.gradient(P64, m64, s64, x, target.astype(np.float64), ari, 0.1)
    g = g.cpu().numpy()
    assert np.all(np.abs(g - go) <= mb.gradient_bound(p, mean, std, x, target, ari, 0.1))
    tol = mb.empirical_tolerance(go, mb.row_abs_mean(p, mean, std, x, target, ari, 0.1), len(x))
    assert np.all(np.abs(g - go) <= tol), np.max(np.abs(g - go) / tol)
    assert abs(float(loss.item()) - lo) <= 1e-5 * max(abs(lo), 1.0)


def test_adam_step_matches_reference():
    from gpu_util import ctx
    B, lr = 32, 1e-3
    p, mean, std, x, target = rand_problem(5, B)
    P = cuda(p)
    m1, m2 = torch.zeros_like(P), torch.zeros_like(P)
    M.mcd_mlp_train_step(ctx(), P, m1, m2, 1, lr, cuda(mean), cuda(std), cuda(x), cuda(target))
    go, _ = mlp.gradient(p.astype(np.float64), mean.astype(np.float64), std.astype(np.float64), x,
                         target.astype(np.float64))
    po, _, _ = mlp.adam_step(p.astype(np.float64), 0 * go, 0 * go, go, 1, lr)
    dp = P.cpu().numpy().astype(np.float64) - p
    dpo = po - p
    sel = np.abs(go) > 1e-4  # where the step's direction is well defined
    assert np.all(np.abs(dp[sel] - dpo[sel]) <= 1e-3 * lr + 1e-6 * np.abs(p[sel]))
    # training decreases the loss
    losses = []
    for s in range(2, 200):
        losses.append(float(M.mcd_mlp_train_step(ctx(), P, m1, m2, s, lr, cuda(mean), cuda(std), cuda(x),
                                                 cuda(target)).item()))
    assert losses[-1] < 0.2 * losses[0]


def test_features_batch():
    from gpu_util import build
    b = gg.sbm_batch(5, n_max=3000)
    n, vbase = b["n"], b["vbase"]
    g = build(b["src"], b["dst"], n)
    t = M.mcd_triangles(g)
    x = M.mcd_features(g, t, cuda(vbase)).cpu().numpy()
    lo, hi = oracle.canon(n, b["src"], b["dst"])
    for k in range(5):
        a, c = vbase[k], vbase[k + 1]
        sel = (lo >= a) & (lo < c)
        l2, h2 = (lo[sel] - a).astype(np.int32), (hi[sel] - a).astype(np.int32)
        deg = oracle.degrees(c - a, l2, h2)
        tk = oracle.triangles(c - a, l2, h2)
        xo = mlp.features(c - a, l2, h2, tk, deg)
        assert np.all(np.abs(x[k] - xo) <= 1e-6 * np.maximum(np.abs(xo), 1e-30))


def test_select_targets_and_per_graph_prune():
    from gpu_util import ctx, build, unpack_bits, canonical_order
    y = np.array([-0.3, 0.0, 0.2, 0.49, 0.5, 0.999, 1.5, 31.5 / 63], np.float32)
    idx, d = M.mcd_grid_select(ctx(), cuda(y), 64, 9, 7, 900)
    io, do = mlp.select(y, 64, 9, 7, 900)
    assert np.array_equal(idx.cpu().numpy(), io) and np.array_equal(d.cpu().numpy(), do)
    ari = np.random.default_rng(3).choice([0.1, 0.4, 0.7], (9, 64))
    for frac in (1.0, 0.95, 0.6):
        ti, ty = M.mcd_sweep_targets(ctx(), cuda(ari), frac)
        io_, yo_ = mlp.targets(ari, frac)
        assert np.array_equal(ti.cpu().numpy(), io_)
        assert np.allclose(ty.cpu().numpy(), yo_, rtol=1e-6)
    # per-graph thresholds
    b = gg.sbm_batch(4, n_max=2000)
    n, vbase = b["n"], b["vbase"]
    deltas = np.array([[9 + 7 * i, 900] for i in (3, 10, 0, 40)], np.int64)
    g = build(b["src"], b["dst"], n)
    t = M.mcd_triangles(g)
    keep, nk = M.mcd_prune_graphs(g, M.MCD_SIM_TECTONIC, t, cuda(deltas), cuda(vbase))
    lab, ncc = M.mcd_components(g, keep)
    _, _, order = canonical_order(g)
    kg = unpack_bits(keep, g.m)[order]
    lo, hi = oracle.canon(n, b["src"], b["dst"])
    deg = oracle.degrees(n, lo, hi)
    to = oracle.triangles(n, lo, hi)
    want = np.zeros(len(lo), np.uint8)
    eg = np.searchsorted(vbase, lo, side="right") - 1
    for k in range(4):
        want[eg == k] = oracle.prune(oracle.TECTONIC, lo, hi, to, deg, *deltas[k])[eg == k]
    assert np.array_equal(kg, want) and int(nk.item()) == int(want.sum())
    lab_o, ncc_o = oracle.components(n, lo, hi, want)
    assert np.array_equal(lab.cpu().numpy(), lab_o) and int(ncc.item()) == ncc_o
    # the same per-graph thresholds through the one-pass weights + prune and
    # components over its kept list
    f = M.mcd_weigh_prune(g, M.MCD_SIM_TECTONIC, t, deltas=cuda(deltas), vbase=cuda(vbase))
    assert np.array_equal(unpack_bits(f["keep_bits"], g.m)[order], want)
    assert int(f["n_kept"].item()) == int(want.sum())
    assert int(f["kept"].counts.sum().item()) == int(want.sum())
    lab2, ncc2 = M.mcd_components_kept(g, f["kept"])
    assert np.array_equal(lab2.cpu().numpy(), lab_o) and int(ncc2.item()) == ncc_o
    # and weights + prune + components in one pass
    pc = M.mcd_prune_components(g, M.MCD_SIM_TECTONIC, t, deltas=cuda(deltas), vbase=cuda(vbase))
    assert np.array_equal(unpack_bits(pc["keep_bits"], g.m)[order], want)
    assert int(pc["n_kept"].item()) == int(want.sum())
    assert np.array_equal(pc["labels"].cpu().numpy(), lab_o) and int(pc["n_components"].item()) == ncc_o


def test_feature_range_and_fallback_guard():
    # the training range and the out-of-range guard on feature rows built
    # around the bounds, against the oracle's fp32 decisions; the threshold
    # each row then uses
    from gpu_util import ctx
    rng = np.random.default_rng(11)
    xt = rng.random((20, M.MLP_IN)).astype(np.float32) * rng.random(M.MLP_IN).astype(np.float32) * 8
    lo_g, hi_g = M.mcd_feature_range(ctx(), cuda(xt))
    lo_o, hi_o = mlp.feature_range(xt)
    assert np.array_equal(lo_g.cpu().numpy(), lo_o) and np.array_equal(hi_g.cpu().numpy(), hi_o)
    margin = np.float32(0.25)
    w = margin * (hi_o - lo_o)
    up, down = hi_o + w, lo_o - w
    rows = [xt[0], xt[7], (lo_o + hi_o) / 2, up, down]
    for j in (0, 17, 65):
        for edge, away in ((up, np.float32(np.inf)), (down, np.float32(-np.inf))):
            r = (lo_o + hi_o) / 2
            r[j] = np.nextafter(edge[j], away)
            rows.append(r.copy())
    rows += list(rng.random((12, M.MLP_IN)).astype(np.float32) * 10)
    x = np.stack(rows).astype(np.float32)
    B = len(x)
    picked = np.stack([9 + 7 * np.arange(B), np.full(B, 900)], 1).astype(np.int64)
    fb = np.stack([np.arange(B), np.full(B, 50)], 1).astype(np.int64)
    flags, delta = M.mcd_picker_fallback(ctx(), cuda(x), lo_g, hi_g, float(margin), picked=cuda(picked),
                                         fallback=cuda(fb))
    fo = mlp.out_of_range(x, lo_o, hi_o, margin)
    assert fo[:5].tolist() == [0, 0, 0, 0, 0] and fo[5:11].tolist() == [1] * 6
    assert np.array_equal(flags.cpu().numpy(), fo)
    assert np.array_equal(delta.cpu().numpy(), mlp.choose_thresholds(fo, picked, fb))
    # the chosen thresholds written over the picked table itself
    pk = cuda(picked)
    M.mcd_picker_fallback(ctx(), cuda(x), lo_g, hi_g, float(margin), picked=pk, fallback=cuda(fb), delta=pk,
                          want_flags=False)
    assert np.array_equal(pk.cpu().numpy(), mlp.choose_thresholds(fo, picked, fb))


def test_picker_end_to_end_small_batch():
    # a reduced planted-partition batch: sweep -> targets -> train -> pick;
    # the picked labels are the oracle's at the picked thresholds, and the
    # trained picker's validation ARI is reported against two baselines
    from gpu_util import ctx, build
    from paper_2412_12382_amd import picker as PK
    G = 48
    b = gg.sbm_batch(G, n_max=6000)
    n, vbase = b["n"], cuda(b["vbase"])
    g = build(b["src"], b["dst"], n)
    t = M.mcd_triangles(g)
    stats, ari, _ = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, PK.GRID, vbase=vbase, truth=cuda(b["truth"]))
    idx, y = M.mcd_sweep_targets(ctx(), ari)
    x = M.mcd_features(g, t, vbase)
    gi = np.arange(G)
    tr, va = gi[gi % 4 != 3], gi[gi % 4 == 3]
    model, losses = PK.train(ctx(), x[torch.from_numpy(tr).cuda()].contiguous(),
                             y[torch.from_numpy(tr).cuda()].contiguous())
    assert losses[-1] < losses[0]
    index, deltas, labels, ncc, flags = PK.pick(g, t, model, vbase)
    A = ari.cpu().numpy()
    pi = index.cpu().numpy()
    picked = A[va, pi[va]].mean()
    best = A[va].max(1).mean()
    glob = A[va][:, np.argmax(A[tr].mean(0))].mean()
    print(f"small batch val ARI: picker {picked:.4f}  per-graph best {best:.4f}  best global {glob:.4f}")
    # the range guard: the oracle's own features of every graph, the range of
    # the training graphs' features, and its fp32 decision per graph
    lo, hi = oracle.canon(n, b["src"], b["dst"])
    deg = oracle.degrees(n, lo, hi)
    to = oracle.triangles(n, lo, hi)
    vb = b["vbase"]
    xo = []
    for k in range(G):
        sel = (lo >= vb[k]) & (lo < vb[k + 1])
        l2, h2 = (lo[sel] - vb[k]).astype(np.int32), (hi[sel] - vb[k]).astype(np.int32)
        nk = int(vb[k + 1] - vb[k])
        xo.append(mlp.features(nk, l2, h2, oracle.triangles(nk, l2, h2), oracle.degrees(nk, l2, h2)))
    xo = np.stack(xo).astype(np.float32)
    lo_f, hi_f = mlp.feature_range(xo[tr])
    flags_o = mlp.out_of_range(xo, lo_f, hi_f, PK.MARGIN)
    assert np.array_equal(flags.cpu().numpy(), flags_o)
    print(f"graphs out of the training range (fallback to the sweep's rule): {int(flags_o.sum())} of {G}")
    # labels equal the oracle's components at the threshold each graph used:
    # the network's grid point, or the oracle's own rule of thumb on its own
    # sweep with modularity where the guard fired; the GPU's index only
    # selects which of the oracle's results to compare with
    st_o, _, labels_o, q_o = oracle.sweep(n, lo, hi, to, deg, oracle.TECTONIC, PK.GRID, vbase=vb,
                                          modularity=True)
    rule_o = np.asarray(oracle.rule_of_thumb(st_o, PK.GRID, vb, q_o))
    chosen = np.where(flags_o == 1, rule_o, pi)
    got = labels.cpu().numpy()
    for k in range(G):
        assert np.array_equal(got[vb[k]:vb[k + 1]], labels_o[chosen[k], vb[k]:vb[k + 1]]), k
        assert tuple(deltas.cpu().numpy()[k]) == PK.GRID[chosen[k]]
    assert int(ncc.item()) == sum(int(np.count_nonzero(labels_o[chosen[k], vb[k]:vb[k + 1]] ==
                                                      np.arange(vb[k], vb[k + 1]))) for k in range(G))
    # forced fallback: every graph takes the rule of thumb
    _, dforce, lforce, _, _ = PK.pick(g, t, model, vbase, fallback="force")
    for k in range(G):
        assert tuple(dforce.cpu().numpy()[k]) == PK.GRID[rule_o[k]], k
        assert np.array_equal(lforce.cpu().numpy()[vb[k]:vb[k + 1]], labels_o[rule_o[k], vb[k]:vb[k + 1]]), k


def test_picker_gain_on_planted_batch():
    # the 256-graph planted-partition batch: train on graphs g % 4 != 3, score
    # the 64 others; the learned per-graph threshold must beat the best single
    # global threshold chosen on the training graphs (the method without it)
    from gpu_util import ctx, build
    from paper_2412_12382_amd import picker as PK
    b = gg.sbm_batch(256)
    vb = cuda(b["vbase"])
    g = build(b["src"], b["dst"], b["n"])
    t = M.mcd_triangles(g)
    _, ari, _ = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, PK.GRID, vbase=vb, truth=cuda(b["truth"]))
    _, y = M.mcd_sweep_targets(ctx(), ari)
    x = M.mcd_features(g, t, vb)
    gi = np.arange(256)
    tr, va = gi[gi % 4 != 3], gi[gi % 4 == 3]
    model, losses = PK.train(ctx(), x[cuda(tr)].contiguous(), y[cuda(tr)].contiguous())
    index, _, _, _, _ = PK.pick(g, t, model, vb)
    A = ari.cpu().numpy()
    pi = index.cpu().numpy()
    picked = A[va, pi[va]].mean()
    best = A[va].max(1).mean()
    glob = A[va][:, np.argmax(A[tr].mean(0))].mean()
    print(f"planted batch val ARI: picker {picked:.4f}  per-graph best {best:.4f}  best global {glob:.4f}")
    assert picked > glob + 0.05
    assert losses[-1] < 0.1 * losses[0]


def _he_uniform_expected(seed):
    """The documented initial weights: weight i of a layer with fan-in f is
    (2 u_i - 1) sqrt(6/f) in fp64, rounded to fp32, u_i the input module's
    Philox uniform of counter i under (seed, "MLP0"); biases zero."""
    import math
    u = gg.uniforms(seed, 0x4D4C5030, mlp.NPAR)
    p = np.zeros(mlp.NPAR, np.float32)
    o = 0
    for fan_out, fan_in in ((64, 66), (64, 64), (1, 64)):
        k = fan_out * fan_in
        p[o:o + k] = ((2.0 * u[o:o + k] - 1.0) * math.sqrt(6.0 / fan_in)).astype(np.float32)
        o += k + fan_out
    return p


def test_picker_object_initial_weights():
    from gpu_util import ctx
    for seed in (0, 7, 2**40 + 3):
        h = M.mcd_picker_create(ctx(), seed)
        st = M.mcd_picker_export(h)
        want = _he_uniform_expected(seed)
        assert np.array_equal(st["params"].cpu().numpy().view(np.int32), want.view(np.int32)), seed
        assert st["margin"] == np.float32(0.25)


def test_picker_fit_equals_the_step_sequence():
    # mcd_picker_fit = standardisation + range + Adam steps from the seeded
    # weights: the same kernels called one by one give the same bits
    from gpu_util import ctx
    B, steps, lr, wd = 24, 5, 3e-3, 1.0
    rng = np.random.default_rng(11)
    x = cuda(rng.uniform(0, 1, (B, mlp.NI)).astype(np.float32))
    y = cuda(rng.uniform(0, 1, B).astype(np.float32))
    h = M.mcd_picker_create(ctx(), 5)
    losses = M.mcd_picker_fit(h, x, y, steps, lr, wd, 1.0, 0.25)
    got = M.mcd_picker_export(h)
    params = cuda(_he_uniform_expected(5))
    m1, m2 = torch.zeros_like(params), torch.zeros_like(params)
    mean, std = M.mcd_feature_stats(ctx(), x, 1.0)
    lo, hi = M.mcd_feature_range(ctx(), x)
    ref_losses = []
    for s in range(1, steps + 1):
        ref_losses.append(M.mcd_mlp_train_step(ctx(), params, m1, m2, s, lr, mean, std, x, y, weight_decay=wd).item())
    assert torch.equal(got["params"], params) and torch.equal(got["mean"], mean) and torch.equal(got["std"], std)
    assert torch.equal(got["lo"], lo) and torch.equal(got["hi"], hi)
    assert losses.cpu().numpy().tolist() == ref_losses


def test_picker_checkpoint_save_load_pick_identical(tmp_path):
    # save -> load -> pick equals the in-memory pick bit for bit; a corrupted
    # file is refused and leaves the loading picker untouched
    from gpu_util import ctx, build
    from paper_2412_12382_amd import picker as PK
    G = 32
    b = gg.sbm_batch(G, n_max=5000)
    vbase = cuda(b["vbase"])
    g = build(b["src"], b["dst"], b["n"])
    t = M.mcd_triangles(g)
    _, ari, _ = M.mcd_sweep(g, M.MCD_SIM_TECTONIC, t, PK.GRID, vbase=vbase, truth=cuda(b["truth"]))
    _, y = M.mcd_sweep_targets(ctx(), ari)
    x = M.mcd_features(g, t, vbase)
    model, _ = PK.train(ctx(), x[: G // 2].contiguous(), y[: G // 2].contiguous(), steps=300)
    path = str(tmp_path / "picker.ckpt")
    model.save(path)
    M.mcd_picker_check_file(path)
    loaded = PK.load(ctx(), path)
    for mode in ("auto", "force", "off"):
        a = PK.pick(g, t, model, vbase, fallback=mode)
        c = PK.pick(g, t, loaded, vbase, fallback=mode)
        for u, v in zip(a, c):
            assert torch.equal(u, v), mode
    for k in ("params", "mean", "std", "lo", "hi"):
        assert torch.equal(getattr(model, k), getattr(loaded, k)), k
    # import of the exported state picks the same
    other = M.mcd_picker_create(ctx(), 99)
    M.mcd_picker_import(other, model.params, model.mean, model.std, model.lo, model.hi, model.margin)
    a = PK.pick(g, t, model, vbase)
    c = M.mcd_picker_pick(other, g, M.MCD_SIM_TECTONIC, t, vbase=vbase)
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1]) and torch.equal(a[2], c[3])
    # a corrupted checkpoint: refused, the picker keeps its state
    data = bytearray(open(path, "rb").read())
    data[64 + 4 * 1000] ^= 1
    bad = str(tmp_path / "bad.ckpt")
    open(bad, "wb").write(bytes(data))
    before = M.mcd_picker_export(loaded.handle)
    with pytest.raises(M.MCDError) as ei:
        M.mcd_picker_load(loaded.handle, bad)
    assert ei.value.status == -9
    after = M.mcd_picker_export(loaded.handle)
    for k in ("params", "mean", "std", "lo", "hi"):
        assert torch.equal(before[k], after[k]), k
