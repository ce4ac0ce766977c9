"""Pins of the MLP parity tolerance (tests/mlp_bound.py) on the CPU: the
derived bound covers an fp32 evaluation of the network and its gradient, and
it is tight enough to reject plausible mistakes planted in the float64
reference (through its inputs)."""
import numpy as np
import pytest

import mlp_bound as mb
from oracle import mlp

F = np.float32


def rand_problem(seed, B):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.NPAR).astype(F)
    x = rng.normal(0, 1, (B, mlp.NI)).astype(F)
    mean = rng.normal(0, 0.1, mlp.NI).astype(F)
    std = rng.uniform(0.5, 2.0, mlp.NI).astype(F)
    target = rng.uniform(0, 1, B).astype(F)
    return p, mean, std, x, target


def fp32_network(p, mean, std, x, target, ari=None, mse_w=1.0):
    """The network, loss slope and gradient evaluated in fp32 throughout
    (numpy's single-precision products and sums, any order)."""
    P = {k: v.astype(F) for k, v in mlp.unpack(p).items()}
    xs = (x.astype(F) - mean.astype(F)) / std.astype(F)
    a1 = xs @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, F(0))
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, F(0))
    y = h2 @ P["W3"] + P["b3"][0]
    B = len(y)
    dl = F(2 * mse_w) * (y - target.astype(F))
    if ari is not None:
        K = ari.shape[1]
        z = np.clip(F(K - 1) * y, F(0), F(K - 1))
        i0 = np.minimum(np.floor(z).astype(np.int64), K - 2)
        r = np.arange(B)
        a0, a1v = ari[r, i0].astype(F), ari[r, i0 + 1].astype(F)
        inside = (F(K - 1) * y > 0) & (F(K - 1) * y < F(K - 1))
        dl = dl - np.where(inside, F(K - 1) * (a1v - a0), F(0))
    dy = (dl / F(B)).astype(F)
    dh2 = np.outer(dy, P["W3"]) * (h2 > 0)
    dh1 = (dh2 @ P["W2"]) * (h1 > 0)
    g = {"W3": dy @ h2, "b3": np.array([dy.sum()], F), "W2": dh2.T @ h1, "b2": dh2.sum(0),
         "W1": dh1.T @ xs, "b1": dh1.sum(0)}
    for v in g.values():
        assert v.dtype == F
    return y.astype(np.float64), mlp.pack(g)


def f64(*a):
    return [np.asarray(v, np.float64) for v in a]


@pytest.mark.parametrize("B", [1, 7, 192])
def test_bound_covers_an_fp32_evaluation(B):
    p, mean, std, x, target = rand_problem(100 + B, B)
    keep = mb.rows_with_clear_masks(p, mean, std, x)
    assert keep.sum() >= max(1, int(0.9 * B))
    x, target = x[keep], target[keep]
    y32, g32 = fp32_network(p, mean, std, x, target)
    P, M, S = f64(p, mean, std)
    y64, _ = mlp.forward(P, M, S, x)
    g64, _ = mlp.gradient(P, M, S, x, target.astype(np.float64))
    assert np.all(np.abs(y32 - y64) <= mb.forward_bound(p, mean, std, x))
    assert np.all(np.abs(g32 - g64) <= mb.gradient_bound(p, mean, std, x, target))
    # the empirical tolerance holds with at least twice its size to spare
    emp = mb.empirical_tolerance(g64, mb.row_abs_mean(p, mean, std, x, target), len(x))
    assert np.all(np.abs(g32 - g64) <= 0.5 * emp)


def test_bound_covers_an_fp32_evaluation_with_ari():
    B = 64
    p, mean, std, x, target = rand_problem(7, B)
    p[8448:8512] *= 0.02
    P, M, S = f64(p, mean, std)
    yo, _ = mlp.forward(P, M, S, x)
    p[8512] += F(0.5 - np.median(yo))
    P = np.asarray(p, np.float64)
    yo, _ = mlp.forward(P, M, S, x)
    z, zb = 63 * yo, mb.grid_position_bound(p, mean, std, x, 64)
    keep = (z > zb) & (z < 63 - zb) & (np.abs(z - np.round(z)) > zb)
    keep &= mb.rows_with_clear_masks(p, mean, std, x)
    x, target = x[keep], target[keep]
    assert len(x) >= 40
    ari = np.random.default_rng(8).uniform(-0.1, 1.0, (len(x), 64))
    _, g32 = fp32_network(p, mean, std, x, target, ari, 0.1)
    g64, _ = mlp.gradient(P, M, S, x, target.astype(np.float64), ari, 0.1)
    assert np.all(np.abs(g32 - g64) <= mb.gradient_bound(p, mean, std, x, target, ari, 0.1))
    emp = mb.empirical_tolerance(g64, mb.row_abs_mean(p, mean, std, x, target, ari, 0.1), len(x))
    assert np.all(np.abs(g32 - g64) <= 0.5 * emp)


def test_bound_rejects_planted_mistakes():
    # each mistake is planted in the float64 reference through its inputs; the
    # correct fp32 evaluation must fall outside the a priori bound for gross
    # mistakes and outside the empirical tolerance for slight ones
    B = 192
    p, mean, std, x, target = rand_problem(5, B)
    keep = mb.rows_with_clear_masks(p, mean, std, x)
    x, target = x[keep], target[keep]
    y32, g32 = fp32_network(p, mean, std, x, target)
    fb = mb.forward_bound(p, mean, std, x)
    gb = mb.gradient_bound(p, mean, std, x, target)
    P, M, S = f64(p, mean, std)
    T = target.astype(np.float64)
    W2 = slice(64 * 66 + 64, 64 * 66 + 64 + 64 * 64)

    def outside(P_, M_, S_):
        y, _ = mlp.forward(P_, M_, S_, x)
        g, _ = mlp.gradient(P_, M_, S_, x, T)
        emp = mb.empirical_tolerance(g, mb.row_abs_mean(P_, M_, S_, x, T), len(x))
        return (np.any(np.abs(y32 - y) > fb) or np.any(np.abs(g32 - g) > gb), np.any(np.abs(g32 - g) > emp))

    assert outside(P, M, S) == (False, False)
    m = M.copy(); m[64] = -m[64]                       # x + mean in the degree-ratio column
    assert outside(P, m, S) == (True, True)
    s = S.copy(); s[65] = 1.0                          # max-degree column left unscaled
    assert outside(P, M, s) == (True, True)
    q = P.copy(); q[W2] = q[W2].reshape(64, 64).T.reshape(-1)   # W2 transposed
    assert outside(q, M, S) == (True, True)
    q = P.copy(); q[-1] = 0.0                          # b3 dropped
    assert outside(q, M, S) == (True, True)
    s = S.copy(); s[65] *= 1 + 1e-2                    # its scale off by 1 %
    assert outside(P, M, s) == (True, True)
    # slight: within the a priori bound, caught by the empirical tolerance
    s = S.copy(); s[65] *= 1 + 3e-4                    # a scale off by 0.03 %
    assert outside(P, M, s) == (False, True)
    m = M.copy(); m[3] += 1e-4                         # a mean off by 1e-4
    assert outside(P, m, S) == (False, True)


def test_gamma_and_depths():
    # gamma_k from its definition, and the depth rules of the module header
    assert mb.gamma(1, 2.0 ** -24) == 2.0 ** -24 / (1 - 2.0 ** -24)
    xs = 2
    a1 = xs + 1 + 66
    a2 = a1 + 1 + 64
    y = a2 + 1 + 6 + 1
    dy = y + 1 + 2 + 1 + 1
    assert (mb.DEPTH_A1, mb.DEPTH_A2, mb.DEPTH_Y) == (a1, a2, y)
    assert mb.DEPTH_GRAD == {"W3": dy + a2 + 1, "b3": dy, "W2": dy + 1 + a1 + 1, "b2": dy + 1,
                             "W1": dy + 1 + 1 + 64 + xs + 1, "b1": dy + 1 + 1 + 64}
