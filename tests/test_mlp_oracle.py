"""Pins for the float64 picker reference: central differences, Adam's first
step in closed form, targets and snapping on hand-made cases."""
import numpy as np

from oracle import mlp


def rand_problem(seed, B=7):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.NPAR)
    x = rng.normal(0, 1, (B, mlp.NI))
    mean, std = rng.normal(0, 0.1, mlp.NI), rng.uniform(0.5, 2.0, mlp.NI)
    target = rng.uniform(0, 1, B)
    return p, mean, std, x, target


def test_gradient_central_differences():
    p, mean, std, x, target = rand_problem(0)
    g, _ = mlp.gradient(p, mean, std, x, target)
    rng = np.random.default_rng(1)
    h = 1e-6
    for q in rng.choice(mlp.NPAR, 200, replace=False).tolist() + [mlp.NPAR - 1]:
        e = np.zeros(mlp.NPAR)
        e[q] = h
        num = (mlp.loss(p + e, mean, std, x, target) - mlp.loss(p - e, mean, std, x, target)) / (2 * h)
        assert abs(num - g[q]) <= 1e-6 * max(abs(num), 1.0), (q, num, g[q])


def test_adam_first_step_is_signed_lr():
    # after one step from zero moments: m/(1-b1) = g, v/(1-b2) = g^2, so the
    # update is lr * g / (|g| + eps)
    p = np.zeros(5)
    g = np.array([3.0, -0.5, 1e-3, -2e-2, 0.0])
    p1, m, v = mlp.adam_step(p, np.zeros(5), np.zeros(5), g, 1, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    p, mean, std, x, target = rand_problem(2, B=32)
    m, v = np.zeros_like(p), np.zeros_like(p)
    l0 = mlp.loss(p, mean, std, x, target)
    for s in range(1, 201):
        g, _ = mlp.gradient(p, mean, std, x, target)
        p, m, v = mlp.adam_step(p, m, v, g, s, 1e-3)
    assert mlp.loss(p, mean, std, x, target) < 0.1 * l0


def test_targets_and_select():
    ari = np.array([[0.1, 0.5, 0.5, 0.5, 0.2, 0.5],
                    [0.9, 0.1, 0.2, 0.3, 0.4, 0.5],
                    [0.0, 0.0, 0.3, 0.3, 0.0, 0.0]])
    # exact maxima (frac 1): centroids 2.75 -> 3, 0, 2.5 -> 2 (half rounds down)
    assert mlp.targets(ari, 1.0)[0].tolist() == [3, 0, 2]
    # within 20% of the best: row 0 keeps 0.5s (0.4 cut), row 1 only 0.9, row 2 the 0.3s
    assert mlp.targets(ari, 0.8)[0].tolist() == [3, 0, 2]
    assert np.allclose(mlp.targets(ari, 1.0)[1], np.array([2.75, 0, 2.5]) / 5)
    i, d = mlp.select([-0.2, 0.0, 0.49, 0.5, 1.7], 64, 9, 7, 900)
    assert i.tolist() == [0, 0, 31, 32, 63]
    assert d[1].tolist() == [9, 900] and d[4].tolist() == [9 + 7 * 63, 900]


def test_range_guard_hand_cases():
    # training range [0, 1] and [0, 2], margin 1/4: bounds [-1/4, 5/4] and
    # [-1/2, 5/2] (exact in fp32); the bounds themselves are inside
    train = np.array([[0.0, 2.0], [1.0, 0.0], [0.5, 1.0]], np.float32)
    lo, hi = mlp.feature_range(train)
    assert lo.tolist() == [0.0, 0.0] and hi.tolist() == [1.0, 2.0]
    x = np.array([[1.25, 2.5], [np.nextafter(np.float32(1.25), np.float32(2)), 0.0], [-0.5, -0.5],
                  [0.0, np.nextafter(np.float32(-0.5), np.float32(-1))], [0.5, 1.0], [-0.25, 0.0]], np.float32)
    assert mlp.out_of_range(x, lo, hi, 0.25).tolist() == [0, 1, 1, 1, 0, 0]
    # margin 0: exactly the training range; training rows are never out of it
    assert mlp.out_of_range(x, lo, hi, 0.0).tolist() == [1, 1, 1, 1, 0, 1]
    assert mlp.out_of_range(train, lo, hi, 0.0).tolist() == [0, 0, 0]
    picked = np.array([[9, 900]] * 6)
    fb = np.array([[k, 50] for k in range(6)])
    got = mlp.choose_thresholds(mlp.out_of_range(x, lo, hi, 0.25), picked, fb)
    assert got.tolist() == [[9, 900], [1, 50], [2, 50], [3, 50], [9, 900], [9, 900]]


def _flat(kind, i, j=0):
    """Index of one parameter in the flat vector, from the documented layout
    W1[64][66], b1[64], W2[64][64], b2[64], W3[64], b3 (row-major, output
    index first)."""
    return {"W1": i * 66 + j, "b1": 4224 + i, "W2": 4288 + i * 64 + j, "b2": 8384 + i, "W3": 8448 + i,
            "b3": 8512}[kind]


def test_forward_hand_computed_sparse_network():
    # a network with a handful of nonzero weights, evaluated by hand; every
    # value is dyadic, so the fp64 forward must reproduce it exactly.  The
    # standardisation (x - mean)/std, both ReLUs, the orientation of W2 and
    # the flat layout all change the result if mistaken.
    p = np.zeros(mlp.NPAR)
    for (k, i, j), val in {("W1", 0, 3): 1.5, ("W1", 0, 65): 0.5, ("b1", 0, 0): -1.0, ("W1", 1, 3): -1.0,
                           ("b1", 1, 0): 0.5, ("W1", 2, 65): 1.0, ("W2", 0, 0): 1.0, ("W2", 0, 2): 2.0,
                           ("W2", 2, 0): -7.0, ("b2", 0, 0): -0.5, ("W2", 1, 1): 5.0, ("b2", 1, 0): 0.25,
                           ("W3", 0, 0): 2.0, ("W3", 1, 0): -4.0, ("W3", 2, 0): 3.0, ("b3", 0, 0): 0.125}.items():
        p[_flat(k, i, j)] = val
    assert mlp.NPAR == 8513
    mean, std = np.zeros(mlp.NI), np.ones(mlp.NI)
    mean[3], std[3], mean[65], std[65] = 1.0, 2.0, -2.0, 4.0
    x = np.zeros((2, mlp.NI))
    x[0, 3], x[0, 65] = 5.0, 6.0   # standardised: 2, 2
    x[1, 3], x[1, 65] = 1.0, -2.0  # standardised: 0, 0
    # row 0: a1 = (1.5*2 + 0.5*2 - 1, -1*2 + 0.5, 1*2) = (3, -1.5, 2) -> h1 = (3, 0, 2)
    #        a2 = (3 + 2*2 - 0.5, 5*0 + 0.25, -7*3) = (6.5, 0.25, -21) -> h2 = (6.5, 0.25, 0)
    #        y = 2*6.5 - 4*0.25 + 3*0 + 0.125 = 12.125
    # row 1: a1 = (-1, 0.5, 0) -> h1 = (0, 0.5, 0); a2 = (-0.5, 2.75, 0) -> h2 = (0, 2.75, 0)
    #        y = -4*2.75 + 0.125 = -10.875
    y, _ = mlp.forward(p, mean, std, x)
    assert y.tolist() == [12.125, -10.875]


def _features_of(n, edges):
    import oracle
    e = np.array(sorted((min(a, b), max(a, b)) for a, b in edges), np.int32).reshape(-1, 2)
    lo, hi = e[:, 0].copy(), e[:, 1].copy()
    deg = oracle.degrees(n, lo, hi)
    t = oracle.triangles(n, lo, hi)
    return mlp.features(n, lo, hi, t, deg)


def test_features_on_complete_graph_and_star():
    import math
    # K5 (+ 3 isolated vertices): t = 3, deg u + deg v = 8 on every edge, so
    # every edge falls in bin floor(128*3/8) = 48; 2m/n = 20/8, max degree 4
    x = _features_of(8, [(a, b) for a in range(5) for b in range(a + 1, 5)])
    want = np.zeros(mlp.NI)
    want[48] = 1.0
    want[64], want[65] = math.log(3.5), math.log(5.0)
    assert np.allclose(x, want, rtol=1e-15, atol=0)
    # star with 7 leaves: no triangles, every edge in bin 0; 2m/n = 14/8, max degree 7
    x = _features_of(8, [(0, k) for k in range(1, 8)])
    want = np.zeros(mlp.NI)
    want[0] = 1.0
    want[64], want[65] = math.log(2.75), math.log(8.0)
    assert np.allclose(x, want, rtol=1e-15, atol=0)
    # the wheel W5 (hub 0, rim 1..5): rim edges t = 1, D = 6 -> bin 21; spokes
    # t = 2, D = 8 -> bin 32; 2m/n = 20/6, max degree 5
    rim = [(k, k % 5 + 1) for k in range(1, 6)]
    x = _features_of(6, [(0, k) for k in range(1, 6)] + rim)
    want = np.zeros(mlp.NI)
    want[21], want[32] = 0.5, 0.5
    want[64], want[65] = math.log1p(20 / 6), math.log(6.0)
    assert np.allclose(x, want, rtol=1e-15, atol=0)


def test_ari_loss_hand_cases():
    # three grid thresholds with ARI 0.1, 0.5, 0.3; mse weight 0.25, target 0.5
    ari = np.array([[0.1, 0.5, 0.3]] * 4)
    y = np.array([0.25, 0.75, -0.5, 1.2])
    L, g = mlp.row_loss(y, np.full(4, 0.5), ari, mse_w=0.25)
    # z = 2y: 0.5 -> 0.1 + 0.5 * 0.4 = 0.3, slope 2 * 0.4; 1.5 -> 0.5 - 0.5 * 0.2 = 0.4,
    # slope -2 * 0.2; -1 and 2.4 clamp to the ends (0.1 and 0.3) with slope 0
    assert np.allclose(L, 0.25 * (y - 0.5) ** 2 - np.array([0.3, 0.4, 0.1, 0.3]), rtol=0, atol=1e-15)
    assert np.allclose(g, 0.5 * (y - 0.5) - np.array([0.8, -0.4, 0.0, 0.0]), rtol=0, atol=1e-15)
    # without a table: the squared error alone
    L0, g0 = mlp.row_loss(y, np.full(4, 0.5))
    assert np.array_equal(L0, (y - 0.5) ** 2) and np.array_equal(g0, 2 * (y - 0.5))


def test_ari_loss_gradient_central_differences():
    # away from the grid points the loss is smooth: central differences of the
    # whole network's loss match the analytic gradient
    p, mean, std, x, target = rand_problem(3, B=24)
    rng = np.random.default_rng(4)
    ari = rng.uniform(-0.1, 1.0, (24, 64))
    # rescale the last layer so that (K-1) y spreads over (0, 63)
    p = p.copy()
    y, _ = mlp.forward(p, mean, std, x)
    sd = np.std(y) if np.std(y) > 0 else 1.0
    p[8448:8512] *= (10.0 / 63) / sd
    y, _ = mlp.forward(p, mean, std, x)
    p[8512] += 0.5 - np.median(y)
    y, _ = mlp.forward(p, mean, std, x)
    z = 63 * y
    keep = (z > 0.01) & (z < 62.99) & (np.abs(z - np.round(z)) > 0.01)
    x, target, ari = x[keep], target[keep], ari[keep]
    assert len(x) >= 8
    g, _ = mlp.gradient(p, mean, std, x, target, ari, mse_w=0.1)
    h = 1e-7
    for q in rng.choice(mlp.NPAR, 200, replace=False).tolist() + [mlp.NPAR - 1]:
        e = np.zeros(mlp.NPAR)
        e[q] = h
        num = (mlp.loss(p + e, mean, std, x, target, ari, 0.1) - mlp.loss(p - e, mean, std, x, target, ari, 0.1)) / (2 * h)
        assert abs(num - g[q]) <= 1e-5 * max(abs(num), 1.0), (q, num, g[q])
