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
