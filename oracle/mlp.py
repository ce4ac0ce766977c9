"""Float64 reference of the learned threshold picker (test infrastructure).

A plain numpy statement of the network and its training rule:
  y = W3 . relu(W2 relu(W1 xs + b1) + b2) + b3,   xs = (x - mean) / std,
  L = (1/B) sum_r [mse_w (y_r - target_r)^2 - A_r((K-1) y_r)]
  (A_r: the row's ARI curve over the threshold grid, linearly interpolated;
  without it, mse_w = 1 gives the plain squared error),
  Adam (Kingma & Ba, ICLR 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
  p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
Parameters are one flat vector: W1[64][66], b1[64], W2[64][64], b2[64], W3[64], b3.
The GPU library shares no code with this file.
"""
import numpy as np

NI, NH = 66, 64
SIZES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
NPAR = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SIZES:
        k = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + k], np.float64).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, mean, std, x):
    P = unpack(p)
    xs = (np.asarray(x, np.float64) - mean) / std
    a1 = xs @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ P["W3"] + P["b3"][0]
    return y, (xs, a1, h1, a2, h2)


def row_loss(y, target, ari=None, mse_w=1.0):
    """Per-row training loss and its derivative in y:
        mse_w (y - target)^2 - A_r((K-1) y),
    A_r the row's ARI curve over the K grid thresholds, interpolated linearly
    at z clamped to [0, K-1] (slope 0 outside 0 < z < K-1).  The segment
    index is decided in fp32, the precision of the network output, as on the
    GPU; the value and slope are formed in fp64."""
    y = np.asarray(y, np.float64)
    d = y - np.asarray(target, np.float64)
    L = mse_w * d * d
    g = 2.0 * mse_w * d
    if ari is not None:
        ari = np.asarray(ari, np.float64)
        K = ari.shape[1]
        zy32 = np.float32(K - 1) * y.astype(np.float32)
        z32 = np.clip(zy32, np.float32(0), np.float32(K - 1))
        i0 = np.minimum(np.floor(z32).astype(np.int64), K - 2)
        rows = np.arange(len(y))
        a0, a1 = ari[rows, i0], ari[rows, i0 + 1]
        z = np.clip((K - 1) * y, 0.0, K - 1.0)
        L = L - (a0 + (z - i0) * (a1 - a0))
        inside = (zy32 > 0) & (zy32 < np.float32(K - 1))
        g = g - np.where(inside, (K - 1) * (a1 - a0), 0.0)
    return L, g


def loss(p, mean, std, x, target, ari=None, mse_w=1.0):
    y, _ = forward(p, mean, std, x)
    return float(np.mean(row_loss(y, target, ari, mse_w)[0]))


def gradient(p, mean, std, x, target, ari=None, mse_w=1.0):
    """Analytic gradient of the loss (chain rule, ReLU derivative 1 iff > 0)."""
    P = unpack(p)
    y, (xs, a1, h1, a2, h2) = forward(p, mean, std, x)
    B = len(y)
    rl, dl = row_loss(y, target, ari, mse_w)
    dy = dl / B
    g = {"W3": dy @ h2, "b3": np.array([dy.sum()])}
    dh2 = np.outer(dy, P["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ P["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ xs
    g["b1"] = dh1.sum(0)
    return pack(g), float(np.mean(rl))


def adam_step(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return p, m, v


def feature_stats(x):
    x = np.asarray(x, np.float64)
    mu = x.mean(0)
    sd = x.std(0)
    return mu, np.where(sd > 1e-12, sd, 1.0)


def features(n, lo, hi, t, deg):
    """Picker inputs of one graph: fraction of edges per Tectonic bin
    floor(128 t / D) (64 bins on [0, 1/2)), log1p(2m/n), log1p(max degree)."""
    from . import histogram
    h = histogram(lo, hi, t, deg).astype(np.float64)
    m = len(lo)
    x = np.zeros(NI)
    x[:64] = h / m if m else 0.0
    x[64] = np.log1p(2.0 * m / n) if n else 0.0
    x[65] = np.log1p(deg.max() if len(deg) else 0)
    return x


def targets(ari, frac=0.95):
    """Centroid c of the thresholds with ARI >= best - (1 - frac)|best|;
    returns (index = round half down of c, y = c / (K - 1))."""
    ari = np.asarray(ari, np.float64)
    K = ari.shape[1]
    idx = np.zeros(ari.shape[0], np.int64)
    y = np.zeros(ari.shape[0])
    for g, row in enumerate(ari):
        best = row.max()
        sel = np.nonzero(row >= best - (1 - frac) * abs(best))[0]
        s, c = int(sel.sum()), len(sel)
        idx[g] = (2 * s + c - 1) // (2 * c)
        y[g] = s / c / (K - 1)
    return idx, y


def select(y, K, a, b, c):
    """Grid snap i = clamp(round((K-1) y), 0, K-1) (round half to even), delta =
    (a+b i)/c.  The product is rounded in fp32, the precision of the network
    output, so both sides take the integer decision in the same precision."""
    q = np.float32(K - 1) * np.asarray(y, np.float32)
    i = np.clip(np.rint(q), 0, K - 1).astype(np.int64)
    return i, np.stack([a + b * i, np.full_like(i, c)], 1)


def feature_range(x):
    """Column minimum and maximum of the training features."""
    x = np.asarray(x, np.float32)
    return x.min(0), x.max(0)


def out_of_range(x, lo, hi, margin):
    """Guard of the learned threshold (the sweep is its fallback): a graph is
    flagged when some feature lies outside [lo - margin w, hi + margin w],
    w = hi - lo.  Each bound is formed in fp32 with one rounding per
    operation, the precision of the features, so both sides take the same
    decision."""
    x = np.asarray(x, np.float32)
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    w = np.float32(margin) * (hi - lo)
    below = x < (lo - w)
    above = x > (hi + w)
    return (below | above).any(1).astype(np.int32)


def choose_thresholds(flags, picked, fallback):
    """Per graph: the fallback's threshold where flagged, else the picked one."""
    flags = np.asarray(flags).astype(bool)
    return np.where(flags[:, None], np.asarray(fallback), np.asarray(picked))
